"""Pins of the oracle's axis-aligned perfectly matched layers (paper Sec. 3.3):
the anisotropic element matrix against brute-force quadrature, and the
stretched plane wave e^{ik x~(x)} (which decays through the layers as
e^{-int sigma}) as an exact solution of the layered problem."""
import numpy as np

import workloads as W
from oracle import dp_elementwise as dpe
from oracle import element as el
from oracle import problem as pb
from test_oracle_element import basis_np
import numpy.polynomial.legendre as npl


def brute_aniso(n, hx, hy, axx, ayy, beta):
    """int of axx psi_x phi_x + ayy psi_y phi_y + beta psi phi over [0,hx]x[0,hy]
    by tensor Gauss quadrature (x index fastest)."""
    u, w = npl.leggauss(n + 3)
    N, dN = basis_np(u, n)
    Jx, Jy = hx / 2, hy / 2
    A = np.zeros((n * n, n * n), complex)
    for qi in range(len(u)):
        for qj in range(len(u)):
            phi = np.kron(N[:, qj], N[:, qi])
            dx = np.kron(N[:, qj], dN[:, qi]) / Jx
            dy = np.kron(dN[:, qj], N[:, qi]) / Jy
            wt = w[qi] * w[qj] * Jx * Jy
            A += wt * (axx * np.outer(dx, dx) + ayy * np.outer(dy, dy) + beta * np.outer(phi, phi))
    return A


def test_anisotropic_element_matrix_matches_quadrature():
    """alpha = diag(s_y/s_x, s_x/s_y) on a non-square element: a swapped axis or
    a dropped factor changes the matrix."""
    n, hx, hy, k = 6, 0.3, 0.7, 9.0
    sx, sy = 1 + 0.8j, 1 + 0.3j
    axx, ayy, beta = sy / sx, sx / sy, -k ** 2 * 2.0 * sx * sy
    A = el.element_matrix(n, hx, hy, alpha=(axx, ayy), beta=beta)
    assert np.allclose(A, brute_aniso(n, hx, hy, axx, ayy, beta), atol=1e-12)
    assert not np.allclose(A, brute_aniso(n, hx, hy, ayy, axx, beta), atol=1e-6)


def _layered_channel(nx_phys, n_pml, ny, p, k, sigma):
    """[0, (nx_phys + n_pml) h] x [0, ny h] with h = 1/8, layers in the last n_pml
    element columns with sigma_x graded per column, sigma_y = 0."""
    h = 1.0 / 8
    nx = nx_phys + n_pml
    leaves = W.morton_leaves(nx, ny)
    sig = np.zeros((len(leaves), 2))
    for e, (_, ix, iy) in enumerate(leaves):
        if ix >= nx_phys:
            sig[e, 0] = sigma * ((ix - nx_phys + 1) / n_pml) ** 2
    return dict(domain=(0.0, nx * h, 0.0, ny * h), base=(nx, ny), leaves=leaves, degree=np.full(len(leaves), p),
                k=k, eps_r=np.ones(len(leaves)), bc="impedance", l=2, pml_sigma=sig,
                rhs=dict(kind="none")), h


def _stretched_wave(w, h, nx_phys, k):
    """x~(x) = int_0^x s_x: x in the physical part, then s_x of each column times
    the distance covered in it; u = e^{ik x~} solves the layered equation with
    the flux alpha_xx u_x = ik u continuous across columns."""
    sig = np.asarray(w["pml_sigma"])
    col_s = {}
    for e, (_, ix, iy) in enumerate(w["leaves"]):
        col_s[ix] = 1 + 1j * sig[e, 0] / k

    def xt(x):
        out = np.zeros_like(x, dtype=complex)
        for i, xv in np.ndenumerate(x):
            col = min(int(xv / h), max(col_s))
            acc = sum(col_s[c] * h for c in range(col))
            out[i] = acc + col_s[col] * (xv - col * h)
        return out

    return lambda x, y: np.exp(1j * k * xt(np.asarray(x, float)))


def _manufactured_loads(disc, u, k):
    """Impedance data q = ik(d.n - 1) u with d = (1, 0) on the outer sides: the
    flux alpha grad(u).n equals ik (d.n) u for the stretched wave (alpha_xx u_x =
    ik u, alpha_yy u_y = 0)."""
    m = disc.mesh
    loads = []
    for e in range(m.E):
        n = int(disc.degrees[e]) + 1
        b = np.zeros(n * n, complex)
        for side in (1, 2, 3, 4):
            if not m.boundary_side(e, side):
                continue
            xy, h_edge = pb.edge_param(m, e, side)
            dn = pb.NORMALS[side][0]

            def q(s, xy=xy, dn=dn):
                x, y = xy(s)
                return 1j * k * (dn - 1.0) * u(x, y)
            b += el.edge_load(n, h_edge, side, el.legendre_coeffs_1d(q, n))
        loads.append(b)
    return loads


def _local_values(w, disc, phis, t):
    """Field on the local tensor grid t x t of every element, keyed by the leaf's
    (ix, iy), x fastest."""
    vals = pb.sample_field(disc.mesh, disc.degrees, phis, lambda n: t)
    return {(ix, iy): vals[e] for e, (_, ix, iy) in enumerate(w["leaves"])}


def test_stretched_plane_wave_solves_the_layered_problem():
    k, nx_phys, n_pml = 12.0, 6, 2
    w, h = _layered_channel(nx_phys, n_pml, 2, 10, k, sigma=30.0)
    disc = pb.Discretisation(w)
    u = _stretched_wave(w, h, nx_phys, k)
    disc.b = _manufactured_loads(disc, u, k)
    phis = dpe.ElementwiseDP(disc, 2).solve(tol=1e-13, max_iter=400)
    t = np.linspace(-1, 1, 7)
    got = _local_values(w, disc, phis, t)
    err = 0.0
    for (ix, iy), v in got.items():
        X, Y = np.meshgrid(ix * h + (t + 1) * h / 2, iy * h + (t + 1) * h / 2)   # rows y, columns x
        err = max(err, np.abs(v - u(X.reshape(-1), Y.reshape(-1))).max())
    assert err < 1e-7
    # the wave decays through the layers as e^{-int sigma}
    assert abs(u(np.array([(nx_phys + n_pml) * h]), 0)[0]) < 0.1
