"""Pins of the oracle's element matrices and loads (paper Sec. 2.1.5, 2.2.1, 3.2):
brute-force Gauss quadrature with an independently built basis, the plane-wave
Legendre closed form, complex symmetry and the printed element resonance."""
import numpy as np
import numpy.polynomial.legendre as npl
import pytest
import scipy.linalg as sla
from scipy.special import spherical_jn

from oracle import element as el
from oracle import legendre as lg


def basis_np(x, n):
    """N_0..N_{n-1} and derivatives at x from NumPy's Legendre series."""
    vals, ders = [], []
    for k in range(n):
        if k == 0:
            c = np.array([1 / np.sqrt(2)])
        elif k == 1:
            c = np.array([0.0, 1 / np.sqrt(2)])
        else:
            ck = np.zeros(k)
            ck[k - 1] = np.sqrt((2 * k - 1) / 2.0)
            c = npl.legint(ck, lbnd=-1)
        vals.append(npl.legval(x, c))
        ders.append(npl.legval(x, npl.legder(c)))
    return np.array(vals), np.array(ders)


def brute_element(n, hx, hy, alpha, beta, robin):
    """int over [0,hx]x[0,hy] of alpha grad(psi).grad(phi) + beta psi phi plus
    int over Robin sides of gamma psi phi, by tensor Gauss quadrature."""
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
            A += wt * (alpha * (np.outer(dx, dx) + np.outer(dy, dy)) + beta * np.outer(phi, phi))
    ends = {1: -1.0, 2: 1.0, 3: -1.0, 4: 1.0}
    for side, g in robin.items():
        Ne, _ = basis_np(np.array([ends[side]]), n)
        for q in range(len(u)):
            if side in (1, 2):
                phi = np.kron(N[:, q], Ne[:, 0])
                A += g * w[q] * Jy * np.outer(phi, phi)
            else:
                phi = np.kron(Ne[:, 0], N[:, q])
                A += g * w[q] * Jx * np.outer(phi, phi)
    return A


@pytest.mark.parametrize("robin", [{}, {2: -3j}, {1: 2.0 - 1j, 4: -5j}, {3: -1j, 2: -1j, 1: 0.5}])
def test_element_matrix_matches_quadrature(robin):
    n, hx, hy, alpha, beta = 6, 0.3, 0.7, 1.7, -23.0
    A = el.element_matrix(n, hx, hy, alpha=alpha, beta=beta, robin=robin)
    assert np.allclose(A, brute_element(n, hx, hy, alpha, beta, robin), atol=1e-12)
    assert np.allclose(A, A.T)   # complex symmetric


def test_loads_match_quadrature():
    n, hx, hy = 7, 0.4, 0.25
    k, d = 9.0, np.array([np.cos(0.7), np.sin(0.7)])
    f = lambda u, v: np.exp(1j * k * (d[0] * (u + 1) * hx / 2 + d[1] * (v + 1) * hy / 2))
    b = el.volume_load(n, hx, hy, el.legendre_coeffs_2d(f, n))
    u, w = npl.leggauss(40)
    N, _ = basis_np(u, n)
    ref = np.zeros(n * n, complex)
    for i in range(40):
        for j in range(40):
            ref += w[i] * w[j] * hx * hy / 4 * f(u[i], u[j]) * np.kron(N[:, j], N[:, i])
    assert np.allclose(b, ref, atol=1e-13)
    q = lambda s: np.cos(3 * s) + 1j * s ** 2
    for side, end in ((1, -1.0), (2, 1.0), (3, -1.0), (4, 1.0)):
        r = el.edge_load(n, hy if side < 3 else hx, side, el.legendre_coeffs_1d(q, n))
        Ne, _ = basis_np(np.array([end]), n)
        h = hy if side < 3 else hx
        ref = np.zeros(n * n, complex)
        for i in range(40):
            tr = np.kron(N[:, i], Ne[:, 0]) if side < 3 else np.kron(Ne[:, 0], N[:, i])
            ref += w[i] * h / 2 * q(u[i]) * tr
        assert np.allclose(r, ref, atol=1e-13)


def test_plane_wave_legendre_closed_form():
    # int_{-1}^{1} e^{i w t} p_n(t) dt = sqrt(2(2n+1)) i^n j_n(w)
    for om in (0.3, 2.5, 11.0):
        c = el.legendre_coeffs_1d(lambda s: np.exp(1j * om * s), 20)
        nn = np.arange(20)
        ref = np.sqrt(2 * (2 * nn + 1)) * (1j ** nn) * spherical_jn(nn, om)
        assert np.allclose(c, ref, rtol=0, atol=1e-13)


def test_point_load_and_vertex_basis():
    n = 5
    b = el.point_load(n, 1.0, -1.0)   # corner x=+1, y=-1
    bt = el.to_vertex_basis(n) @ b     # vertex-basis coefficients
    # in the vertex basis the corner value picks out exactly one vertex mode
    e = np.zeros(n * n)
    e[0 + n * 1] = 1.0
    assert np.allclose(bt, e, atol=1e-14)


def test_element_resonance_of_removed_mode_block():
    """Sec. 3.2: an element of size 0.25 with p = 32 and l = 3 resonates at
    k = 16.56157163134991 once the vertex modes and the first l-1 bubbles of each
    side are removed (the block A_11 of one element, natural boundary)."""
    n, h, l = 33, 0.25, 3
    Bz = el.to_vertex_basis(n)
    K = (Bz @ el.element_matrix(n, h, h) @ Bz).real
    M = (Bz @ el.element_matrix(n, h, h, alpha=0.0, beta=1.0) @ Bz).real
    ix, iy = np.arange(n * n) % n, np.arange(n * n) // n
    removed = ((ix < 2) & (iy < 2)) | ((ix < 2) & (iy <= l)) | ((iy < 2) & (ix <= l))
    I = ~removed
    ev = np.sqrt(np.sort(sla.eigvalsh(K[np.ix_(I, I)], M[np.ix_(I, I)])))
    k = ev[np.argmin(np.abs(ev - 16.56157163134991))]
    assert abs(k - 16.56157163134991) < 1e-10
    # removing only the vertex modes gives no eigenvalue there
    Iv = ~((ix < 2) & (iy < 2))
    ev2 = np.sqrt(np.sort(sla.eigvalsh(K[np.ix_(Iv, Iv)], M[np.ix_(Iv, Iv)])))
    assert np.abs(ev2 - 16.56157163134991).min() > 1e-3
