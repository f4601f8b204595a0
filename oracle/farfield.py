"""Far field and radar cross section (paper Sec. 3.3.1, eqs. rcs_def and far_field),
written for the e^{-i omega t} convention.  Test infrastructure only.

E_far(phi) = oint_Gamma [ (xhat . n') u_s(x') + (i k)^-1 n'.grad u_s(x') ] e^{-i k xhat.x'} dGamma'
sigma_2D   = (k / 4) |E_far|^2
with n' the outward normal of the region enclosed by Gamma.  Gamma is a union
of element sides; traces and normal derivatives are taken from the element
outside Gamma; each side is integrated with Gauss-Legendre quadrature.
"""
import numpy as np

from . import legendre as lg
from .mesh import OPPOSITE

OUT_NORMAL = {1: (-1.0, 0.0), 2: (1.0, 0.0), 3: (0.0, -1.0), 4: (0.0, 1.0)}


def gamma_sides(mesh, inside):
    """(outside element, its side) pairs whose neighbour across the side is inside."""
    out = []
    for e in range(mesh.E):
        if inside[e]:
            continue
        for side in (1, 2, 3, 4):
            if mesh.boundary_side(e, side):
                continue
            nb = mesh.neighbours(e, side)
            if nb and all(inside[f] for f, _ in nb):
                out.append((e, side))
    return out


def far_field(mesh, degrees, phis, k, inside, angles, extra_nodes=12):
    angles = np.asarray(angles, float)
    xh = np.stack([np.cos(angles), np.sin(angles)], axis=1)
    E = np.zeros(len(angles), complex)
    for (e, side) in gamma_sides(mesh, inside):
        n = int(degrees[e]) + 1
        Phi = phis[e].reshape(n, n, order="F")
        (ox, oy), (hx, hy) = mesh.origin(e), mesh.size(e)
        s, wq = np.polynomial.legendre.leggauss(n + extra_nodes)
        if side in (1, 2):
            u = np.full_like(s, -1.0 if side == 1 else 1.0)
            v = s
            jac = hy / 2
        else:
            u = s
            v = np.full_like(s, -1.0 if side == 3 else 1.0)
            jac = hx / 2
        Nu, Nv = lg.basis_N(u, n), lg.basis_N(v, n)
        dNu, dNv = lg.basis_dN(u, n), lg.basis_dN(v, n)
        val = np.einsum("iq,ij,jq->q", Nu, Phi, Nv)
        dx = (2 / hx) * np.einsum("iq,ij,jq->q", dNu, Phi, Nv)
        dy = (2 / hy) * np.einsum("iq,ij,jq->q", Nu, Phi, dNv)
        x = ox + (u + 1) * hx / 2
        y = oy + (v + 1) * hy / 2
        # n' points out of the enclosed region, i.e. into this outside element
        nrm = -np.array(OUT_NORMAL[side])
        dn = dx * nrm[0] + dy * nrm[1]
        xn = xh @ nrm
        phase = np.exp(-1j * k * (np.outer(xh[:, 0], x) + np.outer(xh[:, 1], y)))
        integrand = xn[:, None] * val[None, :] + dn[None, :] / (1j * k)
        E += (integrand * phase) @ (wq * jac)
    return E


def rcs(E_far, k):
    return 0.25 * k * np.abs(E_far) ** 2


def interpolate_function(mesh, degrees, fun):
    """Modal coefficients (basis N) interpolating fun at each element's GLL nodes."""
    phis = []
    for e in range(mesh.E):
        n = int(degrees[e]) + 1
        (ox, oy), (hx, hy) = mesh.origin(e), mesh.size(e)
        t = lg.gll_nodes(n)
        X, Y = np.meshgrid(ox + (t + 1) * hx / 2, oy + (t + 1) * hy / 2, indexing="ij")
        U = fun(X, Y)                      # U[i, j] at (t_i, t_j), i along x
        V = lg.basis_N(t, n).T              # V[i, k] = N_k(t_i)
        Vi = np.linalg.inv(V)
        Phi = Vi @ U @ Vi.T
        phis.append(Phi.reshape(-1, order="F"))
    return phis
