"""Gradient of a far-field intensity with respect to the per-element relative
permittivity, by the adjoint of the discrete system.  Test infrastructure only.

J(eps) = |E_far(phi)|^2 with phi the conforming Galerkin solution of the
scattered-field problem (f = k^2 (eps_r - 1) u_inc, homogeneous impedance
condition) and E_far the far field of Sec. 3.3.1, which is linear in phi:
E = g^T phi.  With A phi = b (A complex symmetric: a(psi, phi) is a bilinear
form, Sec. 2.3.4) and A lambda = g in the same conforming space,
    dJ/d eps_e = 2 Re( conj(E) lambda^T (db/d eps_e - dA/d eps_e phi) ),
where only element e's blocks depend on eps_e:
    dA_e/d eps_e = element matrix of beta = -k^2 (mass term only),
    db_e/d eps_e = volume load of f = k^2 u_inc.
"""
import numpy as np

from . import element as el
from . import legendre as lg
from . import problem as pb
from .direct import conforming_solution
from .farfield import OUT_NORMAL, gamma_sides


def far_functional(mesh, degrees, k, inside, angle, extra_nodes=12):
    """Element vectors g_e (paper basis, x index fastest) with E_far(angle) = sum_e g_e^T phi_e:
    the far-field integrand of Sec. 3.3.1 differentiated with respect to each coefficient."""
    xh = np.array([np.cos(angle), np.sin(angle)])
    g = [np.zeros((int(p) + 1) ** 2, complex) for p in degrees]
    for (e, side) in gamma_sides(mesh, inside):
        n = int(degrees[e]) + 1
        (ox, oy), (hx, hy) = mesh.origin(e), mesh.size(e)
        s, wq = np.polynomial.legendre.leggauss(n + extra_nodes)
        if side in (1, 2):
            u, v, jac = np.full_like(s, -1.0 if side == 1 else 1.0), s, hy / 2
        else:
            u, v, jac = s, np.full_like(s, -1.0 if side == 3 else 1.0), hx / 2
        Nu, Nv = lg.basis_N(u, n), lg.basis_N(v, n)
        dNu, dNv = lg.basis_dN(u, n), lg.basis_dN(v, n)
        nrm = -np.array(OUT_NORMAL[side])
        x = ox + (u + 1) * hx / 2
        y = oy + (v + 1) * hy / 2
        c = wq * jac * np.exp(-1j * k * (xh[0] * x + xh[1] * y))
        # d/dPhi_ij of sum_q c_q [ (xh.n) u_q + (ik)^-1 n.grad u_q ]
        G = (xh @ nrm) * np.einsum("q,iq,jq->ij", c, Nu, Nv)
        G += (nrm[0] * (2 / hx) * np.einsum("q,iq,jq->ij", c, dNu, Nv)
              + nrm[1] * (2 / hy) * np.einsum("q,iq,jq->ij", c, Nu, dNv)) / (1j * k)
        g[e] += G.reshape(-1, order="F")
    return g


def eps_gradient(w, incidence, far_angle, inside, solver="direct", tol=1e-13):
    """(J, dJ/d eps_r per element) for the scattered field of the plane wave with
    propagation angle ``incidence``; ``inside`` marks the region whose boundary
    carries the far-field integral.  solver: "direct" (dense null-space solve of
    the conforming system, small meshes) or "elementwise" (the element-by-element
    dual-primal method driven to ``tol``, conforming meshes of any size; the
    adjoint solve reuses its factorisations)."""
    w = dict(w, rhs=dict(kind="plane_wave_scattered", angles=[incidence]))
    disc = pb.Discretisation(w)
    mesh, k = disc.mesh, disc.k
    g = far_functional(mesh, disc.degrees, k, inside, far_angle)
    if solver == "direct":
        phi = conforming_solution(disc)
        lam = conforming_solution(disc, loads=g)
    else:
        from .dp_elementwise import ElementwiseDP
        D = ElementwiseDP(disc, pb.coarse_order(w, mesh))
        phi = D.solve(tol=tol, max_iter=400)
        D.set_loads(g)
        lam = D.solve(tol=tol, max_iter=400)
    E = sum(ge @ pe for ge, pe in zip(g, phi))
    d = np.array([np.cos(incidence), np.sin(incidence)])
    grad = np.zeros(mesh.E)
    for e in range(mesh.E):
        n = int(disc.degrees[e]) + 1
        (ox, oy), (hx, hy) = mesh.origin(e), mesh.size(e)
        dA = el.element_matrix(n, hx, hy, alpha=0.0, beta=-k ** 2)

        def f(uu, vv):
            return k ** 2 * np.exp(1j * k * (d[0] * (ox + (uu + 1) * hx / 2) + d[1] * (oy + (vv + 1) * hy / 2)))
        db = el.volume_load(n, hx, hy, el.legendre_coeffs_2d(f, n))
        grad[e] = 2 * np.real(np.conj(E) * (lam[e] @ (db - dA @ phi[e])))
    return abs(E) ** 2, grad, E


def far_intensity(w, incidence, far_angle, inside):
    """J alone (for finite differences)."""
    w = dict(w, rhs=dict(kind="plane_wave_scattered", angles=[incidence]))
    disc = pb.Discretisation(w)
    phi = conforming_solution(disc)
    g = far_functional(disc.mesh, disc.degrees, disc.k, inside, far_angle)
    return abs(sum(ge @ pe for ge, pe in zip(g, phi))) ** 2
