"""Pins of the oracle's adjoint gradient (dJ/d eps_r of a far-field intensity):
the far-field functional reproduces the far field by linearity, and the
adjoint gradient equals central finite differences of the oracle's own J."""
import numpy as np

import workloads as W
from oracle import adjoint as adj, direct, farfield as ff, problem as pb


def design_case():
    w = W.small_uniform(6, 4, 6.0, domain=(-1.0, 1.0, -1.0, 1.0), l=2)
    c = W.leaf_centres(w)
    inside = (np.abs(c[:, 0]) < 0.4) & (np.abs(c[:, 1]) < 0.4)
    eps = np.where(inside, np.random.default_rng(3).uniform(1.0, 4.0, len(c)), 1.0)
    return dict(w, eps_r=eps), inside


def test_far_functional_is_the_far_field():
    w, inside = design_case()
    w = dict(w, rhs=dict(kind="plane_wave_scattered", angles=[0.3]))
    disc = pb.Discretisation(w)
    phi = direct.conforming_solution(disc)
    for ang in (0.0, 1.1, 2.9):
        g = adj.far_functional(disc.mesh, disc.degrees, disc.k, inside, ang)
        E = sum(ge @ pe for ge, pe in zip(g, phi))
        ref = ff.far_field(disc.mesh, disc.degrees, phi, disc.k, inside, [ang])[0]
        assert abs(E - ref) < 1e-12 * abs(ref)


def test_adjoint_gradient_equals_central_differences():
    w, inside = design_case()
    J, grad, _ = adj.eps_gradient(w, 0.0, 0.0, inside)
    idx = np.nonzero(inside)[0]
    rng = np.random.default_rng(1)
    h = 1e-6
    for e in rng.choice(idx, 3, replace=False):
        ep, em = w["eps_r"].copy(), w["eps_r"].copy()
        ep[e] += h
        em[e] -= h
        fd = (adj.far_intensity(dict(w, eps_r=ep), 0.0, 0.0, inside)
              - adj.far_intensity(dict(w, eps_r=em), 0.0, 0.0, inside)) / (2 * h)
        assert abs(fd - grad[e]) < 1e-6 * max(abs(grad).max(), 1e-30)
    # elements outside the design region get gradients too (eps enters every element)
    assert np.abs(grad[~inside]).max() > 0


def test_elementwise_adjoint_equals_direct_adjoint():
    """The element-by-element dual-primal solves (forward and adjoint, the latter
    reusing the factorisations) give the direct solves' J and gradient."""
    import workloads as W
    from oracle import adjoint as adj
    w = W.small_uniform(6, 4, 6.0, domain=(-1.0, 1.0, -1.0, 1.0), l=2)
    c = W.leaf_centres(w)
    inside = (np.abs(c[:, 0]) < 0.4) & (np.abs(c[:, 1]) < 0.4)
    w["eps_r"] = np.where(inside, np.random.default_rng(3).uniform(1.0, 4.0, len(c)), 1.0)
    J0, g0, _ = adj.eps_gradient(w, 0.0, 0.0, inside)
    J1, g1, _ = adj.eps_gradient(w, 0.0, 0.0, inside, solver="elementwise", tol=1e-14)
    assert abs(J1 - J0) < 1e-10 * J0
    assert np.linalg.norm(g1 - g0) < 1e-9 * np.linalg.norm(g0)
