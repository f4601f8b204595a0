"""GPU adjoint gradient of a far-field intensity with respect to the per-leaf
permittivity (hdp_far_intensity_gradient, and the torch.autograd wrapper),
against the oracle's adjoint (plain conforming solves) on a small design
problem, and against central finite differences of the GPU's own J at the
full 64x64 design-block size."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as adj

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def hdp():
    import paper_1808_04713_amd as m
    return m


def design_case():
    w = W.small_uniform(6, 4, 6.0, domain=(-1.0, 1.0, -1.0, 1.0), l=2)
    c = W.leaf_centres(w)
    inside = (np.abs(c[:, 0]) < 0.4) & (np.abs(c[:, 1]) < 0.4)
    eps = np.where(inside, np.random.default_rng(3).uniform(1.0, 4.0, len(c)), 1.0)
    return dict(w, eps_r=eps), inside


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gradient_matches_oracle_adjoint(precision):
    w, inside = design_case()
    J0, g0, E0 = adj.eps_gradient(w, 0.0, 0.0, inside)
    s = hdp().Solver(w, precision=precision, tol=1e-13, max_iter=400)
    J, g, st = s.far_intensity_gradient(0.0, 0.0, inside)
    s.close()
    assert st["converged"]
    tol = 1e-9 if precision == "fp64" else 1e-7
    assert abs(J - J0) < tol * J0
    assert np.linalg.norm(g - g0) < tol * np.linalg.norm(g0)


def test_autograd_function_returns_the_adjoint_gradient():
    w, inside = design_case()
    _, g0, _ = adj.eps_gradient(w, 0.0, 0.0, inside)
    eps = torch.tensor(w["eps_r"], dtype=torch.float64, requires_grad=True)
    J = hdp().far_intensity(eps, w, 0.0, 0.0, inside, tol=1e-13, max_iter=400)
    (3.0 * J).backward()
    assert np.linalg.norm(eps.grad.numpy() - 3.0 * g0) < 1e-9 * 3.0 * np.linalg.norm(g0)


def test_full_size_design_block_against_central_differences():
    """64x64 elements, p = 12, k = 150, eps_r ~ U[1,4] on the central 16x16 block,
    J = |E_far(0)|^2 for normal incidence; central differences of the GPU's J on
    four random design parameters.  J (about 1.5) is reproducible to about 1e-10
    between set-ups (each set-up factors the coarse matrix anew), so a difference
    quotient carries about 1e-10/h of noise: at h = 1e-6 it is
    off by 6e-3 relative, at 1e-5 by 7e-4, at 1e-4 by 1e-4, at 1e-3 by 3e-5 on
    the first sampled element.  h = 3e-4 balances noise and truncation."""
    w = W.design_block_64x64()
    c = W.leaf_centres(w)
    h_el = 2.0 / 64
    inside = (np.abs(c[:, 0]) < 8 * h_el) & (np.abs(c[:, 1]) < 8 * h_el)
    opts = dict(tol=1e-13, max_iter=400)
    s = hdp().Solver(w, **opts)
    J, g, st = s.far_intensity_gradient(0.0, 0.0, inside)
    s.close()
    assert st["converged"] and J > 0
    idx = np.nonzero(inside)[0]
    assert len(idx) == 256
    rng = np.random.default_rng(11)
    h = 3e-4
    for e in rng.choice(idx, 4, replace=False):
        Js = []
        for sgn in (1, -1):
            eps = w["eps_r"].copy()
            eps[e] += sgn * h
            s2 = hdp().Solver(dict(w, eps_r=eps), **opts)
            Js.append(s2.far_intensity_gradient(0.0, 0.0, inside)[0])
            s2.close()
        fd = (Js[0] - Js[1]) / (2 * h)
        assert abs(fd - g[e]) < 1e-3 * abs(g[e]) + 1e-6, (e, fd, g[e])
