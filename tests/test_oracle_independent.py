"""Pins of the oracle against solves that do not use it (Sec. 2.3.1 and the
globally conforming space of Sec. 1), CPU only.

- The sparse LU of the constrained system eq. (large_saddle) with every
  continuity row kept equals the oracle's null-space solve (direct.py) on
  conforming and hanging meshes.
- A nodal C^0 spectral element solve on one global GLL lattice, with its own
  basis, exact quadrature and impedance terms (independent.py shares nothing
  with the modal oracle), equals the oracle's direct solve for the
  plane-wave (total field), point-source and scattered-field right-hand
  sides, and equals the converged element-by-element dual-primal iteration.
"""
import numpy as np
import pytest

import workloads as W
from oracle import direct, dp, dp_elementwise as dpe, independent as ind, problem as pb


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _field(disc, phis):
    return np.concatenate(pb.gll_field(disc.mesh, disc.degrees, phis))


def _scattered(n=4, p=6, k=12.0, theta=0.7):
    w = W.small_uniform(n, p, k, domain=(-1.0, 1.0, -1.0, 1.0),
                        rhs=dict(kind="plane_wave_scattered", angles=[theta]))
    c = W.leaf_centres(w)
    w["eps_r"] = np.where((np.abs(c[:, 0]) < 0.5) & (np.abs(c[:, 1]) < 0.5), 4.0, 1.0)
    return w


def _hanging(base, pvals, seed, l, k=6.0):
    lv = W.refine_where(W.morton_leaves(base, base), 0, 1, 0, 1, base, base,
                        lambda x, y: (x - 0.5) ** 2 + (y - 0.5) ** 2 < 0.03, 2)
    deg = np.random.default_rng(seed).integers(pvals[0], pvals[1] + 1, len(lv))
    return dict(domain=(0.0, 1.0, 0.0, 1.0), base=(base, base), leaves=lv, degree=deg, k=k, l=l,
                bc="impedance", eps_r=np.ones(len(lv)), rhs=dict(kind="plane_wave_total", angles=[0.4]))


@pytest.mark.parametrize("make", [lambda: W.small_uniform(3, 5, 9.0),
                                  lambda: _hanging(3, (3, 6), 1, 2)])
def test_saddle_point_lu_equals_null_space_solve(make):
    w = make()
    disc = pb.Discretisation(w)
    sad, m = ind.saddle_solution(disc)
    assert m > 0
    assert rel(_field(disc, sad), _field(disc, direct.conforming_solution(disc))) < 1e-12


def test_independent_rows_drop_exactly_the_dependent_ones():
    rng = np.random.default_rng(3)
    B = rng.standard_normal((4, 9))
    C = np.vstack([B, B[0] + 2 * B[2], B[1]])        # two dependent rows
    keep = ind.independent_rows(C)
    assert len(keep) == 4 and np.linalg.matrix_rank(C[keep]) == 4


@pytest.mark.parametrize("make", [W.plane_wave_4x4,
                                  lambda: W.small_uniform(4, 6, 7.0, rhs=dict(kind="point", points=[[0.5, 0.5]])),
                                  _scattered])
def test_nodal_assembly_equals_modal_direct_solve(make):
    w = make()
    disc = pb.Discretisation(w)
    assert rel(ind.nodal_solution(w), _field(disc, direct.conforming_solution(disc))) < 1e-12


def test_nodal_assembly_reproduces_the_plane_wave_spectrally():
    """The nodal solve alone (no oracle): the impedance data of an exact plane
    wave is reproduced with an error that falls fast with p."""
    errs = []
    for p in (4, 6, 8):
        w = W.small_uniform(4, p, 10.0, rhs=dict(kind="plane_wave_total", angles=[np.pi / 6]))
        u = ind.nodal_solution(w)
        x0, x1, y0, y1 = w["domain"]
        xi = ind._gll(p)
        h = (x1 - x0) / 4
        pts = []
        for _, ix, iy in np.asarray(w["leaves"]).reshape(-1, 3):
            X, Y = np.meshgrid(x0 + ix * h + (xi + 1) * h / 2, y0 + iy * h + (xi + 1) * h / 2)
            pts.append((X.ravel(), Y.ravel()))
        ex = np.concatenate([np.exp(1j * 10.0 * (np.cos(np.pi / 6) * X + np.sin(np.pi / 6) * Y)) for X, Y in pts])
        errs.append(rel(u, ex))
    assert errs[1] < errs[0] / 30 and errs[2] < errs[1] / 30 and errs[2] < 1e-6


@pytest.mark.parametrize("make", [W.plane_wave_4x4, lambda: _scattered(n=6, p=6, k=20.0)])
def test_dual_primal_iteration_converges_to_the_nodal_solution(make):
    w = make()
    disc = pb.Discretisation(w)
    l = pb.coarse_order(w, disc.mesh) if w.get("l", -1) >= 1 else min(3, int(w["degree"][0]) - 1)
    E = dpe.ElementwiseDP(disc, l)
    phis = E.solve(tol=1e-14, max_iter=400)
    assert E.iters > 3
    assert rel(_field(disc, phis), ind.nodal_solution(w)) < 1e-11


def test_literal_dual_primal_converges_to_the_nodal_solution():
    w = W.small_uniform(3, 5, 9.0, l=2)
    disc = pb.Discretisation(w)
    D = dp.LiteralDP(disc, 2)
    phis = D.solve(tol=1e-14, max_iter=200)
    assert rel(_field(disc, phis), ind.nodal_solution(w)) < 1e-11
