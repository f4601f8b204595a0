"""Pins of the oracle's per-edge coarse order (the non-uniform l the paper's
conclusions propose for non-uniformly refined meshes; the rule itself is the
dispersion criterion of Sec. 2.3.4 evaluated edge by edge)."""
import numpy as np
import pytest

import workloads as W
from oracle import constraints as cs
from oracle import direct, dp
from oracle import legendre as lg
from oracle import problem as pb


def _disk(k=40.0, passes=2, p=(4, 7), seed=0):
    """[0,1]^2 from a 4x4 base refined twice near the centre, a dielectric disk
    (eps_r = 2.25) in the refined part."""
    lv = W.refine_where(W.morton_leaves(4, 4), 0, 1, 0, 1, 4, 4,
                        lambda x, y: (x - 0.5) ** 2 + (y - 0.5) ** 2 < 0.05, passes)
    rng = np.random.default_rng(seed)
    w = dict(domain=(0.0, 1.0, 0.0, 1.0), base=(4, 4), leaves=lv, degree=rng.integers(p[0], p[1] + 1, len(lv)),
             k=k, l=-1, bc="impedance", rhs=dict(kind="plane_wave_scattered", angles=[0.3]))
    c = W.leaf_centres(w)
    w["eps_r"] = np.where(((c - 0.5) ** 2).sum(1) < 0.05, 2.25, 1.0)
    return w


def test_uniform_mesh_gets_the_global_order_on_every_edge():
    w = W.small_uniform(5, 6, 17.0)
    mesh = pb.make_mesh(w)
    lg_ = pb.coarse_order(w, mesh)
    lf = pb.edge_orders(w, mesh)
    assert all(lf(e, s) == lg_ for e in range(mesh.E) for s in (1, 2, 3, 4))


def test_edge_orders_follow_the_local_mesh_size_and_wavenumber():
    w = _disk()
    mesh = pb.make_mesh(w)
    lf = pb.edge_orders(w, mesh)
    lglob = pb.coarse_order(w, mesh)
    eps = np.asarray(w["eps_r"])
    vals = []
    for e in range(mesh.E):
        hx, hy = mesh.size(e)
        for s in (1, 2, 3, 4):
            v = lf(e, s)
            vals.append(v)
            assert v <= lglob
            # never below the element's own value on that side
            own = lg.dispersion_l(w["k"] * np.sqrt(eps[e]) * (hy if s in (1, 2) else hx), 1.0)
            assert v >= own
            # the two sides of an edge agree (hanging edges included)
            if not mesh.boundary_side(e, s):
                for f, sf in mesh.neighbours(e, s):
                    assert lf(f, sf) == v
    assert min(vals) < lglob


def test_per_edge_order_keeps_the_galerkin_solution_with_a_smaller_coarse_space():
    w = _disk()
    disc = pb.Discretisation(w)
    mesh = disc.mesh
    lf = pb.edge_orders(w, mesh)
    lglob = pb.coarse_order(w, mesh)
    n2 = {}
    for name, l in (("global", lglob), ("edge", lf)):
        status = cs.algorithm1(mesh, disc.degrees, l, disc.bc)
        n2[name] = sum(int((st == 2).sum()) for st in status)
    assert n2["edge"] < n2["global"]
    D = dp.LiteralDP(disc, lf)
    ref = direct.conforming_solution(disc)

    def err(phis):
        return max(np.abs(a - b).max() for a, b in zip(phis, ref)) / max(np.abs(b).max() for b in ref)
    # the interface system is solved exactly: the constraint set is complete
    assert err(D.recover(D.direct_interface())) < 1e-11
    # GMRES to a preconditioned residual of 1e-14 (F has condition number ~5e9 here)
    assert err(D.solve(tol=1e-14, max_iter=600)) < 1e-9
