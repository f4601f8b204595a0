"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, and its host-only analysis (hdp_inspect) validates input and reports
the sizes the oracle computes."""
import os
import re

import numpy as np
import pytest

import paper_1808_04713_amd as hdp
import workloads as W
from oracle import dp_elementwise as dpe, problem as pb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hdp.h")).read()
    return sorted(set(re.findall(r"\b(hdp_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = hdp.load_library()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert sorted(hdp.EXPORTS) == names


@pytest.mark.parametrize("make,l,nlam,nK", [(W.plane_wave_4x4, 1, 168, 25),
                                             (W.point_source_32x32, 2, 27776, 3201),
                                             (W.square_scatterer_64x64, 6, 48384, 45825)])
def test_inspect_sizes(make, l, nlam, nK):
    st = hdp.inspect(make())
    assert (st["l"], st["n_lambda"], st["n_coarse"]) == (l, nlam, nK)
    assert st["min_element_margin"] > 1e-8


@pytest.mark.parametrize("n,p,k,l", [(3, 5, 9.0, 2), (4, 6, 7.0, 3), (3, 7, 20.0, -1)])
def test_inspect_matches_oracle_counts(n, p, k, l):
    w = W.small_uniform(n, p, k, l=l)
    disc = pb.Discretisation(w)
    lo = pb.coarse_order(w, disc.mesh)
    E = dpe.ElementwiseDP(disc, lo)
    st = hdp.inspect(w)
    assert (st["l"], st["n_lambda"], st["n_coarse"]) == (lo, E.nlam, E.nK)
    assert st["dof"] == n * n * (p + 1) ** 2


def _hanging(base, pvals, seed, l, k=6.0, passes=2):
    lv = W.refine_where(W.morton_leaves(base, base), 0, 1, 0, 1, base, base,
                        lambda x, y: (x - 0.5) ** 2 + (y - 0.5) ** 2 < (0.03 if base % 2 else 0.05), passes)
    rng = np.random.default_rng(seed)
    deg = rng.integers(pvals[0], pvals[1] + 1, len(lv))
    return dict(domain=(0.0, 1.0, 0.0, 1.0), base=(base, base), leaves=lv, degree=deg, k=k, l=l,
                bc="impedance", eps_r=np.ones(len(lv)), rhs=dict(kind="plane_wave_total", angles=[0.4]))


@pytest.mark.parametrize("base,pvals,seed,l", [(3, (4, 4), 0, 1), (3, (3, 6), 1, 2), (4, (2, 5), 2, 3),
                                                (3, (3, 7), 3, 7)])
def test_inspect_matches_literal_oracle_on_hanging_meshes(base, pvals, seed, l):
    """Dual rows and coarse unknowns on meshes with hanging edges (up to three
    hanging nodes per edge), uneven degrees and l above some degrees: the
    library's counts equal the literal oracle's (dual rows of C_d, type-2
    columns of Z from Algorithm 1)."""
    from oracle import constraints as cs
    w = _hanging(base, pvals, seed, l)
    disc = pb.Discretisation(w)
    con = cs.Constraints(disc.mesh, disc.degrees, l, disc.bc)
    n_dual = int((~con.primal).sum())
    status = cs.algorithm1(disc.mesh, disc.degrees, l, disc.bc)
    n_type2 = sum(int((st == 2).sum()) for st in status)
    st = hdp.inspect(w)
    assert disc.mesh.Lmax == 2
    assert (st["l"], st["n_lambda"], st["n_coarse"]) == (l, n_dual, n_type2)


def test_inspect_rejects_bad_input():
    w = W.plane_wave_4x4()
    bad = dict(w, k=float("nan"))
    with pytest.raises(hdp.HdpError) as e:
        hdp.inspect(bad)
    assert e.value.status == -1
    # leaves that do not tile the domain
    with pytest.raises(hdp.HdpError) as e:
        hdp.inspect(dict(w, leaves=w["leaves"][:-1], degree=w["degree"][:-1], eps_r=w["eps_r"][:-1]))
    assert e.value.status == -2


def test_inspect_reports_element_resonance():
    # The centre element of a 3x3 mesh of unit squares has natural (Neumann)
    # sides; at k = pi its separable operator has the eigenvalue
    # (pi/h)^2 + 0 within the polynomial approximation, and setup must refuse
    # (Sec. 2.3.4: spurious element resonances make the local problems singular).
    w = W.small_uniform(3, 8, np.pi, domain=(0.0, 3.0, 0.0, 3.0), l=1)
    with pytest.raises(hdp.HdpError) as e:
        hdp.inspect(w)
    assert e.value.status == -3
    near = hdp.inspect(W.small_uniform(3, 8, np.pi * 1.001, domain=(0.0, 3.0, 0.0, 3.0), l=1))
    far = hdp.inspect(W.small_uniform(3, 8, 2.0, domain=(0.0, 3.0, 0.0, 3.0), l=1))
    assert near["min_element_margin"] < 1e-2 * far["min_element_margin"]


def test_robin_modified_local_problems_remove_the_element_resonance():
    """Sec. 2.3.4: with +-ik Robin terms on the sides between elements of opposite
    label every local problem is uniquely solvable, so the set-up that refuses
    k = pi above accepts it, with a margin of the size found away from resonance."""
    w = dict(W.small_uniform(3, 8, np.pi, domain=(0.0, 3.0, 0.0, 3.0), l=1), robin_modified=True)
    st = hdp.inspect(w)
    far = hdp.inspect(W.small_uniform(3, 8, 2.0, domain=(0.0, 3.0, 0.0, 3.0), l=1))
    assert st["min_element_margin"] > 1e-2 * far["min_element_margin"]
    # elements now also differ by label (the sign of their terms): on a 6x6 mesh
    # the 4 corner, 4 side and 1 interior classes become 4 corners (one label
    # each), 8 side classes and 2 interior ones
    w6 = W.small_uniform(6, 5, 2.0, l=1)
    assert hdp.inspect(w6)["n_classes"] == 9
    assert hdp.inspect(dict(w6, robin_modified=True))["n_classes"] == 14


def test_robin_modified_rejects_sides_with_both_labels():
    """On a quadtree mesh a coarse side can meet fine leaves of both labels; its
    term would cover part of the side, which the separable local solver cannot
    take: the set-up reports an unsupported input."""
    lv = W.refine_where(W.morton_leaves(3, 3), 0, 1, 0, 1, 3, 3,
                        lambda x, y: (x - 0.5) ** 2 + (y - 0.5) ** 2 < 0.02, 1)
    w = dict(domain=(0.0, 1.0, 0.0, 1.0), base=(3, 3), leaves=lv, degree=np.full(len(lv), 4), k=6.0,
             eps_r=np.ones(len(lv)), l=-1, robin_modified=True)
    with pytest.raises(hdp.HdpError) as e:
        hdp.inspect(w)
    assert e.value.status == -7


def test_layers_are_checked_and_refused_with_hanging_edges():
    w = W.small_uniform(8, 4, 10.0, domain=(-1.0, 1.0, -1.0, 1.0), l=2)
    sig = W.pml_sigma(w["leaves"], (8, 8), 4, 2, 40.0)
    st = hdp.inspect(dict(w, pml_sigma=sig))
    # stretched elements differ from plain ones of the same position: the layer
    # rings add classes to the 9 of the plain 8x8 mesh
    assert hdp.inspect(w)["n_classes"] == 9
    assert st["n_classes"] > 9
    bad = sig.copy()
    bad[3, 0] = -1.0
    with pytest.raises(hdp.HdpError) as e:
        hdp.inspect(dict(w, pml_sigma=bad))
    assert e.value.status == -1
    lv = W.refine_where(W.morton_leaves(3, 3), 0, 1, 0, 1, 3, 3,
                        lambda x, y: (x - 0.5) ** 2 + (y - 0.5) ** 2 < 0.02, 1)
    wh = dict(domain=(0.0, 1.0, 0.0, 1.0), base=(3, 3), leaves=lv, degree=np.full(len(lv), 4), k=6.0,
              eps_r=np.ones(len(lv)), l=-1, pml_sigma=np.full((len(lv), 2), 1.0))
    with pytest.raises(hdp.HdpError) as e:
        hdp.inspect(wh)
    assert e.value.status == -7


@pytest.mark.parametrize("k,seed", [(30.0, 0), (45.0, 1)])
def test_per_edge_order_counts_match_the_oracle(k, seed):
    """Per-edge coarse orders on a refined mesh with a dielectric disk: the
    library's largest order, dual rows and coarse unknowns equal the oracle's
    (its Constraints and Algorithm 1 with the same per-edge function), and the
    coarse space is smaller than with the one global order."""
    from oracle import constraints as cs
    import test_oracle_edge_l as tel
    w = dict(tel._disk(k=k, seed=seed), l_per_edge=True)
    disc = pb.Discretisation(w)
    lf = pb.edge_orders(w, disc.mesh)
    con = cs.Constraints(disc.mesh, disc.degrees, lf, disc.bc)
    status = cs.algorithm1(disc.mesh, disc.degrees, lf, disc.bc)
    n_dual = int((~con.primal).sum())
    n_type2 = sum(int((st == 2).sum()) for st in status)
    st = hdp.inspect(w)
    lmax = max(lf(e, s) for e in range(disc.mesh.E) for s in (1, 2, 3, 4))
    assert (st["l"], st["n_lambda"], st["n_coarse"]) == (lmax, n_dual, n_type2)
    assert st["n_coarse"] < hdp.inspect(dict(w, l_per_edge=False))["n_coarse"]


def test_inspect_free_space_reading_of_the_rule():
    """l_free_space evaluates the dispersion rule with k instead of k sqrt(eps_r):
    on the 64x64 dielectric-square scatterer (h = 1/32, k = 150, eps_r = 4) the
    local reading gives l = 6 and the free-space reading l = 3, matching the
    oracle's rule in both readings."""
    w = W.square_scatterer_64x64()
    for free, l in ((False, 6), (True, 3)):
        ww = dict(w, l_free_space=free)
        assert hdp.inspect(ww)["l"] == l == pb.coarse_order(ww)
