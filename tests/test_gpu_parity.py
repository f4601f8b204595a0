"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tolerances: FP64 path 1e-10 relative L2 on the field (solves driven to 1e-12),
1e-12 on single operator applications; mixed path 1e-8 on the field."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import dp, dp_elementwise as dpe, element as el, problem as pb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def hdp():
    import paper_1808_04713_amd as m
    return m


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def small_cases():
    sq = W.small_uniform(6, 6, 12.0, domain=(-1.0, 1.0, -1.0, 1.0), l=2,
                         rhs=dict(kind="plane_wave_scattered", angles=[0.7]))
    c = W.leaf_centres(sq)
    sq["eps_r"] = np.where((np.abs(c[:, 0]) < 0.4) & (np.abs(c[:, 1]) < 0.4), 4.0, 1.0)
    return {
        "plane_wave_4x4": W.plane_wave_4x4(),
        "uniform_4x4_p6_l2": W.small_uniform(4, 6, 7.0, l=2),
        "uniform_5x5_p7_l3": W.small_uniform(5, 7, 11.0, l=3),
        "point_4x4_p6": W.small_uniform(4, 6, 9.0, rhs=dict(kind="point", points=[(0.5, 0.5)]), l=2),
        "scatterer_6x6_p6": sq,
    }


CASES = small_cases()


@pytest.fixture(scope="module")
def oracles():
    out = {}
    for name, w in CASES.items():
        disc = pb.Discretisation(w)
        l = pb.coarse_order(w, disc.mesh)
        out[name] = (disc, l, dpe.ElementwiseDP(disc, l))
    return out


def vertex_element_matrices(disc):
    mats = []
    for e in range(disc.mesh.E):
        n = int(disc.degrees[e]) + 1
        B = el.to_vertex_basis(n)
        mats.append(B @ disc.A[e] @ B)
    return mats


@pytest.mark.parametrize("name", ["plane_wave_4x4", "scatterer_6x6_p6"])
def test_local_solve_separable(name, oracles):
    disc, l, _ = oracles[name]
    w = CASES[name]
    s = hdp().Solver(w)
    R = 3
    rng = np.random.default_rng(7)
    y = rng.standard_normal((s.dof, R)) + 1j * rng.standard_normal((s.dof, R))
    x = s.local_solve(torch.from_numpy(y).cuda()).cpu().numpy()
    off = 0
    for A in vertex_element_matrices(disc):
        n2 = A.shape[0]
        ref = np.linalg.solve(A, y[off:off + n2])
        assert rel(x[off:off + n2], ref) < 1e-11
        off += n2
    s.close()


@pytest.mark.parametrize("R", [16, 32, 64])
@pytest.mark.parametrize("name", ["uniform_4x4_p6_l2", "scatterer_6x6_p6"])
def test_fp32_operators_at_many_columns(name, R, oracles):
    """F v and P^-1 v of the mixed path at 16, 32 and 64 columns (the FP32
    matrix-core slot kernels, FP32 accumulation) against the oracle column by
    column, at FP32 accuracy."""
    disc, l, E = oracles[name]
    s = hdp().Solver(CASES[name], max_rhs=R)
    rng = np.random.default_rng(R + 1)
    v = rng.standard_normal((E.nlam, R)) + 1j * rng.standard_normal((E.nlam, R))
    vd = torch.from_numpy(v).cuda()
    Fv = s.apply_interface(vd, "mixed").cpu().numpy()
    Pv = s.apply_precond(vd, "mixed").cpu().numpy()
    for r in range(R):
        assert rel(Fv[:, r], E.apply_F(v[:, r])) < 1e-5
        assert rel(Pv[:, r], E.apply_P(v[:, r])) < 1e-5
    s.close()


@pytest.mark.parametrize("R", [16, 32, 64])
@pytest.mark.parametrize("name", ["uniform_4x4_p6_l2", "uniform_5x5_p7_l3"])
def test_operators_at_many_columns(name, R, oracles):
    """F v and P^-1 v at 16, 32 and 64 columns (the matrix-core slot kernels)
    against the oracle column by column."""
    disc, l, E = oracles[name]
    s = hdp().Solver(CASES[name], max_rhs=R)
    rng = np.random.default_rng(R)
    v = rng.standard_normal((E.nlam, R)) + 1j * rng.standard_normal((E.nlam, R))
    vd = torch.from_numpy(v).cuda()
    Fv = s.apply_interface(vd, "fp64").cpu().numpy()
    Pv = s.apply_precond(vd, "fp64").cpu().numpy()
    for r in range(R):
        assert rel(Fv[:, r], E.apply_F(v[:, r])) < 1e-12
        assert rel(Pv[:, r], E.apply_P(v[:, r])) < 1e-12
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_interface_operator_and_preconditioner(name, oracles):
    disc, l, E = oracles[name]
    s = hdp().Solver(CASES[name], max_rhs=2)
    assert s.n_lambda == E.nlam and s.n_coarse == E.nK
    rng = np.random.default_rng(11)
    v = rng.standard_normal((E.nlam, 2)) + 1j * rng.standard_normal((E.nlam, 2))
    vd = torch.from_numpy(v).cuda()
    Fv = s.apply_interface(vd, "fp64").cpu().numpy()
    Pv = s.apply_precond(vd, "fp64").cpu().numpy()
    for r in range(2):
        assert rel(Fv[:, r], E.apply_F(v[:, r])) < 1e-12
        assert rel(Pv[:, r], E.apply_P(v[:, r])) < 1e-12
    Fv32 = s.apply_interface(vd, "mixed").cpu().numpy()
    Pv32 = s.apply_precond(vd, "mixed").cpu().numpy()
    assert rel(Fv32[:, 0], E.apply_F(v[:, 0])) < 1e-4
    assert rel(Pv32[:, 0], E.apply_P(v[:, 0])) < 1e-5
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_interface_rhs(name, oracles):
    disc, l, E = oracles[name]
    w = CASES[name]
    s = hdp().Solver(w)
    kind, vals = hdp().rhs_values(w)
    g = s.interface_rhs(kind, vals).cpu().numpy()[:, 0]
    assert rel(g, E.interface_rhs()) < 1e-12
    s.close()


@pytest.mark.parametrize("name,kind", [("plane_wave_4x4", "plane_wave_total"),
                                       ("scatterer_6x6_p6", "plane_wave_scattered"),
                                       ("scatterer_6x6_p6", "plane_wave_total")])
def test_interface_rhs_several_angles(name, kind):
    """Device-computed plane-wave loads, three angles in a stride of four columns:
    each column equals the oracle's interface data for that angle alone."""
    w = CASES[name]
    angles = [0.3, 2.0, 4.4]
    s = hdp().Solver(w, max_rhs=4)
    g = s.interface_rhs(kind, angles).cpu().numpy()
    assert g.shape[1] >= len(angles)
    for i, a in enumerate(angles):
        w1 = dict(w, rhs=dict(kind=kind, angles=[a]))
        d1 = pb.Discretisation(w1)
        ref = dpe.ElementwiseDP(d1, pb.coarse_order(w1, d1.mesh)).interface_rhs()
        assert rel(g[:, i], ref) < 1e-12
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_solve_fp64_matches_oracle(name, oracles):
    disc, l, E = oracles[name]
    w = CASES[name]
    s = hdp().Solver(w, tol=1e-12, max_iter=400)
    kind, vals = hdp().rhs_values(w)
    field, st = s.solve(kind, vals)
    gpu = field.cpu().numpy()[0]
    phis = E.solve(tol=1e-12, max_iter=400)
    ref = np.concatenate(pb.gll_field(disc.mesh, disc.degrees, phis))
    assert st["converged"]
    assert rel(gpu, ref) < 1e-10
    assert abs(st["iterations"] - E.iters) <= 1
    s.close()


@pytest.mark.parametrize("cap", [1, 6])
def test_iteration_cap_matches_the_oracle_partial_solution(cap, oracles):
    """Stopped at the iteration cap (max_iter, no convergence) the GPU returns the
    GMRES iterate of that many steps: the same residual history and field as the
    oracle's GMRES with the same cap (the Krylov basis holds max_iter + 1 vectors
    and one more candidate at the end)."""
    name = "uniform_5x5_p7_l3"
    disc, l, E = oracles[name]
    w = CASES[name]
    s = hdp().Solver(w, tol=1e-14, max_iter=cap)
    kind, vals = hdp().rhs_values(w)
    field, st = s.solve(kind, vals)
    assert not st["converged"]
    assert st["iterations"] == cap
    hist = np.asarray(s.residual_history())
    phis = E.solve(tol=1e-14, max_iter=cap)
    assert E.iters == cap
    assert np.abs(hist[:cap + 1] - np.asarray(E.hist[:cap + 1])).max() < 1e-10
    ref = np.concatenate(pb.gll_field(disc.mesh, disc.degrees, phis))
    assert rel(field.cpu().numpy()[0], ref) < 1e-10
    s.close()


def test_plane_wave_against_literal_method_and_exact_solution():
    w = W.plane_wave_4x4()
    disc = pb.Discretisation(w)
    D = dp.LiteralDP(disc, 1)
    phis = D.solve(tol=1e-10, max_iter=300)
    ref = np.concatenate(pb.gll_field(disc.mesh, disc.degrees, phis))
    s = hdp().Solver(w, tol=1e-10)
    field, st = s.solve("plane_wave_total", w["rhs"]["angles"])
    gpu = field.cpu().numpy()[0]
    assert rel(gpu, ref) < 1e-9
    assert abs(st["iterations"] - D.iters) <= 1
    # the discrete solution approximates the exact plane wave (p = 8)
    ex = pb.exact_plane_wave(w)
    from oracle import legendre as lg
    vals = []
    for e in range(disc.mesh.E):
        (ox, oy), (hx, hy) = disc.mesh.origin(e), disc.mesh.size(e)
        t = lg.gll_nodes(9)
        X, Y = np.meshgrid(ox + (t + 1) * hx / 2, oy + (t + 1) * hy / 2, indexing="xy")
        vals.append(ex(X.ravel(), Y.ravel()))
    assert np.abs(gpu - np.concatenate(vals)).max() < 1e-7
    s.close()


@pytest.mark.parametrize("name", ["plane_wave_4x4", "uniform_5x5_p7_l3", "scatterer_6x6_p6"])
def test_mixed_precision_solve(name, oracles):
    disc, l, E = oracles[name]
    w = CASES[name]
    s = hdp().Solver(w, precision="mixed", tol=1e-12, max_iter=400)
    kind, vals = hdp().rhs_values(w)
    field, st = s.solve(kind, vals)
    phis = E.solve(tol=1e-12, max_iter=400)
    ref = np.concatenate(pb.gll_field(disc.mesh, disc.degrees, phis))
    assert st["converged"] and st["refinements"] >= 1
    assert rel(field.cpu().numpy()[0], ref) < 1e-8
    s.close()


def test_batched_rhs_equal_single_solves():
    w = small_cases()["scatterer_6x6_p6"]
    angles = np.array([0.0, 0.9, 2.1, 4.0, 5.5])
    s = hdp().Solver(w, tol=1e-12, max_rhs=len(angles))
    fb, stb = s.solve("plane_wave_scattered", angles)
    fb = fb.cpu().numpy()
    for i, a in enumerate(angles):
        f1, st1 = s.solve("plane_wave_scattered", [a])
        assert rel(fb[i], f1.cpu().numpy()[0]) < 1e-11
    s.close()


@pytest.mark.parametrize("coarse", ["dense", "nd"])
@pytest.mark.parametrize("name", ["uniform_5x5_p7_l3", "scatterer_6x6_p6"])
def test_coarse_solvers_against_the_oracle(name, coarse, oracles):
    """Both coarse factors give the oracle's interface operator at 1, 5, 16 and 64
    columns and its field: the dense inverse (streamed symmetric tiles at one
    column, tile products of the inverse from 4 columns on, on the matrix cores
    at 16..64) and the nested-dissection factor (one-column rows, tile products,
    the top depths as one dense block at several columns); 5 columns exercise the
    masked lanes of the vector path."""
    disc, l, E = oracles[name]
    w = CASES[name]
    s = hdp().Solver(w, tol=1e-12, max_iter=400, max_rhs=64, coarse=coarse)
    st = s.info
    assert st["coarse_mode"] == (0 if coarse == "dense" else 2) and st["coarse_residual"] < 1e-12
    assert coarse == "dense" or st["coarse_blocks"] >= 3
    assert coarse == "dense" or (0 < st["coarse_top_unknowns"] < st["n_coarse"] and st["coarse_top_check"] < 1e-12)
    rng = np.random.default_rng(5)
    for R in (1, 5, 16, 64):
        v = rng.standard_normal((E.nlam, R)) + 1j * rng.standard_normal((E.nlam, R))
        Fg = s.apply_interface(torch.from_numpy(v).cuda(), "fp64").cpu().numpy()
        ref = np.stack([E.apply_F(v[:, r]) for r in range(R)], axis=1)
        assert rel(Fg, ref) < 1e-12, (R, rel(Fg, ref))
    kind, vals = hdp().rhs_values(w)
    f, _ = s.solve(kind, vals)
    phis = E.solve(tol=1e-12, max_iter=400)
    ref = np.concatenate(pb.gll_field(disc.mesh, disc.degrees, phis))
    assert rel(f.cpu().numpy()[0], ref) < 1e-10
    s.close()


def test_handle_memory_from_the_callers_allocator(oracles):
    """hdp_options.allocator: with torch's caching allocator the handle's device
    memory comes from torch's pool (torch.cuda.memory_allocated grows by at least
    the coarse inverse and returns to its value after close), and the solve is the
    same as with hipMalloc."""
    name = "scatterer_6x6_p6"
    w = CASES[name]
    kind, vals = hdp().rhs_values(w)
    s0 = hdp().Solver(w, tol=1e-12, max_iter=400, max_rhs=4)
    f0, st0 = s0.solve(kind, vals)
    s0.close()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    s = hdp().Solver(w, tol=1e-12, max_iter=400, max_rhs=4, torch_memory=True)
    grown = torch.cuda.memory_allocated() - before
    assert grown >= 16 * s.n_coarse ** 2
    f, st = s.solve(kind, vals)
    got = f.cpu().numpy()
    del f
    assert st["iterations"] == st0["iterations"]
    assert rel(got, f0.cpu().numpy()) < 1e-14
    s.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_autotuned_nested_dissection_split(oracles):
    """The set-up autotuner times the nested-dissection sweeps at every split
    target and keeps the fastest; the interface operator with the chosen task
    cut equals the dense-inverse one at 5, 16 and 64 columns."""
    disc, l, E = oracles["scatterer_6x6_p6"]
    w = CASES["scatterer_6x6_p6"]
    sa = hdp().Solver(w, tol=1e-12, max_iter=400, max_rhs=64, coarse="nd", autotune=True)
    sd = hdp().Solver(w, tol=1e-12, max_iter=400, max_rhs=64, coarse="dense")
    rows = [t for t in sa.autotune_table() if t["kernel"] == "coarse_nd_split"]
    assert sorted(t["cols"] for t in rows) == [256, 512, 1024, 2048]
    assert sum(t["chosen"] for t in rows) == 1
    assert min(rows, key=lambda t: t["ms"])["chosen"]
    rng = np.random.default_rng(6)
    for R in (5, 16, 64):
        v = rng.standard_normal((E.nlam, R)) + 1j * rng.standard_normal((E.nlam, R))
        vd = torch.from_numpy(v).cuda()
        assert rel(sa.apply_interface(vd, "fp64").cpu().numpy(), sd.apply_interface(vd, "fp64").cpu().numpy()) < 1e-12
    sa.close()
    sd.close()


def test_point_source_32x32_against_stored_oracle_samples():
    """Full-size workload: sampled field values, F v and P^-1 v rows written by
    tests/golden/make_point_source_32x32.py from the oracle."""
    path = os.path.join(GOLD, "point_source_32x32_samples.txt")
    meta, field, Fv, Pv = {}, [], [], []
    for line in open(path):
        if line.startswith("#"):
            continue
        t = line.split()
        if t[0] == "field":
            field.append((int(t[1]), float(t[2]) + 1j * float(t[3])))
        elif t[0] == "Fv":
            Fv.append((int(t[1]), float(t[2]) + 1j * float(t[3])))
        elif t[0] == "Pv":
            Pv.append((int(t[1]), float(t[2]) + 1j * float(t[3])))
        else:
            meta[t[0]] = int(t[1])
    w = W.point_source_32x32()
    s = hdp().Solver(w, tol=1e-13, max_iter=400)
    assert (s.n_lambda, s.n_coarse, s.info["l"]) == (meta["n_lambda"], meta["n_coarse"], meta["l"])
    rng = np.random.default_rng(meta["vector_seed"])
    v = rng.standard_normal(s.n_lambda) + 1j * rng.standard_normal(s.n_lambda)
    vd = torch.from_numpy(v.reshape(-1, 1)).cuda()
    Fg = s.apply_interface(vd).cpu().numpy()[:, 0]
    Pg = s.apply_precond(vd).cpu().numpy()[:, 0]
    iF, vF = zip(*Fv)
    iP, vP = zip(*Pv)
    assert rel(Fg[list(iF)], vF) < 1e-11
    assert rel(Pg[list(iP)], vP) < 1e-12
    f, st = s.solve("point", [0.5, 0.5])
    g = f.cpu().numpy()[0]
    idx, vals = zip(*field)
    # both sides driven to a preconditioned residual of 1e-13
    assert rel(g[list(idx)], vals) < 1e-10
    assert st["converged"]
    # At this size the residual history is sensitive at the rounding level:
    # the oracle itself needs 111 -> 120 iterations (to 1e-8) and 149 -> 157
    # (to 1e-12) when F's output carries 1e-11 relative noise.  Iteration
    # counts are therefore compared within that measured band.
    hist = s.residual_history(0)
    it12 = next(i for i, h in enumerate(hist) if h <= 1e-12)
    assert abs(it12 - meta["iterations_1e-12"]) <= 10
    assert abs(st["iterations"] - meta["iterations_1e-13"]) <= 10
    s.close()
    s8 = hdp().Solver(w, tol=1e-8, max_iter=400)
    _, st8 = s8.solve("point", [0.5, 0.5], want_field=False)
    assert abs(st8["iterations"] - meta["iterations_1e-8"]) <= 10
    s8.close()


def test_graph_replays_match_eager_launches():
    """The GMRES iteration replayed as a captured graph gives the same solves as
    launching every kernel, over several solves with eager work in between."""
    w = CASES["uniform_5x5_p7_l3"]
    kind, vals = hdp().rhs_values(w)
    sg = hdp().Solver(w, tol=1e-11, graphs=True)
    se = hdp().Solver(w, tol=1e-11, graphs=False)
    ref, st_ref = se.solve(kind, vals)
    ref = ref.cpu().numpy()
    rng = np.random.default_rng(5)
    for rep in range(3):
        v = torch.from_numpy(rng.standard_normal((sg.n_lambda, 1)) + 0j).cuda()
        sg.apply_interface(v)
        torch.cuda.synchronize()
        f, st = sg.solve(kind, vals)
        assert st["iterations"] == st_ref["iterations"]
        assert rel(f.cpu().numpy(), ref) < 1e-13
    for prec in ("mixed",):
        sm = hdp().Solver(w, tol=1e-11, precision=prec, graphs=True)
        sme = hdp().Solver(w, tol=1e-11, precision=prec, graphs=False)
        a, _ = sm.solve(kind, vals)
        b, _ = sme.solve(kind, vals)
        a2, _ = sm.solve(kind, vals)
        assert rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-12
        assert rel(a2.cpu().numpy(), b.cpu().numpy()) < 1e-12
        sm.close()
        sme.close()
    sg.close()
    se.close()


def test_far_field_matches_oracle(oracles):
    """E_far over the boundary of the dielectric block (Sec. 3.3.1, e^{-iwt} form)."""
    from oracle import farfield as ff
    name = "scatterer_6x6_p6"
    disc, l, E = oracles[name]
    w = CASES[name]
    inside = (np.asarray(w["eps_r"]) != 1.0)
    angles = np.linspace(0, 2 * np.pi, 37)
    s = hdp().Solver(w, tol=1e-12, max_iter=400, max_rhs=2)
    kind, vals = hdp().rhs_values(w)
    vals2 = np.array([vals[0], vals[0] + 1.3])
    field, far, st = s.solve(kind, vals2, far_angles=angles, far_inside=inside)
    far = far.cpu().numpy()
    for r, a in enumerate(vals2):
        w1 = dict(w, rhs=dict(kind=kind, angles=[a]))
        d1 = pb.Discretisation(w1)
        E1 = dpe.ElementwiseDP(d1, l)
        phis = E1.solve(tol=1e-12, max_iter=400)
        ref = ff.far_field(d1.mesh, d1.degrees, phis, d1.k, inside, angles)
        assert rel(far[r], ref) < 1e-9
    s.close()
