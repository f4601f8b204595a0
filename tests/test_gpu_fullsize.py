"""Full-size parity of the HIP path against stored oracle samples, through the
C ABI (samples written by the committed scripts in tests/golden/, which call
only oracle/):

- the 64x64 dielectric-square scatterer (p = 12, k = 150, eps_r = 4, l = 6,
  692,224 unknowns) solved for all 64 incidence angles in one batched call:
  at the two stored angles the field samples and the 360-angle far field equal
  the oracle's to 1e-10 (FP64, both sides driven to 1e-12 / 1e-13) and to 1e-8
  on the mixed path; single applications of F and P^-1 to 1e-12; iterations to
  1e-8 within one of the oracle's (the per-column residual history);
- the 32x32 point source (p = 16, k = 100, 295,936 unknowns): the mixed path's
  field equals the oracle's to 1e-8;
- the refined disk (712 leaves, up to three hanging nodes per edge, p 8..24,
  230,391 unknowns): F v and the interface right-hand side to 1e-11, the field
  to 1e-10 (FP64) and 1e-8 (mixed), against the quadtree element-wise oracle,
  with l = 14 and with the per-edge coarse orders;
- the layered scatterer (80x80 elements with 8 PML rings) and the
  Robin-modified point source against the element-wise oracle: F v, P^-1 v, the
  interface right-hand side, the field and the iteration count.
"""
import os

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def hdp():
    import paper_1808_04713_amd as m
    return m


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _scatterer_samples():
    meta, Fv, Pv = {}, [], []
    field, far, iters = {}, {}, {}
    for line in open(os.path.join(GOLD, "square_scatterer_64x64_samples.txt")):
        if line.startswith("#"):
            continue
        t = line.split()
        if t[0] in ("Fv", "Pv"):
            (Fv if t[0] == "Fv" else Pv).append((int(t[1]), float(t[2]) + 1j * float(t[3])))
        elif t[0] == "field":
            field.setdefault(int(t[1]), []).append((int(t[2]), float(t[3]) + 1j * float(t[4])))
        elif t[0] == "far":
            far.setdefault(int(t[1]), []).append((int(t[2]), float(t[3]) + 1j * float(t[4])))
        elif t[0] == "angle":
            iters[int(t[1])] = (int(t[3]), int(t[5]))
        else:
            meta[t[0]] = int(t[1])
    return meta, Fv, Pv, field, far, iters


@pytest.fixture(scope="module")
def scatterer():
    return W.square_scatterer_64x64(), _scatterer_samples()


def test_square_scatterer_operators(scatterer):
    w, (meta, Fv, Pv, _, _, _) = scatterer
    s = hdp().Solver(w, max_rhs=1, max_iter=5)
    assert (s.n_lambda, s.n_coarse, s.info["l"]) == (meta["n_lambda"], meta["n_coarse"], meta["l"])
    rng = np.random.default_rng(meta["vector_seed"])
    v = rng.standard_normal(s.n_lambda) + 1j * rng.standard_normal(s.n_lambda)
    vd = torch.from_numpy(v.reshape(-1, 1)).cuda()
    Fg = s.apply_interface(vd).cpu().numpy()[:, 0]
    Pg = s.apply_precond(vd).cpu().numpy()[:, 0]
    iF, vF = zip(*Fv)
    iP, vP = zip(*Pv)
    assert rel(Fg[list(iF)], vF) < 1e-12
    assert rel(Pg[list(iP)], vP) < 1e-12
    s.close()


@pytest.mark.parametrize("precision,tol,bar", [("fp64", 1e-12, 1e-10), ("mixed", 1e-10, 1e-8)])
def test_square_scatterer_batched_solve(scatterer, precision, tol, bar):
    w, (meta, _, _, field, far, iters) = scatterer
    s = hdp().Solver(w, precision=precision, tol=tol, max_iter=60, max_rhs=64, autotune=True)
    angles = np.asarray(w["rhs"]["angles"])
    inside = np.asarray(w["eps_r"]) != 1.0
    print(f"scatterer 64 angles {precision} tol {tol}", flush=True)
    f, E, st = s.solve("plane_wave_scattered", angles, far_angles=w["far_angles"], far_inside=inside)
    assert st["converged"], st
    f = f.cpu().numpy()
    E = E.cpu().numpy()
    for m in field:
        idx, vals = zip(*field[m])
        assert rel(f[m][list(idx)], vals) < bar, (m, rel(f[m][list(idx)], vals))
        q, fv = zip(*far[m])
        assert rel(E[m][list(q)], fv) < bar, (m, rel(E[m][list(q)], fv))
        if precision == "fp64":
            hist = s.residual_history(m)
            it8 = next(i for i, h in enumerate(hist) if h <= 1e-8)
            assert abs(it8 - iters[m][0]) <= 1
    s.close()


def test_point_source_mixed_full_size():
    path = os.path.join(GOLD, "point_source_32x32_samples.txt")
    field = []
    for line in open(path):
        t = line.split()
        if t and t[0] == "field":
            field.append((int(t[1]), float(t[2]) + 1j * float(t[3])))
    w = W.point_source_32x32()
    s = hdp().Solver(w, precision="mixed", tol=1e-10, max_iter=400)
    f, st = s.solve("point", [0.5, 0.5])
    assert st["converged"]
    idx, vals = zip(*field)
    assert rel(f.cpu().numpy()[0][list(idx)], vals) < 1e-8
    s.close()


def _disk_samples(name):
    meta, field, Fv, g = {}, [], [], []
    for line in open(os.path.join(GOLD, name + "_samples.txt")):
        if line.startswith("#"):
            continue
        t = line.split()
        if t[0] in ("field", "Fv", "g"):
            {"field": field, "Fv": Fv, "g": g}[t[0]].append((int(t[1]), float(t[2]) + 1j * float(t[3])))
        else:
            meta[t[0]] = int(t[1])
    return meta, field, Fv, g


@pytest.mark.parametrize("name", ["refined_disk", "refined_disk_per_edge"])
def test_refined_disk_full_size_against_the_oracle(name):
    """The 712-leaf refined disk (p 8..24, k = 200, l = 14 or the per-edge
    orders, discard threshold 1e-3, up to three hanging nodes per edge) against
    the element-wise oracle on quadtree meshes (samples by
    tests/golden/make_refined_disk.py): rows of F v
    to 1e-11, of the interface right-hand side to 1e-10 (it carries one coarse
    solve by itself, and the nested-dissection factor's set-up check on this
    mesh, ||K x - b|| / ||b||, is about 1e-10), the field to 1e-10 (FP64, GMRES
    to 1e-12) and to 1e-8 (mixed, to 1e-10)."""
    meta, field, Fv_ref, g_ref = _disk_samples(name)
    w = W.refined_disk()
    if name.endswith("per_edge"):
        w = dict(w, l_per_edge=True)
    kind, vals = hdp().rhs_values(w)
    s = hdp().Solver(w, tol=1e-12, max_iter=800)
    assert (s.n_lambda, s.n_coarse) == (meta["n_lambda"], meta["n_coarse"])
    assert "l" not in meta or s.info["l"] == meta["l"]
    rng = np.random.default_rng(meta["vector_seed"])
    v = rng.standard_normal(s.n_lambda) + 1j * rng.standard_normal(s.n_lambda)
    Fv = s.apply_interface(torch.from_numpy(v[:, None].copy()).cuda(), "fp64").cpu().numpy()[:, 0]
    idx, ref = zip(*Fv_ref)
    assert rel(Fv[list(idx)], ref) < 1e-11
    g = s.interface_rhs(kind, vals).cpu().numpy()[:, 0]
    idx, ref = zip(*g_ref)
    print("coarse check", s.info["coarse_residual"], "g", rel(g[list(idx)], ref), flush=True)
    assert rel(g[list(idx)], ref) < 1e-10
    f, st = s.solve(kind, vals)
    assert st["converged"]
    idx, ref = zip(*field)
    print("iterations", st["iterations"], "field", rel(f.cpu().numpy()[0][list(idx)], ref), flush=True)
    assert rel(f.cpu().numpy()[0][list(idx)], ref) < 1e-10
    s.close()
    s = hdp().Solver(w, precision="mixed", tol=1e-10, max_iter=800)
    f, st = s.solve(kind, vals)
    assert st["converged"]
    assert rel(f.cpu().numpy()[0][list(idx)], ref) < 1e-8
    s.close()


def _widened_samples(name):
    meta, rows = {}, {"field": [], "Fv": [], "Pv": [], "g": []}
    for line in open(os.path.join(GOLD, name + "_samples.txt")):
        if line.startswith("#"):
            continue
        t = line.split()
        if t[0] in rows:
            rows[t[0]].append((int(t[1]), float(t[2]) + 1j * float(t[3])))
        else:
            meta[t[0]] = int(t[1])
    return meta, rows


@pytest.mark.parametrize("name", ["pml_scatterer_80x80", "point_source_32x32_robin_modified"])
def test_layers_and_robin_modified_full_size_against_the_oracle(name):
    """The layered scatterer (80x80 elements, 8 layer rings, p = 12, k = 150)
    and the Robin-modified 32x32 point source (p = 16, k = 100) against the
    element-wise oracle (samples by tests/golden/make_pml_and_robin_modified.py):
    rows of F v and P^-1 v to 1e-11; the interface right-hand side, which also
    carries a full-element separable solve of every loaded element (eigenbasis
    contractions, held to 1e-11 against dense solves per element by
    test_gpu_parity) and a coarse solve, to 1e-10; the field to 1e-10 (FP64,
    GMRES to 1e-12); iterations to 1e-8 within the rounding sensitivity of the
    residual history: on the 32x32 point source a relative perturbation of 1e-11
    in F's output moves the oracle's count from 111 to 120, so the window is
    max(10, 8 % of the oracle's count).
    Robin-modified elements next to the impedance boundary carry +ik on one end
    of a 1-D pencil and -ik on the other; that pencil's eigenbasis, which the
    separable solver and the class operators are built from, has condition
    number 1.8e3 at p = 16, k h = 3.1 (1.2e2 with equal or no Robin terms), so the
    library's element solves carry up to cond(E_x) cond(E_y) eps ~ 7e-10 of
    rounding there: that variant is held to 1e-9 throughout."""
    meta, rows = _widened_samples(name)
    if name.startswith("pml"):
        w = W.pml_scatterer_64x64()
        bars = {"Fv": 1e-11, "Pv": 1e-11, "g": 1e-10, "field": 1e-10}
    else:
        w = dict(W.point_source_32x32(), robin_modified=True)
        bars = {"Fv": 1e-9, "Pv": 1e-9, "g": 1e-9, "field": 1e-9}
    kind, vals = hdp().rhs_values(w)
    s = hdp().Solver(w, tol=1e-12, max_iter=800)
    assert (s.n_lambda, s.n_coarse, s.info["l"]) == (meta["n_lambda"], meta["n_coarse"], meta["l"])
    rng = np.random.default_rng(meta["vector_seed"])
    v = rng.standard_normal(s.n_lambda) + 1j * rng.standard_normal(s.n_lambda)
    vd = torch.from_numpy(v.reshape(-1, 1)).cuda()
    got = {"Fv": s.apply_interface(vd).cpu().numpy()[:, 0], "Pv": s.apply_precond(vd).cpu().numpy()[:, 0],
           "g": s.interface_rhs(kind, vals).cpu().numpy()[:, 0]}
    for key in ("Fv", "Pv", "g"):
        idx, ref = zip(*rows[key])
        print(name, key, rel(got[key][list(idx)], ref), flush=True)
        assert rel(got[key][list(idx)], ref) < bars[key]
    f, st = s.solve(kind, vals)
    assert st["converged"]
    idx, ref = zip(*rows["field"])
    it8 = next(i for i, h in enumerate(s.residual_history(0)) if h <= 1e-8)
    print(name, "field", rel(f.cpu().numpy()[0][list(idx)], ref), "it8", it8, meta["iterations_1e-8"], flush=True)
    assert rel(f.cpu().numpy()[0][list(idx)], ref) < bars["field"]
    assert abs(it8 - meta["iterations_1e-8"]) <= max(10, 0.08 * meta["iterations_1e-8"])
    s.close()
