"""GPU checks of the separable element solve (Sec. 2.2.1, remark on the fast
solver) through the C ABI: X = Ex [(Ex^T Y Ey) ./ D] Ey^T on every element,
on the matrix cores for classes of at most 32 modes per direction (real
eigenbasis on interior elements, complex on impedance-boundary elements) and on
the vector ALUs above, against dense solves of each element matrix, at column
counts that exercise every column-block width; and the element solves of the
interface right-hand side and the recovery (coarse pass, coarse solve,
corrected full solve) against the oracle's block elimination."""
import numpy as np
import pytest

import workloads as W
from oracle import dp, dp_elementwise as dpe, element as el, problem as pb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def hdp():
    import paper_1808_04713_amd as m
    return m


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _mixed_degrees():
    """4x4 mesh with degrees 2..12 (several classes, real and complex bases)."""
    w = W.small_uniform(4, 6, 9.0, l=2)
    w["degree"] = np.random.default_rng(11).integers(2, 13, 16)
    return w


def _dense_ref(w, y):
    disc = pb.Discretisation(w)
    out = np.zeros_like(y)
    off = 0
    for e in range(disc.mesh.E):
        n = int(disc.degrees[e]) + 1
        B = el.to_vertex_basis(n)
        A = B @ disc.A[e] @ B
        out[off:off + n * n] = np.linalg.solve(A, y[off:off + n * n])
        off += n * n
    return out


@pytest.mark.parametrize("R", [1, 3, 8, 16, 64])
def test_local_solve_all_widths(R):
    w = _mixed_degrees()
    s = hdp().Solver(w, max_rhs=min(R, 64))
    rng = np.random.default_rng(R)
    y = rng.standard_normal((s.dof, R)) + 1j * rng.standard_normal((s.dof, R))
    print(f"local solve R={R}", flush=True)
    x = s.local_solve(torch.from_numpy(y).cuda()).cpu().numpy()
    assert rel(x, _dense_ref(w, y)) < 1e-11
    s.close()


@pytest.mark.parametrize("cols", [1, 2, 4, 8, 16])
def test_local_solve_every_tile_width(cols):
    w = _mixed_degrees()
    s = hdp().Solver(w, max_rhs=16, tile_fdm=cols)
    rng = np.random.default_rng(cols)
    y = rng.standard_normal((s.dof, 16)) + 1j * rng.standard_normal((s.dof, 16))
    x = s.local_solve(torch.from_numpy(y).cuda()).cpu().numpy()
    assert rel(x, _dense_ref(w, y)) < 1e-11
    s.close()


def test_autotuner_table_and_tuned_solve():
    """HDP_FLAG_AUTOTUNE times every tile width that fits and keeps the fastest;
    the tuned solver gives the same field as the untuned one."""
    w = _mixed_degrees()
    kind, vals = hdp().rhs_values(w)
    vals16 = np.linspace(0.0, 2 * np.pi, 16, endpoint=False)
    st = hdp().Solver(w, max_rhs=16, tol=1e-12, autotune=True)
    su = hdp().Solver(w, max_rhs=16, tol=1e-12)
    tab = st.autotune_table()
    fams = {t["kernel"] for t in tab}
    assert fams == {"fdm_element_solve", "slot_operator"}
    for fam in fams:
        rows = [t for t in tab if t["kernel"] == fam]
        assert sum(t["chosen"] for t in rows) == 1
        best = min(rows, key=lambda t: t["ms"])
        assert best["chosen"] and best["ms"] > 0
    assert {t["cols"] for t in tab if t["kernel"] == "fdm_element_solve"} == {1, 2, 4, 8, 16}
    a, _ = st.solve("plane_wave_total", vals16)
    b, _ = su.solve("plane_wave_total", vals16)
    assert rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-10
    assert su.autotune_table() == []
    st.close()
    su.close()


def test_local_solve_above_32_modes():
    """p = 34 (35 modes): the vector-ALU separable solve."""
    w = W.small_uniform(2, 34, 5.0, l=2)
    s = hdp().Solver(w)
    rng = np.random.default_rng(3)
    y = rng.standard_normal((s.dof, 2)) + 1j * rng.standard_normal((s.dof, 2))
    x = s.local_solve(torch.from_numpy(y).cuda()).cpu().numpy()
    assert rel(x, _dense_ref(w, y)) < 1e-10
    s.close()


@pytest.mark.parametrize("make", [_mixed_degrees, lambda: W.small_uniform(2, 34, 5.0, l=2)])
def test_interface_rhs_and_field_of_mixed_degrees(make):
    """The interface right-hand side (first element solve) and the field (the
    recovery) on a mesh of uneven degree, FP64, against the literal oracle."""
    w = make()
    disc = pb.Discretisation(w)
    l = pb.coarse_order(w, disc.mesh)
    D = dp.LiteralDP(disc, l)
    s = hdp().Solver(w, tol=1e-12, max_iter=300)
    kind, vals = hdp().rhs_values(w)
    g = s.interface_rhs(kind, vals).cpu().numpy()[:, 0]
    assert rel(g, D.g) < 1e-11
    field, st = s.solve(kind, vals)
    phis = D.solve(tol=1e-12, max_iter=300)
    ref = np.concatenate(pb.gll_field(disc.mesh, disc.degrees, phis))
    assert rel(field.cpu().numpy()[0], ref) < 1e-10
    s.close()
