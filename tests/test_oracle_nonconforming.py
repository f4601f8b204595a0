"""Pins of the element-by-element dual-primal oracle on quadtree meshes
(oracle/dp_nonconforming.py) against the literal projected-basis method
(oracle/dp.py, Sec. 2.3.1-2.3.3) and against the conforming element-wise
oracle: the interface operator F, the interface right-hand side and the field
are properties of the constrained space, not of its basis, so all three must
agree; the preconditioner is basis-dependent and is not compared."""
import numpy as np
import pytest

import workloads as W
from oracle import dp, dp_elementwise as dpe, dp_nonconforming as dnc, problem as pb

CASES = W.hanging_cases()


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


@pytest.fixture(scope="module")
def pairs():
    out = {}
    for name, w in CASES.items():
        disc = pb.Discretisation(w)
        l = pb.coarse_order(w, disc.mesh)
        out[name] = (dp.LiteralDP(disc, l), dnc.NonconformingDP(disc, l))
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_interface_operator_and_rhs_equal_the_literal_method(name, pairs):
    L, N = pairs[name]
    assert N.nlam == L.F.shape[0]
    rng = np.random.default_rng(2)
    for _ in range(2):
        v = rng.standard_normal(N.nlam) + 1j * rng.standard_normal(N.nlam)
        assert rel(N.apply_F(v), L.F @ v) < 1e-12
    assert rel(N.interface_rhs(), L.g) < 1e-12
    # hanging edges make C_2 non-zero (the dual rows reach the coarse side's modes)
    assert N.C2.nnz > 0


@pytest.mark.parametrize("name", ["h3_p3to6_l2", "h3_p3to6_l2_tau", "disk_6x6_p3to6"])
def test_field_of_a_direct_interface_solve_equals_the_literal_method(name, pairs):
    """nu = F^-1 g (dense, no iteration) and the recovered field against the
    literal method's direct interface solve."""
    L, N = pairs[name]
    Fd = np.stack([N.apply_F(e) for e in np.eye(N.nlam, dtype=complex)], axis=1)
    nu = np.linalg.solve(Fd, N.interface_rhs())
    f = np.concatenate(N.recover(nu))
    f0 = np.concatenate(L.recover(L.direct_interface()))
    assert rel(f, f0) < 1e-11


def test_iterative_solve_reaches_the_literal_field(pairs):
    """GMRES with the oracle's own preconditioner to 1e-12 lands within the
    tolerance's reach of the literal method's solution."""
    L, N = pairs["disk_6x6_p3to6"]
    phis = N.solve(tol=1e-12, max_iter=400)
    f0 = np.concatenate(L.recover(L.direct_interface()))
    assert rel(np.concatenate(phis), f0) < 1e-9


def test_conforming_mesh_equals_the_conforming_element_wise_oracle():
    """No hanging edge: C_2 = 0 and F, the right-hand side and the coarse size
    are those of oracle/dp_elementwise.py."""
    w = W.small_uniform(4, 6, 7.0, l=2)
    disc = pb.Discretisation(w)
    l = pb.coarse_order(w, disc.mesh)
    N = dnc.NonconformingDP(disc, l)
    Ew = dpe.ElementwiseDP(disc, l)
    assert N.C2.nnz == 0 and N.nK == Ew.nK and N.nlam == Ew.nlam
    v = np.random.default_rng(3).standard_normal(N.nlam) + 0j
    assert rel(N.apply_F(v), Ew.apply_F(v)) < 1e-12
    assert rel(N.interface_rhs(), Ew.interface_rhs()) < 1e-12


def test_what_the_discard_threshold_changes():
    """Sec. 2.2.4 drops the dual rows of a hanging edge whose L_c^f diagonal a^k
    has decayed below a user threshold tau; the rows are part of the discrete
    problem, so dropping them changes the solution.  On the small refined disk
    (p 3..6, two refinement levels, a = 1/4): tau = 1e-8 and 1e-4 drop nothing
    and give the Galerkin solution of the conforming space (direct solve, every
    row); tau = 1e-3 drops the rows of degree 5 and 6 (427 -> 389 dual rows) and
    moves the field by 2.7e-3 relative; tau = 1e-2 drops degree 4 too (359) and
    moves it by 1.5e-2.  The refined-disk workload uses tau = 1e-3."""
    from oracle import direct
    w0 = W.small_disk(tau=0.0)
    d0 = pb.Discretisation(w0)
    exact = np.concatenate(pb.gll_field(d0.mesh, d0.degrees, direct.conforming_solution(d0)))
    got = {}
    for tau in (1e-8, 1e-4, 1e-3, 1e-2):
        w = W.small_disk(tau=tau)
        disc = pb.Discretisation(w)
        N = dnc.NonconformingDP(disc, pb.coarse_order(w, disc.mesh))
        Fd = np.stack([N.apply_F(e) for e in np.eye(N.nlam, dtype=complex)], axis=1)
        nu = np.linalg.solve(Fd, N.interface_rhs())
        got[tau] = (N.nlam, rel(np.concatenate(pb.gll_field(disc.mesh, disc.degrees, N.recover(nu))), exact))
    assert got[1e-8][0] == got[1e-4][0] == 427 and got[1e-3][0] == 389 and got[1e-2][0] == 359
    assert got[1e-8][1] < 1e-12 and got[1e-4][1] < 1e-12
    assert 2e-3 < got[1e-3][1] < 4e-3
    assert 1e-2 < got[1e-2][1] < 2e-2
