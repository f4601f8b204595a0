"""GPU parity of the Robin-modified local problems (paper Sec. 2.3.4) against the
oracle, through the C ABI: interface operator, preconditioner and field on
small meshes, the element-resonance experiment of Sec. 3.2 at a small size, and
the full-size point source.  Tolerances as for the unmodified path."""
import numpy as np
import pytest

import workloads as W
from oracle import direct, dp_elementwise as dpe, problem as pb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def hdp():
    import paper_1808_04713_amd as m
    return m


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


CASES = {
    "uniform_4x4_p6_l2": dict(W.small_uniform(4, 6, 7.0, l=2), robin_modified=True),
    "uniform_5x5_p7_l3": dict(W.small_uniform(5, 7, 11.0, l=3), robin_modified=True),
    "point_4x4_p6": dict(W.small_uniform(4, 6, 9.0, rhs=dict(kind="point", points=[(0.5, 0.5)]), l=2),
                         robin_modified=True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_modified_operator_preconditioner_and_field(name):
    w = CASES[name]
    disc = pb.Discretisation(w)
    l = pb.coarse_order(w, disc.mesh)
    E = dpe.ElementwiseDP(disc, l)
    s = hdp().Solver(w, tol=1e-12, max_iter=400, max_rhs=2)
    assert s.n_lambda == E.nlam and s.n_coarse == E.nK
    rng = np.random.default_rng(3)
    v = rng.standard_normal((E.nlam, 2)) + 1j * rng.standard_normal((E.nlam, 2))
    vd = torch.from_numpy(v).cuda()
    Fv = s.apply_interface(vd, "fp64").cpu().numpy()
    Pv = s.apply_precond(vd, "fp64").cpu().numpy()
    for r in range(2):
        assert rel(Fv[:, r], E.apply_F(v[:, r])) < 1e-12
        assert rel(Pv[:, r], E.apply_P(v[:, r])) < 1e-12
    kind, vals = hdp().rhs_values(w)
    f, st = s.solve(kind, vals)
    assert st["converged"]
    ref = np.concatenate(pb.gll_field(disc.mesh, disc.degrees, direct.conforming_solution(disc)))
    assert rel(f.cpu().numpy()[0], ref) < 1e-10
    s.close()


def test_modified_solver_at_an_element_resonance():
    """At a wavenumber where the interior elements' A_11 is singular the
    Robin-modified solver still reaches the Galerkin solution."""
    import test_oracle_robin as tor
    l = 2
    w0 = W.small_uniform(4, 6, 8.0, l=l)
    kr = tor._interior_resonance(w0, l)
    w = dict(w0, k=float(kr), robin_modified=True)
    disc = pb.Discretisation(w)
    ref = np.concatenate(pb.gll_field(disc.mesh, disc.degrees, direct.conforming_solution(disc)))
    s = hdp().Solver(w, tol=1e-12, max_iter=200)
    kind, vals = hdp().rhs_values(w)
    f, st = s.solve(kind, vals)
    assert st["converged"]
    assert rel(f.cpu().numpy()[0], ref) < 1e-10
    s.close()


def test_point_source_32x32_modified_equals_unmodified():
    """Full size: the modified local problems change the interface problem (more
    iterations, as Sec. 2.3.4 remarks) but not the field."""
    w = W.point_source_32x32()
    kind, vals = hdp().rhs_values(w)
    fields, its = {}, {}
    for mod in (False, True):
        s = hdp().Solver(dict(w, robin_modified=mod), tol=1e-10, max_iter=600)
        f, st = s.solve(kind, vals)
        assert st["converged"]
        fields[mod] = f.cpu().numpy()[0]
        its[mod] = st["iterations"]
        s.close()
    assert rel(fields[True], fields[False]) < 1e-8
    assert its[True] > its[False]
