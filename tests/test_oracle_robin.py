"""Pins of the oracle's Robin-modified local problems (paper Sec. 2.3.4, and the
resonance experiment of Sec. 3.2): labels, cancellation in the assembled system,
convergence to the unmodified Galerkin solution, and robustness at an element
resonance where the unmodified local problems are singular."""
import warnings

import numpy as np
import pytest

import workloads as W
from oracle import constraints as cs
from oracle import direct, dp, dp_elementwise as dpe
from oracle import element as el
from oracle import problem as pb


def _uniform(n, p, k, **kw):
    w = W.small_uniform(n=n, p=p, k=k, **kw)
    return w


def _field_err(a, b):
    return max(np.abs(x - y).max() for x, y in zip(a, b)) / max(np.abs(y).max() for y in b)


def test_labels_alternate_on_a_conforming_grid():
    """A conforming grid graph is bipartite, so breadth-first levels alternate
    across every interior side: the labels form a checkerboard and every
    interior side carries the term."""
    w = _uniform(5, 3, 4.0)
    mesh = pb.make_mesh(w)
    lab = pb.robin_labels(mesh)
    for e, (_, ix, iy) in enumerate(mesh.leaves):
        assert lab[e] == (1 if (ix + iy) % 2 == 0 else -1)
        sides = pb.robin_sides(mesh, e, lab)
        interior = [s for s in (1, 2, 3, 4) if not mesh.boundary_side(e, s)]
        assert sides == interior


def test_labels_on_a_quadtree_mesh_reach_every_element():
    """Every element has a neighbour of the other label (the weak 2-colouring the
    method needs); where a coarse side meets fine leaves of both labels the term
    would cover part of a side only, which is refused."""
    lv = W.refine_where(W.morton_leaves(3, 3), 0, 1, 0, 1, 3, 3,
                        lambda x, y: (x - 0.5) ** 2 + (y - 0.5) ** 2 < 0.02, 1)
    mesh = pb.Mesh(0, 1, 0, 1, 3, 3, lv)
    lab = pb.robin_labels(mesh)
    for e in range(mesh.E):
        others = {lab[f] for s in (1, 2, 3, 4) for f, _ in mesh.neighbours(e, s)}
        assert -lab[e] in others
    with pytest.raises(NotImplementedError):
        for e in range(mesh.E):
            pb.robin_sides(mesh, e, lab)


def test_modified_terms_cancel_in_the_assembled_system():
    """The added terms are +ik and -ik times the same edge mass matrix on the two
    sides of an edge, so the globally conforming Galerkin solution does not
    change; the element matrices themselves do."""
    w = _uniform(4, 5, 7.0)
    d0 = pb.Discretisation(w)
    d1 = pb.Discretisation(dict(w, robin_modified=True))
    assert max(np.abs(a - b).max() for a, b in zip(d0.A, d1.A)) > 1.0
    # on an interior element all four sides carry the term: A1 - A0 is the sum of
    # gamma |J| times the edge mass matrices (closed form of Sec. 2.2.1)
    mesh = d0.mesh
    e = next(e for e in range(mesh.E) if not any(mesh.boundary_side(e, s) for s in (1, 2, 3, 4)))
    n = int(d0.degrees[e]) + 1
    g = d1.labels[e] * 1j * d1.k
    hx, hy = mesh.size(e)
    expect = el.element_matrix(n, hx, hy, robin={s: g for s in (1, 2, 3, 4)}) - el.element_matrix(n, hx, hy)
    assert np.abs((d1.A[e] - d0.A[e]) - expect).max() < 1e-12
    u0 = direct.conforming_solution(d0)
    u1 = direct.conforming_solution(d1)
    assert _field_err(u1, u0) < 1e-12


@pytest.mark.parametrize("n,p,k,l", [(4, 6, 7.0, 2), (5, 5, 12.0, 3)])
def test_modified_dual_primal_method_reaches_the_galerkin_solution(n, p, k, l):
    """Literal dual-primal method on the modified local problems: a different
    interface operator (complex symmetric, the dual variables change meaning)
    with the same converged field."""
    w = _uniform(n, p, k, l=l)
    d0 = pb.Discretisation(w)
    d1 = pb.Discretisation(dict(w, robin_modified=True))
    D0 = dp.LiteralDP(d0, l)
    D1 = dp.LiteralDP(d1, l)
    assert np.linalg.norm(D1.F - D0.F) > 1e-3 * np.linalg.norm(D0.F)
    assert np.abs(D1.F - D1.F.T).max() < 1e-9 * np.abs(D1.F).max()
    ref = direct.conforming_solution(d0)
    phis = D1.solve(tol=1e-12, max_iter=400)
    assert _field_err(phis, ref) < 1e-9


def _interior_resonance(w, l):
    """A wavenumber at which the type-1 block A_11 of the interior elements (no
    boundary side, no Robin term) is singular: A_11(k) = K_11 - k^2 M_11 is real,
    so its singular points are the square roots of the generalised eigenvalues of
    (K_11, M_11)."""
    mesh = pb.make_mesh(w)
    e = next(e for e in range(mesh.E) if not any(mesh.boundary_side(e, s) for s in (1, 2, 3, 4)))
    status = cs.algorithm1(mesh, np.asarray(w["degree"]), l, {s: "robin" for s in (1, 2, 3, 4)})
    I = np.nonzero(status[e] == 1)[0]
    n = int(w["degree"][e]) + 1
    hx, hy = mesh.size(e)
    B = el.to_vertex_basis(n)
    K = (B @ el.element_matrix(n, hx, hy) @ B)[np.ix_(I, I)].real
    M = -(B @ el.element_matrix(n, hx, hy, beta=1.0) @ B - B @ el.element_matrix(n, hx, hy) @ B)[np.ix_(I, I)].real
    lam = np.sort(np.linalg.eigvals(np.linalg.solve(-M, K)).real)
    return np.sqrt(lam[(lam > 4.0 ** 2) & (lam < 20.0 ** 2)][0])


def test_modified_method_converges_at_an_element_resonance():
    """At a wavenumber where the interior elements' A_11 is singular (Sec. 2.3.4)
    the unmodified method cannot form A_11^-1, while the Robin-modified local
    problems stay uniquely solvable and the method converges to the Galerkin
    solution (the experiment of Sec. 3.2, at a size the oracle handles)."""
    l = 2
    w0 = _uniform(4, 6, 8.0, l=l)
    kr = _interior_resonance(w0, l)
    w = dict(w0, k=float(kr))
    d0 = pb.Discretisation(w)
    d1 = pb.Discretisation(dict(w, robin_modified=True))
    ref = direct.conforming_solution(d0)
    # the unmodified interior block is singular to rounding
    mesh = d0.mesh
    e = next(e for e in range(mesh.E) if not any(mesh.boundary_side(e, s) for s in (1, 2, 3, 4)))
    status = cs.algorithm1(mesh, d0.degrees, l, d0.bc)
    I = np.nonzero(status[e] == 1)[0]
    B = el.to_vertex_basis(int(d0.degrees[e]) + 1)
    assert np.linalg.cond((B @ d0.A[e] @ B)[np.ix_(I, I)]) > 1e11
    assert np.linalg.cond((B @ d1.A[e] @ B)[np.ix_(I, I)]) < 1e6
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")   # the singular factorisation warns
        E0 = dpe.ElementwiseDP(d0, l)
        bad = E0.solve(tol=1e-12, max_iter=400)
    assert _field_err(bad, ref) > 1e-4
    E1 = dpe.ElementwiseDP(d1, l)
    phis = E1.solve(tol=1e-12, max_iter=400)
    assert _field_err(phis, ref) < 1e-10
