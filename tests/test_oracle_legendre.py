"""Pins of the oracle's 1-D toolkit (paper Sec. 2.1.1, 2.1.6, 2.2.4, 2.3.4)
against closed forms, NumPy's own Legendre series module and printed values."""
import os

import numpy as np
import numpy.polynomial.legendre as npl
import pytest

from oracle import legendre as lg
from oracle.mesh import Mesh
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def np_orthonormal(k):
    """p_k from NumPy's Legendre series: sqrt((2k+1)/2) P_k."""
    c = np.zeros(k + 1)
    c[k] = np.sqrt((2 * k + 1) / 2.0)
    return c


def np_integrated(k):
    """Integrated Legendre basis built independently: N_0 = 1/sqrt2,
    N_1 = x/sqrt2, N_k = int_{-1}^{x} p_{k-1} for k >= 2."""
    if k == 0:
        return np.array([1 / np.sqrt(2)])
    if k == 1:
        return np.array([0.0, 1 / np.sqrt(2)])
    return npl.legint(np_orthonormal(k - 1), lbnd=-1)


def test_orthonormal_recurrence_matches_numpy_and_is_orthonormal():
    x = np.linspace(-1, 1, 23)
    P = lg.legendre_p(x, 12)
    for k in range(12):
        assert np.allclose(P[k], npl.legval(x, np_orthonormal(k)), atol=1e-13)
    assert np.isclose(P[0, 0], 1 / np.sqrt(2)) and np.allclose(P[1], np.sqrt(1.5) * x)
    xq, wq = npl.leggauss(20)
    Pq = lg.legendre_p(xq, 12)
    assert np.allclose((Pq * wq) @ Pq.T, np.eye(12), atol=1e-13)


def test_differentiation_matrix():
    x = np.linspace(-0.9, 0.95, 17)
    n = 11
    dP = np.array([npl.legval(x, npl.legder(np_orthonormal(k))) for k in range(n)])
    assert np.allclose(lg.diff_matrix(n) @ lg.legendre_p(x, n), dP, atol=1e-11)


def test_integrated_basis_S_and_matrices():
    n = 10
    x = np.linspace(-1, 1, 31)
    N = lg.basis_N(x, n)
    for k in range(n):
        assert np.allclose(N[k], npl.legval(x, np_integrated(k)), atol=1e-13)
    # bubbles vanish at +-1; N(+-1) = (e1 +- e2)/sqrt2
    assert np.allclose(lg.basis_N(np.array([-1.0, 1.0]), n)[2:], 0, atol=1e-14)
    assert np.allclose(lg.basis_N(np.array(1.0), n), lg.N_at_pm1(n, +1))
    assert np.allclose(lg.basis_N(np.array(-1.0), n), lg.N_at_pm1(n, -1))
    # K^ = diag(0,1,...,1), M^ pentadiagonal with zero first off-diagonals, M^_33 = 2/5
    assert np.allclose(lg.stiffness_1d(n), np.diag([0.0] + [1.0] * (n - 1)))
    M = lg.mass_1d(n)
    xq, wq = npl.leggauss(n + 2)
    Nq = np.array([npl.legval(xq, np_integrated(k)) for k in range(n)])
    assert np.allclose(M, (Nq * wq) @ Nq.T, atol=1e-14)
    assert np.isclose(M[2, 2], 0.4)
    assert np.allclose(np.diag(M, 1), 0) and np.allclose(np.triu(M, 3), 0)
    dNq = np.array([npl.legval(xq, npl.legder(np_integrated(k))) for k in range(n)])
    assert np.allclose(lg.stiffness_1d(n), (dNq * wq) @ dNq.T, atol=1e-13)


def test_Q_and_B_are_involutory_and_give_vertex_functions():
    n = 7
    B = lg.B_matrix(n)
    assert np.allclose(lg.Q_matrix() @ lg.Q_matrix(), np.eye(2))
    assert np.allclose(B @ B, np.eye(n))
    x = np.linspace(-1, 1, 9)
    Nt = B @ lg.basis_N(x, n)
    assert np.allclose(Nt[0], (1 + x) / 2) and np.allclose(Nt[1], (1 - x) / 2)


@pytest.mark.parametrize("a,b", [(0.5, 0.5), (0.5, -0.5), (0.125, -0.125), (0.25, 0.625), (1.0, 0.0)])
def test_affine_L(a, b):
    n = 14
    L = lg.affine_L(n, a, b)
    x = np.linspace(-1, 1, 13)
    # the defining identity p(ax+b) = L p(x), evaluated pointwise
    assert np.allclose(lg.legendre_p(a * x + b, n), L @ lg.legendre_p(x, n), atol=1e-12)
    assert np.allclose(L, lg.affine_L_quadrature(n, a, b), atol=1e-13)
    assert np.allclose(np.triu(L, 1), 0)
    assert np.allclose(np.diag(L), a ** np.arange(n), rtol=1e-12)
    Nf = lg.basis_N(a * x + b, n)
    assert np.allclose(Nf, lg.affine_L_basis(n, a, b) @ lg.basis_N(x, n), atol=1e-12)


def test_affine_L_identity_composition_and_decay():
    n = 12
    assert np.allclose(lg.affine_L(n, 1.0, 0.0), np.eye(n), atol=1e-14)
    a1, b1, a2, b2 = 0.5, -0.5, 0.5, 0.5
    # p(a1 (a2 x + b2) + b1) = L(a1,b1) L(a2,b2) p(x)
    assert np.allclose(lg.affine_L(n, a1, b1) @ lg.affine_L(n, a2, b2),
                       lg.affine_L(n, a1 * a2, a1 * b2 + b1), atol=1e-13)
    # one level of refinement at degree 32: the diagonal has decayed to 2^-32 ~ 2.3e-10
    assert np.isclose(lg.affine_L(33, 0.5, 0.5)[32, 32], 2.0 ** -32, rtol=1e-9)


def test_affine_parameters_figure_example_and_geometry():
    # Fig. 2 example: a level-3 fine element below a level-0 coarse element whose
    # signs are (s1, s2, s3) = (+, +, -): a = 1/8, b = -1/8, i.e. the fine edge is
    # the coarse sub-interval [-1/4, 0].
    lv = W.refine_where([(0, 0, 0)], 0, 1, 0, 2, 1, 2, lambda x, y: True, 3) + [(0, 0, 1)]
    m = Mesh(0, 1, 0, 2, 1, 2, lv)
    fine = m.leaves.index((3, 3, 7))
    (c, sc), = m.neighbours(fine, 4)
    assert m.leaves[c] == (0, 0, 1) and sc == 3
    assert m.affine_params(fine, 4, c) == (0.125, -0.125)
    assert np.allclose(m.affine_params_geometric(fine, 4, c), (0.125, -0.125))
    # on a refined mesh the sign-sequence formula equals the coordinates
    lv = W.refine_where(W.morton_leaves(4, 4), 0, 1, 0, 1, 4, 4,
                        lambda x, y: (x - 0.4) ** 2 + (y - 0.45) ** 2 < 0.05, 2)
    mesh = Mesh(0, 1, 0, 1, 4, 4, lv)
    seen = 0
    for e in range(mesh.E):
        for side in (1, 2, 3, 4):
            if mesh.boundary_side(e, side):
                continue
            nb = mesh.neighbours(e, side)
            if len(nb) == 1 and mesh.leaves[nb[0][0]][0] < mesh.leaves[e][0]:
                assert np.allclose(mesh.affine_params(e, side, nb[0][0]),
                                   mesh.affine_params_geometric(e, side, nb[0][0]))
                seen += 1
    assert seen > 8


def test_dispersion_rule_printed_threshold():
    # k = 10.75, h = 1: criterion holds for l >~ 5.9785 (Sec. 2.3.4)
    x = 0.5 * (10.75 + 10.75 ** (1 / 3) - 1)
    assert abs(x - 5.9785) < 5e-5
    assert lg.dispersion_l(10.75, 1.0) == 6
    assert lg.dispersion_l(0.1, 1.0) == 1


def test_dispersion_rule_reproduces_table2_bold_pattern():
    rows = [l.split() for l in open(os.path.join(GOLD, "table2_bold.txt")) if l[0] != "#"]
    for k, N, lb in rows:
        h = 2.0 / np.sqrt(int(N))
        lmin = lg.dispersion_l(float(k), h)
        assert min(lmin, 5) == int(lb), (k, N)


def test_gll_nodes():
    for n in (3, 5, 9, 17):
        t = lg.gll_nodes(n)
        p = n - 1
        assert len(t) == n and t[0] == -1 and t[-1] == 1 and np.all(np.diff(t) > 0)
        c = np.zeros(p + 1)
        c[p] = 1
        assert np.allclose(npl.legval(t[1:-1], npl.legder(c)), 0, atol=1e-10)
        assert np.allclose(t, -t[::-1])
