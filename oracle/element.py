"""Element matrices and loads on an axis-aligned rectangle (paper Sec. 2.1.5, 2.2.1).
Test infrastructure only.

Unknowns of one element are vec(Phi) with the x-mode index fastest, so the
element matrix is a sum of Kronecker products written (y-factor) (x) (x-factor),
Sec. 2.2.1.  Sides are numbered as the paper's Gamma_1..Gamma_4: 1 left (x=-1),
2 right (x=+1), 3 bottom (y=-1), 4 top (y=+1).
"""
import numpy as np

from . import legendre as lg


def side_vector(n, side):
    """e_1 + (-1)^i e_2 of the Robin, Dirichlet and constraint formulas (Sec. 2.2.1)."""
    v = np.zeros(n)
    v[0] = 1.0
    if n > 1:
        v[1] = (-1.0) ** side
    return v


def element_matrix(n, hx, hy, alpha=1.0, beta=0.0, robin=None):
    """A_j for constant alpha = alpha*I, or alpha = diag(alpha[0], alpha[1]) when a
    pair is given, and constant beta on an hx-by-hy rectangle.

    Volume terms from the Kronecker identity of Sec. 2.2.1 (eq. complicated_integral
    with the X_i of Table tab:volume_integrals); for constant coefficients only
    T_0 = I/sqrt(2) enters, so S_11 ~ M^ (x) K^, S_22 ~ K^ (x) M^, M ~ M^ (x) M^.
    The mapping of [-1,1] onto an interval of length h has J = h/2; derivative
    terms carry sign(J) J^-1 and integral terms |J| (Sec. 2.1.5), per axis.
    ``robin`` maps a side (1..4) to a constant gamma; its term is
    R_i = |J_edge| gamma M^ (x) (1/2) v v^T (sides 1,2) or (1/2) v v^T (x) M^ (sides 3,4),
    v = e_1 + (-1)^i e_2 (Sec. 2.2.1).
    """
    K = lg.stiffness_1d(n)
    M = lg.mass_1d(n)
    Jx, Jy = hx / 2.0, hy / 2.0
    axx, ayy = (alpha, alpha) if np.isscalar(alpha) else alpha
    # vec order x fastest: kron(M, K) carries the x derivatives, kron(K, M) the y ones
    A = (axx * (Jy / Jx) * np.kron(M, K) + ayy * (Jx / Jy) * np.kron(K, M)
         + beta * Jx * Jy * np.kron(M, M)).astype(complex)
    for side, gamma in (robin or {}).items():
        v = side_vector(n, side)
        vv = 0.5 * np.outer(v, v)
        if side in (1, 2):
            A = A + gamma * Jy * np.kron(M, vv)
        else:
            A = A + gamma * Jx * np.kron(vv, M)
    return A


def legendre_coeffs_1d(fun, n, nq=None):
    """Legendre coefficients int_{-1}^{1} f(s) p(s) ds by Gauss quadrature
    (eq. legendre_coefficients; direct evaluation for small K_f, Sec. 2.1.2)."""
    nq = nq or (n + 40)
    s, w = np.polynomial.legendre.leggauss(nq)
    return lg.legendre_p(s, n) @ (w * fun(s))


def legendre_coeffs_2d(fun, n, nq=None):
    """F^ with F^_ij = int int f(u,v) p_i(u) p_j(v) du dv (Sec. 2.2.1, quadrature form)."""
    nq = nq or (n + 40)
    s, w = np.polynomial.legendre.leggauss(nq)
    U, V = np.meshgrid(s, s, indexing="ij")
    F = fun(U, V) * np.outer(w, w)
    P = lg.legendre_p(s, n)
    return P @ F @ P.T


def volume_load(n, hx, hy, Fhat):
    """f~ = |J| vec((S U) Sigma (S V)^T) with U Sigma V^T = F^ (Sec. 2.2.1),
    returned as vec with the x index fastest."""
    S = lg.basis_S(n)
    G = (hx / 2.0) * (hy / 2.0) * (S @ Fhat @ S.T)
    return G.reshape(-1, order="F")


def edge_load(n, h_edge, side, qhat):
    """r_i = |J_edge| S q_i (x) v/sqrt2 (sides 1,2) or v/sqrt2 (x) S q_i (sides 3,4),
    v = e_1 + (-1)^i e_2, Sec. 2.2.1; qhat holds the Legendre coefficients of q
    along the edge."""
    S = lg.basis_S(n)
    v = side_vector(n, side) / np.sqrt(2.0)
    Sq = (h_edge / 2.0) * (S @ qhat)
    if side in (1, 2):
        return np.kron(Sq, v)
    return np.kron(v, Sq)


def point_load(n, u, v):
    """int N(x) delta(x - x0) = N(u) (x) ... evaluated at the local point (u, v):
    vec with x fastest is kron(N(v), N(u))."""
    return np.kron(lg.basis_N(np.array(v), n), lg.basis_N(np.array(u), n))


def dirichlet_rows(n, side):
    """C_i of Sec. 2.2.1: I (x) v^T (sides 1,2) or v^T (x) I (sides 3,4), v = e_1 + (-1)^i e_2."""
    v = side_vector(n, side)[None, :]
    I = np.eye(n)
    if side in (1, 2):
        return np.kron(I, v)
    return np.kron(v, I)


def dirichlet_data(n, phat):
    """d_i = sqrt(2) S^{-T} p_i (Sec. 2.2.1)."""
    S = lg.basis_S(n)
    return np.sqrt(2.0) * np.linalg.solve(S.T, phat)


def to_vertex_basis(n):
    """B (x) B, mapping N~-coefficients to N-coefficients (Sec. 2.3.2, B_j = B (x) B)."""
    B = lg.B_matrix(n)
    return np.kron(B, B)
