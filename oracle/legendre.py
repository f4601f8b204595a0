"""1-D Legendre toolkit (paper Sec. 2.1.1 and Sec. 2.1.6).  Test infrastructure only.

Conventions: ``n`` is the number of modes (degree p = n - 1); all vectors and
matrices are indexed from 0 (the paper indexes from 1).
"""
import numpy as np


def legendre_p(x, n):
    """Orthonormal Legendre polynomials p_0..p_{n-1} at points x.

    Three-term recurrence, Sec. 2.1, eq. (recurrence_relation):
    p_0 = 1/sqrt(2), p_1 = sqrt(3/2) x and, for k >= 2,
    p_k = sqrt((2k+1)(2k-1))/k * x p_{k-1} - (k-1)/k sqrt((2k+1)/(2k-3)) p_{k-2}.
    Returns an array of shape (n,) + x.shape.
    """
    x = np.asarray(x, dtype=float)
    P = np.zeros((n,) + x.shape)
    P[0] = 1.0 / np.sqrt(2.0)
    if n > 1:
        P[1] = np.sqrt(1.5) * x
    for k in range(2, n):
        P[k] = (np.sqrt((2 * k + 1) * (2 * k - 1)) / k * x * P[k - 1]
                - (k - 1) / k * np.sqrt((2 * k + 1) / (2 * k - 3)) * P[k - 2])
    return P


def diff_matrix(n):
    """D with d/dx p(x) = D p(x), Sec. 2.1 (entries after eq. derivative_property).

    1-based: d_ij = sqrt((2i-1)(2j-1)) when i+j is odd and i > j, else 0.
    """
    D = np.zeros((n, n))
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            if (i + j) % 2 == 1 and i > j:
                D[i - 1, j - 1] = np.sqrt((2 * i - 1) * (2 * j - 1))
    return D


def shift_down(n):
    """S_DL with (s_DL)_ij = delta_{i,j+1}, Sec. 2.1.1."""
    return np.eye(n, k=-1)


def basis_S(n):
    """S with N(x) = S p(x) for the integrated Legendre basis, Sec. 2.1.1,
    eq. (define_basis_functions): S = diag(g) - S_DL diag(g) S_DL with
    g_1 = 1 and g_i = 1/sqrt((2i-1)(2i-3)) (1-based)."""
    g = np.ones(n)
    for i in range(2, n + 1):
        g[i - 1] = 1.0 / np.sqrt((2 * i - 1) * (2 * i - 3))
    SDL = shift_down(n)
    return np.diag(g) - SDL @ np.diag(g) @ SDL


def stiffness_1d(n):
    """K^ = int N' N'^T = S_DL S_DL^T (uses dN/dx = S_DL p, eq. differentiation_property)."""
    SDL = shift_down(n)
    return SDL @ SDL.T


def mass_1d(n):
    """M^ = int N N^T = S S^T (orthonormality of p)."""
    S = basis_S(n)
    return S @ S.T


def basis_N(x, n):
    """N(x) = S p(x), shape (n,) + x.shape."""
    return np.tensordot(basis_S(n), legendre_p(x, n), axes=1)


def basis_dN(x, n):
    """d/dx N(x) = S_DL p(x)."""
    return np.tensordot(shift_down(n), legendre_p(x, n), axes=1)


def Q_matrix():
    """Q relating (N_0, N_1) to the interpolatory pair (l_0, l_1), Sec. 2.1.1."""
    return np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)


def B_matrix(n):
    """B = blockdiag(Q, I) with N~ = B N (eq. interpolatory_relation).

    In N~ the first function is l_0 = (1+x)/2 (value 1 at x=+1) and the second
    l_1 = (1-x)/2 (value 1 at x=-1); B is involutory.
    """
    B = np.eye(n)
    B[:2, :2] = Q_matrix()
    return B


def N_at_pm1(n, sign):
    """N(+1) = (e1+e2)/sqrt2 and N(-1) = (e1-e2)/sqrt2, Sec. 2.1.1."""
    v = np.zeros(n)
    v[0] = 1.0 / np.sqrt(2.0)
    if n > 1:
        v[1] = sign / np.sqrt(2.0)
    return v


def jacobi_matrix(n):
    """Truncated Jacobi matrix J_n of the orthonormal Legendre recurrence,
    Sec. 2.1.6 eq. (modified_recurrence): zero diagonal, off-diagonal
    sqrt(beta_k) = k / sqrt((2k+1)(2k-1)), k = 1..n-1."""
    J = np.zeros((n, n))
    for k in range(1, n):
        J[k - 1, k] = J[k, k - 1] = k / np.sqrt((2 * k + 1) * (2 * k - 1))
    return J


def affine_L(n, a, b):
    """Lower-triangular L with p(a x + b) = L p(x), Sec. 2.1.6.

    Rows are generated one after another from the Sylvester equation
    (eq. displacement_rank) A~ L - L B~ = -e_{n+1} p_{n+1}^T with
    A~ = J - b I, B~ = a J: row k of that equation (away from the last row)
    links rows k-1, k, k+1 of L, and the first row is e_1^T because an affine
    change of variable maps the constant p_0 to itself.  The matrices are
    enlarged by one row and column so the last needed row never touches the
    right-hand side term.
    """
    m = n + 1
    J = jacobi_matrix(m)
    At = J - b * np.eye(m)
    Bt = a * J
    L = np.zeros((m, m))
    L[0, 0] = 1.0
    for k in range(0, m - 1):
        row = L[k] @ Bt - At[k, k] * L[k]
        if k > 0:
            row = row - At[k, k - 1] * L[k - 1]
        L[k + 1] = row / At[k, k + 1]
    return L[:n, :n]


def affine_L_quadrature(n, a, b):
    """L = int_{-1}^{1} p(a x + b) p(x)^T dx by Gauss-Legendre quadrature
    (the defining integral quoted in Sec. 2.1.6)."""
    x, w = np.polynomial.legendre.leggauss(n + 2)
    Pa = legendre_p(a * x + b, n)
    P = legendre_p(x, n)
    return (Pa * w) @ P.T


def affine_L_basis(n, a, b):
    """L_c^f = S L S^{-1} so that N(a x + b) = L_c^f N(x), Sec. 2.2.4."""
    S = basis_S(n)
    return S @ affine_L(n, a, b) @ np.linalg.inv(S)


def gll_nodes(n):
    """Gauss-Lobatto-Legendre nodes for degree p = n-1 (n nodes), ascending:
    -1, +1 and the roots of P_p'(x)."""
    p = n - 1
    if p == 1:
        return np.array([-1.0, 1.0])
    c = np.zeros(p + 1)
    c[p] = 1.0
    r = np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c))
    return np.concatenate(([-1.0], np.sort(r.real), [1.0]))


def dispersion_l(k, h):
    """Coarse order from the dispersion criterion, Sec. 2.3.4 eq. (dispersion_criterion):
    the smallest integer l with l > (kh + (kh)^(1/3) - 1)/2, and never below 1."""
    x = 0.5 * (k * h + (k * h) ** (1.0 / 3.0) - 1.0)
    return max(1, int(np.floor(x)) + 1)
