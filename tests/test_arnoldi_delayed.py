"""The delayed-reorthogonalisation Arnoldi step of the GPU's GMRES, written out
in NumPy from the recurrences the kernels implement, against explicit classical
Gram-Schmidt with one reorthogonalisation (the two are equal in exact
arithmetic).  Host-side check of the algebra; the kernels themselves are
compared with the oracle's GMRES in the GPU parity tests."""
import numpy as np


def _cgs2(A, b, K):
    n = len(b)
    Q = np.zeros((n, K + 1), complex)
    H = np.zeros((K + 1, K), complex)
    Q[:, 0] = b / np.linalg.norm(b)
    for j in range(K):
        w = A @ Q[:, j]
        h1 = Q[:, :j + 1].conj().T @ w
        w = w - Q[:, :j + 1] @ h1
        h2 = Q[:, :j + 1].conj().T @ w
        w = w - Q[:, :j + 1] @ h2
        H[:j + 1, j] = h1 + h2
        H[j + 1, j] = np.linalg.norm(w)
        Q[:, j + 1] = w / H[j + 1, j]
    return Q, H


def _delayed(A, b, K):
    """Iteration j: u = V[:, j] once projected and scaled, z = A u; one pass of
    dot products, then column j-1 of H, q_j, the first-pass coefficients of
    column j and the next candidate."""
    n = len(b)
    V = np.zeros((n, K + 2), complex)
    H = np.zeros((K + 1, K), complex)
    V[:, 0] = b / np.linalg.norm(b)
    hprev, rho = None, None
    for j in range(K + 1):
        u = V[:, j]
        z = A @ u
        Q = V[:, :j]
        s, t = Q.conj().T @ u, Q.conj().T @ z
        uz, uu, zz = np.vdot(u, z), np.vdot(u, u).real, np.vdot(z, z).real
        nu = np.sqrt(uu - np.vdot(s, s).real)
        if j >= 1:
            H[:j, j - 1] = hprev[:j] + rho * s
            H[j, j - 1] = rho * nu
        tau = (uz - np.vdot(s, t)) / nu
        hprev = (np.concatenate([t, [tau]]) - H[:j + 1, :j] @ s) / nu
        sigma = np.sqrt(zz - np.vdot(t, t).real - abs(tau) ** 2)
        rho = sigma / nu
        q = (u - Q @ s) / nu
        V[:, j + 1] = (z - Q @ t - q * tau) / sigma
        V[:, j] = q
    return V[:, :K + 1], H


def test_delayed_reorthogonalisation_equals_cgs2():
    rng = np.random.default_rng(1)
    n, K = 300, 60
    A = np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Q, H = _cgs2(A, b, K)
    V, Hd = _delayed(A, b, K)
    assert np.abs(H - Hd).max() < 1e-13
    assert np.abs(Q - V).max() < 1e-13
    assert np.abs(V.conj().T @ V - np.eye(K + 1)).max() < 1e-14
    assert np.abs(A @ V[:, :K] - V @ Hd).max() < 1e-14
