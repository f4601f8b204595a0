"""Left-preconditioned GMRES (paper Sec. 2.3.4 and Sec. 3.2).  Test infrastructure only.

Full (unrestarted) GMRES with modified Gram-Schmidt, zero initial iterate
(Sec. 3, opening paragraph), stopped when the preconditioned relative residual
||P^-1 r_k|| / ||P^-1 r_0|| falls to tol (the quantity plotted in the
residual-convergence figure of Sec. 3.2).
"""
import numpy as np


def gmres(apply_F, apply_P, rhs, tol, max_iter):
    """Solve P^-1 F x = P^-1 rhs.  apply_F, apply_P act on 1-D complex vectors.

    Returns (x, iterations, history) with history[k] = ||P^-1 r_k|| / ||P^-1 r_0||.
    """
    r0 = apply_P(rhs)
    beta = np.linalg.norm(r0)
    n = rhs.shape[0]
    if beta == 0.0:
        return np.zeros(n, complex), 0, [0.0]
    V = [r0 / beta]
    H = np.zeros((max_iter + 1, max_iter), complex)
    cs = np.zeros(max_iter, complex)
    sn = np.zeros(max_iter, complex)
    g = np.zeros(max_iter + 1, complex)
    g[0] = beta
    hist = [1.0]
    k = 0
    for j in range(max_iter):
        w = apply_P(apply_F(V[j]))
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        # apply previous rotations to the new column
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        a, b = H[j, j], H[j + 1, j]
        den = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
        cs[j] = abs(a) / den if den else 1.0
        sn[j] = (a / abs(a)) * np.conj(b) / den if abs(a) else 1.0
        H[j, j] = cs[j] * a + sn[j] * b
        H[j + 1, j] = 0.0
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        hist.append(abs(g[j + 1]) / beta)
        if hist[-1] <= tol:
            break
        if H[j + 1, j] == 0.0 and np.linalg.norm(w) == 0.0:
            break
        V.append(w / np.linalg.norm(w))
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
    x = np.zeros(n, complex)
    for i in range(k):
        x = x + y[i] * V[i]
    return x, k, hist
