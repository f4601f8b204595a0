"""Direct solves that check the dual-primal oracle from outside.  Test
infrastructure only.

saddle_solution: the constrained system of Sec. 2.3.1 (eq. large_saddle) with
    every continuity row kept, [A C^T; C 0][phi; nu] = [b; d], solved by one
    sparse LU (SciPy spsolve) after the rows that depend on others are removed
    (rank-revealing QR of the dense C; Sec. 2.2.4 notes the redundancy).  It
    shares the element matrices and constraint rows with the rest of the
    oracle; it checks the linear algebra of the null-space and dual-primal
    solves, not their ingredients.

nodal_solution: the same Galerkin problem written without any of the oracle's
    machinery, for uniform conforming meshes: continuous piecewise Q_p on a
    single global lattice of Gauss-Lobatto-Legendre nodes (Lagrange basis),
    element matrices and loads integrated exactly (Gauss-Legendre quadrature
    of enough points; not GLL quadrature, which would change the discrete
    problem), impedance condition d_n u - i k u = g on the outer boundary
    (Robin coefficient gamma = -i k), assembled and solved by sparse LU.  The
    space is the conforming space of Sec. 1 (globally conforming method), so
    its solution equals the limit of the dual-primal iteration; its values at
    the element GLL nodes are the nodal coefficients themselves.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import constraints as cs


def independent_rows(C, tol=1e-10):
    """Indices of a maximal set of linearly independent rows of a dense C
    (QR of C^T with column pivoting, numerical rank by the diagonal of R)."""
    if C.shape[0] == 0:
        return np.zeros(0, int)
    _, R, piv = sla.qr(C.T.conj(), mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    r = int((d > tol * d[0]).sum()) if d.size and d[0] > 0 else 0
    return np.sort(piv[:r])


def saddle_solution(disc):
    """Element coefficient vectors (paper basis) from one sparse LU of eq. large_saddle."""
    A = sp.block_diag([sp.csr_matrix(a) for a in disc.A]).tocsr()
    b = np.concatenate(disc.b)
    con = cs.Constraints(disc.mesh, disc.degrees, 10 ** 6, disc.bc, disc.dirichlet_fun())
    Cd = con.C.toarray()
    keep = independent_rows(Cd)
    C = sp.csr_matrix(Cd[keep])
    d = np.asarray(con.d, complex)[keep] if len(keep) else np.zeros(0, complex)
    n, m = A.shape[0], C.shape[0]
    S = sp.bmat([[A, C.T], [C, None]], format="csc")
    x = spla.spsolve(S, np.concatenate([b, d]))
    phi = x[:n]
    off = cs.offsets(disc.degrees)
    return [phi[off[e]:off[e + 1]] for e in range(disc.mesh.E)], m


# ---------------------------------------------------------------------------
# nodal C^0 spectral elements (independent of the modal oracle)

def _gll(p):
    """GLL nodes of degree p: -1, the roots of the derivative of the Legendre
    polynomial P_p, +1 (ascending)."""
    if p == 1:
        return np.array([-1.0, 1.0])
    c = np.zeros(p + 1)
    c[p] = 1.0
    r = np.polynomial.legendre.Legendre(c).deriv().roots()
    return np.concatenate(([-1.0], np.sort(r.real), [1.0]))


def _lagrange(nodes, x):
    """Values and derivatives of the Lagrange polynomials of `nodes` at x:
    (len(x), len(nodes)) each, from the product formula."""
    n = len(nodes)
    V = np.ones((len(x), n))
    D = np.zeros((len(x), n))
    for a in range(n):
        others = [nodes[b] for b in range(n) if b != a]
        den = np.prod([nodes[a] - t for t in others])
        fac = np.array([x - t for t in others])          # (n-1, len(x))
        V[:, a] = np.prod(fac, axis=0) / den
        for j in range(n - 1):
            D[:, a] += np.prod(np.delete(fac, j, axis=0), axis=0) / den
    return V, D


def nodal_solution(w, nq_extra=30):
    """Field at the tensor GLL nodes of every element (x index fastest,
    elements in the workload's leaf order) of the conforming Galerkin solution
    on a uniform mesh of one degree, impedance boundary, and the workload's
    plane-wave (total or scattered field) or point-source right-hand side."""
    x0, x1, y0, y1 = w["domain"]
    nx, ny = w["base"]
    deg = np.asarray(w["degree"])
    p = int(deg[0])
    assert np.all(deg == p) and all(int(l[0]) == 0 for l in np.asarray(w["leaves"]).reshape(-1, 3))
    k = float(w["k"])
    eps = np.asarray(w.get("eps_r", np.ones(len(deg))), float)
    hx, hy = (x1 - x0) / nx, (y1 - y0) / ny
    n = p + 1
    xi = _gll(p)
    # exact quadrature for the polynomial parts (degree 2p), generous for loads
    gq, gw = np.polynomial.legendre.leggauss(p + 2)
    lq, lw = np.polynomial.legendre.leggauss(p + nq_extra)
    B, Dr = _lagrange(xi, gq)
    M1 = B.T @ (gw[:, None] * B)          # 1-D mass on [-1, 1]
    S1 = Dr.T @ (gw[:, None] * Dr)        # 1-D stiffness on [-1, 1]
    BL, _ = _lagrange(xi, lq)
    NX, NY = nx * p + 1, ny * p + 1
    gamma = -1j * k
    rhs = w["rhs"]
    rows, cols, vals = [], [], []
    b = np.zeros(NX * NY, complex)
    leaves = np.asarray(w["leaves"]).reshape(-1, 3)
    gidx = []
    for e, (_, ix, iy) in enumerate(leaves):
        ix, iy = int(ix), int(iy)
        g = ((iy * p + np.arange(n))[:, None] * NX + (ix * p + np.arange(n))[None, :]).reshape(-1)  # x fastest
        gidx.append(g)
        beta = -k * k * eps[e]
        Ke = ((hy / hx) * np.kron(M1, S1) + (hx / hy) * np.kron(S1, M1)
              + beta * (hx * hy / 4) * np.kron(M1, M1)).astype(complex)
        ox, oy = x0 + ix * hx, y0 + iy * hy
        # impedance terms on outer sides: only the nodes on that side are non-zero there
        loc = np.arange(n * n).reshape(n, n)   # [iy, ix]
        sides = []
        if ix == 0:
            sides.append((loc[:, 0], hy, (-1.0, 0.0), lambda s: (np.full_like(s, ox), oy + (s + 1) * hy / 2)))
        if ix == nx - 1:
            sides.append((loc[:, -1], hy, (1.0, 0.0), lambda s: (np.full_like(s, ox + hx), oy + (s + 1) * hy / 2)))
        if iy == 0:
            sides.append((loc[0, :], hx, (0.0, -1.0), lambda s: (ox + (s + 1) * hx / 2, np.full_like(s, oy))))
        if iy == ny - 1:
            sides.append((loc[-1, :], hx, (0.0, 1.0), lambda s: (ox + (s + 1) * hx / 2, np.full_like(s, oy + hy))))
        for idx, hs, nrm, xy in sides:
            Ke[np.ix_(idx, idx)] += gamma * (hs / 2) * M1
            if rhs["kind"] == "plane_wave_total":
                th = rhs["angles"][0]
                d = np.array([np.cos(th), np.sin(th)])
                X, Y = xy(lq)
                q = 1j * k * (d @ np.array(nrm) - 1.0) * np.exp(1j * k * (d[0] * X + d[1] * Y))
                b[g[idx]] += (hs / 2) * (BL.T @ (lw * q))
        if rhs["kind"] == "plane_wave_scattered" and eps[e] != 1.0:
            th = rhs["angles"][0]
            X = ox + (lq + 1) * hx / 2
            Y = oy + (lq + 1) * hy / 2
            fx = np.exp(1j * k * np.cos(th) * X)
            fy = np.exp(1j * k * np.sin(th) * Y)
            bx = BL.T @ (lw * fx)
            by = BL.T @ (lw * fy)
            b[g] += k * k * (eps[e] - 1.0) * (hx * hy / 4) * np.kron(by, bx)
        r, c = np.meshgrid(g, g, indexing="ij")
        rows.append(r.ravel())
        cols.append(c.ravel())
        vals.append(Ke.ravel())
    if rhs["kind"] == "point":
        for px, py in np.asarray(rhs["points"], float).reshape(-1, 2):
            jx = (px - x0) / hx * p
            jy = (py - y0) / hy * p
            assert abs(jx - round(jx)) < 1e-9 and abs(jy - round(jy)) < 1e-9, "point source off the lattice"
            b[int(round(jy)) * NX + int(round(jx))] += 1.0
    K = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(NX * NY,) * 2)
    u = spla.spsolve(K, b)
    return np.concatenate([u[g] for g in gidx])
