"""The dual-primal method element by element on quadtree meshes with hanging
edges (paper Sec. 2.2.4, 2.3.1-2.3.3), for impedance (Robin) outer boundaries.
Test infrastructure only.

The partially assembled space is null(C_p) (the primal rows of eq.
final_constraint, vertex basis).  Algorithm 1 (Sec. 2.3.2) splits the local
modes: type 1 (kept, touched by no primal row), type 2 (kept, in some primal
row; on a hanging edge every coarse-side edge mode) and discarded.  Here the
space is written in the basis those kept modes give directly:
  - each type-1 mode is its own unit vector (so A_11 is block diagonal);
  - each type-2 mode is one global coarse unknown; its column carries the
    values the primal rows force on the discarded modes, x_D = T_D x_2 with
    C_p,D T_D = -C_p,2 (C_p,D has full column rank, because Algorithm 1 discards
    exactly rank(C_p) modes; solved through the normal equations).
With T = [I; T_D] over the type-2 and discarded modes (rows of element e: T_e),
  A_11 = blockdiag(A_II^e),   K = sum_e T_e^T (A_RR - A_RI A_II^-1 A_IR)_e T_e,
  C_1 = C_d on the type-1 modes,   C_2 = C_d,R T,
and A^ is inverted by block elimination (eq. block_matrix_inversion).  The
projected basis of Sec. 2.3.2 spans the same space, so F = C^ A^-1 C^T, the
interface right-hand side and the recovered field are the paper's (they do not
depend on the basis).  The preconditioner of Sec. 2.3.3 does depend on it: it is
written here in this basis (Dirichlet blocks on the type-1 edge modes, W_2 = I,
X = C_1 C_1^T + C_2 C_2^T, C_2 K_L C_2^T kept) and serves only to converge; it
is not a reference for the library's preconditioner.
On a conforming mesh T_D copies each kept value onto its discarded copies and
C_2 = 0, which is oracle/dp_elementwise.py.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import constraints as cs
from . import element as el
from .dp import interior_mask
from .gmres import gmres


def _discarded_from_kept(CpD, Cp2, block=2048):
    """T_D with CpD T_D = -Cp2 (CpD full column rank): normal equations, sparse
    LU, right-hand sides in blocks; entries below 1e-14 of the largest dropped."""
    nD, n2 = CpD.shape[1], Cp2.shape[1]
    if nD == 0:
        return sp.csr_matrix((0, n2))
    N = (CpD.T @ CpD).tocsc()
    S = (CpD.T @ Cp2).tocsc()
    lu = spla.splu(N)
    cols = []
    for j0 in range(0, n2, block):
        X = -lu.solve(S[:, j0:j0 + block].toarray())
        cols.append(sp.csc_matrix(np.where(np.abs(X) > 1e-14, X, 0.0)))
    TD = sp.hstack(cols).tocsr() if cols else sp.csr_matrix((nD, 0))
    TD.eliminate_zeros()
    return TD


class NonconformingDP:
    def __init__(self, disc, l):
        self.disc, self.l = disc, l
        mesh, deg = disc.mesh, disc.degrees
        self.mesh, self.deg = mesh, deg
        assert all(v == "robin" for v in disc.bc.values())
        tau = disc.w.get("discard_tol", 0.0)
        con = cs.Constraints(mesh, deg, l, disc.bc, tau=tau)
        Cp, _, Cd, _, _ = con.split()
        status = cs.algorithm1(mesh, deg, l, disc.bc)
        off = cs.offsets(deg)
        E = mesh.E
        Bz = sp.block_diag([sp.csr_matrix(el.to_vertex_basis(int(p) + 1)) for p in deg]).tocsc()
        CpB = (Cp @ Bz).tocsc()
        CdB = (Cd @ Bz).tocsc()
        st = np.concatenate(status)
        g1 = np.nonzero(st == 1)[0]
        g2 = np.nonzero(st == 2)[0]
        g0 = np.nonzero(st == 0)[0]
        # no primal row may touch a type-1 mode (Algorithm 1's split)
        if CpB.shape[0] and len(g1):
            assert abs(CpB[:, g1]).max() < 1e-12
        # coarse unknowns: the type-2 modes in global order; T over the type-2
        # and discarded modes (identity on the type-2 rows)
        self.nK = len(g2)
        TD = _discarded_from_kept(CpB[:, g0], CpB[:, g2]).tocoo()
        if CpB.shape[0] and len(g2):
            res = CpB[:, g0] @ TD + CpB[:, g2]
            assert abs(res).max() < 1e-10, "primal rows not satisfied by the kept-mode basis"
        ndof = int(off[-1])
        Tall = sp.csr_matrix((np.concatenate([np.ones(len(g2)), TD.data]),
                              (np.concatenate([g2, g0[TD.row]]), np.concatenate([np.arange(len(g2)), TD.col]))),
                             shape=(ndof, self.nK))
        self.I = [np.nonzero(status[e] == 1)[0] for e in range(E)]
        self.R = [np.nonzero(status[e] != 1)[0] for e in range(E)]
        self.T = [Tall[off[e] + self.R[e]] for e in range(E)]
        # C_1 (type-1 columns, element-major) and C_2 = C_d,R T
        self.C1 = CdB[:, g1].tocsr()
        self.C1.eliminate_zeros()
        gR = np.concatenate([off[e] + self.R[e] for e in range(E)])
        Tglob = Tall[gR]
        self.C2 = (CdB[:, gR] @ Tglob).tocsr()
        self.C2.eliminate_zeros()
        self.I_off = np.concatenate(([0], np.cumsum([len(i) for i in self.I])))
        self.nlam = self.C1.shape[0]
        # element blocks
        self.lu, self.Phi, self.b1, self.bR, self.Se = [], [], [], [], []
        Kblk, KLblk = [], []
        for e in range(E):
            n = int(deg[e]) + 1
            Bl = el.to_vertex_basis(n)
            At = Bl @ disc.A[e] @ Bl
            AtL = Bl @ disc.A_lap[e] @ Bl
            bt = Bl @ disc.b[e]
            I, R = self.I[e], self.R[e]
            lu = sla.lu_factor(At[np.ix_(I, I)])
            Phi = sla.lu_solve(lu, At[np.ix_(I, R)])
            Kj = At[np.ix_(R, R)] - At[np.ix_(R, I)] @ Phi
            Kblk.append(Kj)
            self.lu.append(lu)
            self.Phi.append(Phi)
            self.b1.append(bt[I])
            self.bR.append(bt[R])
            A11L = AtL[np.ix_(I, I)]
            KLj = AtL[np.ix_(R, R)] - AtL[np.ix_(R, I)] @ np.linalg.solve(A11L, AtL[np.ix_(I, R)])
            KLblk.append(KLj)
            inner = interior_mask(n)[I]
            ie, ii = np.nonzero(~inner)[0], np.nonzero(inner)[0]
            Se = (A11L[np.ix_(ie, ie)]
                  - A11L[np.ix_(ie, ii)] @ np.linalg.solve(A11L[np.ix_(ii, ii)], A11L[np.ix_(ii, ie)]))
            self.Se.append((ie, Se))
        # K = sum_e T_e^T K_e T_e (and the Laplace-only K_L) as T^T blockdiag(K_e) T
        self.K = (Tglob.T @ sp.block_diag(Kblk, format="csr") @ Tglob).tocsc()
        self.K_lu = spla.splu(self.K)
        self.KL = (Tglob.T @ sp.block_diag(KLblk, format="csr") @ Tglob).tocsr()
        X = (self.C1 @ self.C1.T + self.C2 @ self.C2.T).astype(complex).tocsc()
        self.X_lu = spla.splu(X)

    # -- element operations -------------------------------------------------
    def _split(self, y):
        return [y[self.I_off[e]:self.I_off[e + 1]] for e in range(self.mesh.E)]

    def _solve_block(self, yI, y2):
        """A^ [x_1; x_2] = [y_1; y_2] by block elimination: x_2 = K^-1 (y_2 -
        A_21 A_11^-1 y_1), x_1 = A_11^-1 (y_1 - A_12 x_2)."""
        E = self.mesh.E
        z = [sla.lu_solve(self.lu[e], yI[e]) for e in range(E)]
        g = np.asarray(y2, complex).copy()
        for e in range(E):
            g -= self.T[e].T @ (self.Phi[e].T @ yI[e])
        w = self.K_lu.solve(g)
        x = [z[e] - self.Phi[e] @ (self.T[e] @ w) for e in range(E)]
        return x, w

    def apply_F(self, v):
        x, w = self._solve_block(self._split(self.C1.T @ v), self.C2.T @ v)
        return self.C1 @ np.concatenate(x) + self.C2 @ w

    def apply_P(self, u):
        s = self.X_lu.solve(np.asarray(u, complex))
        y = self._split(self.C1.T @ s)
        out = []
        for e in range(self.mesh.E):
            ie, Se = self.Se[e]
            z = np.zeros_like(y[e])
            z[ie] = Se @ y[e][ie]
            out.append(z)
        t = self.C1 @ np.concatenate(out) + self.C2 @ (self.KL @ (self.C2.T @ s))
        return self.X_lu.solve(t)

    def b2(self):
        g = np.zeros(self.nK, complex)
        for e in range(self.mesh.E):
            g += self.T[e].T @ self.bR[e]
        return g

    def interface_rhs(self):
        x, w = self._solve_block(self.b1, self.b2())
        return self.C1 @ np.concatenate(x) + self.C2 @ w

    def recover(self, nu):
        """phi = A^-1 (b^ - C^T nu) in the element modes (vertex basis back to
        the paper basis)."""
        r = self._split(self.C1.T @ nu)
        yI = [self.b1[e] - r[e] for e in range(self.mesh.E)]
        x, w = self._solve_block(yI, self.b2() - self.C2.T @ nu)
        phis = []
        for e in range(self.mesh.E):
            n = int(self.deg[e]) + 1
            full = np.zeros(n * n, complex)
            full[self.I[e]] = x[e]
            full[self.R[e]] = self.T[e] @ w
            phis.append(el.to_vertex_basis(n) @ full)
        return phis

    def solve(self, tol=1e-10, max_iter=300):
        g = self.interface_rhs()
        nu, it, hist = gmres(self.apply_F, self.apply_P, g, tol, max_iter)
        self.nu, self.iters, self.hist = nu, it, hist
        return self.recover(nu)
