"""The dual-primal method written element by element (paper Sec. 2.3.3),
for conforming meshes with impedance (Robin) outer boundaries.
Test infrastructure only.

With Z = [Z_1 Z_2], Z_1 the kept type-1 unit vectors and Z_2 the assembled
coarse functions (one column per coarse unknown, equal on every copy),
A_11 is block diagonal and
  F = C_1 [A_11^-1 + A_11^-1 A_12 K^-1 A_12^T A_11^-1] C_1^T,
  K = A_22 - A_12^T A_11^-1 A_12                      (eq. complicated_schur_system)
applied with one dense LU of each element block A_11^(j) (plain per-element
factorisations, no sharing between equal elements).  Z_2 here differs from the
projected basis of Sec. 2.3.2 only by a column scaling; F, its right-hand side
and, on a conforming mesh, the preconditioner do not depend on that choice.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import constraints as cs
from . import element as el
from .dp import interior_mask
from .gmres import gmres


class ElementwiseDP:
    def __init__(self, disc, l):
        self.disc, self.l = disc, l
        mesh, deg = disc.mesh, disc.degrees
        self.mesh, self.deg = mesh, deg
        assert all(v == "robin" for v in disc.bc.values())
        con = cs.Constraints(mesh, deg, l, disc.bc)
        _, _, Cd, _, _ = con.split()
        status = cs.algorithm1(mesh, deg, l, disc.bc)
        off = cs.offsets(deg)
        E = mesh.E
        self.I = [np.nonzero(status[e] == 1)[0] for e in range(E)]
        self.R = [np.nonzero(status[e] != 1)[0] for e in range(E)]
        # C_1 = C_d B_z restricted to the type-1 columns, element-major order
        Bz = sp.block_diag([sp.csr_matrix(el.to_vertex_basis(int(p) + 1)) for p in deg]).tocsc()
        CdB = (Cd @ Bz).tocsc()
        cols = np.concatenate([off[e] + self.I[e] for e in range(E)])
        self.C1 = CdB[:, cols].tocsr()
        self.C1.eliminate_zeros()
        self.I_off = np.concatenate(([0], np.cumsum([len(i) for i in self.I])))
        # global coarse numbering: vertices by point, low edge bubbles by edge
        self.T = self._coarse_maps(status)
        nK = 1 + max(int(t.max()) for t in self.T)
        self.nK = nK
        # per-element blocks (vertex basis)
        self.lu, self.Phi, self.Se, self.b1, self.bR = [], [], [], [], []
        Krows, Kcols, Kvals = [], [], []
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
            t = self.T[e]
            Krows.append(np.repeat(t, len(t)))
            Kcols.append(np.tile(t, len(t)))
            Kvals.append(Kj.reshape(-1))
            self.lu.append(lu)
            self.Phi.append(Phi)
            self.b1.append(bt[I])
            self.bR.append(bt[R])
            # Dirichlet preconditioner block, Laplace-only (Sec. 2.3.3)
            A11L = AtL[np.ix_(I, I)]
            inner = interior_mask(n)[I]
            ie, ii = np.nonzero(~inner)[0], np.nonzero(inner)[0]
            Se = (A11L[np.ix_(ie, ie)]
                  - A11L[np.ix_(ie, ii)] @ np.linalg.solve(A11L[np.ix_(ii, ii)], A11L[np.ix_(ii, ie)]))
            self.Se.append((ie, Se))
        self.K = sp.csc_matrix((np.concatenate(Kvals), (np.concatenate(Krows), np.concatenate(Kcols))),
                               shape=(nK, nK))
        self.K_lu = spla.splu(self.K)
        self.nlam = self.C1.shape[0]
        self.X = np.asarray(self.C1.multiply(self.C1).sum(axis=1)).ravel()

    def set_loads(self, loads):
        """Replace the element loads (one vector per element, paper basis) while
        keeping every factorisation: the right-hand side of an adjoint solve."""
        for e in range(self.mesh.E):
            n = int(self.deg[e]) + 1
            bt = el.to_vertex_basis(n) @ loads[e]
            self.b1[e] = bt[self.I[e]]
            self.bR[e] = bt[self.R[e]]

    def _coarse_maps(self, status):
        mesh, deg = self.mesh, self.deg
        ids = {}
        T = []
        for e in range(mesh.E):
            n = int(deg[e]) + 1
            cp = mesh.corner_points(e)
            t = []
            for m in self.R[e]:
                ix, iy = m % n, m // n
                if ix < 2 and iy < 2:
                    key = ("v", cp[(ix, iy)])
                else:
                    if ix == 0:
                        side, k = 2, iy
                    elif ix == 1:
                        side, k = 1, iy
                    elif iy == 0:
                        side, k = 4, ix
                    else:
                        side, k = 3, ix
                    seg = mesh.side_segment(e, side)
                    key = ("e", seg, k)
                if key not in ids:
                    ids[key] = len(ids)
                t.append(ids[key])
            T.append(np.array(t, int))
        return T

    # -- element operations -------------------------------------------------
    def _split(self, y):
        return [y[self.I_off[e]:self.I_off[e + 1]] for e in range(self.mesh.E)]

    def _solve_block(self, yI, yR_global):
        """Solve A^ [x_I; x_R] = [y_I; y_R] with block elimination (eq. block_matrix_inversion).
        Returns the list of element x_I and the global x_R."""
        E = self.mesh.E
        z = [sla.lu_solve(self.lu[e], yI[e]) for e in range(E)]
        g = yR_global.astype(complex).copy()
        for e in range(E):
            np.add.at(g, self.T[e], -(self.Phi[e].T @ yI[e]))
        w = self.K_lu.solve(g)
        x = [z[e] - self.Phi[e] @ w[self.T[e]] for e in range(E)]
        return x, w

    def apply_F(self, v):
        y = self._split(self.C1.T @ v)
        x, _ = self._solve_block(y, np.zeros(self.nK))
        return self.C1 @ np.concatenate(x)

    def apply_P(self, u):
        """P^-1 = X^-1 C_1 S_e C_1^T X^-1 with X = C_1 C_1^T (diagonal, conforming)."""
        s = u / self.X
        y = self._split(self.C1.T @ s)
        out = []
        for e in range(self.mesh.E):
            ie, Se = self.Se[e]
            z = np.zeros_like(y[e])
            z[ie] = Se @ y[e][ie]
            out.append(z)
        return (self.C1 @ np.concatenate(out)) / self.X

    def b2(self):
        g = np.zeros(self.nK, complex)
        for e in range(self.mesh.E):
            np.add.at(g, self.T[e], self.bR[e])
        return g

    def interface_rhs(self):
        x, _ = self._solve_block(self.b1, self.b2())
        return self.C1 @ np.concatenate(x)

    def recover(self, nu):
        r = self._split(self.C1.T @ nu)
        yI = [self.b1[e] - r[e] for e in range(self.mesh.E)]
        x, w = self._solve_block(yI, self.b2())
        phis = []
        for e in range(self.mesh.E):
            n = int(self.deg[e]) + 1
            full = np.zeros(n * n, complex)
            full[self.I[e]] = x[e]
            full[self.R[e]] = w[self.T[e]]
            phis.append(el.to_vertex_basis(n) @ full)
        return phis

    def solve(self, tol=1e-10, max_iter=300):
        g = self.interface_rhs()
        nu, it, hist = gmres(self.apply_F, self.apply_P, g, tol, max_iter)
        self.nu, self.iters, self.hist = nu, it, hist
        return self.recover(nu)
