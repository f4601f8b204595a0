"""Literal partial-nullspace dual-primal method (paper Sec. 2.3.1-2.3.4), dense.
Test infrastructure only; meant for meshes of a few thousand unknowns.

Every quantity is formed exactly as written in the paper:
  phi = Z phi_p + phi_z, phi_z = C_p^+ d_p                (eq. null_space_identity)
  A^ = Z^T A Z, C^ = C_d Z, b^ = Z^T(b - A phi_z), d^ = d_d - C_d phi_z
  C^ A^-1 C^T nu_d = C^ A^-1 b^ - d^                    (eq. schur_complement_system)
  P^-1 = (C^ W C^T)^-T C^ W^T A^ W C^T (C^ W C^T)^-1     (eq. general_preconditioner)
with W from eq. (weight_matrix) built on the Laplace-only part of A^ (Sec. 2.3.3).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import constraints as cs
from .gmres import gmres


def interior_mask(n):
    """Vertex-basis local modes with both indices >= 2 (vanish on every side)."""
    ix = np.arange(n * n) % n
    iy = np.arange(n * n) // n
    return (ix >= 2) & (iy >= 2)


class LiteralDP:
    def __init__(self, disc, l, precond="dirichlet", scaling=False, keep_c2kc2=True):
        self.disc, self.l = disc, l
        mesh, deg = disc.mesh, disc.degrees
        self.mesh, self.deg = mesh, deg
        A = sp.block_diag([sp.csr_matrix(a) for a in disc.A]).toarray()
        AL = sp.block_diag([sp.csr_matrix(a) for a in disc.A_lap]).toarray()
        b = np.concatenate(disc.b)
        self.A, self.b = A, b
        con = cs.Constraints(mesh, deg, l, disc.bc, disc.dirichlet_fun(), tau=disc.w.get("discard_tol", 0.0))
        self.con = con
        Cp, dp, Cd, dd, _ = con.split()
        status = cs.algorithm1(mesh, deg, l, disc.bc)
        self.status = status
        Z, J1, J2 = cs.literal_Z(mesh, deg, status, Cp)
        self.Z, self.J1, self.J2 = Z, J1, J2
        n1 = len(J1)
        self.n1 = n1
        Cpd = Cp.toarray()
        phi_z = cs.pinv(Cpd) @ dp if Cpd.shape[0] else np.zeros(A.shape[0])
        self.phi_z = phi_z
        Cdd = Cd.toarray()
        self.Cp, self.Cd = Cpd, Cdd
        Ah = Z.T @ A @ Z
        AhL = Z.T @ AL @ Z
        bh = Z.T @ (b - A @ phi_z)
        Ch = Cdd @ Z
        dh = dd - Cdd @ phi_z
        self.Ah, self.AhL, self.bh, self.Ch, self.dh = Ah, AhL, bh, Ch, dh
        self.A11 = Ah[:n1, :n1]
        self.A12 = Ah[:n1, n1:]
        self.A22 = Ah[n1:, n1:]
        self.C1, self.C2 = Ch[:, :n1], Ch[:, n1:]
        self.b1, self.b2 = bh[:n1], bh[n1:]
        # interface operator and right-hand side
        lu = sla.lu_factor(Ah)
        self.Ah_lu = lu
        self.F = Ch @ sla.lu_solve(lu, Ch.T)
        self.g = Ch @ sla.lu_solve(lu, bh) - dh
        self.Pinv = self._preconditioner(precond, scaling, keep_c2kc2)

    # ------------------------------------------------------------------
    def _element_of_type1(self):
        """For each type-1 column: (element, local mode)."""
        off = cs.offsets(self.deg)
        el_of = np.searchsorted(off, self.J1, side="right") - 1
        return el_of, self.J1 - off[el_of]

    def _preconditioner(self, kind, scaling, keep_c2kc2):
        n1 = self.n1
        AL = self.AhL
        A11L = AL[:n1, :n1]
        A12L = AL[:n1, n1:]
        A22L = AL[n1:, n1:]
        conforming = np.abs(self.C2).max(initial=0.0) == 0.0
        # W_1, block diagonal over elements (Sec. 2.3.3)
        W1 = np.eye(n1, dtype=complex)
        if kind == "dirichlet":
            el_of, loc = self._element_of_type1()
            W1 = np.zeros((n1, n1), complex)
            for e in range(self.mesh.E):
                idx = np.nonzero(el_of == e)[0]
                n = int(self.deg[e]) + 1
                inner = interior_mask(n)[loc[idx]]
                ie, ii = idx[~inner], idx[inner]
                Aee = A11L[np.ix_(ie, ie)]
                Aie = A11L[np.ix_(ii, ie)]
                Aii = A11L[np.ix_(ii, ii)]
                top = np.eye(len(ie))
                if scaling:
                    top = np.diag(1.0 / np.diag(Aee))
                W1[np.ix_(ie, ie)] = top
                if len(ii):
                    W1[np.ix_(ii, ie)] = -np.linalg.solve(Aii, Aie) @ top
        C1, C2 = self.C1, self.C2
        X = C1 @ W1 @ C1.T
        Y = C1 @ W1.T @ A11L @ W1 @ C1.T
        if not conforming:
            # W_2 = I; the cross term of eq. (first_precond_comp) is dropped,
            # C_2 K C_2^T is kept (Sec. 2.3.3 and the remark that follows it)
            X = X + C2 @ C2.T
            if keep_c2kc2:
                KL = A22L - A12L.T @ np.linalg.solve(A11L, A12L)
                Y = Y + C2 @ KL @ C2.T
        Xi = np.linalg.inv(X)
        return Xi.T @ Y @ Xi

    # ------------------------------------------------------------------
    def solve(self, tol=1e-10, max_iter=200):
        nu, it, hist = gmres(lambda v: self.F @ v, lambda v: self.Pinv @ v, self.g, tol, max_iter)
        self.nu, self.iters, self.hist = nu, it, hist
        return self.recover(nu)

    def recover(self, nu):
        """phi_p = A^-1 (b^ - C^T nu_d), phi = Z phi_p + phi_z (Sec. 2.3.1)."""
        php = sla.lu_solve(self.Ah_lu, self.bh - self.Ch.T @ nu)
        phi = self.Z @ php + self.phi_z
        off = cs.offsets(self.deg)
        return [phi[off[e]:off[e + 1]] for e in range(self.mesh.E)]

    def direct_interface(self):
        """nu_d from a dense solve of the interface system (no iteration)."""
        return np.linalg.solve(self.F, self.g)
