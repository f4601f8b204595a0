"""Globally conforming Galerkin solution by a direct solve.  Test infrastructure only.

With every continuity moment of every edge enforced (all rows of C), the
method's converged answer is the conforming Galerkin solution (Sec. 1 calls
the method globally conforming; with l >= p the partial nullspace method is
the nullspace method, Sec. 2.3.2).  This module computes it from its plain
definition: phi = phi_d + Y psi with Y a basis of null(C), phi_d = C^+ d, and
Y^T A Y psi = Y^T (b - A phi_d), using a dense SVD null space.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import constraints as cs


def conforming_solution(disc, loads=None):
    """Element coefficient vectors of the conforming solution; ``loads`` (one
    vector per element, paper basis) replaces the discretisation's loads."""
    A = sp.block_diag([sp.csr_matrix(a) for a in disc.A]).toarray()
    b = np.concatenate(disc.b if loads is None else loads)
    con = cs.Constraints(disc.mesh, disc.degrees, 10 ** 6, disc.bc, disc.dirichlet_fun())
    C = con.C.toarray()
    if C.shape[0]:
        phi_d = cs.pinv(C) @ con.d
        Y = sla.null_space(C)
    else:
        phi_d = np.zeros(A.shape[0], complex)
        Y = np.eye(A.shape[0])
    psi = np.linalg.solve(Y.T @ A @ Y, Y.T @ (b - A @ phi_d))
    phi = phi_d + Y @ psi
    off = cs.offsets(disc.degrees)
    return [phi[off[e]:off[e + 1]] for e in range(disc.mesh.E)]
