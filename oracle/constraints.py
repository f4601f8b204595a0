"""Hierarchical moment constraints and the type-1/type-2 split (paper Sec. 2.2.4,
2.3.2 and Algorithm 1).  Test infrastructure only.

Global unknowns are the concatenated element vectors vec(Phi_e) (x index
fastest) in the paper's basis N.  Vertex-basis mode labels use the basis
N~ = B N: along one direction index 0 is the vertex function at +1, index 1
the vertex function at -1, indices >= 2 the bubbles.
"""
import numpy as np
import scipy.sparse as sp

from . import element as el
from . import legendre as lg
from .mesh import OPPOSITE


def offsets(degrees):
    n = np.asarray(degrees) + 1
    return np.concatenate(([0], np.cumsum(n * n)))


def trace_rows(n, side):
    """Trace coefficients of a side (Sec. 2.2.1, C_i): rows k = 0..n-1 of
    I (x) v^T (sides 1,2) or v^T (x) I (sides 3,4), v = e_1 + (-1)^i e_2."""
    return el.dirichlet_rows(n, side)


def side_modes(n, side):
    """Vertex-basis local indices (ix, iy) of the bubbles k = 2..n-1 on a side,
    as flat indices ix + n*iy (right: ix=0, left: ix=1, top: iy=0, bottom: iy=1)."""
    out = []
    for k in range(2, n):
        if side == 2:
            ix, iy = 0, k
        elif side == 1:
            ix, iy = 1, k
        elif side == 4:
            ix, iy = k, 0
        else:
            ix, iy = k, 1
        out.append(ix + n * iy)
    return out


def side_vertices(n, side):
    """Vertex-basis flat indices of the two vertex modes on a side."""
    if side == 2:
        pairs = [(0, 0), (0, 1)]
    elif side == 1:
        pairs = [(1, 0), (1, 1)]
    elif side == 4:
        pairs = [(0, 0), (1, 0)]
    else:
        pairs = [(0, 1), (1, 1)]
    return [a + n * b for (a, b) in pairs], pairs


def side_l(l, e, side):
    """The coarse order of an element side: l itself, or l(e, side) when l is a
    per-edge function (the same value on both sides of an edge)."""
    return l(e, side) if callable(l) else l


def edge_l(l, na, nb):
    """Number of primal rows minus one on an edge between elements with na and nb
    modes per direction: min(l, p_a, p_b).  A primal row above the smaller degree
    would only involve the other side's mode and zero a kept unknown; it stays
    dual instead (Sec. 2.3.2 reading: with l at or above every degree every
    shared mode is primal and the method is the nullspace method)."""
    return min(l, na - 1, nb - 1)


class Constraints:
    """Global C (rows per edge, k ascending), data d, primal flags and edge list.

    Edges are visited as in Algorithm 1: finest level first, elements in input
    order, sides left, right, bottom, top.  An interior edge is imposed from the
    visiting (finer or same-level) element f toward its neighbour c as
    (L_c^f)^T C_j^c phi_c - C_i^f phi_f = 0 (eq. final_constraint), with both
    sides zero-padded to L = max(p_c, p_f) (eq. fine_constraints); a Dirichlet
    side gives C_i phi = d_i.  Rows k <= min(l, p_c, p_f) are primal (C_p), the rest
    dual (C_d).
    Rows that only zero coarse modes already zeroed by a sibling fine edge are
    dropped (Sec. 2.2.4, degree-reduction redundancy), and so are dual rows
    whose diagonal entry of L_c^f lies below tau (Sec. 2.2.4, discard
    threshold for decayed constraints; tau = 0 keeps all).
    """

    def __init__(self, mesh, degrees, l, bc, dirichlet_fun=None, tau=0.0):
        self.mesh, self.degrees, self.l = mesh, np.asarray(degrees), l
        self.off = offsets(degrees)
        self.ndof = int(self.off[-1])
        rows, cols, vals = [], [], []
        self.d = []
        self.primal = []
        self.kind = []      # 'edge' or 'dirichlet'
        self.row_edge = []
        self.row_k = []
        self.edges = []     # (f, side_f, c, side_c, a, b) or (e, side, None, bnd, 0, 0)
        visited = set()
        zeroed = {}
        r = 0
        for e in mesh.visit_order():
            ne = int(self.degrees[e]) + 1
            for side in (1, 2, 3, 4):
                bnd = mesh.boundary_side(e, side)
                if bnd:
                    if bc.get(bnd) != "dirichlet":
                        continue
                    eid = len(self.edges)
                    self.edges.append((e, side, None, bnd, 0.0, 0.0))
                    T = trace_rows(ne, side)
                    hdat = np.zeros(ne, complex)
                    if dirichlet_fun is not None:
                        hdat = dirichlet_fun(e, side, ne)
                    dd = el.dirichlet_data(ne, hdat)
                    for k in range(ne):
                        nz = np.nonzero(T[k])[0]
                        rows += [r] * len(nz)
                        cols += list(self.off[e] + nz)
                        vals += list(T[k, nz])
                        self.d.append(dd[k])
                        self.primal.append(k <= side_l(l, e, side))
                        self.kind.append("dirichlet")
                        self.row_edge.append(eid)
                        self.row_k.append(k)
                        r += 1
                    continue
                if (e, side) in visited:
                    continue
                nbrs = mesh.neighbours(e, side)
                lev_e = mesh.leaves[e][0]
                if len(nbrs) != 1 or mesh.leaves[nbrs[0][0]][0] > lev_e:
                    # finer neighbours: imposed earlier from their side
                    visited.add((e, side))
                    continue
                c, sc = nbrs[0]
                if mesh.leaves[c][0] == lev_e:
                    a, b = 1.0, 0.0
                    visited.add((c, sc))
                else:
                    a, b = mesh.affine_params(e, side, c)
                visited.add((e, side))
                nc = int(self.degrees[c]) + 1
                L = max(ne, nc)
                Lcf = lg.affine_L_basis(L, a, b)
                Tc = np.zeros((L, nc * nc))
                Tc[:nc] = trace_rows(nc, sc)
                Tf = np.zeros((L, ne * ne))
                Tf[:ne] = trace_rows(ne, side)
                Rc = Lcf.T @ Tc
                eid = len(self.edges)
                self.edges.append((e, side, c, sc, a, b))
                zkey = (c, sc)
                zset = zeroed.setdefault(zkey, set())
                le = edge_l(side_l(l, e, side), ne, nc)
                for k in range(L):
                    if k > le and abs(Lcf[k, k]) < tau:
                        # decayed diagonal of L_c^f: the dual constraint is dropped
                        # (Sec. 2.2.4 discard threshold; primal rows are kept)
                        continue
                    if k >= ne:
                        # only coarse modes enter this row: it zeroes them
                        if k in zset:
                            continue
                        zset.add(k)
                    nzc = np.nonzero(np.abs(Rc[k]) > 0)[0]
                    nzf = np.nonzero(Tf[k])[0]
                    rows += [r] * (len(nzc) + len(nzf))
                    cols += list(self.off[c] + nzc) + list(self.off[e] + nzf)
                    vals += list(Rc[k, nzc]) + list(-Tf[k, nzf])
                    self.d.append(0.0)
                    self.primal.append(k <= le)
                    self.kind.append("edge")
                    self.row_edge.append(eid)
                    self.row_k.append(k)
                    r += 1
        self.nrows = r
        self.C = sp.csr_matrix((vals, (rows, cols)), shape=(r, self.ndof))
        self.d = np.array(self.d, complex)
        self.primal = np.array(self.primal, bool)
        self.row_edge = np.array(self.row_edge)
        self.row_k = np.array(self.row_k)

    def split(self):
        P = np.nonzero(self.primal)[0]
        D = np.nonzero(~self.primal)[0]
        return self.C[P], self.d[P], self.C[D], self.d[D], D


def algorithm1(mesh, degrees, l, bc):
    """Index set J of Sec. 2.3.2 (Algorithm 1) as a per-element status array.

    status[e][m] for each vertex-basis local mode m: 0 discarded, 1 type 1,
    2 type 2.  Edge unknowns ``first l-1`` are the bubbles k = 2..l.  Vertex
    copies: one copy of every geometric vertex is kept, unless the vertex lies
    on a Dirichlet side or is a hanging node; a copy on the fine side of a
    hanging edge is never the kept one.  (Which copy is kept does not change
    the projected basis: copies linked by primal constraints project to the
    same column.)
    """
    degrees = np.asarray(degrees)
    status = [np.full((int(p) + 1) ** 2, -1, dtype=int) for p in degrees]
    visited_edge = set()
    kept_point = set()
    dirichlet_points = set()
    for e in range(mesh.E):
        for side in (1, 2, 3, 4):
            bnd = mesh.boundary_side(e, side)
            if bnd and bc.get(bnd) == "dirichlet":
                n = int(degrees[e]) + 1
                _, pairs = side_vertices(n, side)
                cp = mesh.corner_points(e)
                for pr in pairs:
                    dirichlet_points.add(cp[pr])
    # vertex copies on a side that faces a coarser neighbour are discarded
    # whichever side of the element is visited first, so that the one kept copy
    # of every vertex is never such a copy
    on_coarse_edge = set()
    for e in range(mesh.E):
        n = int(degrees[e]) + 1
        for side in (1, 2, 3, 4):
            if mesh.boundary_side(e, side):
                continue
            nbrs = mesh.neighbours(e, side)
            if len(nbrs) == 1 and mesh.leaves[nbrs[0][0]][0] < mesh.leaves[e][0]:
                on_coarse_edge.update((e, m) for m in side_vertices(n, side)[0])
    order = mesh.visit_order()
    for e in order:
        n = int(degrees[e]) + 1
        for side in (1, 2, 3, 4):
            bnd = mesh.boundary_side(e, side)
            nbrs = [] if bnd else mesh.neighbours(e, side)
            le = side_l(l, e, side)
            if len(nbrs) == 1:
                le = edge_l(le, n, int(degrees[nbrs[0][0]]) + 1)
            first = side_modes(n, side)[: max(0, le - 1)]
            coarse_nbr = False
            if bnd:
                if bc.get(bnd) == "dirichlet":
                    for m in first:
                        status[e][m] = 0
                else:
                    for m in first:
                        if status[e][m] != 0:
                            status[e][m] = 2
            elif (e, side) not in visited_edge:
                nbrs = mesh.neighbours(e, side)
                lev_e = mesh.leaves[e][0]
                if len(nbrs) == 1 and mesh.leaves[nbrs[0][0]][0] == lev_e:
                    c, sc = nbrs[0]
                    for m in first:
                        if status[e][m] != 0:
                            status[e][m] = 2
                    nc = int(degrees[c]) + 1
                    for m in side_modes(nc, sc)[: max(0, le - 1)]:
                        status[c][m] = 0
                    visited_edge.add((c, sc))
                elif len(nbrs) == 1 and mesh.leaves[nbrs[0][0]][0] < lev_e:
                    c, sc = nbrs[0]
                    coarse_nbr = True
                    for m in first:
                        status[e][m] = 0
                    nc = int(degrees[c]) + 1
                    for m in side_modes(nc, sc):
                        if status[c][m] != 0:
                            status[c][m] = 2
                    visited_edge.add((c, sc))
                visited_edge.add((e, side))
            else:
                nbrs = mesh.neighbours(e, side)
                if len(nbrs) == 1 and mesh.leaves[nbrs[0][0]][0] < mesh.leaves[e][0]:
                    coarse_nbr = True
            vids, pairs = side_vertices(n, side)
            cp = mesh.corner_points(e)
            for m, pr in zip(vids, pairs):
                pt = cp[pr]
                if coarse_nbr or pt in dirichlet_points or mesh.is_hanging_point(pt) \
                        or (e, m) in on_coarse_edge:
                    status[e][m] = 0
                elif pt not in kept_point and status[e][m] != 0:
                    status[e][m] = 2
                    kept_point.add(pt)
    # every copy not kept is discarded; everything left over is type 1
    for e in range(mesh.E):
        n = int(degrees[e]) + 1
        for a in (0, 1):
            for b in (0, 1):
                m = a + n * b
                if status[e][m] != 2:
                    status[e][m] = 0
        status[e][status[e] == -1] = 1
    return status


def pinv(M):
    """Moore-Penrose pseudo-inverse by the SVD with the numerical-rank cutoff
    max(rows, cols) * eps * sigma_max: constraint matrices with redundant rows
    have exact zero singular values that rounding lifts to about 1e-15, and a
    looser cutoff would invert them."""
    M = np.asarray(M)
    if M.size == 0:
        return np.zeros(M.shape[::-1], M.dtype)
    U, S, Vh = np.linalg.svd(M, full_matrices=False)
    tol = max(M.shape) * np.finfo(float).eps * (S[0] if len(S) else 0.0)
    r = int((S > tol).sum())
    return (Vh[:r].conj().T / S[:r]) @ U[:, :r].conj().T


def literal_Z(mesh, degrees, status, Cp):
    """Z = (I - C_p^+ C_p) B_z I(:, J), Sec. 2.3.2, with J ordered type 1 then
    type 2 (Z = [Z_1 Z_2]).  Dense; for small meshes.  Returns Z, the global
    indices of J1 and J2 (positions in the vertex-basis vector)."""
    off = offsets(degrees)
    ndof = int(off[-1])
    Bz = sp.block_diag([sp.csr_matrix(el.to_vertex_basis(int(p) + 1)) for p in degrees]).toarray()
    J1 = [int(off[e]) + m for e in range(mesh.E) for m in np.nonzero(status[e] == 1)[0]]
    J2 = [int(off[e]) + m for e in range(mesh.E) for m in np.nonzero(status[e] == 2)[0]]
    Cpd = Cp.toarray()
    if Cpd.shape[0]:
        Pn = np.eye(ndof) - pinv(Cpd) @ Cpd
    else:
        Pn = np.eye(ndof)
    Z = Pn @ Bz[:, J1 + J2]
    return Z, np.array(J1, int), np.array(J2, int)
