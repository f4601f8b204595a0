"""Element-by-element discretisation of a workload (paper Sec. 2.2.1 with the
Helmholtz data of Sec. 2.3.4 and Sec. 3).  Test infrastructure only.

Time convention e^{-i omega t}: the outgoing impedance condition is
d_n u - i k u = g, i.e. the Robin form n.grad(phi) + gamma phi = q with
gamma = -i k and q = g.  Helmholtz: alpha = I, beta = -k^2 eps_r.
"""
import numpy as np
from scipy.special import hankel2

from . import element as el
from . import legendre as lg
from .mesh import Mesh

NORMALS = {1: (-1.0, 0.0), 2: (1.0, 0.0), 3: (0.0, -1.0), 4: (0.0, 1.0)}


def make_mesh(w):
    x0, x1, y0, y1 = w["domain"]
    bnx, bny = w["base"]
    return Mesh(x0, x1, y0, y1, bnx, bny, w["leaves"])


def coarse_order(w, mesh=None):
    """l: explicit, or from the dispersion rule of Sec. 2.3.4 evaluated per element
    with its longest edge and its local wavenumber k sqrt(eps_r), taking the largest
    (with eps_r = 1: the free-space k and the longest edge, as in Sec. 3.3.1); with
    w["l_free_space"] the free-space k everywhere (the reading of the dielectric
    cylinder of Sec. 3.3.1); with w["l_per_edge"] the per-edge orders of
    edge_orders (a function of (e, side))."""
    if w.get("l", -1) >= 1:
        return int(w["l"])
    mesh = mesh or make_mesh(w)
    if w.get("l_per_edge", False):
        return edge_orders(w, mesh)
    eps = np.asarray(w.get("eps_r", np.ones(mesh.E)))
    if w.get("l_free_space", False):
        eps = np.ones(mesh.E)
    kh = max(w["k"] * np.sqrt(eps[e]) * max(mesh.size(e)) for e in range(mesh.E))
    return lg.dispersion_l(kh, 1.0)


def edge_orders(w, mesh=None, safety=0):
    """Per-edge coarse order (the non-uniform choice of l that the conclusions
    propose for non-uniformly refined meshes): the dispersion rule of Sec. 2.3.4
    evaluated on each edge with, for every element touching the edge, its own
    side length along the edge and its local wavenumber k sqrt(eps_r), the
    largest value taken.  A hanging edge is the coarse side with all the fine
    leaves along it, so both of its sides get one value.  Returns l(e, side)."""
    mesh = mesh or make_mesh(w)
    eps = np.asarray(w.get("eps_r", np.ones(mesh.E)))
    if w.get("l_free_space", False):
        eps = np.ones(mesh.E)
    k = float(w["k"])

    def side_len(e, side):
        hx, hy = mesh.size(e)
        return hy if side in (1, 2) else hx

    def value(e, side):
        if not mesh.boundary_side(e, side):
            nbrs = mesh.neighbours(e, side)
            if len(nbrs) == 1 and mesh.leaves[nbrs[0][0]][0] < mesh.leaves[e][0]:
                e, side = nbrs[0]          # the coarse side holds the edge
        touching = [(e, side)] + ([] if mesh.boundary_side(e, side) else mesh.neighbours(e, side))
        return max(lg.dispersion_l(k * np.sqrt(eps[f]) * side_len(f, sf), 1.0) for f, sf in touching) + safety

    cache = {}

    def l_of(e, side):
        if (e, side) not in cache:
            cache[(e, side)] = value(e, side)
        return cache[(e, side)]
    return l_of


def robin_labels(mesh):
    """Signs for the Robin-modified local problems (Sec. 2.3.4): a breadth-first
    spanning tree of the element adjacency graph from leaf 0, labelled +1 on even
    and -1 on odd levels.  Neighbours are taken side by side (left, right, bottom,
    top) and, across one side, in increasing leaf order, so that the labelling is
    reproducible."""
    lab = np.zeros(mesh.E, int)
    depth = -np.ones(mesh.E, int)
    depth[0] = 0
    queue = [0]
    while queue:
        nxt = []
        for e in queue:
            for side in (1, 2, 3, 4):
                for f, _ in sorted(mesh.neighbours(e, side)):
                    if depth[f] < 0:
                        depth[f] = depth[e] + 1
                        nxt.append(f)
        queue = nxt
    if (depth < 0).any():
        raise ValueError("mesh is not connected")
    lab[:] = np.where(depth % 2 == 0, 1, -1)
    return lab


def robin_sides(mesh, e, lab):
    """Interior sides of element e that carry the Robin term: those whose
    neighbours all have the opposite label.  A side whose neighbours carry both
    labels would need the term on part of the side only, which this
    discretisation does not form."""
    out = []
    for side in (1, 2, 3, 4):
        if mesh.boundary_side(e, side):
            continue
        others = {lab[f] for f, _ in mesh.neighbours(e, side)}
        if others == {-lab[e]}:
            out.append(side)
        elif len(others) > 1:
            raise NotImplementedError("Robin-modified local problems: a side whose neighbours carry both labels")
    return out


def edge_param(mesh, e, side):
    """Map s in [-1,1] along a side to (x, y)."""
    (ox, oy), (hx, hy) = mesh.origin(e), mesh.size(e)
    if side in (1, 2):
        xc = ox if side == 1 else ox + hx
        return lambda s: (np.full_like(s, xc), oy + (s + 1) * hy / 2), hy
    yc = oy if side == 3 else oy + hy
    return lambda s: (ox + (s + 1) * hx / 2, np.full_like(s, yc)), hx


class Discretisation:
    """A_e (paper basis N), the Laplace-only part, loads b_e, Dirichlet data."""

    def __init__(self, w, mesh=None, bc=None, alpha=None, poisson=False, modified=None):
        self.w = w
        self.mesh = mesh or make_mesh(w)
        m = self.mesh
        # Robin-modified local problems (Sec. 2.3.4): gamma = +-ik on the interior
        # sides between elements of opposite label; the two terms of a side cancel
        # in the assembled system, which is therefore unchanged
        self.modified = bool(w.get("robin_modified", False) if modified is None else modified)
        self.labels = robin_labels(m) if self.modified else None
        self.k = float(w.get("k", 0.0))
        self.degrees = np.asarray(w["degree"])
        # axis-aligned perfectly matched layers (Sec. 3.3): complex stretching
        # s_i = 1 + i sigma_i / k (the paper's 1 - j sigma_i / omega in the e^{-i omega t}
        # convention, omega = k in scaled units), piecewise constant per element;
        # alpha = diag(s_y / s_x, s_x / s_y) and beta = -k^2 eps s_x s_y
        sig = w.get("pml_sigma")
        self.stretch = None
        if sig is not None:
            sig = np.asarray(sig, float).reshape(m.E, 2)
            self.stretch = 1.0 + 1j * sig / self.k
        eps = np.asarray(w.get("eps_r", np.ones(m.E)))
        alpha = np.ones(m.E) if alpha is None else np.asarray(alpha)
        if bc is None:
            bc = {s: ("dirichlet" if w.get("bc") == "dirichlet" else "robin") for s in (1, 2, 3, 4)}
        self.bc = bc
        gamma = -1j * self.k
        self.A, self.A_lap, self.b = [], [], []
        rhs = w.get("rhs", {"kind": "none"})
        for e in range(m.E):
            n = int(self.degrees[e]) + 1
            hx, hy = m.size(e)
            beta = 0.0 if poisson else -self.k ** 2 * eps[e]
            al = alpha[e]
            if self.stretch is not None:
                sx, sy = self.stretch[e]
                al = (alpha[e] * sy / sx, alpha[e] * sx / sy)
                beta = beta * sx * sy
            robin = {}
            for side in (1, 2, 3, 4):
                bnd = m.boundary_side(e, side)
                if bnd and bc[bnd] == "robin":
                    robin[side] = gamma
            terms = dict(robin)
            if self.modified:
                for side in robin_sides(m, e, self.labels):
                    terms[side] = self.labels[e] * 1j * self.k
            self.A.append(el.element_matrix(n, hx, hy, alpha=al, beta=beta, robin=terms))
            self.A_lap.append(el.element_matrix(n, hx, hy, alpha=al))
            self.b.append(self._load(e, n, hx, hy, eps[e], rhs, robin))

    def _load(self, e, n, hx, hy, eps_e, rhs, robin):
        m = self.mesh
        kind = rhs["kind"]
        k = self.k
        b = np.zeros(n * n, complex)
        (ox, oy) = m.origin(e)
        if kind == "plane_wave_total":
            th = rhs["angles"][0]
            d = np.array([np.cos(th), np.sin(th)])
            for side in robin:
                xy, h_edge = edge_param(m, e, side)
                nrm = np.array(NORMALS[side])

                def q(s, xy=xy, nrm=nrm):
                    x, y = xy(s)
                    return 1j * k * (d @ nrm - 1.0) * np.exp(1j * k * (d[0] * x + d[1] * y))
                b += el.edge_load(n, h_edge, side, el.legendre_coeffs_1d(q, n))
        elif kind == "plane_wave_scattered":
            th = rhs["angles"][0]
            d = np.array([np.cos(th), np.sin(th)])
            if eps_e != 1.0:
                def f(u, v):
                    x = ox + (u + 1) * hx / 2
                    y = oy + (v + 1) * hy / 2
                    return k ** 2 * (eps_e - 1.0) * np.exp(1j * k * (d[0] * x + d[1] * y))
                b += el.volume_load(n, hx, hy, el.legendre_coeffs_2d(f, n))
        elif kind == "point":
            for (px, py) in rhs["points"]:
                owners = [f for f in range(m.E) if _contains(m, f, px, py)]
                if e in owners:
                    u = 2 * (px - ox) / hx - 1
                    v = 2 * (py - oy) / hy - 1
                    b += el.point_load(n, u, v) / len(owners)
        elif kind == "random":
            rng = np.random.default_rng(rhs.get("seed", 0) + e)
            b += rng.uniform(0.0, 1.0, n * n)
        return b

    def dirichlet_fun(self):
        """Legendre coefficients of the Dirichlet data along a side, or None."""
        rhs = self.w.get("rhs", {"kind": "none"})
        if rhs["kind"] != "dirichlet_hankel":
            return None
        xc, yc = rhs["center"]
        k = self.k
        m = self.mesh

        def fun(e, side, n):
            xy, _ = edge_param(m, e, side)

            def pfun(s):
                x, y = xy(s)
                return -0.25j * hankel2(0, k * np.hypot(x - xc, y - yc))
            return el.legendre_coeffs_1d(pfun, n)
        return fun


def _contains(m, e, px, py):
    (ox, oy), (hx, hy) = m.origin(e), m.size(e)
    tol = 1e-12
    return (ox - tol <= px <= ox + hx + tol) and (oy - tol <= py <= oy + hy + tol)


def exact_plane_wave(w):
    th = w["rhs"]["angles"][0]
    k = w["k"]
    return lambda x, y: np.exp(1j * k * (np.cos(th) * x + np.sin(th) * y))


def sample_field(mesh, degrees, phis, pts_fun):
    """Evaluate each element expansion phi = N(u)^T Phi N(v) on a local tensor grid
    given by pts_fun(n) -> 1-D points; returns list of (n_pts^2,) arrays, x fastest."""
    out = []
    for e in range(mesh.E):
        n = int(degrees[e]) + 1
        t = pts_fun(n)
        Nt = lg.basis_N(t, n)          # (n, npts)
        Phi = phis[e].reshape(n, n, order="F")
        out.append((Nt.T @ Phi @ Nt).reshape(-1, order="F"))
    return out


def gll_field(mesh, degrees, phis):
    """Field at the tensor GLL nodes of each element, x fastest."""
    return sample_field(mesh, degrees, phis, lg.gll_nodes)
