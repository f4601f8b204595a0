"""Quadtree leaves, neighbours and affine edge parameters (paper Sec. 2.2.3-2.2.4).
Test infrastructure only.

A mesh is a base grid of bnx-by-bny squares on [x0,x1]x[y0,y1], each the root
of a quadtree; a leaf is (level, ix, iy) with ix, iy counted on the grid of
that level.  Element sides follow Gamma_1..Gamma_4 = left, right, bottom, top.
"""
import numpy as np

OPPOSITE = {1: 2, 2: 1, 3: 4, 4: 3}


class Mesh:
    def __init__(self, x0, x1, y0, y1, bnx, bny, leaves):
        self.x0, self.x1, self.y0, self.y1 = x0, x1, y0, y1
        self.bnx, self.bny = bnx, bny
        self.leaves = [tuple(int(t) for t in lf) for lf in leaves]
        self.E = len(self.leaves)
        self.Lmax = max(lf[0] for lf in self.leaves)
        # integer extents on the finest grid
        self.ext = []
        for (lev, ix, iy) in self.leaves:
            s = 2 ** (self.Lmax - lev)
            self.ext.append((ix * s, (ix + 1) * s, iy * s, (iy + 1) * s))
        self.fine_hx = (x1 - x0) / (bnx * 2 ** self.Lmax)
        self.fine_hy = (y1 - y0) / (bny * 2 ** self.Lmax)
        self.NX = bnx * 2 ** self.Lmax
        self.NY = bny * 2 ** self.Lmax
        self._build_lines()

    # geometry -------------------------------------------------------------
    def size(self, e):
        lev = self.leaves[e][0]
        return ((self.x1 - self.x0) / (self.bnx * 2 ** lev),
                (self.y1 - self.y0) / (self.bny * 2 ** lev))

    def origin(self, e):
        X0, _, Y0, _ = self.ext[e]
        return self.x0 + X0 * self.fine_hx, self.y0 + Y0 * self.fine_hy

    def center(self, e):
        (ox, oy), (hx, hy) = self.origin(e), self.size(e)
        return ox + hx / 2, oy + hy / 2

    def side_segment(self, e, side):
        """(line key, lo, hi) of a side in finest-grid integers."""
        X0, X1, Y0, Y1 = self.ext[e]
        if side == 1:
            return ("v", X0), Y0, Y1
        if side == 2:
            return ("v", X1), Y0, Y1
        if side == 3:
            return ("h", Y0), X0, X1
        return ("h", Y1), X0, X1

    def _build_lines(self):
        self.lines = {}
        for e in range(self.E):
            for side in (1, 2, 3, 4):
                key, lo, hi = self.side_segment(e, side)
                self.lines.setdefault(key, []).append((lo, hi, e, side))

    def boundary_side(self, e, side):
        """Domain side (1..4) if this element side lies on the outer boundary, else 0."""
        (kind, c), _, _ = self.side_segment(e, side)
        if kind == "v" and c == 0:
            return 1
        if kind == "v" and c == self.NX:
            return 2
        if kind == "h" and c == 0:
            return 3
        if kind == "h" and c == self.NY:
            return 4
        return 0

    def neighbours(self, e, side):
        """Leaves across a side: list of (leaf, their side) overlapping it."""
        key, lo, hi = self.side_segment(e, side)
        want = OPPOSITE[side]
        out = []
        for (l2, h2, f, s2) in self.lines[key]:
            if f != e and s2 == want and min(hi, h2) > max(lo, l2):
                out.append((f, s2))
        return out

    def along_index(self, e, side):
        """Index along the edge direction at the element's own level."""
        lev, ix, iy = self.leaves[e]
        return iy if side in (1, 2) else ix

    def affine_params(self, fine, side, coarse):
        """(a, b) of eq. (affine_parameters), Sec. 2.2.4: climb from the fine
        element's same-level neighbour to the coarse leaf; step i records
        s_i = +1 if the node sits in the upper/right half of its parent.
        a = 2^-m, b = 2^-m sum_i s_i 2^(i-1)."""
        m = self.leaves[fine][0] - self.leaves[coarse][0]
        idx = self.along_index(fine, side)
        b = 0.0
        for i in range(1, m + 1):
            s = 1.0 if (idx >> (i - 1)) & 1 else -1.0
            b += s * 2.0 ** (i - 1)
        return 2.0 ** (-m), b * 2.0 ** (-m)

    def affine_params_geometric(self, fine, side, coarse):
        """The same (a, b) from coordinates: the fine edge as a sub-interval
        a*s+b of the coarse edge's parameter in [-1,1]."""
        _, lo_f, hi_f = self.side_segment(fine, side)
        _, lo_c, hi_c = self.side_segment(coarse, OPPOSITE[side])
        t0 = -1.0 + 2.0 * (lo_f - lo_c) / (hi_c - lo_c)
        t1 = -1.0 + 2.0 * (hi_f - lo_c) / (hi_c - lo_c)
        return (t1 - t0) / 2.0, (t1 + t0) / 2.0

    def visit_order(self):
        """Elements finest level first, input order within a level (Algorithm 1)."""
        levels = sorted({lf[0] for lf in self.leaves}, reverse=True)
        return [e for lev in levels for e in range(self.E) if self.leaves[e][0] == lev]

    def corner_points(self, e):
        """Finest-grid integer corners keyed by the element's vertex modes of the
        vertex basis: index 0 of a direction is the +1 end, index 1 the -1 end."""
        X0, X1, Y0, Y1 = self.ext[e]
        xs = {0: X1, 1: X0}
        ys = {0: Y1, 1: Y0}
        return {(a, b): (xs[a], ys[b]) for a in (0, 1) for b in (0, 1)}

    def is_hanging_point(self, pt):
        """True if pt lies strictly inside a side of some leaf (a hanging node)."""
        X, Y = pt
        for e in range(self.E):
            X0, X1, Y0, Y1 = self.ext[e]
            if (X in (X0, X1) and Y0 < Y < Y1) or (Y in (Y0, Y1) and X0 < X < X1):
                return True
        return False

