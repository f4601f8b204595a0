"""Seeded synthetic workloads shared by the tests, the oracle and the benchmark.

This module only describes inputs (mesh leaves, per-element degrees and
relative permittivities, wavenumber, boundary conditions and right-hand-side
kind).  It holds none of the method's arithmetic.

The workloads stand in for the paper's test problems (whose meshes come from
its own generator): a small plane-wave check, a 32x32 point-source case, a
quadtree-refined dielectric disk with uneven degrees, a square dielectric
scatterer lit from 64 directions, a permittivity design block, and the square
scatterer inside perfectly matched layers.
"""
import math

import numpy as np


def morton_leaves(nx, ny, level=0):
    """Leaves (level, ix, iy) of an nx-by-ny grid in z (Morton) order."""
    def key(t):
        ix, iy = t
        k = 0
        for bit in range(20):
            k |= ((ix >> bit) & 1) << (2 * bit)
            k |= ((iy >> bit) & 1) << (2 * bit + 1)
        return k
    cells = sorted(((ix, iy) for ix in range(nx) for iy in range(ny)), key=key)
    return [(level, ix, iy) for ix, iy in cells]


def refine_where(leaves, x0, x1, y0, y1, bnx, bny, inside, passes):
    """Split every leaf whose centre satisfies inside(x, y), `passes` times.
    Children replace their parent in z order (the order of a depth-first
    quadtree walk)."""
    for _ in range(passes):
        out = []
        for (lev, ix, iy) in leaves:
            hx = (x1 - x0) / (bnx * 2 ** lev)
            hy = (y1 - y0) / (bny * 2 ** lev)
            cx, cy = x0 + (ix + 0.5) * hx, y0 + (iy + 0.5) * hy
            if inside(cx, cy):
                for (dx, dy) in ((0, 0), (1, 0), (0, 1), (1, 1)):
                    out.append((lev + 1, 2 * ix + dx, 2 * iy + dy))
            else:
                out.append((lev, ix, iy))
        leaves = out
    return leaves


def leaf_centres(w):
    x0, x1, y0, y1 = w["domain"]
    bnx, bny = w["base"]
    out = []
    for (lev, ix, iy) in w["leaves"]:
        hx = (x1 - x0) / (bnx * 2 ** lev)
        hy = (y1 - y0) / (bny * 2 ** lev)
        out.append((x0 + (ix + 0.5) * hx, y0 + (iy + 0.5) * hy))
    return np.array(out)


def _uniform(name, domain, n, p, k, **kw):
    w = dict(name=name, domain=domain, base=(n, n), leaves=morton_leaves(n, n),
             degree=np.full(n * n, p, dtype=np.int32), k=float(k),
             eps_r=np.ones(n * n), bc="impedance", l=-1, tol=1e-10)
    w.update(kw)
    return w


def plane_wave_4x4():
    """Unit square, 4x4 quads, p=8, k=10, impedance data from the plane wave
    e^{ik(x cos30 + y sin30)} (the exact solution); coarse space = vertices."""
    return _uniform("plane_wave_4x4_p8_k10", (0.0, 1.0, 0.0, 1.0), 4, 8, 10.0,
                    l=1, rhs=dict(kind="plane_wave_total", angles=[math.radians(30.0)]))


def point_source_32x32():
    """Unit square, 32x32 quads, p=16, k=100, point source at the vertex
    (0.5, 0.5), homogeneous impedance condition; l from the dispersion rule."""
    return _uniform("point_source_32x32_p16_k100", (0.0, 1.0, 0.0, 1.0), 32, 16, 100.0,
                    tol=1e-8, rhs=dict(kind="point", points=[(0.5, 0.5)]))


def square_scatterer_64x64(n_angles=64):
    """[-1,1]^2, 64x64 quads, p=12, k=150, a square [-1/4,1/4]^2 with eps_r=4,
    plane waves from n_angles directions evenly spaced in [0, 2pi), scattered-
    field formulation with a homogeneous impedance condition."""
    w = _uniform("square_scatterer_64x64_p12_k150", (-1.0, 1.0, -1.0, 1.0), 64, 12, 150.0,
                 tol=1e-8)
    c = leaf_centres(w)
    inside = (np.abs(c[:, 0]) < 0.25) & (np.abs(c[:, 1]) < 0.25)
    w["eps_r"] = np.where(inside, 4.0, 1.0)
    w["rhs"] = dict(kind="plane_wave_scattered",
                    angles=[2 * math.pi * m / n_angles for m in range(n_angles)])
    w["far_angles"] = [2 * math.pi * q / 360 for q in range(360)]
    return w


def design_block_64x64(seed=5):
    """Square-scatterer mesh with per-element eps_r ~ U[1,4] on the central
    16x16 element block (a permittivity design region), normal incidence."""
    w = square_scatterer_64x64(1)
    w["name"] = "design_block_64x64_p12_k150"
    rng = np.random.default_rng(seed)
    c = leaf_centres(w)
    h = 2.0 / 64
    block = (np.abs(c[:, 0]) < 8 * h) & (np.abs(c[:, 1]) < 8 * h)
    eps = np.ones(len(c))
    eps[block] = rng.uniform(1.0, 4.0, size=int(block.sum()))
    w["eps_r"] = eps
    w["rhs"] = dict(kind="plane_wave_scattered", angles=[0.0])
    w["far_angles"] = [0.0]
    w["seed"] = seed
    return w


def refined_disk(seed=0):
    """[-1,1]^2 from a 16x16 base, leaves with centre inside r<0.4 split twice,
    p ~ U{8..24} per leaf (seeded, z order), refractive index 1.5 inside the
    disk, k=200, plane-wave incidence, impedance condition."""
    x0, x1, y0, y1 = -1.0, 1.0, -1.0, 1.0
    leaves = morton_leaves(16, 16)
    leaves = refine_where(leaves, x0, x1, y0, y1, 16, 16,
                          lambda x, y: x * x + y * y < 0.16, 2)
    rng = np.random.default_rng(seed)
    w = dict(name="refined_disk_k200", domain=(x0, x1, y0, y1), base=(16, 16),
             leaves=leaves, degree=rng.integers(8, 25, size=len(leaves)).astype(np.int32),
             k=200.0, bc="impedance", l=-1, tol=1e-8, seed=seed)
    c = leaf_centres(w)
    w["eps_r"] = np.where((c ** 2).sum(1) < 0.16, 2.25, 1.0)
    w["rhs"] = dict(kind="plane_wave_scattered", angles=[0.0])
    # dual constraints on hanging edges whose change-of-basis diagonal a^k has
    # decayed below 1e-3 are dropped (the threshold is left to the user)
    w["discard_tol"] = 1e-3
    return w


def pml_sigma(leaves, base, n_phys, n_layer, sigma_max):
    """Per-leaf (sigma_x, sigma_y) for layers of n_layer element rings around an
    n_phys x n_phys block of a uniform base grid: ring r (0 innermost) carries
    sigma_max ((r + 1/2) / n_layer)^2 along the axis it crosses (both in corners)."""
    sig = np.zeros((len(leaves), 2))
    for e, (lev, ix, iy) in enumerate(leaves):
        for a, i in enumerate((ix, iy)):
            r = n_layer - 1 - i if i < n_layer else i - n_layer - n_phys if i >= n_layer + n_phys else -1
            if r >= 0:
                sig[e, a] = sigma_max * ((r + 0.5) / n_layer) ** 2
    return sig


def pml_scatterer_64x64(n_layer=8, sigma_max=144.0):
    """The square scatterer (64x64 physical elements on [-1,1]^2, p=12, k=150,
    eps_r=4 on [-1/4,1/4]^2, normal incidence, scattered field) surrounded by
    n_layer rings of perfectly matched layers with a quadratic profile (about
    e^{-12} attenuation across them), impedance condition outside."""
    n = 64 + 2 * n_layer
    h = 2.0 / 64
    L = 1.0 + n_layer * h
    w = _uniform(f"pml_scatterer_64x64_p12_k150_{n_layer}layers", (-L, L, -L, L), n, 12, 150.0, tol=1e-8)
    c = leaf_centres(w)
    w["eps_r"] = np.where((np.abs(c[:, 0]) < 0.25) & (np.abs(c[:, 1]) < 0.25), 4.0, 1.0)
    w["pml_sigma"] = pml_sigma(w["leaves"], (n, n), 64, n_layer, sigma_max)
    w["rhs"] = dict(kind="plane_wave_scattered", angles=[0.0])
    w["far_angles"] = [2 * math.pi * q / 360 for q in range(360)]
    return w


def small_uniform(n=4, p=6, k=7.0, domain=(0.0, 1.0, 0.0, 1.0), l=-1, rhs=None, eps=None):
    """A small uniform mesh for parity tests at sizes the oracle finishes quickly."""
    w = _uniform(f"uniform_{n}x{n}_p{p}_k{k:g}", domain, n, p, k, l=l,
                 rhs=rhs or dict(kind="plane_wave_total", angles=[0.3]))
    if eps is not None:
        w["eps_r"] = np.asarray(eps, float)
    return w


ALL = {
    "plane_wave_4x4": plane_wave_4x4,
    "point_source_32x32": point_source_32x32,
    "refined_disk": refined_disk,
    "square_scatterer_64x64": square_scatterer_64x64,
    "design_block_64x64": design_block_64x64,
    "pml_scatterer_64x64": pml_scatterer_64x64,
}


def hanging_square(base, pvals, seed, l, k=6.0, rhs="plane_wave_total"):
    """[0,1]^2 from a base x base grid, leaves near the centre split twice (up to
    three hanging nodes per edge), p ~ U{pvals} per leaf (seeded); with a
    scattered-field right-hand side, eps_r = 2.25 in a disk of radius 0.2."""
    lv = refine_where(morton_leaves(base, base), 0, 1, 0, 1, base, base,
                      lambda x, y: (x - 0.5) ** 2 + (y - 0.5) ** 2 < (0.03 if base % 2 else 0.05), 2)
    deg = np.random.default_rng(seed).integers(pvals[0], pvals[1] + 1, len(lv))
    w = dict(domain=(0.0, 1.0, 0.0, 1.0), base=(base, base), leaves=lv, degree=deg, k=k, l=l,
             bc="impedance", eps_r=np.ones(len(lv)), rhs=dict(kind=rhs, angles=[0.4]))
    if rhs == "plane_wave_scattered":
        c = leaf_centres(w)
        w["eps_r"] = np.where((c[:, 0] - 0.5) ** 2 + (c[:, 1] - 0.5) ** 2 < 0.04, 2.25, 1.0)
    return w


def small_disk(base=6, pvals=(3, 6), seed=4, k=12.0, tau=1e-3):
    """The refined-disk layout at a small size: [-1,1]^2, leaves with centre in
    r < 0.4 split twice, eps_r = 2.25 inside, uneven p, discard threshold tau."""
    lv = refine_where(morton_leaves(base, base), -1, 1, -1, 1, base, base,
                      lambda x, y: x * x + y * y < 0.16, 2)
    deg = np.random.default_rng(seed).integers(pvals[0], pvals[1] + 1, len(lv))
    w = dict(domain=(-1.0, 1.0, -1.0, 1.0), base=(base, base), leaves=lv, degree=deg, k=k, l=-1,
             bc="impedance", rhs=dict(kind="plane_wave_scattered", angles=[0.0]), discard_tol=tau)
    c = leaf_centres(w)
    w["eps_r"] = np.where((c ** 2).sum(1) < 0.16, 2.25, 1.0)
    return w


def hanging_cases():
    """The quadtree meshes of the parity tests, by name."""
    return {
        "h3_p4_l1": hanging_square(3, (4, 4), 0, 1),
        "h3_p3to6_l2": hanging_square(3, (3, 6), 1, 2),
        "h4_p2to5_l3": hanging_square(4, (2, 5), 2, 3),
        "h3_p3to7_l7": hanging_square(3, (3, 7), 3, 7),
        "h4_p4to6_l2_lens": hanging_square(4, (4, 6), 5, 2, k=9.0, rhs="plane_wave_scattered"),
        "h3_p3to6_l2_tau": dict(hanging_square(3, (3, 6), 1, 2), discard_tol=1e-2),
        "h4_p2to5_l3_tau": dict(hanging_square(4, (2, 5), 2, 3), discard_tol=3e-3),
        "disk_6x6_p3to6": small_disk(),
    }

