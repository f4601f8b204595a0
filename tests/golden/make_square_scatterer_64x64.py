"""Write square_scatterer_64x64_samples.txt from the CPU oracle only.

Workload: [-1,1]^2, 64x64 quads, p = 12, k = 150, the square [-1/4,1/4]^2 with
eps_r = 4, scattered-field plane waves, homogeneous impedance condition, l from
the dispersion rule with the local wavenumber (l = 6).  The oracle is the
element-by-element dual-primal method (oracle/dp_elementwise.py) solved to a
preconditioned relative residual of 1e-13, for two of the 64 incidence angles
(m = 0 and m = 5 of 2 pi m / 64).  Stored per angle: the iteration count at
which the residual history first falls below 1e-8, a seeded sample of 400
field values at GLL nodes, and the far field E_far at the 360 angles 2 pi q / 360
over the boundary of the dielectric square (Sec. 3.3.1, e^{-i w t} form);
once: a seeded sample of rows of F v and P^-1 v for a seeded random dual vector.
Run: python tests/golden/make_square_scatterer_64x64.py   (several minutes)
"""
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import dp_elementwise as dpe, farfield as ff, problem as pb  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "square_scatterer_64x64_samples.txt")
ANGLE_INDICES = (0, 5)


def main():
    base = W.square_scatterer_64x64()
    inside = np.asarray(base["eps_r"]) != 1.0
    far_angles = np.asarray(base["far_angles"])
    lines = []
    rng = np.random.default_rng(4321)
    for j, m in enumerate(ANGLE_INDICES):
        theta = 2 * math.pi * m / 64
        w = dict(base, rhs=dict(kind="plane_wave_scattered", angles=[theta]))
        disc = pb.Discretisation(w)
        l = pb.coarse_order(w, disc.mesh)
        E = dpe.ElementwiseDP(disc, l)
        if j == 0:
            lines += [f"l {l}", f"n_lambda {E.nlam}", f"n_coarse {E.nK}", "vector_seed 4321"]
            v = rng.standard_normal(E.nlam) + 1j * rng.standard_normal(E.nlam)
            Fv, Pv = E.apply_F(v), E.apply_P(v)
            ridx = np.sort(rng.choice(E.nlam, 200, replace=False))
            for i in ridx:
                lines.append(f"Fv {i} {Fv[i].real:.17e} {Fv[i].imag:.17e}")
                lines.append(f"Pv {i} {Pv[i].real:.17e} {Pv[i].imag:.17e}")
        phis = E.solve(tol=1e-13, max_iter=400)
        it8 = next(i for i, h in enumerate(E.hist) if h <= 1e-8)
        field = np.concatenate(pb.gll_field(disc.mesh, disc.degrees, phis))
        far = ff.far_field(disc.mesh, disc.degrees, phis, disc.k, inside, far_angles)
        lines.append(f"angle {m} iterations_1e-8 {it8} iterations_1e-13 {E.iters}")
        fidx = np.sort(rng.choice(field.size, 400, replace=False))
        for i in fidx:
            lines.append(f"field {m} {i} {field[i].real:.17e} {field[i].imag:.17e}")
        for q, a in enumerate(far):
            lines.append(f"far {m} {q} {a.real:.17e} {a.imag:.17e}")
        print(f"angle index {m}: iterations to 1e-8 {it8}, to 1e-13 {E.iters}", flush=True)
    with open(OUT, "w") as f:
        f.write("# oracle samples for square_scatterer_64x64 (see make_square_scatterer_64x64.py)\n")
        f.write("\n".join(lines) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
