"""Write point_source_32x32_samples.txt from the CPU oracle only.

Workload: unit square, 32x32 quads, p = 16, k = 100, point source at the
vertex (0.5, 0.5), homogeneous impedance condition, l from the dispersion
rule (l = 2).  The oracle is the element-by-element dual-primal method
(oracle/dp_elementwise.py), solved to a preconditioned relative residual of
1e-13.  Stored: the iteration counts at which the residual history first falls
below 1e-8 and 1e-12, a seeded sample of field values at GLL nodes, and a seeded
sample of rows of F v and P^-1 v for a seeded random dual vector v.
Run: python tests/golden/make_point_source_32x32.py   (about three minutes)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import dp_elementwise as dpe, problem as pb  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "point_source_32x32_samples.txt")


def main():
    w = W.point_source_32x32()
    disc = pb.Discretisation(w)
    l = pb.coarse_order(w, disc.mesh)
    E = dpe.ElementwiseDP(disc, l)
    rng = np.random.default_rng(1234)
    v = rng.standard_normal(E.nlam) + 1j * rng.standard_normal(E.nlam)
    Fv = E.apply_F(v)
    Pv = E.apply_P(v)
    phis = E.solve(tol=1e-13, max_iter=400)
    it8 = next(i for i, h in enumerate(E.hist) if h <= 1e-8)
    it12 = next(i for i, h in enumerate(E.hist) if h <= 1e-12)
    field = np.concatenate(pb.gll_field(disc.mesh, disc.degrees, phis))
    fidx = np.sort(rng.choice(field.size, 400, replace=False))
    ridx = np.sort(rng.choice(E.nlam, 200, replace=False))
    with open(OUT, "w") as f:
        f.write("# oracle samples for point_source_32x32 (see make_point_source_32x32.py)\n")
        f.write(f"l {l}\nn_lambda {E.nlam}\nn_coarse {E.nK}\niterations_1e-8 {it8}\n")
        f.write(f"iterations_1e-12 {it12}\niterations_1e-13 {E.iters}\nvector_seed 1234\n")
        for i in fidx:
            f.write(f"field {i} {field[i].real:.17e} {field[i].imag:.17e}\n")
        for i in ridx:
            f.write(f"Fv {i} {Fv[i].real:.17e} {Fv[i].imag:.17e}\n")
            f.write(f"Pv {i} {Pv[i].real:.17e} {Pv[i].imag:.17e}\n")
    print("wrote", OUT, "iterations to 1e-8:", it8, "to 1e-12:", it12, "to 1e-13:", E.iters)


if __name__ == "__main__":
    main()
