"""Write pml_scatterer_80x80_samples.txt and
point_source_32x32_robin_modified_samples.txt from the CPU oracle only.

Workloads (conforming, impedance condition outside):
  - the layered scatterer: 80x80 elements on [-1.25,1.25]^2 (the 64x64 physical
    square scatterer, p = 12, k = 150, eps_r = 4 on [-1/4,1/4]^2, plus 8 rings
    of perfectly matched layers with a quadratic profile, Sec. 3.3), normal
    incidence, scattered field;
  - the 32x32 point source (p = 16, k = 100) with Robin-modified local problems
    (gamma = +-ik on the interior sides between elements of opposite label,
    Sec. 2.3.4).
The oracle is the element-by-element dual-primal method
(oracle/dp_elementwise.py) with the Dirichlet preconditioner, solved to a
preconditioned relative residual of 1e-13.  Stored: the iteration count at
which the residual history first falls below 1e-8, seeded samples of field
values at GLL nodes, and seeded samples of rows of F v, P^-1 v and of the
interface right-hand side for a seeded random dual vector v.
Run: python tests/golden/make_pml_and_robin_modified.py [pml|robin]
(a few minutes each; both without an argument)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import dp_elementwise as dpe, problem as pb  # noqa: E402

GOLD = os.path.dirname(os.path.abspath(__file__))


def write(w, out, seed, max_iter):
    disc = pb.Discretisation(w)
    l = pb.coarse_order(w, disc.mesh)
    E = dpe.ElementwiseDP(disc, l)
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(E.nlam) + 1j * rng.standard_normal(E.nlam)
    Fv = E.apply_F(v)
    Pv = E.apply_P(v)
    g = E.interface_rhs()
    phis = E.solve(tol=1e-13, max_iter=max_iter)
    it8 = next(i for i, h in enumerate(E.hist) if h <= 1e-8)
    field = np.concatenate(pb.gll_field(disc.mesh, disc.degrees, phis))
    fidx = np.sort(rng.choice(field.size, 400, replace=False))
    ridx = np.sort(rng.choice(E.nlam, 200, replace=False))
    with open(out, "w") as f:
        f.write(f"# oracle samples for {os.path.basename(out)[:-12]} (see make_pml_and_robin_modified.py)\n")
        f.write(f"l {l}\nn_lambda {E.nlam}\nn_coarse {E.nK}\nvector_seed {seed}\n")
        f.write(f"iterations_1e-8 {it8}\niterations_1e-13 {E.iters}\n")
        for i in fidx:
            f.write(f"field {i} {field[i].real:.17e} {field[i].imag:.17e}\n")
        for i in ridx:
            f.write(f"Fv {i} {Fv[i].real:.17e} {Fv[i].imag:.17e}\n")
            f.write(f"Pv {i} {Pv[i].real:.17e} {Pv[i].imag:.17e}\n")
            f.write(f"g {i} {g[i].real:.17e} {g[i].imag:.17e}\n")
    print("wrote", out, "iterations to 1e-8:", it8, "to 1e-13:", E.iters, flush=True)


def main():
    which = sys.argv[1:] or ["pml", "robin"]
    if "pml" in which:
        write(W.pml_scatterer_64x64(), os.path.join(GOLD, "pml_scatterer_80x80_samples.txt"), 5151, 400)
    if "robin" in which:
        write(dict(W.point_source_32x32(), robin_modified=True),
              os.path.join(GOLD, "point_source_32x32_robin_modified_samples.txt"), 6161, 800)


if __name__ == "__main__":
    main()
