"""Write design_block_64x64_gradient.txt from the CPU oracle only.

Workload: the 64x64 square-scatterer mesh ([-1,1]^2, p = 12, k = 150) with
eps_r ~ U[1,4] (seeded) on the central 16x16 elements, J = |E_far(0)|^2 over the
boundary of that block for normal incidence.  The oracle's adjoint gradient
(oracle/adjoint.py, element-by-element dual-primal forward and adjoint solves to
a preconditioned residual of 1e-13) is stored for the 256 design elements
together with J and E_far.
Run: python tests/golden/make_design_block_64x64.py   (several minutes)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import adjoint as adj  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "design_block_64x64_gradient.txt")


def main():
    w = W.design_block_64x64()
    c = W.leaf_centres(w)
    h = 2.0 / 64
    inside = (np.abs(c[:, 0]) < 8 * h) & (np.abs(c[:, 1]) < 8 * h)
    J, g, E = adj.eps_gradient(w, 0.0, 0.0, inside, solver="elementwise", tol=1e-13)
    with open(OUT, "w") as f:
        f.write("# oracle adjoint gradient for design_block_64x64 (see make_design_block_64x64.py)\n")
        f.write(f"J {J:.17e}\nE {E.real:.17e} {E.imag:.17e}\n")
        for e in np.nonzero(inside)[0]:
            f.write(f"grad {e} {g[e]:.17e}\n")
    print("wrote", OUT, "J", J)


if __name__ == "__main__":
    main()
