"""Write refined_disk_samples.txt from the CPU oracle only.

Workload: [-1,1]^2 from a 16x16 base, leaves with centre in r < 0.4 split twice
(712 leaves, up to three hanging nodes per edge), p ~ U{8..24} (seed 0), k = 200,
eps_r = 2.25 in the disk, one plane wave (theta = 0, scattered field),
impedance condition, l from the dispersion rule (14), discard threshold 1e-3.
The oracle is the element-by-element dual-primal method on quadtree meshes
(oracle/dp_nonconforming.py), solved to a preconditioned relative residual of
1e-13 with its own preconditioner.  Stored: a seeded sample of rows of F v for
a seeded random dual vector v, of the interface right-hand side g, and of the
field at GLL nodes.  The preconditioner depends on the basis of the
constrained space and the iteration count on the preconditioner, so neither is
stored.
The same for the per-edge coarse order (the dispersion rule edge by edge, the
conclusions' proposal) in refined_disk_per_edge_samples.txt.
Run: python tests/golden/make_refined_disk.py [plain|per_edge]   (about six
minutes each; both without an argument)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import dp_nonconforming as dnc, problem as pb  # noqa: E402

GOLD = os.path.dirname(os.path.abspath(__file__))


def write(w, out, seed):
    disc = pb.Discretisation(w)
    l = pb.coarse_order(w, disc.mesh)
    N = dnc.NonconformingDP(disc, l)
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(N.nlam) + 1j * rng.standard_normal(N.nlam)
    Fv = N.apply_F(v)
    g = N.interface_rhs()
    phis = N.solve(tol=1e-13, max_iter=800)
    field = np.concatenate(pb.gll_field(disc.mesh, disc.degrees, phis))
    fidx = np.sort(rng.choice(field.size, 400, replace=False))
    ridx = np.sort(rng.choice(N.nlam, 200, replace=False))
    with open(out, "w") as f:
        f.write(f"# oracle samples for {os.path.basename(out)[:-12]} (see make_refined_disk.py)\n")
        if not callable(l):
            f.write(f"l {l}\n")
        f.write(f"n_lambda {N.nlam}\nn_coarse {N.nK}\nvector_seed {seed}\n")
        f.write(f"oracle_iterations_1e-13 {N.iters}\n")
        for i in fidx:
            f.write(f"field {i} {field[i].real:.17e} {field[i].imag:.17e}\n")
        for i in ridx:
            f.write(f"Fv {i} {Fv[i].real:.17e} {Fv[i].imag:.17e}\n")
            f.write(f"g {i} {g[i].real:.17e} {g[i].imag:.17e}\n")
    print("wrote", out, "oracle iterations to 1e-13:", N.iters, flush=True)


def main():
    which = sys.argv[1:] or ["plain", "per_edge"]
    w = W.refined_disk()
    if "plain" in which:
        write(w, os.path.join(GOLD, "refined_disk_samples.txt"), 4321)
    if "per_edge" in which:
        write(dict(w, l_per_edge=True), os.path.join(GOLD, "refined_disk_per_edge_samples.txt"), 4322)


if __name__ == "__main__":
    main()
