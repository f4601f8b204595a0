"""Benchmark: Helmholtz DOF/s to a preconditioned relative residual of 1e-8.

Workload (one "step" = one full solve: element loads, interface right-hand
side, GMRES on the interface problem, recovery of the field and its GLL
samples): the 32x32 unit-square mesh, p = 16 on every element, k = 100, point
source at the vertex (0.5, 0.5), impedance boundary, coarse order l from the
dispersion rule (l = 2).  Inputs are synthetic; the mesh and source are
resident before the timed region, which brackets K solves with device
synchronisations.

Both the plain FP64 path and the mixed path (FP32 local operators inside
FP64 GMRES-IR) are timed; `value` is the faster path that reaches 1e-8.  A
second, profiled pass over the same K solves brackets each kernel launch with
HIP events on the solver's stream to give the dominant kernel's average launch
duration and its roofline fraction.  The CPU oracle is timed on a bounded
sample (a 12x12 sub-square with the same h, p and k) on this host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
HBM_FAMILIES = {"coarse_gemv", "coarse_reduce", "coarse_assemble", "row_gather", "gmres_dots", "gmres_update",
                "gmres_norm_scale", "element_coarse_fix", "precision_cast", "hanging_blocks"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "point_source_32x32_hbm_counters.md")


def kernels_digest():
    """Digest of the kernel source; counter figures taken on another source are stale."""
    import hashlib
    with open(os.path.join(ROOT, "paper_1808_04713_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the kernel families recorded in the point-source
    counter summary (FETCH_SIZE + WRITE_SIZE scaled by a plain copy), if that
    summary was taken on the current kernel source; else {}."""
    out, digest = {}, None
    if not os.path.exists(TRAFFIC_FILE):
        return out
    for line in open(TRAFFIC_FILE):
        t = line.split()
        if len(t) == 3 and t[0] == "traffic_per_launch":
            out[t[1]] = float(t[2])
        elif len(t) == 2 and t[0] == "kernels_sha256_16":
            digest = t[1]
    return out if digest == kernels_digest() else {}


def load_samples():
    path = os.path.join(ROOT, "tests", "golden", "point_source_32x32_samples.txt")
    if not os.path.exists(path):
        return None
    idx, vals = [], []
    for line in open(path):
        t = line.split()
        if t and t[0] == "field":
            idx.append(int(t[1]))
            vals.append(float(t[2]) + 1j * float(t[3]))
    return idx, vals


def time_path(hdp, torch, w, precision, steps, warmup, samples):
    import numpy as np
    kind, vals = hdp.rhs_values(w)
    s = hdp.Solver(w, precision=precision, tol=1e-8, max_iter=400)
    field = None
    for _ in range(warmup):
        field, st = s.solve(kind, vals)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        field, st = s.solve(kind, vals)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    err = None
    if samples is not None:
        f = field[0].cpu().numpy()
        idx, ref = samples
        ref = np.asarray(ref)
        err = float(np.linalg.norm(f[idx] - ref) / np.linalg.norm(ref))
    # profiled pass over the same number of solves
    s.profile(True)
    for _ in range(steps):
        s.solve(kind, vals)
    torch.cuda.synchronize()
    kt = s.kernel_times()
    s.profile(False)
    out = dict(ms_per_solve=ms, dof_per_s=s.dof / (ms * 1e-3), iterations=st["iterations"],
               refinements=st["refinements"], rel_residual=st["rel_residual"], converged=st["converged"],
               err_vs_oracle_samples=err, kernels=kt, setup_ms=s.info["setup_ms"])
    info = dict(s.info)
    s.close()
    return out, info


def roofline(kernels, precision, info, name=None):
    """Roofline of the dominant kernel family (or `name`).  The coarse solve is
    credited with the bytes of the method's own coarse factor (a banded LU of K
    in its natural order, from the library's set-up statistics), not with the
    dense inverse this build streams; other families with their algorithmic
    bytes and flops."""
    live = [k for k in kernels if k["launches"] > 0]
    dom = max(live, key=lambda k: k["total_ms"]) if name is None else next(k for k in live if k["name"] == name)
    avg_ms = dom["total_ms"] / dom["launches"]
    bytes_per = dom["bytes"] / dom["launches"]
    flops_per = dom["flops"] / dom["launches"]
    method_bytes = bytes_per
    if dom["name"] == "coarse_gemv":
        method_bytes = info["coarse_band_bytes"] + 32.0 * info["n_coarse"]   # factor + g and w
    ai = flops_per / bytes_per if bytes_per else float("inf")
    peak_tf = FP64_PEAK_TFLOPS if precision == "fp64" else FP32_PEAK_TFLOPS
    ridge = peak_tf * 1e12 / (HBM_PEAK_GBS * 1e9)
    if dom["name"] in HBM_FAMILIES or ai < ridge:
        achieved = method_bytes / (avg_ms * 1e-3) / 1e9
        r = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s")
    else:
        achieved = flops_per / (avg_ms * 1e-3) / 1e12
        r = dict(bound="mfma", achieved=achieved, peak=peak_tf, unit="TFLOP/s")
    traffic = measured_traffic().get(dom["name"])
    r.update(frac=r["achieved"] / r["peak"], traffic=traffic, kernel=dom["name"],
             avg_launch_us=avg_ms * 1e3, launches_per_step=None,
             algorithmic_bytes_per_launch=method_bytes, kernel_bytes_per_launch=bytes_per,
             kernel_stream_frac=bytes_per / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
             algorithmic_flops_per_launch=flops_per,
             share_of_kernel_time=dom["total_ms"] / sum(k["total_ms"] for k in live))
    return r


def batched_scatterer(hdp, torch, steps, warmup):
    """The 64-angle dielectric-square workload (64x64 elements on [-1,1]^2, p=12,
    k=150, eps_r=4 on [-1/4,1/4]^2, scattered-field formulation, 360 far-field
    angles): the plain FP64 path with one right-hand side per call (timed on a
    sample of angles and scaled to 64) against the FP64 and mixed paths with all
    64 angles in one batched solve."""
    import numpy as np
    import workloads as W
    w = W.square_scatterer_64x64()
    ang = np.asarray(w["rhs"]["angles"])
    fa = np.asarray(w["far_angles"])
    inside = np.asarray(w["eps_r"]) != 1.0
    out = {}
    fars = {}
    # the one-angle-per-call baseline on a handle set up for one column (its own
    # coarse ordering and sweeps), as a caller solving angle by angle would use
    s1 = hdp.Solver(w, precision="fp64", tol=1e-8, max_iter=300, max_rhs=1)
    n1 = 4
    for _ in range(max(1, warmup)):
        s1.solve("plane_wave_scattered", ang[:1], want_field=False, far_angles=fa, far_inside=inside)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a in ang[:n1]:
        _, _, st1 = s1.solve("plane_wave_scattered", [a], want_field=False, far_angles=fa, far_inside=inside)
    torch.cuda.synchronize()
    ms1 = (time.perf_counter() - t0) * 1e3 / n1
    out["fp64_one_rhs_per_call"] = dict(ms_per_rhs=ms1, ms_for_64=ms1 * len(ang), iterations=st1["iterations"],
                                        sample=f"{n1} of the 64 angles, one per call (handle for one column), "
                                               "scaled to 64")
    s1.close()
    for prec in ("fp64", "mixed"):
        s = hdp.Solver(w, precision=prec, tol=1e-8, max_iter=300, max_rhs=len(ang), autotune=True)
        for _ in range(warmup):
            s.solve("plane_wave_scattered", ang, want_field=False, far_angles=fa, far_inside=inside)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, far, st = s.solve("plane_wave_scattered", ang, want_field=False, far_angles=fa, far_inside=inside)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        fars[prec] = far.cpu().numpy()
        out[prec + "_batched_64"] = dict(ms_per_solve=ms, dof_per_s=s.dof * len(ang) / (ms * 1e-3),
                                         iterations=st["iterations"], refinements=st["refinements"],
                                         converged=st["converged"], rhs_ms=st["rhs_ms"], gmres_ms=st["gmres_ms"],
                                         recover_ms=st["recover_ms"], setup_ms=s.info["setup_ms"],
                                         autotune=s.autotune_table())
        # one profiled solve: per-family HIP-event times, algorithmic bytes and flops
        s.profile(True)
        s.solve("plane_wave_scattered", ang, want_field=False, far_angles=fa, far_inside=inside)
        torch.cuda.synchronize()
        kt = [k for k in s.kernel_times() if k["launches"]]
        s.profile(False)
        peak = FP64_PEAK_TFLOPS * 1e12
        fams = {}
        for k in kt:
            sec = k["total_ms"] * 1e-3
            fams[k["name"]] = dict(launches=k["launches"], ms=k["total_ms"],
                                   tflops=k["flops"] / sec / 1e12 if sec else None,
                                   gbs=k["bytes"] / sec / 1e9 if sec else None,
                                   mfma_frac_fp64=k["flops"] / sec / peak if sec else None,
                                   hbm_frac=k["bytes"] / sec / (HBM_PEAK_GBS * 1e9) if sec else None)
        out[prec + "_batched_64"]["kernels"] = fams
        out["dof"] = s.dof
        out["l"] = s.info["l"]
        out["n_lambda"] = s.info["n_lambda"]
        out["n_coarse"] = s.info["n_coarse"]
        s.close()
        print(f"bench: batched scatterer {prec} done ({ms:.1f} ms per 64-angle solve)", file=sys.stderr, flush=True)
    a, b = fars["mixed"], fars["fp64"]
    out["far_field_rel_diff_mixed_vs_fp64"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out["speedup_mixed_batched_vs_fp64_one_rhs_per_call"] = (
        out["fp64_one_rhs_per_call"]["ms_for_64"] / out["mixed_batched_64"]["ms_per_solve"])
    out["speedup_fp64_batched_vs_fp64_one_rhs_per_call"] = (
        out["fp64_one_rhs_per_call"]["ms_for_64"] / out["fp64_batched_64"]["ms_per_solve"])
    out["workload"] = "square_scatterer_64x64_p12_k150_eps4_64angles_360far"
    return out


def refined_disk(hdp, torch, steps, warmup):
    """The non-conforming workload: [-1,1]^2 from a 16x16 base, leaves with centre
    in r < 0.4 split twice (up to three hanging nodes per edge), p ~ U{8..24},
    k = 200, eps_r = 2.25 in the disk, one plane wave, FP64 and mixed paths."""
    import workloads as W
    w = W.refined_disk()
    out = {"workload": "refined_disk_16x16_2levels_p8to24_k200", "discard_tol": w["discard_tol"]}
    for prec in ("fp64", "mixed"):
        s = hdp.Solver(w, precision=prec, tol=1e-8, max_iter=400)
        for _ in range(max(1, warmup)):
            s.solve("plane_wave_scattered", [0.0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st = s.solve("plane_wave_scattered", [0.0])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        out[prec] = dict(ms_per_solve=ms, dof_per_s=s.dof / (ms * 1e-3), iterations=st["iterations"],
                         refinements=st["refinements"], rel_residual=st["rel_residual"],
                         true_residual=st["true_residual"], converged=st["converged"], setup_ms=s.info["setup_ms"],
                         setup_host_ms=s.info["setup_host_ms"], setup_classes_ms=s.info["setup_classes_ms"],
                         setup_coarse_ms=s.info["setup_coarse_ms"])
        out.update(dof=s.dof, elements=s.info["n_elements"], l=s.info["l"], n_lambda=s.info["n_lambda"],
                   n_coarse=s.info["n_coarse"], classes=s.info["n_classes"])
        s.close()
        print(f"bench: refined disk {prec} done ({ms:.1f} ms per solve)", file=sys.stderr, flush=True)
    # the per-edge coarse order (smaller coarse space on the refined part), FP64
    s = hdp.Solver(dict(w, l_per_edge=True), tol=1e-8, max_iter=600)
    for _ in range(max(1, warmup)):
        s.solve("plane_wave_scattered", [0.0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = s.solve("plane_wave_scattered", [0.0])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    out["fp64_per_edge_l"] = dict(ms_per_solve=ms, dof_per_s=s.dof / (ms * 1e-3), iterations=st["iterations"],
                                  true_residual=st["true_residual"], converged=st["converged"],
                                  setup_ms=s.info["setup_ms"], n_lambda=s.info["n_lambda"],
                                  n_coarse=s.info["n_coarse"], l_max=s.info["l"])
    s.close()
    print(f"bench: refined disk per-edge l done ({ms:.1f} ms per solve)", file=sys.stderr, flush=True)
    return out


def design_gradient(hdp, torch, steps, warmup):
    """The 64x64 design block (p = 12, k = 150, eps_r ~ U[1,4] on the central 16x16
    elements): J = |E_far(0)|^2 for normal incidence and dJ/d eps_r for all 4096
    elements by one forward and one adjoint solve."""
    import numpy as np
    import workloads as W
    w = W.design_block_64x64()
    c = W.leaf_centres(w)
    he = 2.0 / 64
    inside = (np.abs(c[:, 0]) < 8 * he) & (np.abs(c[:, 1]) < 8 * he)
    s = hdp.Solver(w, tol=1e-8, max_iter=300)
    for _ in range(max(1, warmup)):
        s.far_intensity_gradient(0.0, 0.0, inside)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        J, g, st = s.far_intensity_gradient(0.0, 0.0, inside)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    out = dict(workload="design_block_64x64_p12_k150_16x16_design", ms_forward_adjoint_gradient=ms, J=J,
               parameters=int(inside.sum()), iterations_forward=st["iterations"], setup_ms=s.info["setup_ms"],
               classes=s.info["n_classes"], converged=st["converged"])
    s.close()
    print(f"bench: design gradient done ({ms:.1f} ms for J and 4096 derivatives)", file=sys.stderr, flush=True)
    return out


def robin_modified(hdp, torch, steps, warmup):
    """The point-source workload with Robin-modified local problems (gamma = +-ik
    on the interior sides between elements of opposite label): same field, a
    different interface problem; FP64 path, against the unmodified solve."""
    import numpy as np
    import workloads as W
    w = W.point_source_32x32()
    out = {"workload": "point_source_32x32_p16_k100_robin_modified"}
    fields = {}
    for mod in (False, True):
        s = hdp.Solver(dict(w, robin_modified=mod), tol=1e-8, max_iter=600)
        for _ in range(max(1, warmup)):
            s.solve("point", [(0.5, 0.5)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            f, st = s.solve("point", [(0.5, 0.5)])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        fields[mod] = f.cpu().numpy()[0]
        out["modified" if mod else "unmodified"] = dict(
            ms_per_solve=ms, dof_per_s=s.dof / (ms * 1e-3), iterations=st["iterations"],
            true_residual=st["true_residual"], converged=st["converged"], setup_ms=s.info["setup_ms"],
            classes=s.info["n_classes"])
        s.close()
    out["field_rel_diff"] = float(np.linalg.norm(fields[True] - fields[False]) / np.linalg.norm(fields[False]))
    print(f"bench: robin-modified point source done ({out['modified']['ms_per_solve']:.1f} ms per solve)",
          file=sys.stderr, flush=True)
    return out


def pml_scatterer(hdp, torch, steps, warmup):
    """The square scatterer inside 8 rings of perfectly matched layers (80x80
    elements, p = 12, k = 150, normal incidence, 360 far-field angles), FP64 path,
    beside the same scatterer truncated by the impedance condition alone."""
    import numpy as np
    import workloads as W
    out = {"workload": "pml_scatterer_64x64_p12_k150_8layers"}
    fars = {}
    for name, w in (("layers", W.pml_scatterer_64x64()), ("impedance_only", W.square_scatterer_64x64(1))):
        fa = np.asarray(w["far_angles"])
        inside = np.asarray(w["eps_r"]) != 1.0
        s = hdp.Solver(w, tol=1e-8, max_iter=400)
        for _ in range(max(1, warmup)):
            s.solve("plane_wave_scattered", [0.0], want_field=False, far_angles=fa, far_inside=inside)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, far, st = s.solve("plane_wave_scattered", [0.0], want_field=False, far_angles=fa, far_inside=inside)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        fars[name] = far.cpu().numpy()[0]
        out[name] = dict(ms_per_solve=ms, dof_per_s=s.dof / (ms * 1e-3), dof=s.dof, iterations=st["iterations"],
                         true_residual=st["true_residual"], converged=st["converged"], setup_ms=s.info["setup_ms"],
                         classes=s.info["n_classes"], n_coarse=s.info["n_coarse"])
        s.close()
    a, b = fars["layers"], fars["impedance_only"]
    out["far_field_rel_diff_layers_vs_impedance_only"] = float(np.linalg.norm(a - b) / np.linalg.norm(a))
    print(f"bench: layered scatterer done ({out['layers']['ms_per_solve']:.1f} ms per solve)", file=sys.stderr,
          flush=True)
    return out


def cpu_baseline():
    """The oracle as it stands on a bounded sample of the same workload."""
    import numpy as np
    import workloads as W
    from oracle import dp_elementwise as dpe, problem as pb
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    n = 12
    h = 1.0 / 32
    w = W.small_uniform(n, 16, 100.0, domain=(0.0, n * h, 0.0, n * h),
                        rhs=dict(kind="point", points=[(n * h / 2, n * h / 2)]))
    t0 = time.perf_counter()
    disc = pb.Discretisation(w)
    E = dpe.ElementwiseDP(disc, pb.coarse_order(w, disc.mesh))
    E.solve(tol=1e-8, max_iter=400)
    t = time.perf_counter() - t0
    dof = n * n * 17 * 17
    return dict(value=dof / t, unit="DOF/s", cores=int(threads), kind="oracle",
                sample=f"12x12 sub-square of the 32x32 mesh (h=1/32, p=16, k=100, point source at its "
                       f"centre vertex, l=2): {dof} DOF, oracle setup+solve to 1e-8 in {t:.1f} s, "
                       f"{E.iters} iterations, host cpu_count={os.cpu_count()}")


def cpu_baseline_full():
    """The oracle on whole workloads (not part of the default run): the 4x4
    plane wave, the 32x32 point source and the refined disk (the quadtree
    element-wise oracle), set-up and solve to 1e-8 timed separately, on this
    host's cores."""
    import workloads as W
    from oracle import dp_elementwise as dpe, dp_nonconforming as dnc, problem as pb
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    out = {"cores": int(threads), "cpu_count": os.cpu_count(), "kind": "oracle"}
    for name, w in (("plane_wave_4x4", W.plane_wave_4x4()), ("point_source_32x32", W.point_source_32x32()),
                    ("refined_disk", W.refined_disk())):
        t0 = time.perf_counter()
        disc = pb.Discretisation(w)
        oracle = dnc.NonconformingDP if name == "refined_disk" else dpe.ElementwiseDP
        E = oracle(disc, pb.coarse_order(w, disc.mesh))
        t1 = time.perf_counter()
        E.solve(tol=1e-8, max_iter=400)
        t2 = time.perf_counter()
        dof = int(sum((int(p) + 1) ** 2 for p in w["degree"]))
        out[name] = dict(dof=dof, setup_s=t1 - t0, solve_s=t2 - t1, iterations=E.iters,
                         dof_per_s_solve=dof / (t2 - t1), dof_per_s_setup_and_solve=dof / (t2 - t0))
        print(f"bench: oracle {name} done ({t2 - t0:.1f} s)", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the refined-disk and 64-angle batched scatterer measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy three times (HBM counter calibration)")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="only time the oracle on the whole 4x4 and 32x32 workloads (minutes) and print the record")
    ap.add_argument("--only", choices=["refined_disk", "scatterer", "design", "robin", "pml"],
                    help="profiling aid: run only this secondary workload and print its record")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 512 * 1024 * 1024 // 16
        a = torch.ones(n, dtype=torch.complex128, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": 16 * n, "copy_bytes_written_per_launch": 16 * n,
                          "launches": 3}), flush=True)
        return
    if args.cpu_baseline_full:
        print(json.dumps(cpu_baseline_full()), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the multi-GPU path is not part of this build "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1808_04713_amd as hdp
    import workloads as W
    if args.only:
        fn = {"refined_disk": refined_disk, "scatterer": batched_scatterer, "design": design_gradient,
              "robin": robin_modified, "pml": pml_scatterer}[args.only]
        print(json.dumps(fn(hdp, torch, max(1, args.steps), args.warmup)), flush=True)
        return
    w = W.point_source_32x32()
    samples = load_samples()
    fp64, info = time_path(hdp, torch, w, "fp64", args.steps, args.warmup, samples)
    print(f"bench: point source fp64 done ({fp64['ms_per_solve']:.2f} ms per solve)", file=sys.stderr, flush=True)
    mixed, _ = time_path(hdp, torch, w, "mixed", args.steps, args.warmup, samples)
    print(f"bench: point source mixed done ({mixed['ms_per_solve']:.2f} ms per solve)", file=sys.stderr, flush=True)
    best_name, best = ("mixed", mixed) if (mixed["converged"] and mixed["ms_per_solve"] < fp64["ms_per_solve"]) \
        else ("fp64", fp64)
    line = {
        "metric": "Helmholtz DOF/s to rel.res 1e-8",
        "value": best["dof_per_s"],
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if best_name == "fp64" else "c64 local / c128 outer",
        "data": "synthetic",
        "config": {"workload": "point_source_32x32_p16_k100", "elements": info["n_elements"], "p": 16,
                   "k": 100.0, "l": info["l"], "dof": info["dof"], "n_lambda": info["n_lambda"],
                   "n_coarse": info["n_coarse"], "n_rhs": 1, "tol": 1e-8, "path": best_name},
        "mixed_vs_fp64_speedup": fp64["ms_per_solve"] / mixed["ms_per_solve"],
        "paths": {k: {kk: vv for kk, vv in v.items() if kk != "kernels"} for k, v in
                  (("fp64", fp64), ("mixed", mixed))},
        "roofline": roofline(best["kernels"], best_name, info),
        "roofline_krylov": {k: roofline(best["kernels"], best_name, info, k) for k in ("gmres_dots", "gmres_update")},
        "kernels": sorted([k for k in best["kernels"] if k["launches"]], key=lambda k: -k["total_ms"]),
    }
    for r in [line["roofline"]] + list(line["roofline_krylov"].values()):
        r["launches_per_step"] = next(k["launches"] for k in best["kernels"] if k["name"] == r["kernel"]) / args.steps
    # at one right-hand side the working set stays in the Infinity Cache and every
    # kernel is latency-bound: the wall time per GMRES iteration states that bound
    line["roofline"]["iteration_us"] = best["ms_per_solve"] * 1e3 / max(1, best["iterations"])
    if not args.no_batched:
        line["nonconforming"] = refined_disk(hdp, torch, max(1, min(args.steps, 5)), min(args.warmup, 1))
        line["adjoint_gradient"] = design_gradient(hdp, torch, max(1, min(args.steps, 5)), min(args.warmup, 1))
        line["robin_modified"] = robin_modified(hdp, torch, max(1, min(args.steps, 3)), min(args.warmup, 1))
        line["pml_scatterer"] = pml_scatterer(hdp, torch, max(1, min(args.steps, 3)), min(args.warmup, 1))
        line["batched_rhs"] = batched_scatterer(hdp, torch, max(1, min(args.steps, 3)), min(args.warmup, 1))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
