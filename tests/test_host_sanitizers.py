"""The host set-up code (setup.cpp, coarse_nd.cpp: side analysis, classes,
Algorithm 1, coarse maps and assembly, nested-dissection ordering and factor)
built with AddressSanitizer and UndefinedBehaviorSanitizer for the host only
(no device code is involved) and run on meshes with hanging edges, uneven
degrees, discarded constraints and per-edge coarse orders, up to the full
refined disk.  Any sanitizer report fails the run (exit status non-zero); the
sizes it prints equal those of the library's own host analysis."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("san") / "sanitize_host")
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
           "-fsanitize=undefined", "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "sanitize_host.cpp"),
           os.path.join(ROOT, "paper_1808_04713_amd", "csrc", "setup.cpp"),
           os.path.join(ROOT, "paper_1808_04713_amd", "csrc", "coarse_nd.cpp"), "-o", exe, "-pthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def _run(exe, w, per_edge=False):
    lv = np.asarray(w["leaves"]).reshape(-1, 3)
    deg = np.asarray(w["degree"])
    eps = np.asarray(w.get("eps_r", np.ones(len(deg))))
    x0, x1, y0, y1 = w["domain"]
    def g(v):
        return f"{float(v):.17g}"
    text = (f"{g(x0)} {g(x1)} {g(y0)} {g(y1)} {int(w['base'][0])} {int(w['base'][1])} {len(deg)} {g(w['k'])} "
            f"{int(w.get('l', -1))} {g(w.get('discard_tol', 0.0))} {int(per_edge)}\n")
    text += "\n".join(f"{int(a)} {int(b)} {int(c)} {int(d)} {g(e)}" for (a, b, c), d, e in zip(lv, deg, eps)) + "\n"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    t = r.stdout.split()
    return dict(n_lambda=int(t[1]), n_coarse=int(t[3]))


def _hanging(base, pvals, seed, l, k=6.0, tau=0.0):
    lv = W.refine_where(W.morton_leaves(base, base), 0, 1, 0, 1, base, base,
                        lambda x, y: (x - 0.5) ** 2 + (y - 0.5) ** 2 < (0.03 if base % 2 else 0.05), 2)
    deg = np.random.default_rng(seed).integers(pvals[0], pvals[1] + 1, len(lv))
    return dict(domain=(0.0, 1.0, 0.0, 1.0), base=(base, base), leaves=lv, degree=deg, k=k, l=l,
                bc="impedance", eps_r=np.ones(len(lv)), discard_tol=tau)


@pytest.mark.parametrize("args,per_edge", [((3, (4, 4), 0, 1), False), ((3, (3, 6), 1, 2), False),
                                           ((4, (2, 5), 2, 3), False), ((3, (3, 7), 3, 7), False),
                                           ((3, (3, 6), 1, 2, 6.0, 1e-2), False), ((4, (3, 7), 4, -1, 30.0), True)])
def test_hanging_meshes_run_clean(checker, args, per_edge):
    import paper_1808_04713_amd as hdp
    w = _hanging(*args)
    got = _run(checker, w, per_edge)
    st = hdp.inspect(dict(w, l_per_edge=per_edge))
    assert (got["n_lambda"], got["n_coarse"]) == (st["n_lambda"], st["n_coarse"])


def test_full_refined_disk_runs_clean(checker):
    import paper_1808_04713_amd as hdp
    w = W.refined_disk()
    got = _run(checker, w)
    st = hdp.inspect(w)
    assert (got["n_lambda"], got["n_coarse"]) == (st["n_lambda"], st["n_coarse"])
