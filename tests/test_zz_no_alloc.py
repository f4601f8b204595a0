"""GPU checks of the allocation-free preconditioner entry point
(hdp_apply_precond_noalloc), called through the C ABI: its result equals
hdp_apply_precond's on the same input, on two calls in a row with the second
smaller (fewer right-hand sides, then a smaller mesh on another handle, so that
the shared scratch array holds the previous call's values), in FP64 and in the
mixed precision, on a conforming mesh and on one with hanging edges; requests
beyond the scratch array's size are refused before any device work."""
import ctypes

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def hdp():
    import paper_1808_04713_amd as m
    return m


def _hanging(base, pvals, seed, l, k=6.0):
    lv = W.refine_where(W.morton_leaves(base, base), 0, 1, 0, 1, base, base,
                        lambda x, y: (x - 0.5) ** 2 + (y - 0.5) ** 2 < 0.05, 2)
    deg = np.random.default_rng(seed).integers(pvals[0], pvals[1] + 1, len(lv))
    return dict(domain=(0.0, 1.0, 0.0, 1.0), base=(base, base), leaves=lv, degree=deg, k=k, l=l,
                bc="impedance", eps_r=np.ones(len(lv)), rhs=dict(kind="plane_wave_total", angles=[0.4]))


def _noalloc(s, v, precision):
    m = hdp()
    u = torch.full_like(v, complex(np.nan, np.nan))
    p = m.HDP_MIXED if precision == "mixed" else m.HDP_FP64
    st = m.load_library().hdp_apply_precond_noalloc(s.h, ctypes.c_void_p(v.data_ptr()),
                                                    ctypes.c_void_p(u.data_ptr()), v.shape[1], p)
    m._check(st)
    torch.cuda.synchronize()
    return u


def _vec(n, R, seed):
    g = torch.Generator().manual_seed(seed)
    v = torch.randn(n, R, dtype=torch.float64, generator=g) + 1j * torch.randn(n, R, dtype=torch.float64, generator=g)
    return v.to(torch.complex128).cuda()


def _rel(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.all(np.isfinite(a))
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-14), ("mixed", 1e-6)])
def test_noalloc_precond_equals_precond_twice_then_smaller(precision, bar):
    m = hdp()
    big = m.Solver(W.small_uniform(8, 8, 20.0), max_rhs=8, max_iter=20)
    small = m.Solver(W.small_uniform(4, 5, 9.0, l=2), max_rhs=1, max_iter=20)
    try:
        for s, R, seed in ((big, 8, 1), (big, 2, 2), (small, 1, 3)):
            print(f"noalloc {precision}: n_lambda {s.n_lambda} R {R}", flush=True)
            v = _vec(s.n_lambda, R, seed)
            ref = s.apply_precond(v, precision=precision)
            out = _noalloc(s, v, precision)
            # same kernels on the same input: equal to rounding (FP32 operators: the
            # same FP32 arithmetic, so the bar is loose only for safety)
            assert _rel(out, ref) <= bar
            if precision == "fp64":
                assert torch.equal(out, ref)
    finally:
        big.close()
        small.close()


def test_noalloc_precond_on_hanging_mesh():
    m = hdp()
    s = m.Solver(_hanging(4, (2, 5), 2, 3), max_rhs=4, max_iter=20)
    try:
        assert s.info["n_lambda"] > 0
        for R, seed in ((4, 5), (1, 6)):
            print(f"noalloc hanging: n_lambda {s.n_lambda} R {R}", flush=True)
            v = _vec(s.n_lambda, R, seed)
            ref = s.apply_precond(v, precision="fp64")
            out = _noalloc(s, v, "fp64")
            assert _rel(out, ref) <= 1e-14
    finally:
        s.close()


def test_noalloc_precond_refuses_requests_beyond_the_scratch_size():
    m = hdp()
    # 32x32 p = 16: 57,344 dual slots; at 64 columns the FP64 slot values alone are
    # 58.7 MB, above the 32 MiB array
    s = m.Solver(W.point_source_32x32(), max_rhs=64, max_iter=2)
    try:
        v = torch.zeros(s.n_lambda, 64, dtype=torch.complex128, device="cuda")
        u = torch.zeros_like(v)
        L = m.load_library()
        st = L.hdp_apply_precond_noalloc(s.h, ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(u.data_ptr()), 64,
                                         m.HDP_FP64)
        assert st == -1
        assert "limit" in L.hdp_last_error_detail().decode()
        assert torch.count_nonzero(u).item() == 0
        # a size that fits still works on the same handle
        v1 = _vec(s.n_lambda, 1, 7)
        assert _rel(_noalloc(s, v1, "fp64"), s.apply_precond(v1, precision="fp64")) <= 1e-14
    finally:
        s.close()
