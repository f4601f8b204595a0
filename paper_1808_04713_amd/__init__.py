"""Python binding of libhdp, the MI355X dual-primal spectral-element Helmholtz
solver (Galagusz & McFee, arXiv:1808.04713).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides device memory and the current stream.  Importing this module
does not need a GPU; creating a Solver does, and it fails loudly when the
library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdp.so")

HDP_FP64, HDP_MIXED = 0, 1
RHS_KINDS = {"plane_wave_total": 0, "point": 1, "plane_wave_scattered": 2, "element_loads": 3}
STATUS_OK, STATUS_NOT_CONVERGED, STATUS_TRUE_RESIDUAL = 0, 1, 2


class HdpError(RuntimeError):
    def __init__(self, status, detail):
        super().__init__(f"hdp status {status}: {detail}")
        self.status = status


class _Mesh(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double), ("base_nx", ctypes.c_int32), ("base_ny", ctypes.c_int32),
                ("n_leaves", ctypes.c_int32), ("leaf", ctypes.POINTER(ctypes.c_int32)),
                ("degree", ctypes.POINTER(ctypes.c_int32))]


class _Problem(ctypes.Structure):
    _fields_ = [("k", ctypes.c_double), ("eps_r", ctypes.POINTER(ctypes.c_double)),
                ("l", ctypes.c_int32), ("l_safety", ctypes.c_int32), ("discard_tol", ctypes.c_double),
                ("robin_modified", ctypes.c_int32), ("pml_sigma", ctypes.POINTER(ctypes.c_double)),
                ("l_per_edge", ctypes.c_int32), ("l_free_space", ctypes.c_int32)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("max_rhs", ctypes.c_int32), ("stream", ctypes.c_void_p), ("flags", ctypes.c_int32),
                ("tile_fdm", ctypes.c_int32), ("tile_slot", ctypes.c_int32), ("allocator", _Allocator)]


class _Rhs(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_rhs", ctypes.c_int32),
                ("angles", ctypes.POINTER(ctypes.c_double)), ("points", ctypes.POINTER(ctypes.c_double)),
                ("loads", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("dof", ctypes.c_int64), ("n_elements", ctypes.c_int32), ("n_lambda", ctypes.c_int32),
                ("n_coarse", ctypes.c_int32), ("l", ctypes.c_int32), ("n_classes", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("min_element_margin", ctypes.c_double),
                ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double), ("rhs_ms", ctypes.c_double),
                ("gmres_ms", ctypes.c_double), ("gmres_launch_ms", ctypes.c_double),
                ("gmres_wait_ms", ctypes.c_double), ("recover_ms", ctypes.c_double),
                ("true_residual", ctypes.c_double), ("coarse_residual", ctypes.c_double),
                ("coarse_mode", ctypes.c_int32), ("coarse_blocks", ctypes.c_int32),
                ("coarse_factor_bytes", ctypes.c_double), ("coarse_band_bytes", ctypes.c_double),
                ("setup_host_ms", ctypes.c_double), ("setup_classes_ms", ctypes.c_double),
                ("setup_coarse_ms", ctypes.c_double), ("coarse_top_unknowns", ctypes.c_int32),
                ("coarse_top_check", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TuneEntry(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_char * 32), ("cols", ctypes.c_int32), ("chosen", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


EXPORTS = ["hdp_inspect", "hdp_setup", "hdp_solve", "hdp_apply_interface", "hdp_apply_precond",
           "hdp_apply_precond_noalloc",
           "hdp_interface_rhs", "hdp_local_solve", "hdp_get_stats", "hdp_profile", "hdp_profile_read",
           "hdp_residual_history", "hdp_far_intensity_gradient", "hdp_autotune_table",
           "hdp_destroy", "hdp_status_string", "hdp_last_error_detail"]

_lib = None


def load_library():
    """Load libhdp.so (no GPU needed) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
    L.hdp_setup.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Problem), ctypes.POINTER(_Options),
                            ctypes.POINTER(vp)]
    L.hdp_solve.argtypes = [vp, ctypes.POINTER(_Rhs), vp, i32, dp, ctypes.POINTER(ctypes.c_uint8), vp,
                            ctypes.POINTER(Stats)]
    L.hdp_apply_interface.argtypes = [vp, vp, vp, i32, i32]
    L.hdp_apply_precond.argtypes = [vp, vp, vp, i32, i32]
    L.hdp_apply_precond_noalloc.argtypes = [vp, vp, vp, i32, i32]
    L.hdp_interface_rhs.argtypes = [vp, ctypes.POINTER(_Rhs), vp]
    L.hdp_local_solve.argtypes = [vp, vp, vp, i32]
    L.hdp_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.hdp_inspect.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Problem), ctypes.POINTER(Stats)]
    L.hdp_profile.argtypes = [vp, i32]
    L.hdp_residual_history.argtypes = [vp, i32, dp, i32, ctypes.POINTER(i32)]
    L.hdp_profile_read.argtypes = [vp, ctypes.POINTER(KernelTime), i32, ctypes.POINTER(i32)]
    L.hdp_far_intensity_gradient.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_uint8),
                                             dp, dp, ctypes.POINTER(Stats)]
    L.hdp_autotune_table.argtypes = [vp, ctypes.POINTER(TuneEntry), i32, ctypes.POINTER(i32)]
    L.hdp_destroy.argtypes = [vp]
    L.hdp_destroy.restype = None
    L.hdp_status_string.restype = ctypes.c_char_p
    L.hdp_last_error_detail.restype = ctypes.c_char_p
    for name in ("hdp_inspect", "hdp_setup", "hdp_solve", "hdp_apply_interface", "hdp_apply_precond",
                 "hdp_apply_precond_noalloc", "hdp_interface_rhs", "hdp_local_solve", "hdp_get_stats", "hdp_profile", "hdp_profile_read",
                 "hdp_residual_history", "hdp_far_intensity_gradient", "hdp_autotune_table"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status, allow_not_converged=False):
    if status == STATUS_OK or (allow_not_converged and status in (STATUS_NOT_CONVERGED, STATUS_TRUE_RESIDUAL)):
        return status
    L = load_library()
    raise HdpError(status, L.hdp_last_error_detail().decode())


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def check_operand(t, rows, max_cols, device, what):
    """Validate a tensor passed to the library as [rows][n_rhs] complex128
    memory of the handle's device (the library reads rows * n_rhs values
    through the raw pointer); returns it contiguous."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != torch.complex128:
        raise ValueError(f"{what}: dtype must be complex128, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{what}: tensor on {t.device}, the solver's device is {device}")
    if t.ndim != 2 or t.shape[0] != rows:
        raise ValueError(f"{what}: shape must be ({rows}, n_rhs), got {tuple(t.shape)}")
    if not 1 <= t.shape[1] <= max_cols:
        raise ValueError(f"{what}: n_rhs = {t.shape[1]} outside 1..{max_cols}")
    return t.contiguous()


def _pow2ceil(x):
    p = 1
    while p < x:
        p <<= 1
    return p


def _structs(w, l_safety=0):
    leaves = np.ascontiguousarray(np.asarray(w["leaves"], dtype=np.int32).reshape(-1, 3))
    deg = np.ascontiguousarray(np.asarray(w["degree"], dtype=np.int32))
    eps = np.ascontiguousarray(np.asarray(w.get("eps_r", np.ones(len(deg))), dtype=np.float64))
    x0, x1, y0, y1 = w["domain"]
    mesh = _Mesh(x0, x1, y0, y1, int(w["base"][0]), int(w["base"][1]), len(deg),
                 leaves.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                 deg.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    sig = None
    if w.get("pml_sigma") is not None:
        sig = np.ascontiguousarray(np.asarray(w["pml_sigma"], dtype=np.float64).reshape(len(deg), 2))
    prob = _Problem(float(w["k"]), eps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    int(w.get("l", -1)), int(l_safety), float(w.get("discard_tol", 0.0)),
                    int(bool(w.get("robin_modified", False))),
                    sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if sig is not None else None,
                    int(bool(w.get("l_per_edge", False))), int(bool(w.get("l_free_space", False))))
    return mesh, prob, (leaves, deg, eps, sig)


def inspect(w, l_safety=0):
    """Host-only analysis (no GPU): sizes, l, classes, smallest solver margin."""
    L = load_library()
    mesh, prob, keep = _structs(w, l_safety)
    st = Stats()
    _check(L.hdp_inspect(ctypes.byref(mesh), ctypes.byref(prob), ctypes.byref(st)))
    return st.as_dict()


class Solver:
    """setup(mesh, degrees, k, coefficients, constraint set) -> solve(rhs) -> field.

    mesh: dict with domain (x0,x1,y0,y1), base (nx,ny), leaves [(level,ix,iy)],
    degree (per leaf), k, eps_r (per leaf) and l (<= 0: dispersion rule).
    """

    def __init__(self, w, precision="fp64", tol=1e-8, max_iter=300, max_rhs=1, l_safety=0, device=0,
                 graphs=False, coarse="auto", autotune=False, tile_fdm=0, tile_slot=0, torch_memory=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("hdp needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.torch = torch
        self.device = torch.device("cuda", device)
        L = load_library()
        mesh, prob, self._keep = _structs(w, l_safety)
        self.precision = HDP_MIXED if precision == "mixed" else HDP_FP64
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            flags = ((1 if graphs else 0) | {"auto": 0, "dense": 4, "nd": 8}[coarse]
                     | (16 if autotune else 0))
            alloc = _Allocator()
            if torch_memory:
                # the handle's device memory from torch's caching allocator (on the
                # caller's stream, which the solver orders after)
                dev = self.device

                def _alloc(nbytes, ctx):
                    try:
                        return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev,
                                                                  stream=torch.cuda.current_stream(dev))
                    except Exception:
                        return None

                def _free(p, ctx):
                    torch.cuda.caching_allocator_delete(p)

                self._allocator_fns = (_ALLOC_FN(_alloc), _FREE_FN(_free))   # alive until close()
                alloc = _Allocator(self._allocator_fns[0], self._allocator_fns[1], None)
            opt = _Options(self.precision, float(tol), int(max_iter), int(max_rhs), ctypes.c_void_p(stream), flags,
                           int(tile_fdm), int(tile_slot), alloc)
            h = ctypes.c_void_p()
            _check(L.hdp_setup(ctypes.byref(mesh), ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(h)))
        self.h = h
        self.max_rhs = max_rhs
        st = Stats()
        _check(L.hdp_get_stats(self.h, ctypes.byref(st)))
        self.info = st.as_dict()
        self.dof, self.n_lambda, self.n_coarse = st.dof, st.n_lambda, st.n_coarse

    def close(self):
        if getattr(self, "h", None):
            load_library().hdp_destroy(self.h)
            self.h = None
        self._allocator_fns = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _rhs(self, kind, values):
        if kind == "element_loads":
            # values: (dof, n_rhs) complex128 device tensor of element load vectors
            loads = check_operand(values, self.dof, self.max_rhs, self.device, "element loads")
            r = _Rhs(RHS_KINDS[kind], loads.shape[1], None, None, ctypes.c_void_p(loads.data_ptr()))
            return r, loads, loads.shape[1]
        vals = np.ascontiguousarray(np.asarray(values, dtype=np.float64))
        n = len(vals) if RHS_KINDS[kind] != 1 else len(vals.reshape(-1, 2))
        r = _Rhs(RHS_KINDS[kind], n, None, None, None)
        ptr = vals.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if kind == "point":
            r.points = ptr
        else:
            r.angles = ptr
        return r, vals, n

    def solve(self, kind, values, want_field=True, far_angles=None, far_inside=None):
        """Returns (field, stats) or, with far_angles, (field, far, stats).

        field: (n_rhs, dof) complex128 GLL-node values (element blocks in leaf
        order, x fastest) or None; far: (n_rhs, n_far) far-field amplitudes
        E_far over the boundary of the leaves with far_inside != 0."""
        torch = self.torch
        r, keep, n = self._rhs(kind, values)
        field = torch.empty((n, self.dof), dtype=torch.complex128, device=self.device) if want_field else None
        far = None
        fa = fi = None
        nfar = 0
        if far_angles is not None:
            fa = np.ascontiguousarray(np.asarray(far_angles, dtype=np.float64))
            fi = np.ascontiguousarray(np.asarray(far_inside, dtype=np.uint8))
            nfar = len(fa)
            far = torch.empty((n, nfar), dtype=torch.complex128, device=self.device)
        st = Stats()
        status = load_library().hdp_solve(
            self.h, ctypes.byref(r), _dptr(field) if want_field else None, nfar,
            fa.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if fa is not None else None,
            fi.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if fi is not None else None,
            _dptr(far) if far is not None else None, ctypes.byref(st))
        _check(status, allow_not_converged=True)
        d = st.as_dict()
        d["converged"] = status == STATUS_OK
        d["status"] = status
        if far_angles is not None:
            return field, far, d
        return field, d

    def far_intensity_gradient(self, incidence, far_angle, far_inside):
        """J = |E_far(far_angle)|^2 for the scattered field of the plane wave with
        propagation angle `incidence`, and dJ/d eps_r per leaf (adjoint solve)."""
        fi = np.ascontiguousarray(np.asarray(far_inside, dtype=np.uint8))
        grad = np.zeros(self.info["n_elements"])
        J = ctypes.c_double()
        st = Stats()
        status = load_library().hdp_far_intensity_gradient(
            self.h, float(incidence), float(far_angle), fi.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
            ctypes.byref(J), grad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(st))
        _check(status, allow_not_converged=True)
        d = st.as_dict()
        d["converged"] = status == STATUS_OK
        d["status"] = status
        return J.value, grad, d

    def apply_interface(self, v, precision=None):
        """u = F v; v is a (n_lambda, n_rhs) complex128 device tensor."""
        v = check_operand(v, self.n_lambda, _pow2ceil(self.max_rhs), self.device, "v")
        u = self.torch.empty_like(v)
        p = self.precision if precision is None else (HDP_MIXED if precision == "mixed" else HDP_FP64)
        _check(load_library().hdp_apply_interface(self.h, _dptr(v), _dptr(u), v.shape[1], p))
        return u

    def apply_precond(self, v, precision=None):
        """u = P^-1 v; v is a (n_lambda, n_rhs) complex128 device tensor."""
        v = check_operand(v, self.n_lambda, _pow2ceil(self.max_rhs), self.device, "v")
        u = self.torch.empty_like(v)
        p = self.precision if precision is None else (HDP_MIXED if precision == "mixed" else HDP_FP64)
        _check(load_library().hdp_apply_precond(self.h, _dptr(v), _dptr(u), v.shape[1], p))
        return u

    def interface_rhs(self, kind, values):
        r, keep, n = self._rhs(kind, values)
        g = self.torch.empty((self.n_lambda, n), dtype=self.torch.complex128, device=self.device)
        _check(load_library().hdp_interface_rhs(self.h, ctypes.byref(r), _dptr(g)))
        return g

    def residual_history(self, rhs=0):
        """Preconditioned relative residual after each iteration of the last GMRES run."""
        L = load_library()
        n = ctypes.c_int32()
        _check(L.hdp_residual_history(self.h, rhs, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value)
        _check(L.hdp_residual_history(self.h, rhs, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      n.value, ctypes.byref(n)))
        return out

    def profile(self, enable=True):
        """Bracket every kernel launch family with HIP events (enable clears totals)."""
        _check(load_library().hdp_profile(self.h, 1 if enable else 0))

    def kernel_times(self):
        """Per launch family: launches, summed event ms, algorithmic bytes and flops."""
        L = load_library()
        buf = (KernelTime * 64)()
        n = ctypes.c_int32()
        _check(L.hdp_profile_read(self.h, buf, 64, ctypes.byref(n)))
        return [dict(name=buf[i].name.decode(), launches=buf[i].launches, total_ms=buf[i].total_ms,
                     bytes=buf[i].bytes, flops=buf[i].flops) for i in range(n.value)]

    def autotune_table(self):
        """The set-up autotuner's measurements: kernel, columns per workgroup, ms, chosen."""
        L = load_library()
        buf = (TuneEntry * 64)()
        n = ctypes.c_int32()
        _check(L.hdp_autotune_table(self.h, buf, 64, ctypes.byref(n)))
        return [dict(kernel=buf[i].kernel.decode(), cols=buf[i].cols, ms=buf[i].ms, chosen=bool(buf[i].chosen))
                for i in range(n.value)]

    def local_solve(self, y):
        """x_e = A_e^-1 y_e by the separable fast solver; y is (dof, n_rhs)."""
        y = check_operand(y, self.dof, 1 << 20, self.device, "y")
        x = self.torch.empty_like(y)
        _check(load_library().hdp_local_solve(self.h, _dptr(y), _dptr(x), y.shape[1]))
        return x


def rhs_values(w):
    """(kind, values) of a workload's right-hand side."""
    rhs = w["rhs"]
    if rhs["kind"] == "point":
        return "point", np.asarray(rhs["points"], float).reshape(-1)
    return rhs["kind"], np.asarray(rhs["angles"], float)


def _far_intensity_function():
    import torch

    class FarFieldIntensity(torch.autograd.Function):
        """J(eps) = |E_far(far_angle)|^2 of the scattered field for one plane-wave
        incidence, as a function of the per-leaf relative permittivity.  Forward
        sets the solver up for eps and runs the forward and adjoint solves; the
        backward pass returns the adjoint gradient (no further solve)."""

        @staticmethod
        def forward(ctx, eps, w, incidence, far_angle, far_inside, options):
            e = eps.detach().to("cpu", torch.float64).numpy()
            s = Solver(dict(w, eps_r=e), **(options or {}))
            try:
                J, grad, _ = s.far_intensity_gradient(incidence, far_angle, far_inside)
            finally:
                s.close()
            ctx.save_for_backward(torch.as_tensor(grad, dtype=eps.dtype, device=eps.device))
            return torch.as_tensor(J, dtype=eps.dtype, device=eps.device)

        @staticmethod
        def backward(ctx, gJ):
            (grad,) = ctx.saved_tensors
            return gJ * grad, None, None, None, None, None

    return FarFieldIntensity


def far_intensity(eps, w, incidence, far_angle, far_inside, **options):
    """Differentiable J = |E_far|^2 with respect to the permittivity tensor eps (one
    value per leaf); options are passed to Solver (tol, max_iter, precision, ...)."""
    return _far_intensity_function().apply(eps, w, incidence, far_angle, far_inside, options)
