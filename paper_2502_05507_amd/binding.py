"""ctypes binding of libbae.so (include/bae.h): argument marshalling only.

Device buffers are torch tensors (their data_ptr() is handed to the library); host
buffers are NumPy arrays.  Every failing call raises BaeError with the library's message.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbae.so")

OK, NOT_CONVERGED = 0, 1
PREC_FP64, PREC_FP32, PREC_FFT = 0, 1, 2
SOLVE_FP64, SOLVE_FP32_REFINED, SOLVE_FFT = 0, 1, 2
LAYER_DOUBLE, LAYER_SINGLE, LAYER_DIRECT = 0, 1, 2
PARTICULAR = {"free": 0, "box": 1}
KINDS = {"sphere": 1, "ellipsoid": 2, "torus": 3, "star": 4, "sampled": 5}


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("origin", C.c_double * 3), ("h", C.c_double), ("sigma", C.c_double)]


class LevelSet(C.Structure):
    _fields_ = [("kind", C.c_int32), ("center", C.c_double * 3), ("params", C.c_double * 8),
                ("phi_samples", C.POINTER(C.c_double))]


class Options(C.Structure):
    _fields_ = [("device", C.c_int32), ("near_radius_fp64", C.c_int32), ("near_radius_fp32", C.c_int32),
                ("max_krylov", C.c_int32), ("max_rhs", C.c_int32), ("sum_wait_polls", C.c_int32)]


class Sizes(C.Structure):
    _fields_ = [("n_mplus", C.c_int64), ("n_gamma_plus", C.c_int64), ("n_gamma_minus", C.c_int64),
                ("n_ext", C.c_int64), ("n_edges", C.c_int64), ("n_sources", C.c_int64),
                ("n_targets", C.c_int64), ("n_empty_d", C.c_int64), ("max_offset", C.c_int32),
                ("table_radius", C.c_int32), ("table_entries", C.c_int64), ("device_bytes", C.c_int64),
                ("lds_radius_fp32", C.c_int32), ("lds_radius_fp64", C.c_int32), ("far_field_fp32", C.c_int32),
                ("far_field_fp64", C.c_int32), ("far_field_err_fp32", C.c_double), ("conv_box", C.c_int32 * 3),
                ("conv_fft", C.c_int32 * 3)]

    def as_dict(self):
        return {k: (list(v) if isinstance(v, C.Array) else v) for k, v in ((k, getattr(self, k)) for k, _ in self._fields_)}


class SolveParams(C.Structure):
    _fields_ = [("precision", C.c_int32), ("tol", C.c_double), ("maxit", C.c_int32), ("inner_tol", C.c_double),
                ("max_outer", C.c_int32), ("compute_grid", C.c_int32), ("recycle_dim", C.c_int32),
                ("formulation", C.c_int32), ("x0_dev", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("outer_steps", C.c_int32),
                ("converged", C.c_int32), ("rel_residual_est", C.c_double), ("rel_residual_true", C.c_double),
                ("seconds", C.c_double), ("matvecs_fp64", C.c_int64), ("matvecs_fp32", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


BoundaryFn = C.CFUNCTYPE(None, C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double))


class ServerOptions(C.Structure):
    _fields_ = [("device", C.c_int32), ("max_slots", C.c_int32), ("hbm_budget", C.c_int64),
                ("precision", C.c_int32), ("tol", C.c_double), ("maxit", C.c_int32), ("max_krylov", C.c_int32),
                ("iters_per_step", C.c_int32), ("setup_threads", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("grid", Grid), ("levelset", LevelSet), ("g", BoundaryFn), ("user", C.c_void_p)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("n_gamma_minus", C.c_int64), ("n_targets", C.c_int64), ("bytes", C.c_int64),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "admitted", "completed", "failed", "steps", "max_active",
                                         "peak_bytes", "bytes_in_use", "waiting", "running")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BaeError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"[{status}] {message}")
        self.status = status


_lib = None
_P = C.c_void_p


def load_library():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise BaeError(-1, f"{LIB_PATH} is missing: build it with `python -m paper_2502_05507_amd.build`")
    # torch ships its own HIP runtime under the same soname as the system one.  Loading
    # torch first makes the dynamic linker bind the library to that runtime, so device
    # pointers and streams from torch and from the library live in one runtime; loaded the
    # other way round, torch would find a foreign runtime and see no device.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    sig = {
        "bae_status_string": (C.c_char_p, [C.c_int]),
        "bae_last_error": (C.c_char_p, []),
        "bae_lgf_table_size": (C.c_int64, [C.c_int32]),
        "bae_lgf_table": (C.c_int, [C.c_double, C.c_int32, _P, _P]),
        "bae_lgf_table_noalloc": (C.c_int, [C.c_double, C.c_int32, _P, _P]),
        "bae_create": (C.c_int, [C.POINTER(Grid), C.POINTER(LevelSet), C.POINTER(Options), C.POINTER(_P)]),
        "bae_destroy": (C.c_int, [_P]),
        "bae_get_sizes": (C.c_int, [_P, C.POINTER(Sizes)]),
        "bae_get_sets": (C.c_int, [_P, _P, _P, _P]),
        "bae_get_boundary_points": (C.c_int, [_P, _P, _P, _P]),
        "bae_set_rhs": (C.c_int, [_P, C.c_int32, _P, _P]),
        "bae_set_rhs_box": (C.c_int, [_P, C.c_int32, _P, _P]),
        "bae_get_particular": (C.c_int, [_P, C.c_int32, _P]),
        "bae_solve": (C.c_int, [_P, C.POINTER(SolveParams), _P]),
        "bae_get_density": (C.c_int, [_P, C.c_int32, _P]),
        "bae_get_density_length": (C.c_int, [_P, C.POINTER(C.c_int64)]),
        "bae_get_gamma_values": (C.c_int, [_P, C.c_int32, _P]),
        "bae_get_solution": (C.c_int, [_P, C.c_int32, _P]),
        "bae_get_history": (C.c_int, [_P, C.c_int32, _P, C.c_int32, C.POINTER(C.c_int32)]),
        "bae_set_rhs_device": (C.c_int, [_P, C.c_int32, _P, _P, C.c_int32, _P]),
        "bae_solve_async": (C.c_int, [_P, C.POINTER(SolveParams), _P]),
        "bae_solve_poll": (C.c_int, [_P, C.POINTER(C.c_int32)]),
        "bae_solve_wait": (C.c_int, [_P, _P, _P]),
        "bae_get_density_device": (C.c_int, [_P, C.c_int32, _P, _P]),
        "bae_get_gamma_values_device": (C.c_int, [_P, C.c_int32, _P, _P]),
        "bae_get_solution_device": (C.c_int, [_P, C.c_int32, _P, _P]),
        "bae_apply_double_layer": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, _P]),
        "bae_apply_operator": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, _P]),
        "bae_apply_single_layer": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, _P]),
        "bae_apply_direct": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, _P]),
        "bae_lgf_eval": (C.c_int, [_P, _P, C.c_int64, _P, C.c_int32, _P]),
        "bae_sum_stats": (C.c_int, [_P, C.c_int32, _P]),
        "bae_lgf_sum_repeat": (C.c_int, [_P, _P, C.c_int32, C.c_int32, C.c_int32, _P]),
        "bae_batch_create": (C.c_int, [_P, C.c_int32, C.POINTER(_P)]),
        "bae_batch_autotune": (C.c_int, [_P, C.c_int32, _P]),
        "bae_batch_solve": (C.c_int, [_P, C.POINTER(SolveParams), C.c_int32, _P]),
        "bae_batch_destroy": (C.c_int, [_P]),
        "bae_batch_sum_stats": (C.c_int, [_P, C.c_int32, _P]),
        "bae_server_create": (C.c_int, [C.POINTER(ServerOptions), C.POINTER(_P)]),
        "bae_server_submit": (C.c_int, [_P, C.POINTER(Request), C.POINTER(C.c_uint64)]),
        "bae_server_wait": (C.c_int, [_P, C.c_uint64, C.c_double, _P, _P]),
        "bae_server_fetch": (C.c_int, [_P, C.c_uint64, _P, C.c_int64, _P, C.c_int64]),
        "bae_server_poll": (C.c_int, [_P, C.c_uint64, C.POINTER(C.c_int32)]),
        "bae_server_stats_get": (C.c_int, [_P, C.POINTER(ServerStats)]),
        "bae_server_destroy": (C.c_int, [_P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc, allow_not_converged=False):
    if rc == OK or (allow_not_converged and rc == NOT_CONVERGED):
        return rc
    lib = load_library()
    raise BaeError(rc, lib.bae_last_error().decode() or lib.bae_status_string(rc).decode())


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _dptr(t):
    """Device pointer of a torch tensor."""
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream)


def lgf_table_size(R):
    return int(load_library().bae_lgf_table_size(R))


def lgf_table(s, R, out, stream=None):
    """FP64 LGF table G_s for 0 <= a <= b <= c <= R into the device tensor `out`."""
    assert out.dtype.is_floating_point and out.element_size() == 8 and out.numel() >= lgf_table_size(R)
    _check(load_library().bae_lgf_table(float(s), int(R), _dptr(out), _stream(stream)))


def lgf_table_noalloc(s, R, out, stream=None):
    """bae_lgf_table_noalloc: the same table, scratch in the library's static device array."""
    assert out.dtype.is_floating_point and out.element_size() == 8 and out.numel() >= lgf_table_size(R)
    _check(load_library().bae_lgf_table_noalloc(float(s), int(R), _dptr(out), _stream(stream)))


class Context:
    """One geometry / grid / sigma (Algorithm 1 set-up), owning its device state."""

    def __init__(self, n, h, origin, sigma, kind, center=(0.0, 0.0, 0.0), params=(), phi=None,
                 device=0, max_krylov=0, max_rhs=0, sum_wait_polls=0):
        lib = load_library()
        g = Grid((C.c_int32 * 3)(*[int(v) for v in n]), (C.c_double * 3)(*[float(v) for v in origin]),
                 float(h), float(sigma))
        p = list(params) + [0.0] * (8 - len(params))
        self._phi = None
        if phi is not None:
            self._phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        ls = LevelSet(KINDS[kind], (C.c_double * 3)(*[float(v) for v in center]),
                      (C.c_double * 8)(*[float(v) for v in p[:8]]),
                      self._phi.ctypes.data_as(C.POINTER(C.c_double)) if self._phi is not None else None)
        opt = Options(int(device), 0, 0, int(max_krylov), int(max_rhs), int(sum_wait_polls))
        h_ = _P()
        _check(lib.bae_create(C.byref(g), C.byref(ls), C.byref(opt), C.byref(h_)))
        self._h = h_
        self.n = tuple(int(v) for v in n)
        self.nrhs = 1
        self.sizes = self.get_sizes()

    @classmethod
    def from_problem(cls, p, **kw):
        return cls(p.n, p.h, p.origin, p.sigma, p.kind, p.center, p.params, **kw)

    def close(self):
        if getattr(self, "_h", None):
            load_library().bae_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def get_sizes(self):
        s = Sizes()
        _check(load_library().bae_get_sizes(self._h, C.byref(s)))
        return s.as_dict()

    def sets(self):
        z = self.sizes
        gp = np.empty((z["n_gamma_plus"], 3), np.int32)
        gm = np.empty((z["n_gamma_minus"], 3), np.int32)
        ex = np.empty((z["n_ext"], 3), np.int32)
        _check(load_library().bae_get_sets(self._h, _ptr(gp), _ptr(gm), _ptr(ex)))
        return gp, gm, ex

    def boundary_points(self):
        m = self.sizes["n_gamma_minus"]
        xs = np.empty((m, 3))
        pa = np.empty(m, np.int32)
        t = np.empty(m)
        _check(load_library().bae_get_boundary_points(self._h, _ptr(xs), _ptr(pa), _ptr(t)))
        return xs, pa, t

    def set_rhs(self, g, f=None, particular="free"):
        """g at x* ([nrhs][|gamma-|]) and optional f on the grid.  particular: "free" (the
        free-space volume potential) or "box" (Algorithm 1's finite-grid solve, bae_set_rhs_box)."""
        g = np.ascontiguousarray(g, dtype=np.float64)
        nrhs = 1 if g.ndim == 1 else g.shape[0]
        if f is not None:
            f = np.ascontiguousarray(f, dtype=np.float64)
        fn = {"free": load_library().bae_set_rhs, "box": load_library().bae_set_rhs_box}[particular]
        _check(fn(self._h, nrhs, _ptr(g), _ptr(f)))
        self.nrhs = nrhs

    def set_rhs_device(self, g, f=None, particular="free", stream=None):
        """Device form of set_rhs on torch tensors g [nrhs][|gamma-|] and f [nrhs][n0 n1 n2] (float64),
        asynchronous on `stream` (default: torch's current stream)."""
        nrhs = 1 if g.dim() == 1 else g.shape[0]
        assert g.is_contiguous() and g.numel() == nrhs * self.sizes["n_gamma_minus"]
        if f is not None:
            assert f.is_contiguous() and f.numel() == nrhs * int(np.prod(self.n))
        _check(load_library().bae_set_rhs_device(self._h, nrhs, _dptr(g), _dptr(f) if f is not None else None,
                                                 PARTICULAR[particular], _stream(stream)))
        self.nrhs = nrhs

    def particular(self, r=0):
        """u_p on the grid after set_rhs(..., particular="box") with f."""
        u = np.empty(self.n)
        _check(load_library().bae_get_particular(self._h, r, _ptr(u)))
        return u

    @staticmethod
    def _params(precision, tol, maxit, inner_tol, max_outer, compute_grid, recycle_dim, formulation, x0):
        return SolveParams(int(precision), float(tol), int(maxit), float(inner_tol), int(max_outer),
                           1 if compute_grid else 0, int(recycle_dim), int(formulation),
                           C.c_void_p(x0.data_ptr()) if x0 is not None else None)

    def solve(self, precision=SOLVE_FP64, tol=1e-10, maxit=0, inner_tol=0.0, max_outer=0, compute_grid=False,
              recycle_dim=0, formulation=0, x0=None):
        """formulation: LAYER_DOUBLE (default) or LAYER_SINGLE (Sec. 3.4); x0: optional device tensor of
        initial densities [nrhs][|gamma-|]."""
        p = self._params(precision, tol, maxit, inner_tol, max_outer, compute_grid, recycle_dim, formulation, x0)
        res = (Result * self.nrhs)()
        rc = load_library().bae_solve(self._h, C.byref(p), res)
        _check(rc, allow_not_converged=True)
        return [r.as_dict() for r in res]

    def solve_async(self, precision=SOLVE_FP64, tol=1e-10, maxit=0, inner_tol=0.0, max_outer=0, compute_grid=False,
                    recycle_dim=0, formulation=0, x0=None, stream=None):
        """bae_solve_async: ordered after `stream` (default: torch's current stream), returns at once."""
        p = self._params(precision, tol, maxit, inner_tol, max_outer, compute_grid, recycle_dim, formulation, x0)
        self._x0 = x0      # kept alive until the solve is collected
        _check(load_library().bae_solve_async(self._h, C.byref(p), _stream(stream)))

    def solve_poll(self):
        d = C.c_int32(0)
        _check(load_library().bae_solve_poll(self._h, C.byref(d)))
        return bool(d.value)

    def solve_wait(self, stream=None):
        res = (Result * self.nrhs)()
        rc = load_library().bae_solve_wait(self._h, _stream(stream), res)
        self._x0 = None
        _check(rc, allow_not_converged=True)
        return [r.as_dict() for r in res]

    def _device_out(self, fn, out, r, length, stream):
        count = length * (self.nrhs if r < 0 else 1)
        assert out.is_contiguous() and out.numel() == count and out.element_size() == 8
        _check(fn(self._h, int(r), _dptr(out), _stream(stream)))

    def density_device(self, out, r=-1, stream=None):
        self._device_out(load_library().bae_get_density_device, out, r, self.density_length(), stream)

    def gamma_values_device(self, out, r=-1, stream=None):
        self._device_out(load_library().bae_get_gamma_values_device, out, r, self.sizes["n_targets"], stream)

    def solution_device(self, out, r=-1, stream=None):
        self._device_out(load_library().bae_get_solution_device, out, r, int(np.prod(self.n)), stream)

    def density_length(self):
        """Length of the last solve's density: |gamma-| (layer potentials), or |gamma| after a
        direct-formulation solve."""
        n = C.c_int64()
        _check(load_library().bae_get_density_length(self._h, C.byref(n)))
        return int(n.value)

    def density(self, r=0):
        q = np.empty(self.density_length())
        _check(load_library().bae_get_density(self._h, r, _ptr(q)))
        return q

    def gamma_values(self, r=0):
        u = np.empty(self.sizes["n_targets"])
        _check(load_library().bae_get_gamma_values(self._h, r, _ptr(u)))
        return u

    def solution(self, r=0):
        u = np.empty(self.n)
        _check(load_library().bae_get_solution(self._h, r, _ptr(u)))
        return u

    def history(self, r=0):
        n = C.c_int32(0)
        _check(load_library().bae_get_history(self._h, r, None, 0, C.byref(n)))
        h = np.empty(n.value)
        _check(load_library().bae_get_history(self._h, r, _ptr(h), n.value, C.byref(n)))
        return h

    def apply_double_layer(self, q, v, precision=PREC_FP64, stream=None):
        """v[nrhs][|gamma|] = [D+ q; D- q] for device tensors q[nrhs][|gamma-|] (float64)."""
        nrhs = 1 if q.dim() == 1 else q.shape[0]
        assert q.is_contiguous() and v.is_contiguous()
        assert q.numel() == nrhs * self.sizes["n_gamma_minus"] and v.numel() == nrhs * self.sizes["n_targets"]
        _check(load_library().bae_apply_double_layer(self._h, _dptr(q), _dptr(v), nrhs, precision, _stream(stream)))

    def apply_single_layer(self, q, v, precision=PREC_FP64, stream=None):
        """v[nrhs][|gamma|] = [S+ q; S- q] for device tensors q[nrhs][|gamma-|] (float64)."""
        nrhs = 1 if q.dim() == 1 else q.shape[0]
        assert q.is_contiguous() and v.is_contiguous()
        assert q.numel() == nrhs * self.sizes["n_gamma_minus"] and v.numel() == nrhs * self.sizes["n_targets"]
        _check(load_library().bae_apply_single_layer(self._h, _dptr(q), _dptr(v), nrhs, precision, _stream(stream)))

    def apply_direct(self, v, y, precision=PREC_FP64, stream=None):
        """y = the direct system's operator (Sec. 3.1) on device tensors v, y [nrhs][|gamma|] (float64)."""
        nrhs = 1 if v.dim() == 1 else v.shape[0]
        assert v.is_contiguous() and y.is_contiguous()
        assert v.numel() == y.numel() == nrhs * self.sizes["n_targets"]
        _check(load_library().bae_apply_direct(self._h, _dptr(v), _dptr(y), nrhs, precision, _stream(stream)))

    def apply_operator(self, q, aq, precision=PREC_FP64, stream=None):
        """aq = (Phi+ D+ + Phi- D-) q for device tensors [nrhs][|gamma-|] (float64)."""
        nrhs = 1 if q.dim() == 1 else q.shape[0]
        assert q.is_contiguous() and aq.is_contiguous()
        assert q.numel() == aq.numel() == nrhs * self.sizes["n_gamma_minus"]
        _check(load_library().bae_apply_operator(self._h, _dptr(q), _dptr(aq), nrhs, precision, _stream(stream)))

    def lgf_sum_repeat(self, q, repeats=1, precision=PREC_FP32, stream=None):
        """The LGF sum alone, `repeats` times, on the weights of device densities q (bae_lgf_sum_repeat)."""
        nrhs = 1 if q.dim() == 1 else q.shape[0]
        assert q.is_contiguous() and q.numel() == nrhs * self.sizes["n_gamma_minus"]
        _check(load_library().bae_lgf_sum_repeat(self._h, _dptr(q), nrhs, precision, int(repeats), _stream(stream)))

    def sum_stats(self, precision=PREC_FP32):
        """Pair counts of the LGF sum by the kernel's block classification (bae_sum_stats)."""
        c = np.zeros(5, np.int64)
        _check(load_library().bae_sum_stats(self._h, precision, _ptr(c)))
        return {"near": int(c[0]), "far": int(c[1]), "far_q2": int(c[2]), "mixed_near": int(c[3]),
                "mixed_far": int(c[4])}

    def lgf_eval(self, offsets, out, precision=PREC_FP64, stream=None):
        """out[i] = the kernel value the LGF sum uses at integer offset offsets[i] (device)."""
        assert offsets.is_contiguous() and offsets.shape[-1] == 3 and out.numel() == offsets.shape[0]
        _check(load_library().bae_lgf_eval(self._h, _dptr(offsets), offsets.shape[0], _dptr(out), precision,
                                           _stream(stream)))


class Batch:
    """Lock-step solves of many single-RHS contexts (bae_batch_*)."""

    def __init__(self, contexts):
        lib = load_library()
        self.contexts = list(contexts)
        arr = (_P * len(self.contexts))(*[c._h for c in self.contexts])
        h = _P()
        _check(lib.bae_batch_create(arr, len(self.contexts), C.byref(h)))
        self._h = h

    def autotune(self, precision=PREC_FP32):
        chosen = np.zeros(2, np.int32)
        _check(load_library().bae_batch_autotune(self._h, precision, _ptr(chosen)))
        return {"blocks_per_chunk": int(chosen[0]), "grid_multiplier": int(chosen[1])}

    def solve(self, precision=SOLVE_FP64, tol=1e-10, maxit=0, inner_tol=0.0, max_outer=0, use_graph=True):
        p = SolveParams(int(precision), float(tol), int(maxit), float(inner_tol), int(max_outer), 0, 0, 0, None)
        res = (Result * len(self.contexts))()
        rc = load_library().bae_batch_solve(self._h, C.byref(p), 1 if use_graph else 0, res)
        _check(rc, allow_not_converged=True)
        return [r.as_dict() for r in res]

    def sum_stats(self, precision=PREC_FP32):
        """Pair counts of the batched LGF sum by its own block classification (bae_batch_sum_stats)."""
        c = np.zeros(5, np.int64)
        _check(load_library().bae_batch_sum_stats(self._h, precision, _ptr(c)))
        return {"near": int(c[0]), "far": int(c[1]), "far_q2": int(c[2]), "mixed_near": int(c[3]),
                "mixed_far": int(c[4])}

    def close(self):
        if getattr(self, "_h", None):
            load_library().bae_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _grid_and_levelset(n, h, origin, sigma, kind, center, params, phi=None):
    g = Grid((C.c_int32 * 3)(*[int(v) for v in n]), (C.c_double * 3)(*[float(v) for v in origin]), float(h),
             float(sigma))
    p = list(params) + [0.0] * (8 - len(params))
    ls = LevelSet(KINDS[kind], (C.c_double * 3)(*[float(v) for v in center]),
                  (C.c_double * 8)(*[float(v) for v in p[:8]]),
                  phi.ctypes.data_as(C.POINTER(C.c_double)) if phi is not None else None)
    return g, ls


class Server:
    """Continuous-batching solve server (bae_server_*).  Boundary data are Python callables
    g(xyz: (N,3) array) -> (N,) array, called on one of the server's set-up threads at admission."""

    def __init__(self, hbm_budget, max_slots=64, precision=SOLVE_FP64, tol=1e-10, maxit=0, max_krylov=200,
                 iters_per_step=4, device=0, setup_threads=0):
        lib = load_library()
        o = ServerOptions(int(device), int(max_slots), int(hbm_budget), int(precision), float(tol), int(maxit),
                          int(max_krylov), int(iters_per_step), int(setup_threads))
        h = _P()
        _check(lib.bae_server_create(C.byref(o), C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, n, h, origin, sigma, kind, center, params, g, phi=None):
        def cb(user, count, xyz, out, _g=g):
            X = np.ctypeslib.as_array(xyz, shape=(count, 3))
            np.ctypeslib.as_array(out, shape=(count,))[:] = _g(X)
        fn = BoundaryFn(cb)
        phi = None if phi is None else np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        grid, ls = _grid_and_levelset(n, h, origin, sigma, kind, center, params, phi)
        req = Request(grid, ls, fn, None)
        t = C.c_uint64(0)
        _check(load_library().bae_server_submit(self._h, C.byref(req), C.byref(t)))
        self._keep[t.value] = fn
        return t.value

    def submit_problem(self, p, g=None):
        g = g if g is not None else (lambda X: p.g(X))
        return self.submit(p.n, p.h, p.origin, p.sigma, p.kind, p.center, p.params, g)

    def wait(self, ticket, timeout=-1.0):
        r = Result()
        info = RequestInfo()
        rc = load_library().bae_server_wait(self._h, ticket, float(timeout), C.byref(r), C.byref(info))
        _check(rc, allow_not_converged=True)
        return r.as_dict(), info.as_dict()

    def poll(self, ticket):
        """0 waiting, 1 admitted, 2 done, 3 failed (never blocks)."""
        st = C.c_int32(0)
        _check(load_library().bae_server_poll(self._h, ticket, C.byref(st)))
        return st.value

    def fetch(self, ticket, n_gamma_minus, n_targets):
        q = np.empty(n_gamma_minus)
        u = np.empty(n_targets)
        _check(load_library().bae_server_fetch(self._h, ticket, _ptr(q), len(q), _ptr(u), len(u)))
        self._keep.pop(ticket, None)
        return q, u

    def result(self, ticket, timeout=-1.0):
        r, info = self.wait(ticket, timeout)
        q, u = self.fetch(ticket, info["n_gamma_minus"], info["n_targets"])
        return r, info, q, u

    def stats(self):
        st = ServerStats()
        _check(load_library().bae_server_stats_get(self._h, C.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            load_library().bae_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
