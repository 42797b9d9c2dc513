"""Thin ctypes binding of the C ABI in include/fftg.h.

Argument marshalling only: every step of the solve runs in libfftg.so's HIP
kernels.  torch supplies device memory (tensors whose data_ptr() is handed
to the library) and the stream.  Names mirror the C entry points.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfftg.so")

FFTG_OK = 0
FFTG_E_INVALID = -1
FFTG_E_NOMEM = -2
FFTG_E_HIP = -3
FFTG_E_NOT_CONVERGED = -4
FFTG_E_BREAKDOWN = -5
FFTG_E_UNSUPPORTED = -6
FFTG_E_NONFINITE = -7

FFTG_FP64 = 0
FFTG_MIXED = 1
FFTG_TANGENT_CURRENT = 0
FFTG_TANGENT_IDENTITY = 1
FFTG_TANGENT_ELASTIC = 2
FFTG_PREDICTOR_TANGENT = 0
FFTG_PREDICTOR_NONE = 1
FFTG_FIELD_FLUCT, FFTG_FIELD_STRAIN, FFTG_FIELD_STRESS, FFTG_FIELD_EPS_P, FFTG_FIELD_EPBAR, FFTG_FIELD_TANGENT = range(6)
FFTG_MAX_NEWTON = 64

# every symbol include/fftg.h declares
EXPORTS = [
    "fftg_options_default", "fftg_plan_create", "fftg_plan_destroy", "fftg_history_create",
    "fftg_history_destroy", "fftg_solve_increment", "fftg_apply_GK", "fftg_eval_constitutive",
    "fftg_get_field", "fftg_set_field", "fftg_history_get_E", "fftg_history_save", "fftg_history_restore",
    "fftg_footprint_bytes", "fftg_batch_create", "fftg_batch_destroy", "fftg_batch_solve_increment",
    "fftg_profiler_start", "fftg_profiler_start_every", "fftg_profiler_stop", "fftg_profiler_seen",
    "fftg_profiler_start_set", "fftg_profiler_kind",
    "fftg_last_error", "fftg_apply_GK_noalloc", "fftg_apply_Gamma",
]
FFTG_KERNEL_ZFWD, FFTG_KERNEL_Y_FWD, FFTG_KERNEL_X_PROJ, FFTG_KERNEL_Y_INV, FFTG_KERNEL_ZINV = range(5)
FFTG_KERNEL_FINALIZE, FFTG_KERNEL_CONSTITUTIVE, FFTG_KERNEL_NEWTON = range(5, 8)


FFTG_LAW_J2, FFTG_LAW_NONLINEAR_ELASTIC, FFTG_LAW_VISCO = 0, 1, 2
FFTG_SCHEME_GALERKIN, FFTG_SCHEME_BASIC = 0, 1


class fftg_material(C.Structure):
    _fields_ = [("K", C.c_double), ("G", C.c_double), ("sigma_y0", C.c_double), ("H", C.c_double),
                ("n", C.c_double), ("law", C.c_int), ("eps0", C.c_double), ("t0", C.c_double)]


def material(row) -> fftg_material:
    """(K, G, sigma_y0, H, n) for an elasto-plastic phase, or
    (K, G, sigma_y0, H, n, law, eps0, t0) naming the law."""
    r = [float(v) for v in row]
    if len(r) == 5:
        r += [FFTG_LAW_J2, 1.0, 1.0]
    if len(r) != 8:
        raise ValueError("material rows are (K, G, s0, H, n) or (K, G, s0, H, n, law, eps0, t0)")
    return fftg_material(r[0], r[1], r[2], r[3], r[4], int(r[5]), r[6], r[7])


class fftg_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("tol_newton", C.c_double), ("tol_cg", C.c_double),
                ("max_newton", C.c_int), ("max_cg", C.c_int), ("predictor", C.c_int),
                ("rhs_floor", C.c_double), ("mixed_cg_floor", C.c_double), ("cg_chunk", C.c_int),
                ("dt", C.c_double), ("scheme", C.c_int)]


class fftg_stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int), ("cg_iters", C.c_int * FFTG_MAX_NEWTON),
                ("newton_res", C.c_double * FFTG_MAX_NEWTON), ("Sigma", C.c_double * 6),
                ("converged", C.c_int), ("total_cg", C.c_int), ("seconds", C.c_double),
                ("rel_equilibrium", C.c_double)]

    def to_dict(self):
        n = min(self.newton_iters, FFTG_MAX_NEWTON)
        return {"newton_iters": self.newton_iters, "cg_iters": list(self.cg_iters[:n]),
                "newton_res": list(self.newton_res[:n]), "Sigma": list(self.Sigma),
                "converged": bool(self.converged), "total_cg": self.total_cg, "seconds": self.seconds,
                "rel_equilibrium": self.rel_equilibrium}


_lib = None


def lib():
    """Loads libfftg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run paper_1601_05970_amd.build.build() first")
    # torch and the library share one HIP runtime; it must be initialised
    # (through torch) before the library's code objects are registered.
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
            torch.empty(1, device="cuda")
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, ip, dp = C.c_void_p, C.c_int, C.POINTER(C.c_double)
    L.fftg_options_default.argtypes = [C.POINTER(fftg_options)]
    L.fftg_options_default.restype = None
    L.fftg_plan_create.argtypes = [C.POINTER(vp), ip, ip, ip, C.c_char_p, ip, C.POINTER(fftg_material),
                                   C.POINTER(fftg_options), vp]
    L.fftg_plan_destroy.argtypes = [vp]
    L.fftg_plan_destroy.restype = None
    L.fftg_history_create.argtypes = [vp, C.POINTER(vp)]
    L.fftg_history_destroy.argtypes = [vp]
    L.fftg_history_destroy.restype = None
    L.fftg_solve_increment.argtypes = [vp, vp, dp, C.POINTER(C.c_int), ip, C.POINTER(fftg_stats)]
    L.fftg_apply_GK.argtypes = [vp, vp, vp, vp, ip]
    L.fftg_eval_constitutive.argtypes = [vp, vp, vp, vp]
    L.fftg_get_field.argtypes = [vp, vp, ip, vp]
    L.fftg_set_field.argtypes = [vp, vp, ip, vp]
    L.fftg_history_get_E.argtypes = [vp, dp, C.POINTER(C.c_int)]
    L.fftg_history_save.argtypes = [vp, vp, vp, C.POINTER(C.c_size_t)]
    L.fftg_history_restore.argtypes = [vp, vp, vp, C.c_size_t]
    L.fftg_footprint_bytes.argtypes = [ip, ip, ip, ip]
    L.fftg_footprint_bytes.restype = C.c_size_t
    L.fftg_batch_create.argtypes = [C.POINTER(vp), ip, C.POINTER(vp), C.POINTER(vp)]
    L.fftg_batch_destroy.argtypes = [vp]
    L.fftg_batch_destroy.restype = None
    L.fftg_batch_solve_increment.argtypes = [vp, dp, C.POINTER(fftg_stats)]
    L.fftg_profiler_start.argtypes = [ip]
    L.fftg_profiler_start_every.argtypes = [ip, ip]
    L.fftg_profiler_seen.argtypes = []
    L.fftg_profiler_seen.restype = C.c_longlong
    L.fftg_profiler_stop.argtypes = [dp, C.POINTER(C.c_longlong), dp]
    L.fftg_profiler_start_set.argtypes = [C.c_uint, ip]
    L.fftg_profiler_kind.argtypes = [ip, dp, C.POINTER(C.c_longlong), dp, C.POINTER(C.c_longlong)]
    L.fftg_apply_GK_noalloc.argtypes = [ip, ip, ip, vp, vp, ip, vp, ip, C.POINTER(fftg_material), vp]
    L.fftg_apply_Gamma.argtypes = [vp, vp, vp, C.c_double, C.c_double]
    L.fftg_last_error.argtypes = []
    L.fftg_last_error.restype = C.c_char_p
    for name in ("fftg_plan_create", "fftg_history_create", "fftg_solve_increment", "fftg_apply_GK",
                 "fftg_eval_constitutive", "fftg_get_field", "fftg_set_field", "fftg_history_get_E",
                 "fftg_history_save", "fftg_history_restore", "fftg_batch_create",
                 "fftg_batch_solve_increment", "fftg_profiler_start", "fftg_profiler_start_every",
                 "fftg_profiler_stop", "fftg_apply_GK_noalloc", "fftg_profiler_start_set",
                 "fftg_profiler_kind", "fftg_apply_Gamma"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


class FFTGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fftg status {status}: {msg}")
        self.status = status


def check(st):
    if st != FFTG_OK:
        raise FFTGError(st, lib().fftg_last_error().decode(errors="replace"))
    return st


def fftg_options_default() -> fftg_options:
    o = fftg_options()
    lib().fftg_options_default(C.byref(o))
    return o


def fftg_footprint_bytes(n0, n1, n2, precision=FFTG_FP64) -> int:
    return int(lib().fftg_footprint_bytes(n0, n1, n2, precision))


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def tensor_to_mandel_components(t6: Sequence[float]) -> np.ndarray:
    """Host 6-vector order used by the ABI: [11, 22, 33, 23, 13, 12]."""
    return np.asarray(t6, dtype=np.float64)


def fftg_profiler_start(kernel_id: int):
    check(lib().fftg_profiler_start(kernel_id))


def fftg_profiler_start_every(kernel_id: int, every: int):
    check(lib().fftg_profiler_start_every(kernel_id, every))


def fftg_profiler_seen() -> int:
    return int(lib().fftg_profiler_seen())


def fftg_profiler_start_set(kernel_ids, every: int):
    mask = 0
    for k in kernel_ids:
        mask |= 1 << int(k)
    check(lib().fftg_profiler_start_set(mask, every))


def fftg_profiler_kind(kernel_id: int):
    """(ms, bracketed launches, voxels, all launches) of one kind after stop."""
    ms, n, vox, seen = C.c_double(), C.c_longlong(), C.c_double(), C.c_longlong()
    check(lib().fftg_profiler_kind(kernel_id, C.byref(ms), C.byref(n), C.byref(vox), C.byref(seen)))
    return ms.value, n.value, vox.value, seen.value


def fftg_profiler_stop():
    """Returns (total_ms, launches, voxels) of the profiled kernel."""
    ms, n, vox = C.c_double(), C.c_longlong(), C.c_double()
    check(lib().fftg_profiler_stop(C.byref(ms), C.byref(n), C.byref(vox)))
    return ms.value, n.value, vox.value


class Plan:
    """fftg_plan_create / fftg_plan_destroy."""

    def __init__(self, phase: np.ndarray, materials, options: Optional[fftg_options] = None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("fftg needs a HIP device")
        ph = np.ascontiguousarray(phase, dtype=np.uint8)
        if ph.ndim != 3:
            raise ValueError("phase must be 3-D")
        self.shape = tuple(int(s) for s in ph.shape)
        mats = (fftg_material * len(materials))(*[material(m) for m in materials])
        self.options = options if options is not None else fftg_options_default()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        check(lib().fftg_plan_create(C.byref(h), self.shape[0], self.shape[1], self.shape[2], ph.tobytes(),
                                     len(materials), mats, C.byref(self.options),
                                     _stream_handle(self.stream)))
        self.handle = h
        self.mixed = self.options.precision == FFTG_MIXED

    @property
    def nvox(self):
        return self.shape[0] * self.shape[1] * self.shape[2]

    def close(self):
        if getattr(self, "handle", None):
            lib().fftg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def field(self, ncomp=6, dtype=None):
        import torch
        return torch.zeros((ncomp,) + self.shape, dtype=dtype or torch.float64, device="cuda")

    def apply_Gamma(self, d_in, d_out, lam0: float, mu0: float):
        """fftg_apply_Gamma: d_out = Gamma_ref(C_ref) : d_in, C_ref = lam0 I(x)I + 2 mu0 I_s."""
        _check_field(d_in, self.shape, 6, "float64")
        _check_field(d_out, self.shape, 6, "float64")
        check(lib().fftg_apply_Gamma(self.handle, _dptr(d_in), _dptr(d_out), float(lam0), float(mu0)))

    def apply_GK(self, d_in, d_out, mode=FFTG_TANGENT_CURRENT, hist: "History" = None):
        """fftg_apply_GK: d_out = G:(C:d_in) on the plan's stream."""
        _check_field(d_in, self.shape, 6, "float64")
        _check_field(d_out, self.shape, 6, "float32" if self.mixed else "float64")
        check(lib().fftg_apply_GK(self.handle, hist.handle if hist else None, _dptr(d_in), _dptr(d_out), mode))


def fftg_apply_GK_noalloc(d_in, d_out, mode=FFTG_TANGENT_IDENTITY, d_phase=None, materials=None, stream=None):
    """fftg_apply_GK_noalloc: d_out = G:(C:d_in) in FP64 without a plan or a
    device allocation (IDENTITY or ELASTIC); d_in, d_out (6,)+grid float64."""
    shape = tuple(d_in.shape[1:])
    _check_field(d_in, shape, 6, "float64")
    _check_field(d_out, shape, 6, "float64")
    if materials:
        mats = (fftg_material * len(materials))(*[material(m) for m in materials])
        nm = len(materials)
    else:
        mats, nm = None, 0
    ph = None
    if d_phase is not None:
        if not (d_phase.is_cuda and d_phase.is_contiguous()) or tuple(d_phase.shape) != shape or \
                str(d_phase.dtype) != "torch.uint8":
            raise ValueError("d_phase must be a contiguous uint8 device tensor of the grid's shape")
        ph = _dptr(d_phase)
    check(lib().fftg_apply_GK_noalloc(shape[0], shape[1], shape[2], _dptr(d_in), _dptr(d_out), mode, ph, nm,
                                      mats, _stream_handle(stream)))


def _check_field(t, shape, ncomp, dtype):
    import torch
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("device tensors must be contiguous CUDA/HIP tensors")
    if tuple(t.shape) != (ncomp,) + tuple(shape):
        raise ValueError(f"expected shape {(ncomp,) + tuple(shape)}, got {tuple(t.shape)}")
    if str(t.dtype) != "torch." + dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")


class History:
    """fftg_history_create / destroy and the per-history entry points."""

    def __init__(self, plan: Plan):
        self.plan = plan
        h = C.c_void_p()
        check(lib().fftg_history_create(plan.handle, C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().fftg_history_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve_increment(self, dE6, lockstep: Optional[List[int]] = None, raise_on_error=True) -> dict:
        """fftg_solve_increment; dE6 = tensor components [11,22,33,23,13,12]."""
        dE = (C.c_double * 6)(*[float(v) for v in dE6])
        st = fftg_stats()
        if lockstep is None:
            ls, nls = None, 0
        else:
            ls = (C.c_int * len(lockstep))(*[int(v) for v in lockstep])
            nls = len(lockstep)
        code = lib().fftg_solve_increment(self.plan.handle, self.handle, dE, ls, nls, C.byref(st))
        d = st.to_dict()
        d["status"] = code
        if raise_on_error:
            check(code)
        return d

    def eval_constitutive(self, d_eps, d_sigma):
        _check_field(d_eps, self.plan.shape, 6, "float64")
        _check_field(d_sigma, self.plan.shape, 6, "float64")
        check(lib().fftg_eval_constitutive(self.plan.handle, self.handle, _dptr(d_eps), _dptr(d_sigma)))

    def get_field(self, which):
        import torch
        if which == FFTG_FIELD_EPBAR:
            out = self.plan.field(1)
        elif which == FFTG_FIELD_TANGENT:
            out = self.plan.field(7, torch.float32 if self.plan.mixed else torch.float64)
        else:
            out = self.plan.field(6)
        check(lib().fftg_get_field(self.plan.handle, self.handle, which, _dptr(out)))
        return out

    def set_field(self, which, d_in):
        n = 1 if which == FFTG_FIELD_EPBAR else 6
        _check_field(d_in, self.plan.shape, n, "float64")
        check(lib().fftg_set_field(self.plan.handle, self.handle, which, _dptr(d_in)))

    def get_E(self):
        E = (C.c_double * 6)()
        inc = C.c_int()
        check(lib().fftg_history_get_E(self.handle, E, C.byref(inc)))
        return list(E), inc.value

    def save(self) -> bytes:
        n = C.c_size_t(0)
        check(lib().fftg_history_save(self.plan.handle, self.handle, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        check(lib().fftg_history_save(self.plan.handle, self.handle, buf, C.byref(n)))
        return buf.raw[:n.value]

    def restore(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        check(lib().fftg_history_restore(self.plan.handle, self.handle, buf, len(data)))

    def checkpoint_bytes(self) -> int:
        n = C.c_size_t(0)
        check(lib().fftg_history_save(self.plan.handle, self.handle, None, C.byref(n)))
        return n.value

    def save_into(self, ptr: int, size: int) -> int:
        """fftg_history_save into caller memory at host address ptr (size
        bytes, e.g. a pinned tensor's data_ptr()); returns the bytes written."""
        n = C.c_size_t(size)
        check(lib().fftg_history_save(self.plan.handle, self.handle, C.c_void_p(ptr), C.byref(n)))
        return n.value

    def restore_from(self, ptr: int, size: int):
        """fftg_history_restore from host address ptr."""
        check(lib().fftg_history_restore(self.plan.handle, self.handle, C.c_void_p(ptr), size))


class Batch:
    """fftg_batch_create / fftg_batch_solve_increment over (plan, history) pairs."""

    def __init__(self, plans: Sequence[Plan], hists: Sequence[History]):
        self.plans, self.hists = list(plans), list(hists)
        n = len(plans)
        P = (C.c_void_p * n)(*[p.handle for p in plans])
        H = (C.c_void_p * n)(*[h.handle for h in hists])
        h = C.c_void_p()
        check(lib().fftg_batch_create(C.byref(h), n, P, H))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().fftg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve_increment(self, dE: np.ndarray, raise_on_error=True):
        n = len(self.plans)
        d = np.ascontiguousarray(dE, dtype=np.float64).reshape(n, 6)
        arr = (C.c_double * (6 * n))(*d.ravel().tolist())
        st = (fftg_stats * n)()
        code = lib().fftg_batch_solve_increment(self.handle, arr, st)
        if raise_on_error:
            check(code)
        out = [s.to_dict() for s in st]
        for o in out:
            o["status"] = code
        return out


def tensor6(E: np.ndarray) -> List[float]:
    """3x3 symmetric tensor -> ABI 6-vector [11, 22, 33, 23, 13, 12]."""
    E = np.asarray(E, dtype=float)
    return [E[0, 0], E[1, 1], E[2, 2], E[1, 2], E[0, 2], E[0, 1]]
