"""ctypes binding of libfew (include/few.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  torch tensors provide device memory; the plan borrows the HIP
stream of ``torch.cuda.current_stream()`` unless one is given.  If the
library is not built, importing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# FEW_LIBRARY selects another build of the same library (the host-sanitizer
# build of build.py), never a different implementation.
LIB_PATH = os.environ.get("FEW_LIBRARY") or os.path.join(HERE, "libfew.so")

FEW_OK = 0
FEW_PENDING = 1
FEW_E_ARG = -1
FEW_E_KNOTS = -2
FEW_E_MODES = -3
FEW_E_RANGE = -4
FEW_E_TOO_LARGE = -5
FEW_E_NOMEM = -6
FEW_E_HIP = -7
FEW_E_STATE = -8
FEW_FP64 = 0
FEW_MIXED = 1
FEW_FLAG_TIMING = 1
FEW_FLAG_TIMING_SUM = 2
FEW_FLAG_VECTOR_ONLY = 4
FEW_FLAG_SELECT_SORTED = 8
FEW_FLAG_TIMING_SPARSE = 16

EXPORTED = [
    "few_plan_create", "few_plan_destroy", "few_spline_fit", "few_spline_free",
    "few_spline_coefs", "few_mode_sum", "few_mode_select", "few_batch", "few_submit",
    "few_poll", "few_wait", "few_plan_log",
    "few_plan_timing", "few_last_error", "few_host_terms", "few_host_interval_starts",
    "few_spline_fit_kerr", "few_host_terms_kerr", "few_inner_product", "few_mode_sum_ssb",
    "few_host_frame",
    "few_host_request_bytes", "few_inner_product_noalloc", "few_host_mfma_path",
    "few_host_mfma_shape", "few_host_xcd_split_step",
]


class FewError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libfew status {code}: {msg}")
        self.code = code


class PlanDesc(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("precision", ctypes.c_int32), ("max_knots", ctypes.c_int32),
                ("max_modes", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("flags", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("n_knots", ctypes.c_int32), ("t_knots", ctypes.c_void_p),
                ("phi_phi", ctypes.c_void_p), ("phi_r", ctypes.c_void_p),
                ("n_modes", ctypes.c_int32), ("lmn", ctypes.c_void_p),
                ("amp", ctypes.c_void_p), ("theta", ctypes.c_double),
                ("phi", ctypes.c_double), ("scale", ctypes.c_double),
                ("t_start", ctypes.c_double), ("dt", ctypes.c_double),
                ("n_samples", ctypes.c_int64), ("out", ctypes.c_void_p)]


class Timing(ctypes.Structure):
    _fields_ = [("spline_ms", ctypes.c_double), ("spline_launches", ctypes.c_int64),
                ("prepare_ms", ctypes.c_double), ("prepare_launches", ctypes.c_int64),
                ("sum_ms", ctypes.c_double), ("sum_launches", ctypes.c_int64)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libfew.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch ships its own HIP runtime with the same soname (libamdhip64.so.7).
    # Loading torch first makes libfew bind to that already-loaded runtime, so
    # both share one HIP context and torch's device memory and streams are
    # valid in libfew.  A second runtime instance in the process would not see
    # the device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    lib.few_plan_create.argtypes = [P(PlanDesc), P(vp)]
    lib.few_plan_destroy.argtypes = [vp]
    lib.few_spline_fit.argtypes = [vp, i32, vp, vp, vp, i32, vp, vp, P(vp)]
    lib.few_spline_fit_kerr.argtypes = [vp, i32, vp, vp, vp, vp, i32, vp, vp, P(vp)]
    lib.few_spline_free.argtypes = [vp]
    lib.few_spline_coefs.argtypes = [vp, i32, vp]
    lib.few_mode_sum.argtypes = [vp, vp, dbl, dbl, dbl, dbl, dbl, i64, vp]
    lib.few_inner_product.argtypes = [vp, vp, dbl, dbl, dbl, dbl, dbl, i64, vp, vp]
    lib.few_inner_product_noalloc.argtypes = [vp, vp, dbl, dbl, dbl, dbl, dbl, i64, vp, vp]
    lib.few_mode_sum_ssb.argtypes = [vp, vp, dbl, dbl, dbl, dbl, dbl, dbl, dbl, i64, vp]
    lib.few_host_frame.argtypes = [dbl, dbl, dbl, dbl, vp]
    lib.few_batch.argtypes = [vp, i32, P(Request)]
    lib.few_mode_select.argtypes = [vp, i32, i32, vp, dbl, vp]
    lib.few_submit.argtypes = [vp, P(Request), P(ctypes.c_uint64)]
    lib.few_poll.argtypes = [vp, ctypes.c_uint64]
    lib.few_wait.argtypes = [vp, ctypes.c_uint64]
    lib.few_plan_log.argtypes = [vp, ctypes.c_char_p]
    lib.few_plan_timing.argtypes = [vp, P(Timing), i32]
    lib.few_last_error.argtypes = []
    lib.few_last_error.restype = ctypes.c_char_p
    lib.few_host_terms.argtypes = [i32, vp, i32, i32, vp, P(i32), i32, vp, P(i32), i32, vp,
                                   P(i32)]
    lib.few_host_terms_kerr.argtypes = [i32, vp, i32, i32, vp, P(i32), i32, vp, P(i32), i32,
                                        vp, P(i32)]
    lib.few_host_interval_starts.argtypes = [i32, vp, dbl, dbl, i64, vp]
    lib.few_host_request_bytes.argtypes = [i32, i32, i32, i32]
    lib.few_host_mfma_path.argtypes = [i32, vp]
    lib.few_host_mfma_shape.argtypes = [vp]
    lib.few_host_xcd_split_step.argtypes = [vp, vp, vp]
    lib.few_host_request_bytes.restype = ctypes.c_uint64
    for name in EXPORTED:
        f = getattr(lib, name)
        if f.restype is None or f.restype is ctypes.c_int:
            f.restype = ctypes.c_int32
    lib.few_last_error.restype = ctypes.c_char_p
    lib.few_host_request_bytes.restype = ctypes.c_uint64
    lib.few_host_mfma_shape.restype = None
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        raise FewError(rc, load().few_last_error().decode(errors="replace"))
    return rc


def _host_f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _host_i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _dev_ptr(t, dtype=None, shape=None, name="tensor") -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


class Spline:
    """A fitted spline resident in the plan arena (few_spline)."""

    def __init__(self, plan: "Plan", handle: int, K: int, M: int, keep, n_phases: int = 2):
        self.plan, self.handle, self.K, self.M = plan, handle, K, M
        self.n_phases = n_phases
        self._keep = keep          # inputs stay alive until the fit has run

    def coefs(self, which: int):
        """Device copy of the coefficients (0: amplitudes [K-1,M,4,2]; 1: phases
        [K-1,P,4,2] with P = 2, or 3 for generic-Kerr splines)."""
        import torch
        shape = (self.K - 1, self.M, 4, 2) if which == 0 else (self.K - 1, self.n_phases, 4, 2)
        out = torch.empty(shape, dtype=torch.float64, device=f"cuda:{self.plan.device}")
        _check(load().few_spline_coefs(self.handle, which, out.data_ptr()))
        return out

    def free(self) -> None:
        if self.handle:
            _check(load().few_spline_free(self.handle))
            self.handle = None


class Plan:
    """few_plan: device arena, precision, stream and the request server.

    timing: False, True (HIP events around every launch, FEW_FLAG_TIMING),
    "sum" (around summation launches only, FEW_FLAG_TIMING_SUM) or "sum_sparse"
    (around every 8th summation launch, FEW_FLAG_TIMING_SUM | _SPARSE).
    vector_only: mixed precision without the matrix-core summation
    (FEW_FLAG_VECTOR_ONLY).
    select_sorted: the mode selector sorts every knot (FEW_FLAG_SELECT_SORTED)."""

    def __init__(self, device: int = 0, precision: str = "fp64", stream: Optional[int] = None,
                 hbm_budget_bytes: int = 0, max_inflight: int = 0, timing=False,
                 max_knots: int = 0, max_modes: int = 0, vector_only: bool = False,
                 select_sorted: bool = False):
        import torch
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        self.device = device
        self.precision = precision
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.stream = stream
        d = PlanDesc(device=device, stream=stream,
                     precision=FEW_MIXED if precision == "mixed" else FEW_FP64,
                     max_knots=max_knots, max_modes=max_modes, max_inflight=max_inflight,
                     hbm_budget_bytes=hbm_budget_bytes,
                     flags=(FEW_FLAG_TIMING_SUM if timing == "sum"
                            else FEW_FLAG_TIMING_SUM | FEW_FLAG_TIMING_SPARSE
                            if timing == "sum_sparse"
                            else FEW_FLAG_TIMING if timing else 0)
                     | (FEW_FLAG_VECTOR_ONLY if vector_only else 0)
                     | (FEW_FLAG_SELECT_SORTED if select_sorted else 0))
        h = ctypes.c_void_p()
        _check(load().few_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h.value
        self._inflight = {}

    @property
    def out_dtype(self):
        import torch
        return torch.complex64 if self.precision == "mixed" else torch.complex128

    def close(self) -> None:
        if self.handle:
            _check(load().few_plan_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def spline_fit(self, t_knots, phi_phi, phi_r, lmn, amp) -> Spline:
        import torch
        t = _host_f64(t_knots)
        lm = _host_i32(lmn).reshape(-1, 3)
        K, M = t.shape[0], lm.shape[0]
        pp = _dev_ptr(phi_phi, torch.float64, (K,), "phi_phi")
        pr = _dev_ptr(phi_r, torch.float64, (K,), "phi_r")
        ap = _dev_ptr(amp, torch.float64, (K, M, 2), "amp")
        h = ctypes.c_void_p()
        _check(load().few_spline_fit(self.handle, K, t.ctypes.data, pp, pr, M, lm.ctypes.data,
                                     ap, ctypes.byref(h)))
        return Spline(self, h.value, K, M, (phi_phi, phi_r, amp))

    def spline_fit_kerr(self, t_knots, phi_phi, phi_theta, phi_r, lmkn, amp) -> "Spline":
        """few_spline_fit_kerr: modes lmkn [M, 4] = (l, m, k, n), three phases."""
        import torch
        t = _host_f64(t_knots)
        lm = _host_i32(lmkn).reshape(-1, 4)
        K, M = t.shape[0], lm.shape[0]
        pp = _dev_ptr(phi_phi, torch.float64, (K,), "phi_phi")
        pt = _dev_ptr(phi_theta, torch.float64, (K,), "phi_theta")
        pr = _dev_ptr(phi_r, torch.float64, (K,), "phi_r")
        ap = _dev_ptr(amp, torch.float64, (K, M, 2), "amp")
        h = ctypes.c_void_p()
        _check(load().few_spline_fit_kerr(self.handle, K, t.ctypes.data, pp, pt, pr, M,
                                          lm.ctypes.data, ap, ctypes.byref(h)))
        return Spline(self, h.value, K, M, (phi_phi, phi_theta, phi_r, amp), n_phases=3)

    def mode_sum(self, spline: Spline, theta: float, phi: float, dt: float, n_samples: int,
                 out=None, t_start: float = 0.0, scale: float = 1.0):
        import torch
        if out is None:
            out = torch.empty(n_samples, dtype=self.out_dtype, device=f"cuda:{self.device}")
        op = _dev_ptr(out, self.out_dtype, (n_samples,), "out")
        _check(load().few_mode_sum(self.handle, spline.handle, float(theta), float(phi),
                                   float(scale), float(t_start), float(dt), int(n_samples), op))
        return out

    def mode_sum_ssb(self, spline: "Spline", theta_s: float, phi_s: float, theta_k: float,
                     phi_k: float, dt: float, n_samples: int, out=None, t_start: float = 0.0,
                     scale: float = 1.0):
        """few_mode_sum_ssb: the waveform in the barycentre frame for sky position
        (theta_s, phi_s) and spin direction (theta_k, phi_k)."""
        import torch
        if out is None:
            out = torch.empty(n_samples, dtype=self.out_dtype, device=f"cuda:{self.device}")
        op = _dev_ptr(out, self.out_dtype, (n_samples,), "out")
        _check(load().few_mode_sum_ssb(self.handle, spline.handle, float(theta_s), float(phi_s),
                                       float(theta_k), float(phi_k), float(scale),
                                       float(t_start), float(dt), int(n_samples), op))
        return out

    def inner_product(self, spline: "Spline", theta: float, phi: float, dt: float,
                      n_samples: int, data, out2=None, t_start: float = 0.0,
                      scale: float = 1.0):
        """few_inner_product: device float64 [2] = (<d|h>, <h|h>) with a unit PSD."""
        import torch
        dp = _dev_ptr(data, self.out_dtype, (n_samples,), "data")
        if out2 is None:
            out2 = torch.empty(2, dtype=torch.float64, device=f"cuda:{self.device}")
        op = _dev_ptr(out2, torch.float64, (2,), "out2")
        _check(load().few_inner_product(self.handle, spline.handle, float(theta), float(phi),
                                        float(scale), float(t_start), float(dt),
                                        int(n_samples), dp, op))
        return out2

    def _request(self, t_knots, phi_phi, phi_r, lmn, amp, theta, phi, dt, n_samples, out,
                 t_start: float = 0.0, scale: float = 1.0):
        import torch
        t = _host_f64(t_knots)
        lm = _host_i32(lmn).reshape(-1, 3)
        K, M = t.shape[0], lm.shape[0]
        r = Request(n_knots=K, t_knots=t.ctypes.data,
                    phi_phi=_dev_ptr(phi_phi, torch.float64, (K,), "phi_phi"),
                    phi_r=_dev_ptr(phi_r, torch.float64, (K,), "phi_r"),
                    n_modes=M, lmn=lm.ctypes.data,
                    amp=_dev_ptr(amp, torch.float64, (K, M, 2), "amp"),
                    theta=float(theta), phi=float(phi), scale=float(scale),
                    t_start=float(t_start), dt=float(dt), n_samples=int(n_samples),
                    out=_dev_ptr(out, self.out_dtype, (n_samples,), "out"))
        return r, (t, lm)

    def mode_select(self, amp, eps: float, keep=None):
        """few_mode_select: int32 device mask [M] of the modes kept at any knot."""
        import torch
        if amp.dim() != 3 or amp.shape[2] != 2:
            raise ValueError("amp must have shape [K, M, 2]")
        K, M = int(amp.shape[0]), int(amp.shape[1])
        ap = _dev_ptr(amp, torch.float64, (K, M, 2), "amp")
        if keep is None:
            keep = torch.empty(M, dtype=torch.int32, device=amp.device)
        kp = _dev_ptr(keep, torch.int32, (M,), "keep")
        _check(load().few_mode_select(self.handle, K, M, ap, float(eps), kp))
        return keep

    def batch(self, requests) -> None:
        """few_batch: each item is a dict of submit() keyword arguments."""
        built = [self._request(**q) for q in requests]
        arr = (Request * len(built))(*[b[0] for b in built])
        _check(load().few_batch(self.handle, len(built), arr))

    def submit(self, t_knots, phi_phi, phi_r, lmn, amp, theta, phi, dt, n_samples, out,
               t_start: float = 0.0, scale: float = 1.0) -> int:
        r, keep = self._request(t_knots, phi_phi, phi_r, lmn, amp, theta, phi, dt, n_samples,
                                out, t_start, scale)
        tk = ctypes.c_uint64()
        _check(load().few_submit(self.handle, ctypes.byref(r), ctypes.byref(tk)))
        self._inflight[tk.value] = (phi_phi, phi_r, amp, out)
        return tk.value

    def poll(self, ticket: int) -> bool:
        rc = load().few_poll(self.handle, ctypes.c_uint64(ticket))
        if rc == FEW_PENDING:
            return False
        self._inflight.pop(ticket, None)
        _check(rc)
        return True

    def wait(self, ticket: int) -> None:
        rc = load().few_wait(self.handle, ctypes.c_uint64(ticket))
        self._inflight.pop(ticket, None)
        _check(rc)

    def request_log(self, path) -> None:
        """few_plan_log: append one JSON line per retired served request to
        `path` (None stops logging)."""
        _check(load().few_plan_log(self.handle, None if path is None else os.fsencode(path)))

    def timing(self, reset: bool = False) -> dict:
        t = Timing()
        _check(load().few_plan_timing(self.handle, ctypes.byref(t), int(reset)))
        return {k: getattr(t, k) for k, _ in Timing._fields_}


def host_terms(lmn, max_gap: int = 4):
    """Folded term layout (few_host_terms, or few_host_terms_kerr for modes
    [M, 4] = (l, m, k, n)): (segs [S,4], term_ptr [T+1], term_src [E,2])."""
    lm = _host_i32(lmn)
    width = 4 if lm.ndim == 2 and lm.shape[1] == 4 else 3
    lm = lm.reshape(-1, width)
    M = lm.shape[0]
    cap_segs = 2 * M + 64
    cap_terms = 2 * M * (max_gap + 1) + 64
    segs = np.zeros(4 * cap_segs, dtype=np.int32)
    tp = np.zeros(cap_terms + 1, dtype=np.int32)
    src = np.zeros(2 * (2 * M + 1), dtype=np.int32)
    ns, nt, ne = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    fn = load().few_host_terms_kerr if width == 4 else load().few_host_terms
    _check(fn(M, lm.ctypes.data, max_gap, cap_segs, segs.ctypes.data, ctypes.byref(ns),
              cap_terms + 1, tp.ctypes.data, ctypes.byref(nt), 2 * M + 1, src.ctypes.data,
              ctypes.byref(ne)))
    return (segs[:4 * ns.value].reshape(-1, 4).copy(), tp[:nt.value + 1].copy(),
            src[:2 * ne.value].reshape(-1, 2).copy())


def host_frame(theta_s: float, phi_s: float, theta_k: float, phi_k: float):
    """few_host_frame: (theta, phi, complex factor) of the detector-frame step."""
    out = np.zeros(4, dtype=np.float64)
    _check(load().few_host_frame(float(theta_s), float(phi_s), float(theta_k), float(phi_k),
                                 out.ctypes.data))
    return float(out[0]), float(out[1]), complex(out[2], out[3])


def host_interval_starts(t_knots, t_start: float, dt: float, n: int) -> np.ndarray:
    t = _host_f64(t_knots)
    out = np.zeros(t.shape[0], dtype=np.int64)
    _check(load().few_host_interval_starts(t.shape[0], t.ctypes.data, float(t_start),
                                           float(dt), int(n), out.ctypes.data))
    return out


def host_request_bytes(precision: str, K: int, M: int, n_terms: int) -> int:
    return int(load().few_host_request_bytes(FEW_MIXED if precision == "mixed" else FEW_FP64,
                                             K, M, n_terms))


def host_mfma_path(lmn) -> bool:
    """few_host_mfma_path: whether a binary32 request with this (l, m, n) list
    is summed on the matrix cores."""
    lm = _host_i32(lmn).reshape(-1, 3)
    return bool(_check(load().few_host_mfma_path(lm.shape[0], lm.ctypes.data)))


def host_xcd_split_step(w_prev, times) -> np.ndarray:
    """few_host_xcd_split_step: the next XCD weights of the matrix-core
    summation from the weights and per-XCD finishing times of a launch."""
    wp = np.ascontiguousarray(w_prev, dtype=np.float64).reshape(8)
    tm = np.ascontiguousarray(times, dtype=np.float64).reshape(8)
    out = np.zeros(8, dtype=np.float64)
    _check(load().few_host_xcd_split_step(wp.ctypes.data, tm.ctypes.data, out.ctypes.data))
    return out


def host_mfma_shape() -> dict:
    """few_host_mfma_shape: launch shape of the matrix-core summation."""
    out = np.zeros(8, dtype=np.int32)
    load().few_host_mfma_shape(out.ctypes.data)
    keys = ("waves", "tiles_per_wave", "row_tiles", "column_steps", "mfma_per_tile",
            "abs_n_limit", "max_rows", "min_terms")
    return dict(zip(keys, (int(v) for v in out)))
