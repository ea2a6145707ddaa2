"""ctypes wrapper over the plain-C oracle (few_oracle.c).

Test infrastructure only.  Functions follow the paper's Sec. III C (spline
and interpolated summation), Sec. III D / Sec. IV (spin-weighted spherical
harmonics) and Eqs. (9)-(10); see the C source for the arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "few_oracle.c")
ORACLE_SO = os.path.join(HERE, "liboracle.so")

_lib = None


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary64 sample times, no FMA contraction)."""
    if force or not os.path.exists(ORACLE_SO):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", ORACLE_SO + ".tmp", SRC, "-lquadmath", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(ORACLE_SO + ".tmp", ORACLE_SO)
    return ORACLE_SO


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(ORACLE_SO):
            build()
        lib = ctypes.CDLL(ORACLE_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.few_oracle_spline.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, dp]
        lib.few_oracle_spline.restype = ctypes.c_int
        lib.few_oracle_swsh.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_double, dp, dp]
        lib.few_oracle_swsh.restype = ctypes.c_int
        lib.few_oracle_phase.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int64, dp, dp]
        lib.few_oracle_phase.restype = ctypes.c_int
        lib.few_oracle_sum.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int, i32p, dp,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                       i64p, ctypes.c_int64, dp, ctypes.c_int]
        lib.few_oracle_sum.restype = ctypes.c_int
        lib.few_oracle_sum_kerr.argtypes = [ctypes.c_int, dp, dp, dp, dp, ctypes.c_int, i32p,
                                            dp, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_int64, i64p,
                                            ctypes.c_int64, dp, ctypes.c_int]
        lib.few_oracle_sum_kerr.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def spline_coefs(t: Sequence[float], y: np.ndarray) -> np.ndarray:
    """Not-a-knot cubic coefficients.  y: [K] or [K, S] (knot-major).

    Returns [K-1, S, 4] (or [K-1, 4] for 1-D y), coefficient of (t - t_i)^p.
    """
    t = _f64(t)
    y = _f64(y)
    one = y.ndim == 1
    y2 = y.reshape(y.shape[0], -1)
    K, S = y2.shape
    out = np.empty((max(K - 1, 1), S, 4), dtype=np.float64)
    _check(load().few_oracle_spline(K, _dp(t), S, _dp(y2), _dp(out)), "spline")
    return out[:, 0, :] if one else out


def swsh(s: int, l: int, m: int, theta: float, phi: float) -> complex:
    """Spin-weighted spherical harmonic sY_lm(theta, phi)."""
    re = ctypes.c_double()
    im = ctypes.c_double()
    _check(load().few_oracle_swsh(s, l, m, theta, phi, ctypes.byref(re), ctypes.byref(im)),
           "swsh")
    return complex(re.value, im.value)


def phase(t: Sequence[float], y: Sequence[float], tq: Sequence[float]) -> np.ndarray:
    """Spline phase at tq, reduced to [-pi, pi)."""
    t = _f64(t)
    y = _f64(y)
    tq = _f64(tq)
    out = np.empty_like(tq)
    _check(load().few_oracle_phase(t.shape[0], _dp(t), _dp(y), tq.shape[0], _dp(tq),
                                   _dp(out)), "phase")
    return out


def mode_sum(t_knots, phi_phi, phi_r, lmn, amp, theta, phi, dt, n_samples,
             t_start: float = 0.0, scale: float = 1.0,
             idx: Optional[np.ndarray] = None, n_threads: Optional[int] = None,
             phi_theta=None) -> np.ndarray:
    """h = h_plus - i h_cross at the samples (all, or the indices idx).

    amp: [K, M, 2] knot-major (re, im); lmn: [M, 3] (l, m, n), or [M, 4]
    (l, m, k, n) for the generic-Kerr sum, which also needs phi_theta [K].
    Returns complex128.
    """
    t = _f64(t_knots)
    pp = _f64(phi_phi)
    pr = _f64(phi_r)
    lmn = np.ascontiguousarray(np.asarray(lmn, dtype=np.int32))
    amp = _f64(amp)
    K = t.shape[0]
    M = lmn.shape[0]
    kerr = lmn.ndim == 2 and lmn.shape[1] == 4
    if kerr and phi_theta is None:
        raise OracleError("the (l, m, k, n) sum needs phi_theta")
    if amp.shape != (K, M, 2):
        raise OracleError(f"amp shape {amp.shape} != {(K, M, 2)}")
    if idx is not None:
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
        n_out = idx.shape[0]
        ip = idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    else:
        n_out = int(n_samples)
        ip = None
    out = np.empty(2 * n_out, dtype=np.float64)
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    mp = lmn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    if kerr:
        pt = _f64(phi_theta)
        rc = load().few_oracle_sum_kerr(K, _dp(t), _dp(pp), _dp(pt), _dp(pr), M, mp,
                                        _dp(amp), float(theta), float(phi), float(scale),
                                        float(t_start), float(dt), int(n_samples), ip, n_out,
                                        _dp(out), int(n_threads))
    else:
        rc = load().few_oracle_sum(K, _dp(t), _dp(pp), _dp(pr), M, mp,
                                   _dp(amp), float(theta), float(phi), float(scale),
                                   float(t_start), float(dt), int(n_samples), ip, n_out,
                                   _dp(out), int(n_threads))
    _check(rc, "mode_sum")
    return out.view(np.complex128)


def mode_sum_waveform(w, idx: Optional[np.ndarray] = None,
                      n_threads: Optional[int] = None) -> np.ndarray:
    """Convenience: oracle sum of a synth.Waveform."""
    return mode_sum(w.t_knots, w.phi_phi, w.phi_r, w.lmn, w.amp, w.theta, w.phi, w.dt,
                    w.n_samples, t_start=w.t_start, scale=w.scale, idx=idx,
                    n_threads=n_threads, phi_theta=getattr(w, "phi_theta", None))
