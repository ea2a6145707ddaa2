"""Error metrics used to compare a waveform with the oracle's.

Mismatch follows Sec. VI (Eqs. (16)-(17)) with the PSD set to 1, as the paper
does for its mismatch studies: the noise-weighted inner product becomes, by
Parseval, the plain sum over time samples of both polarisations, so
    overlap(a, b) = Re sum_j conj(a_j) b_j / (||a|| ||b||),
    mismatch = 1 - overlap,
with no maximisation over time or phase shifts.

Max relative error is max_j |a_j - b_j| / max_j |b_j| (a pointwise ratio is
ill-posed at zeros of h).

inner_flat is the noise-weighted inner product of Sec. VI with S_n = 1,
4 Re int_0^inf conj(a~(f)) b~(f) df summed over both polarisations, which for
sampled h = h_plus - i h_cross is exactly 2 dt Re sum_j conj(a_j) b_j
(discrete Parseval, DC and Nyquist bins counted once).
"""
from __future__ import annotations

import numpy as np


def mismatch(a: np.ndarray, b: np.ndarray) -> float:
    a = np.asarray(a, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    num = np.real(np.vdot(a, b))
    den = np.sqrt(np.real(np.vdot(a, a)) * np.real(np.vdot(b, b)))
    if den == 0.0:
        return 0.0 if np.array_equal(a, b) else 1.0
    return float(1.0 - num / den)


def max_rel_error(a: np.ndarray, ref: np.ndarray) -> float:
    a = np.asarray(a, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    scale = np.max(np.abs(ref)) if ref.size else 0.0
    if scale == 0.0:
        return float(np.max(np.abs(a))) if a.size else 0.0
    return float(np.max(np.abs(a - ref)) / scale)


def inner_flat(a: np.ndarray, b: np.ndarray, dt: float) -> float:
    """<a|b> with a unit PSD: 2 dt Re sum_j conj(a_j) b_j (see module docstring)."""
    a = np.asarray(a, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    return float(2.0 * dt * np.real(np.vdot(a, b)))
