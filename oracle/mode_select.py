"""Oracle of the mode selector (paper Sec. III D) -- test infrastructure only.

At every knot k the power of each listed mode is |A_lmn(t_k)|^2, computed as
re*re + im*im in binary64 (two roundings, no fused multiply-add).  The modes
are ordered by decreasing power (ties by increasing mode index), the powers are
summed sequentially in that order, and the total P_k is the last partial sum.
A mode is kept at knot k when the partial sum before it is still below
(1 - eps) P_k, i.e. the kept modes are the shortest prefix whose power reaches
(1 - eps) of the knot's total (the top mode is always kept).  The selected set
is the union over knots.

Reading of the paper (which describes the steps but no formula): "the
additional power contributed by a mode falls below the threshold" is read as
the remaining power after the prefix being at most eps of the total; the power
of a mode is |A|^2 of the listed (m >= 0) mode.
"""
from __future__ import annotations

import numpy as np


def knot_powers(amp: np.ndarray) -> np.ndarray:
    """|A|^2 per knot and mode from the knot-major [K, M, 2] array."""
    amp = np.asarray(amp, dtype=np.float64)
    re = amp[:, :, 0]
    im = amp[:, :, 1]
    return re * re + im * im


def select_at_knot(p: np.ndarray, eps: float) -> np.ndarray:
    """Mode indices kept at one knot (see module docstring)."""
    p = np.asarray(p, dtype=np.float64)
    order = np.lexsort((np.arange(p.size), -p))       # power desc, index asc
    c = np.add.accumulate(p[order])                   # sequential partial sums
    thr = (1.0 - eps) * c[-1]
    before = np.concatenate([[0.0], c[:-1]])
    return order[before < thr] if c[-1] > 0.0 else order[:1]


def mode_select(amp: np.ndarray, eps: float) -> np.ndarray:
    """int32 mask [M]: 1 where the mode is kept at any knot."""
    p = knot_powers(amp)
    mask = np.zeros(p.shape[1], dtype=np.int32)
    for k in range(p.shape[0]):
        mask[select_at_knot(p[k], eps)] = 1
    return mask
