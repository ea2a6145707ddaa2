"""Pins for the mode-selector oracle (paper Sec. III D): the defining
property (the kept prefix carries at least (1 - eps) of each knot's power),
minimality, special values of eps, monotonicity in eps, the union over knots
and the tie order."""
from fractions import Fraction

import numpy as np
import pytest

from oracle.mode_select import knot_powers, mode_select, select_at_knot
from paper_2104_04582_amd import synth


def exact(p):
    return [Fraction(float(v)) for v in p]


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("eps", [1e-9, 1e-4, 0.01, 0.3])
def test_kept_prefix_is_minimal_and_sufficient(seed, eps):
    """Exact arithmetic: kept power >= (1-eps) P, and without the weakest kept
    mode it is below (random inputs keep clear of the rounding boundary)."""
    rng = np.random.default_rng(seed)
    p = rng.exponential(1.0, 40) ** 3
    kept = select_at_knot(p, eps)
    P = sum(exact(p))
    thr = (1 - Fraction(eps)) * P
    kp = sum(exact(p[kept]))
    assert kp >= thr
    if len(kept) > 1:
        weakest = min(kept, key=lambda j: (p[j], -j))
        assert kp - Fraction(float(p[weakest])) < thr
    # kept modes are the top powers
    rest = np.setdiff1d(np.arange(p.size), kept)
    if rest.size:
        assert p[kept].min() >= p[rest].max()


def test_special_eps_values():
    p = np.array([0.0, 3.0, 1.0, 0.0, 2.0])
    assert sorted(select_at_knot(p, 0.0).tolist()) == [1, 2, 4]     # every mode with power
    assert select_at_knot(p, 0.999999).tolist() == [1]               # only the top mode
    assert select_at_knot(np.zeros(4), 0.1).tolist() == [0]          # no power: top (index 0)


def test_ties_break_by_index():
    p = np.array([1.0, 2.0, 2.0, 2.0, 1.0])
    # total 8: (1 - 0.5) * 8 = 4 is reached after two of the three tied modes
    assert select_at_knot(p, 0.5).tolist() == [1, 2]


def test_monotone_in_eps_and_union_over_knots():
    w = synth.config0()
    masks = [mode_select(w.amp, e) for e in (1e-12, 1e-6, 1e-3, 1e-1, 0.9)]
    for a, b in zip(masks, masks[1:]):
        assert np.all(a >= b)
    # union: a mode dominant at a single knot is kept
    amp = np.zeros((3, 5, 2))
    amp[:, 0, 0] = 1.0
    amp[1, 3, 1] = 10.0
    m = mode_select(amp, 0.01)
    assert m.tolist() == [1, 0, 0, 1, 0]


def test_powers_are_squared_magnitudes():
    amp = np.array([[[3.0, 4.0], [0.5, -0.5]]])
    np.testing.assert_array_equal(knot_powers(amp), [[25.0, 0.5]])
