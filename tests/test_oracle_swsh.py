"""Pins for the oracle's spin-weighted spherical harmonics -2Y_lm.

The paper names the harmonics (Sec. III D; Sec. IV, Schwarzschild limit of
S_lmkn e^{i m phi}) but prints no formula or values.  The convention is fixed
here by the standard l = 2 closed forms, and the implementation is pinned by
normalisation, orthogonality and the conjugation/parity identities that any
correct spin-weighted harmonic satisfies.
"""
import math

import numpy as np
import pytest

import oracle


def y2_closed(m, theta, phi):
    c, s = math.cos(theta), math.sin(theta)
    if m == 2:
        v = math.sqrt(5 / (64 * math.pi)) * (1 + c) ** 2
    elif m == -2:
        v = math.sqrt(5 / (64 * math.pi)) * (1 - c) ** 2
    elif m == 1:
        v = math.sqrt(5 / (16 * math.pi)) * s * (1 + c)
    elif m == -1:
        v = math.sqrt(5 / (16 * math.pi)) * s * (1 - c)
    else:
        v = math.sqrt(15 / (32 * math.pi)) * s * s
    return v * complex(math.cos(m * phi), math.sin(m * phi))


@pytest.mark.parametrize("m", [-2, -1, 0, 1, 2])
def test_l2_closed_forms(m):
    rng = np.random.default_rng(7 + m)
    for _ in range(25):
        th = math.acos(rng.uniform(-1, 1))
        ph = rng.uniform(0, 2 * math.pi)
        got = oracle.swsh(-2, 2, m, th, ph)
        ref = y2_closed(m, th, ph)
        assert abs(got - ref) <= 1e-15


def _grid(nt=48, nph=64):
    x, w = np.polynomial.legendre.leggauss(nt)
    th = np.arccos(x)
    ph = np.arange(nph) * (2 * math.pi / nph)
    return th, w, ph


def _table(s, l, m, th, ph):
    return np.array([[oracle.swsh(s, l, m, a, b) for b in ph] for a in th])


@pytest.mark.parametrize("l,m", [(2, 2), (3, -1), (5, 0), (7, 4), (10, 10), (10, -7)])
def test_unit_norm(l, m):
    th, w, ph = _grid()
    Y = _table(-2, l, m, th, ph)
    integral = np.sum(w[:, None] * np.abs(Y) ** 2) * (2 * math.pi / len(ph))
    assert abs(integral - 1.0) < 1e-13


@pytest.mark.parametrize("m", [0, 2, -1])
def test_orthogonal_in_l(m):
    th, w, ph = _grid()
    ls = [l for l in range(2, 8) if l >= abs(m)]
    tabs = {l: _table(-2, l, m, th, ph) for l in ls}
    for a in ls:
        for b in ls:
            ip = np.sum(w[:, None] * np.conj(tabs[a]) * tabs[b]) * (2 * math.pi / len(ph))
            assert abs(ip - (1.0 if a == b else 0.0)) < 1e-13


@pytest.mark.parametrize("l", [2, 3, 6, 10])
def test_conjugation_identity(l):
    """conj(sY_lm) = (-1)^{s+m} (-s)Y_{l,-m}."""
    rng = np.random.default_rng(l)
    for _ in range(10):
        th = math.acos(rng.uniform(-1, 1))
        ph = rng.uniform(0, 2 * math.pi)
        for m in range(-l, l + 1):
            a = np.conj(oracle.swsh(-2, l, m, th, ph))
            b = (-1) ** ((-2 + m) % 2) * oracle.swsh(2, l, -m, th, ph)
            assert abs(a - b) < 1e-14


@pytest.mark.parametrize("l", [2, 3, 4, 9])
def test_parity_identity(l):
    """sY_lm(pi - theta, phi + pi) = (-1)^l (-s)Y_lm(theta, phi)."""
    rng = np.random.default_rng(50 + l)
    for _ in range(10):
        th = math.acos(rng.uniform(-1, 1))
        ph = rng.uniform(0, 2 * math.pi)
        for m in range(-l, l + 1):
            a = oracle.swsh(-2, l, m, math.pi - th, ph + math.pi)
            b = (-1) ** (l % 2) * oracle.swsh(2, l, m, th, ph)
            assert abs(a - b) < 1e-14


@pytest.mark.parametrize("l", [2, 3, 7, 10])
def test_pole_selects_m_equal_minus_s(l):
    """At theta = 0 only m = -s = 2 survives, with |Y| = sqrt((2l+1)/4pi)."""
    for m in range(-l, l + 1):
        v = oracle.swsh(-2, l, m, 0.0, 0.3)
        if m == 2:
            assert abs(abs(v) - math.sqrt((2 * l + 1) / (4 * math.pi))) < 1e-14
        else:
            assert abs(v) == 0.0


def _mp_swsh(s, l, m, theta, phi, dps=60):
    """sY_lm from Goldberg's sum evaluated with dps decimal digits."""
    import mpmath as mp
    with mp.workdps(dps):
        t = mp.mpf(theta)
        sh, ch = mp.sin(t / 2), mp.cos(t / 2)
        pref = (-1) ** m * mp.sqrt(mp.factorial(l + m) * mp.factorial(l - m) * (2 * l + 1) /
                                   (4 * mp.pi * mp.factorial(l + s) * mp.factorial(l - s)))
        tot = mp.mpf(0)
        for r in range(0, l - s + 1):
            j = r + s - m
            if j < 0 or j > l + s:
                continue
            k = 2 * r + s - m
            tot += mp.binomial(l - s, r) * mp.binomial(l + s, j) * sh ** (2 * l - k) * ch ** k * \
                (-1) ** (l - r - s)
        v = pref * tot * mp.expj(m * mp.mpf(phi))
        return complex(v)


@pytest.mark.parametrize("l", [12, 20, 26, 30])
def test_high_l_against_60_digit_sum(l):
    """The accepted range goes to l = 30, where the alternating sum cancels
    heavily: every -2Y_lm must still be accurate to 1e-14 of its magnitude
    scale (the largest |Y| over m at that l and angle)."""
    for theta in (0.3, 1.1, 2.4):
        vals = {m: (oracle.swsh(-2, l, m, theta, 0.7), _mp_swsh(-2, l, m, theta, 0.7))
                for m in range(-l, l + 1)}
        scale = max(abs(r) for _, r in vals.values())
        for m, (got, ref) in vals.items():
            assert abs(got - ref) <= 1e-14 * scale, (l, m, theta, got, ref)
