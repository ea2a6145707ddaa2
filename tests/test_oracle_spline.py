"""Pins for the oracle's not-a-knot spline (paper Sec. III C).

Each check fixes the spline by something other than the oracle itself: exact
reproduction of cubics, interpolation and smoothness invariants, SciPy's
not-a-knot CubicSpline, and a brute-force solve of the full piecewise system.
"""
import numpy as np
import pytest
from scipy.interpolate import CubicSpline

import oracle
from paper_2104_04582_amd import synth


def random_knots(rng, K, T=1.0):
    g = rng.uniform(0.2, 1.0, K - 1)
    t = np.concatenate([[0.0], np.cumsum(g)])
    return t / t[-1] * T


def eval_coefs(c, t, tq):
    i = np.clip(np.searchsorted(t, tq, side="right") - 1, 0, len(t) - 2)
    x = tq - t[i]
    cc = c[i]
    return cc[..., 0] + x * (cc[..., 1] + x * (cc[..., 2] + x * cc[..., 3]))


@pytest.mark.parametrize("K", [4, 5, 7, 12, 40, 100])
def test_cubic_reproduced_exactly(K):
    rng = np.random.default_rng(K)
    t = random_knots(rng, K, T=50.0)
    p = rng.standard_normal(4)
    y = p[0] + p[1] * t + p[2] * t ** 2 + p[3] * t ** 3
    c = oracle.spline_coefs(t, y)
    tq = rng.uniform(0, 50.0, 500)
    ref = p[0] + p[1] * tq + p[2] * tq ** 2 + p[3] * tq ** 3
    got = eval_coefs(c, t, tq)
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))
    # every interval's cubic is the global cubic re-centred at t_i
    for i in range(K - 1):
        ti = t[i]
        shifted = [p[0] + p[1] * ti + p[2] * ti ** 2 + p[3] * ti ** 3,
                   p[1] + 2 * p[2] * ti + 3 * p[3] * ti ** 2,
                   p[2] + 3 * p[3] * ti,
                   p[3]]
        np.testing.assert_allclose(c[i], shifted, rtol=1e-9, atol=1e-9 * np.abs(shifted).max())


@pytest.mark.parametrize("K", [4, 6, 13, 40])
def test_interpolates_and_is_smooth(K):
    rng = np.random.default_rng(100 + K)
    t = random_knots(rng, K, T=3.0)
    y = rng.standard_normal((K, 3))
    c = oracle.spline_coefs(t, y)                   # [K-1, 3, 4]
    h = np.diff(t)
    a, b, cc, d = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    np.testing.assert_array_equal(a, y[:-1])        # S(t_i) = y_i exactly
    hh = h[:, None]
    right_val = a + b * hh + cc * hh ** 2 + d * hh ** 3
    right_d1 = b + 2 * cc * hh + 3 * d * hh ** 2
    right_d2 = 2 * cc + 6 * d * hh
    np.testing.assert_allclose(right_val, y[1:], rtol=0, atol=1e-12 * np.abs(y).max())
    scale1 = np.abs(b).max()
    scale2 = np.abs(cc).max()
    np.testing.assert_allclose(right_d1[:-1], b[1:], rtol=0, atol=1e-11 * scale1)
    np.testing.assert_allclose(right_d2[:-1], 2 * cc[1:], rtol=0, atol=1e-11 * scale2)
    # not-a-knot: third derivative continuous at t_1 and t_{K-2}
    scale3 = np.abs(d).max()
    np.testing.assert_allclose(d[0], d[1], rtol=0, atol=1e-10 * scale3)
    np.testing.assert_allclose(d[-1], d[-2], rtol=0, atol=1e-10 * scale3)


@pytest.mark.parametrize("K", [4, 5, 8, 20, 40, 100, 150])
def test_matches_scipy_not_a_knot(K):
    rng = np.random.default_rng(200 + K)
    t = random_knots(rng, K, T=10.0)
    y = rng.standard_normal((K, 4))
    c = oracle.spline_coefs(t, y)
    ref = CubicSpline(t, y, bc_type="not-a-knot").c   # [4, K-1, S], highest power first
    for p in range(4):
        np.testing.assert_allclose(c[:, :, p], ref[3 - p], rtol=1e-9,
                                   atol=1e-11 * np.abs(ref[3 - p]).max())


def brute_force_piecewise(t, y):
    """Solve the full 4(K-1) system: interpolation at both ends of each piece,
    C1 and C2 at interior knots, C3 at t_1 and t_{K-2}."""
    K = len(t)
    P = K - 1
    n = 4 * P
    A = np.zeros((n, n))
    r = np.zeros(n)
    row = 0
    h = np.diff(t)
    for i in range(P):
        A[row, 4 * i] = 1.0; r[row] = y[i]; row += 1
        A[row, 4 * i:4 * i + 4] = [1.0, h[i], h[i] ** 2, h[i] ** 3]; r[row] = y[i + 1]; row += 1
    for i in range(P - 1):
        A[row, 4 * i:4 * i + 4] = [0.0, 1.0, 2 * h[i], 3 * h[i] ** 2]
        A[row, 4 * (i + 1) + 1] = -1.0; row += 1
        A[row, 4 * i:4 * i + 4] = [0.0, 0.0, 2.0, 6 * h[i]]
        A[row, 4 * (i + 1) + 2] = -2.0; row += 1
    A[row, 3] = 1.0; A[row, 7] = -1.0; row += 1
    A[row, 4 * (P - 2) + 3] = 1.0; A[row, 4 * (P - 1) + 3] = -1.0; row += 1
    assert row == n
    return np.linalg.solve(A, r).reshape(P, 4)


@pytest.mark.parametrize("K", [4, 5, 6, 9])
def test_matches_brute_force_piecewise_system(K):
    rng = np.random.default_rng(300 + K)
    t = random_knots(rng, K, T=2.0)
    y = rng.standard_normal(K)
    c = oracle.spline_coefs(t, y)
    ref = brute_force_piecewise(t, y)
    np.testing.assert_allclose(c, ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())


def test_generator_amplitudes_are_reproduced():
    """The synthetic amplitudes are cubics in t/T, so the splined amplitude
    equals the generator polynomial everywhere (config-0 inputs)."""
    w = synth.config0()
    y = w.amp.reshape(w.K, -1)
    c = oracle.spline_coefs(w.t_knots, y)
    tq = np.linspace(0, w.T, 777)
    i = np.clip(np.searchsorted(w.t_knots, tq, side="right") - 1, 0, w.K - 2)
    x = (tq - w.t_knots[i])[:, None]
    cc = c[i]                                            # [Q, S, 4]
    got = cc[..., 0] + x * (cc[..., 1] + x * (cc[..., 2] + x * cc[..., 3]))
    s = tq / w.T
    poly = w.amp_poly                                    # [M, 4, 2]
    ref = np.einsum("q p, m p c -> q m c", np.stack([s ** 0, s, s ** 2, s ** 3], 1), poly)
    np.testing.assert_allclose(got, ref.reshape(len(tq), -1), rtol=0,
                               atol=1e-12 * np.abs(ref).max())


def test_knot_validation():
    t = np.array([0.0, 1.0, 2.0])
    with pytest.raises(oracle.OracleError):
        oracle.spline_coefs(t, np.zeros(3))
    t = np.array([0.0, 1.0, 1.0, 3.0])
    with pytest.raises(oracle.OracleError):
        oracle.spline_coefs(t, np.zeros(4))
    t = np.array([0.0, 2.0, 1.0, 3.0])
    with pytest.raises(oracle.OracleError):
        oracle.spline_coefs(t, np.zeros(4))
