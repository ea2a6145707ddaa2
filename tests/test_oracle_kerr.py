"""Pins for the oracle's generic-Kerr spherical-projected sum (paper Sec. VII,
with the amplitude symmetry A_{l,-m,-k,-n} = (-1)^{l+k} conj(A_lmkn)).

Expected waveforms come from routes that share nothing with the oracle's sum:
closed forms when every spline is exact, an explicit +-m expansion of the mode
list, and a 40-digit mpmath evaluation of the definition on tiny inputs.
"""
import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2104_04582_amd import synth
from tests.test_oracle_sum import _mk_knots, _mp_eval, _mp_spline, sample_times
from tests.test_oracle_swsh import y2_closed


@pytest.mark.parametrize("l,m,k,n", [(2, 2, 1, 0), (2, 1, -2, 3), (2, 0, 3, -1), (3, 2, 1, -1),
                                     (3, 1, 0, 2), (4, 3, -3, 0)])
def test_single_mode_linear_phases_closed_form(l, m, k, n):
    """Constant amplitude and linear phases (every spline exact):
    h = A Y_lm e^{-i psi} + [m>0] (-1)^{l+k} conj(A) Y_{l,-m} e^{+i psi},
    psi = m Phi_phi + k Phi_theta + n Phi_r."""
    K, T, N = 9, 5000.0, 311
    t = _mk_knots(K, T, seed=l * 100 + m * 10 + k)
    wf, wt, wr = 0.013, 0.0117, 0.0091
    pp, pt, pr = wf * t + 0.7, wt * t - 0.3, wr * t - 2.1
    A = complex(0.8, -1.3)
    amp = np.zeros((K, 1, 2))
    amp[:, 0, 0], amp[:, 0, 1] = A.real, A.imag
    th, ph = 1.1, 0.4
    dt = T / N
    got = oracle.mode_sum(t, pp, pr, [[l, m, k, n]], amp, th, ph, dt, N, phi_theta=pt)
    ts = sample_times(0.0, dt, N)
    psi = m * (wf * ts + 0.7) + k * (wt * ts - 0.3) + n * (wr * ts - 2.1)
    Yp = y2_closed(m, th, ph) if l == 2 else oracle.swsh(-2, l, m, th, ph)
    Ym = y2_closed(-m, th, ph) if l == 2 else oracle.swsh(-2, l, -m, th, ph)
    ref = A * Yp * np.exp(-1j * psi)
    if m > 0:
        ref = ref + (-1) ** (l + k) * np.conj(A) * Ym * np.exp(1j * psi)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_k_zero_reduces_to_the_schwarzschild_sum():
    """All k = 0: the polar phase drops out and the result equals the (l, m, n)
    sum for any Phi_theta."""
    w = synth.tiny_waveform(seed=9, K=7, M=9, n_samples=90, l_max=4, n_max=3)
    ref = oracle.mode_sum_waveform(w)
    lmkn = np.insert(w.lmn, 2, 0, axis=1)
    pt = np.cumsum(np.random.default_rng(9).uniform(0, 50, w.K))
    got = oracle.mode_sum(w.t_knots, w.phi_phi, w.phi_r, lmkn, w.amp, w.theta, w.phi, w.dt,
                          w.n_samples, phi_theta=pt)
    np.testing.assert_array_equal(got, ref)


def test_explicit_plus_minus_m_expansion():
    """Listing the m < 0 partners explicitly via A_{l,-m,-k,-n} =
    (-1)^{l+k} conj(A) and summing every signed mode directly equals the
    mirrored sum."""
    w = synth.tiny_kerr(seed=5, K=8, M=9, n_samples=120, l_max=4, k_max=3, n_max=3)
    got = oracle.mode_sum_waveform(w)
    ts = sample_times(w.t_start, w.dt, w.n_samples)
    Phf = oracle.phase(w.t_knots, w.phi_phi, ts)
    Pht = oracle.phase(w.t_knots, w.phi_theta, ts)
    Phr = oracle.phase(w.t_knots, w.phi_r, ts)
    coef = oracle.spline_coefs(w.t_knots, w.amp.reshape(w.K, -1))
    i = np.clip(np.searchsorted(w.t_knots, ts, side="right") - 1, 0, w.K - 2)
    x = (ts - w.t_knots[i])[:, None]
    cc = coef[i]
    vals = cc[..., 0] + x * (cc[..., 1] + x * (cc[..., 2] + x * cc[..., 3]))
    A = vals[:, 0::2] + 1j * vals[:, 1::2]
    ref = np.zeros(w.n_samples, dtype=np.complex128)
    for q, (l, m, k, n) in enumerate(w.lmn):
        signed = [(m, k, n, A[:, q])]
        if m > 0:
            signed.append((-m, -k, -n, (-1) ** (l + k) * np.conj(A[:, q])))
        for mm, kk, nn, Amp in signed:
            ref += Amp * oracle.swsh(-2, l, mm, w.theta, w.phi) * \
                np.exp(-1j * (mm * Phf + kk * Pht + nn * Phr))
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_everything_cubic_matches_direct_evaluation():
    """Cubic amplitudes and three cubic phases: no spline is needed at all."""
    rng = np.random.default_rng(21)
    K, T, N = 12, 3000.0, 201
    t = _mk_knots(K, T, seed=21)
    s = t / T
    pf = np.array([0.3, 40.0, 15.0, -6.0])
    pt_ = np.array([1.2, 33.0, -4.0, 5.0])
    pr_ = np.array([-1.0, 25.0, -3.0, 2.0])
    modes = np.array([[2, 2, 1, 0], [2, 1, -2, -2], [3, 3, 0, 1], [3, 0, 2, 2],
                      [4, 2, -1, -1], [2, 0, 0, 0], [3, 1, 3, -3]], dtype=np.int32)
    M = len(modes)
    poly = rng.standard_normal((M, 4, 2))

    def cubic(p, x):
        return p[0] + p[1] * x + p[2] * x ** 2 + p[3] * x ** 3

    amp = np.empty((K, M, 2))
    for q in range(M):
        for c in range(2):
            amp[:, q, c] = cubic(poly[q, :, c], s)
    th, ph = 0.7, 2.9
    dt = T / N
    got = oracle.mode_sum(t, cubic(pf, s), cubic(pr_, s), modes, amp, th, ph, dt, N,
                          phi_theta=cubic(pt_, s))
    ts = sample_times(0.0, dt, N) / T
    Phf, Pht, Phr = cubic(pf, ts), cubic(pt_, ts), cubic(pr_, ts)
    ref = np.zeros(N, dtype=np.complex128)
    for q, (l, m, k, n) in enumerate(modes):
        A = cubic(poly[q, :, 0], ts) + 1j * cubic(poly[q, :, 1], ts)
        psi = m * Phf + k * Pht + n * Phr
        ref += A * oracle.swsh(-2, l, m, th, ph) * np.exp(-1j * psi)
        if m > 0:
            ref += (-1) ** (l + k) * np.conj(A) * oracle.swsh(-2, l, -m, th, ph) * \
                np.exp(1j * psi)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("seed", [1, 2])
def test_brute_force_mpmath_tiny(seed):
    """Whole definition at 40 digits on tiny inputs (K = 5, M = 6, N = 40)."""
    mp.mp.dps = 40
    w = synth.tiny_kerr(seed=seed, K=5, M=6, n_samples=40, l_max=3, k_max=2, n_max=2,
                        phase_scale=200.0)
    got = oracle.mode_sum_waveform(w)
    t = [mp.mpf(float(v)) for v in w.t_knots]
    cf = _mp_spline(t, [mp.mpf(float(v)) for v in w.phi_phi])
    ct = _mp_spline(t, [mp.mpf(float(v)) for v in w.phi_theta])
    cr = _mp_spline(t, [mp.mpf(float(v)) for v in w.phi_r])
    camp = [[_mp_spline(t, [mp.mpf(float(w.amp[i, q, c])) for i in range(w.K)])
             for c in range(2)] for q in range(w.M)]
    ref = []
    for j in range(w.n_samples):
        tj = mp.mpf(float(np.float64(w.t_start) + np.float64(j) * np.float64(w.dt)))
        pf, pt, pr = _mp_eval(t, cf, tj), _mp_eval(t, ct, tj), _mp_eval(t, cr, tj)
        h = mp.mpc(0)
        for q, (l, m, k, n) in enumerate(w.lmn):
            A = mp.mpc(_mp_eval(t, camp[q][0], tj), _mp_eval(t, camp[q][1], tj))
            E = mp.expj(-(int(m) * pf + int(k) * pt + int(n) * pr))
            h += A * mp.mpc(oracle.swsh(-2, int(l), int(m), w.theta, w.phi)) * E
            if m > 0:
                h += (-1) ** int(l + k) * mp.conj(A) * mp.mpc(
                    oracle.swsh(-2, int(l), -int(m), w.theta, w.phi)) / E
        ref.append(complex(h))
    ref = np.array(ref)
    assert np.max(np.abs(got - ref)) <= 1e-15 * np.max(np.abs(ref))


def test_kerr_needs_phi_theta():
    w = synth.tiny_kerr(seed=3)
    with pytest.raises(oracle.OracleError):
        oracle.mode_sum(w.t_knots, w.phi_phi, w.phi_r, w.lmn, w.amp, w.theta, w.phi, w.dt,
                        w.n_samples)
