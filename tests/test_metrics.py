"""Pins for the error metrics (mismatch with unit PSD, Sec. VI Eqs. (16)-(17))."""
import math

import numpy as np
import pytest

from oracle import max_rel_error, mismatch


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def test_mismatch_identities():
    a = _rand(4096, 1)
    assert abs(mismatch(a, a)) < 1e-15
    for c in [1e-4, 0.01, 0.3, 1.0, 2.5]:
        assert abs(mismatch(a, np.exp(1j * c) * a) - (1 - math.cos(c))) < 1e-14
    assert abs(mismatch(a, 3.7 * a)) < 1e-15
    assert abs(mismatch(a, -a) - 2.0) < 1e-15


def test_mismatch_equals_flat_psd_frequency_domain_overlap():
    """Unit-PSD inner product of h_plus and h_cross via FFT (Parseval) equals the
    time-domain form used by mismatch()."""
    a = _rand(2048, 2)
    b = a + 0.05 * _rand(2048, 3)

    def ip(x, y):
        # <x|y> summed over both real polarisations, in the frequency domain
        tot = 0.0
        for f in (np.real, np.imag):
            X = np.fft.fft(f(x))
            Y = np.fft.fft(f(y))
            tot += np.real(np.vdot(X, Y)) / len(X)
        return tot

    ref = 1.0 - ip(a, b) / math.sqrt(ip(a, a) * ip(b, b))
    assert abs(mismatch(a, b) - ref) < 1e-13


def test_max_rel_error():
    ref = np.array([1.0, -2.0j, 0.5])
    assert max_rel_error(ref, ref) == 0.0
    got = ref + np.array([0.0, 1e-3, 0.0])
    assert abs(max_rel_error(got, ref) - 5e-4) < 1e-15


def _one_sided_flat_psd(x, y, dt):
    """4 Re int_0^inf conj(x~) y~ df for each real polarisation, by rfft: the
    continuous transform is dt times the DFT, df = 1 / (N dt), and the DC and
    (even N) Nyquist bins are counted once."""
    n = len(x)
    tot = 0.0
    for f in (np.real, np.imag):
        X = np.fft.rfft(f(x))
        Y = np.fft.rfft(f(y))
        w = np.ones(X.shape[0])
        w[0] = 0.5
        if n % 2 == 0:
            w[-1] = 0.5
        tot += 4.0 * np.real(np.sum(w * np.conj(X) * Y)) * dt * dt / (n * dt)
    return tot


@pytest.mark.parametrize("n", [2048, 1001])
def test_inner_flat_equals_the_frequency_domain_integral(n):
    from oracle import inner_flat
    a = _rand(n, 5)
    b = _rand(n, 6)
    dt = 10.0
    ref = _one_sided_flat_psd(a, b, dt)
    assert abs(inner_flat(a, b, dt) - ref) <= 1e-12 * abs(ref)


def test_inner_flat_identities():
    from oracle import inner_flat
    a, b, c = _rand(700, 7), _rand(700, 8), _rand(700, 9)
    dt = 3.0
    assert abs(inner_flat(a, b, dt) - inner_flat(b, a, dt)) < 1e-10
    assert abs(inner_flat(a, 2 * b + c, dt) - 2 * inner_flat(a, b, dt) - inner_flat(a, c, dt)) < 1e-9
    assert inner_flat(a, a, dt) > 0
    # the overlap built from it is the mismatch's
    ov = inner_flat(a, b, dt) / math.sqrt(inner_flat(a, a, dt) * inner_flat(b, b, dt))
    assert abs((1 - ov) - mismatch(a, b)) < 1e-13
