"""Pins for the error metrics (mismatch with unit PSD, Sec. VI Eqs. (16)-(17))."""
import math

import numpy as np

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
