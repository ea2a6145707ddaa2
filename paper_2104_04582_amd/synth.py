"""Seeded synthetic inputs for the interpolated harmonic-mode summation.

This module only draws inputs: knot times, the two orbital phases at the
knots, the complex mode amplitudes at the knots, the mode list and the
viewing angles.  It holds none of the method's arithmetic (no spline, no
harmonic, no mode sum), so both the CPU oracle and the GPU path can consume
its arrays.

The shapes follow the paper's workload: a sparse trajectory of about 100
points (Sec. III A), the Schwarzschild eccentric mode set l in [2, 10],
m in [0, l], n in [-30, 30] = 3843 modes (Sec. IV B), a 0.1 Hz cadence
(Sec. III C) and year-scale durations (Sec. VI).  The physical trajectory and
RomanNet amplitudes need data that is not available, so:

* phases come from a closed-form chirp, f(t) = f0 (1 - t/tc)^(-3/8),
  Phi_phi = 2 pi f0 tc (8/5) (1 - (1 - t/tc)^(5/8)), Phi_r = kappa Phi_phi;
* amplitudes are random complex cubics in t/T with a weight
  exp(-|n|/5) exp(-(l-2)) on the coefficients;
* knots are log-spaced in time to coalescence (densest near the end).

Generic-Kerr inputs (Sec. VII, spherical projection) add the polar index k
and a third phase: Phi_theta = kappa_theta Phi_phi, kappa_theta in
[0.85, 0.98], amplitude weight exp(-|n|/5) exp(-|k|/2) exp(-(l-2)); the mode
list is (l, m, k, n) with l 2..l_max, m 0..l, |k| <= k_max, |n| <= n_max.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

YEAR_S = 365.25 * 86400.0
DAY_S = 86400.0


def mode_list(l_min: int, l_max: int, n_max: int) -> np.ndarray:
    """All (l, m, n) with l_min <= l <= l_max, 0 <= m <= l, |n| <= n_max.

    Order: l ascending, then m, then n.  Returns int32 [M, 3].
    """
    rows = [(l, m, n)
            for l in range(l_min, l_max + 1)
            for m in range(0, l + 1)
            for n in range(-n_max, n_max + 1)]
    return np.asarray(rows, dtype=np.int32).reshape(-1, 3)


def knot_times(T: float, K: int, tc: float) -> np.ndarray:
    """K knots on [0, T], log-spaced in time to coalescence tc - t."""
    k = np.arange(K, dtype=np.float64)
    t = tc * (1.0 - (1.0 - T / tc) ** (k / (K - 1)))
    t[0] = 0.0
    t[-1] = T
    return t


def chirp_phase(t: np.ndarray, f0: float, tc: float) -> np.ndarray:
    """Closed-form chirp azimuthal phase (the generator's stand-in trajectory)."""
    return 2.0 * math.pi * f0 * tc * (8.0 / 5.0) * (1.0 - (1.0 - t / tc) ** 0.625)


def n_samples_for(T: float, dt: float, t0: float = 0.0) -> int:
    """Dense-grid length n = ceil((T - t0) / dt): the endpoint T is excluded."""
    return int(math.ceil((T - t0) / dt - 1e-12))


@dataclasses.dataclass
class Waveform:
    """One synthetic waveform request (host arrays, float64 / int32)."""
    t_knots: np.ndarray          # [K]
    phi_phi: np.ndarray          # [K]
    phi_r: np.ndarray            # [K]
    lmn: np.ndarray              # [M, 3] int32
    amp: np.ndarray              # [K, M, 2] float64 (re, im), knot-major
    theta: float
    phi: float
    dt: float
    n_samples: int
    t_start: float = 0.0
    scale: float = 1.0
    # generic-Kerr requests: lmn is [M, 4] = (l, m, k, n) and Phi_theta [K]
    phi_theta: Optional[np.ndarray] = None
    # generator bookkeeping (used by tests that pin exact polynomials)
    amp_poly: Optional[np.ndarray] = None   # [M, 4, 2] coefficients in (t/T)^p
    T: float = 0.0
    f0: float = 0.0
    kappa: float = 0.0
    tc: float = 0.0

    @property
    def K(self) -> int:
        return int(self.t_knots.shape[0])

    @property
    def M(self) -> int:
        return int(self.lmn.shape[0])

    @property
    def mode_samples(self) -> int:
        return self.M * self.n_samples


def _amp_weights(lmn: np.ndarray) -> np.ndarray:
    l = lmn[:, 0].astype(np.float64)
    n = lmn[:, -1].astype(np.float64)
    w = np.exp(-np.abs(n) / 5.0) * np.exp(-(l - 2.0))
    if lmn.shape[1] == 4:
        w = w * np.exp(-np.abs(lmn[:, 2].astype(np.float64)) / 2.0)
    return w


def _amp_at_knots(poly: np.ndarray, t: np.ndarray, T: float) -> np.ndarray:
    """Evaluate the generator cubics sum_p c_p (t/T)^p at the knots -> [K, M, 2]."""
    s = t / T
    powers = np.stack([np.ones_like(s), s, s * s, s * s * s], axis=0)   # [4, K]
    return np.ascontiguousarray(np.einsum("pk,mpc->kmc", powers, poly))


def draw_waveform(rng: np.random.Generator, lmn: np.ndarray, T: float, K: int,
                  dt: float) -> Waveform:
    """Draw f0, kappa, cos(theta), phi, then the amplitude cubics, in that order."""
    f0 = rng.uniform(5e-4, 2e-3)
    kappa = rng.uniform(0.6, 0.9)
    cos_t = rng.uniform(-1.0, 1.0)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    M = lmn.shape[0]
    poly = rng.standard_normal((M, 4, 2)) * _amp_weights(lmn)[:, None, None]
    tc = 1.2 * T
    t = knot_times(T, K, tc)
    pp = chirp_phase(t, f0, tc)
    return Waveform(t_knots=t, phi_phi=pp, phi_r=kappa * pp, lmn=lmn.copy(),
                    amp=_amp_at_knots(poly, t, T), theta=math.acos(cos_t),
                    phi=phi, dt=dt, n_samples=n_samples_for(T, dt),
                    amp_poly=poly, T=T, f0=f0, kappa=kappa, tc=tc)


def mode_list_kerr(l_min: int, l_max: int, k_max: int, n_max: int) -> np.ndarray:
    """All (l, m, k, n) with l_min <= l <= l_max, 0 <= m <= l, |k| <= k_max,
    |n| <= n_max.  Order: l, then m, then k, then n ascending.  int32 [M, 4]."""
    rows = [(l, m, k, n)
            for l in range(l_min, l_max + 1)
            for m in range(0, l + 1)
            for k in range(-k_max, k_max + 1)
            for n in range(-n_max, n_max + 1)]
    return np.asarray(rows, dtype=np.int32).reshape(-1, 4)


def draw_kerr(rng: np.random.Generator, lmkn: np.ndarray, T: float, K: int,
              dt: float) -> Waveform:
    """Generic-Kerr draw: f0, kappa, kappa_theta, cos(theta), phi, then the
    amplitude cubics, in that order."""
    f0 = rng.uniform(5e-4, 2e-3)
    kappa = rng.uniform(0.6, 0.9)
    kappa_t = rng.uniform(0.85, 0.98)
    cos_t = rng.uniform(-1.0, 1.0)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    M = lmkn.shape[0]
    poly = rng.standard_normal((M, 4, 2)) * _amp_weights(lmkn)[:, None, None]
    tc = 1.2 * T
    t = knot_times(T, K, tc)
    pp = chirp_phase(t, f0, tc)
    return Waveform(t_knots=t, phi_phi=pp, phi_r=kappa * pp, lmn=lmkn.copy(),
                    amp=_amp_at_knots(poly, t, T), theta=math.acos(cos_t),
                    phi=phi, dt=dt, n_samples=n_samples_for(T, dt),
                    phi_theta=kappa_t * pp, amp_poly=poly, T=T, f0=f0, kappa=kappa,
                    tc=tc)


def kerr_small(seed: int = 0) -> Waveform:
    """Small generic-Kerr case: l 2..4, |k| <= 2, |n| <= 5 (660 modes), 40 knots
    over 1 day, dt 10 s."""
    return draw_kerr(np.random.default_rng(seed), mode_list_kerr(2, 4, 2, 5),
                     DAY_S, 40, 10.0)


def kerr_full(seed: int = 0) -> Waveform:
    """Full generic-Kerr case: l 2..10, |k| <= 4, |n| <= 30 (34,587 modes, about
    nine times the Schwarzschild set), 100 knots over 1 yr, dt 10 s."""
    return draw_kerr(np.random.default_rng(seed), mode_list_kerr(2, 10, 4, 30),
                     YEAR_S, 100, 10.0)


def tiny_kerr(seed: int, K: int = 5, M: int = 4, n_samples: int = 40, l_max: int = 3,
              k_max: int = 2, n_max: int = 2, T: float = 1000.0,
              phase_scale: float = 30.0) -> Waveform:
    """A small random generic-Kerr instance with arbitrary knot data (modes
    drawn at random, repeats possible, from l 2..l_max, |k| <= k_max,
    |n| <= n_max)."""
    rng = np.random.default_rng(seed)
    gaps = rng.uniform(0.3, 1.0, K - 1)
    t = np.concatenate([[0.0], np.cumsum(gaps)])
    t = t / t[-1] * T
    t[-1] = T
    pp = np.cumsum(rng.uniform(0.0, phase_scale, K))
    pt = np.cumsum(rng.uniform(0.0, phase_scale * 0.9, K))
    pr = np.cumsum(rng.uniform(0.0, phase_scale * 0.7, K))
    modes = mode_list_kerr(2, l_max, k_max, n_max)
    lmkn = modes[rng.integers(0, modes.shape[0], M)]
    amp = rng.standard_normal((K, M, 2))
    dt = T / n_samples
    return Waveform(t_knots=t, phi_phi=pp, phi_r=pr, lmn=lmkn, amp=amp,
                    theta=math.acos(rng.uniform(-1, 1)),
                    phi=rng.uniform(0, 2 * math.pi), dt=dt,
                    n_samples=n_samples_for(T, dt), phi_theta=pt, T=T)


def config0(seed: int = 0) -> Waveform:
    """Small case: l 2..4, n -5..5 (132 modes), 40 knots over 1 day, dt 10 s."""
    return draw_waveform(np.random.default_rng(seed), mode_list(2, 4, 5),
                         DAY_S, 40, 10.0)


def config1(seed: int = 0) -> Waveform:
    """Full case: 3843 modes, 100 knots over 1 yr, dt 10 s (3,155,760 samples)."""
    return draw_waveform(np.random.default_rng(seed), mode_list(2, 10, 30),
                         YEAR_S, 100, 10.0)


def top_modes(w: Waveform, S: int) -> Waveform:
    """Keep the S modes with the largest sum over knots of |A|^2.

    Ties break by (l, m, n) ascending (a stable sort on the mode-list order,
    which is itself (l, m, n) ascending).
    """
    power = np.sum(w.amp[:, :, 0] ** 2 + w.amp[:, :, 1] ** 2, axis=0)
    order = np.argsort(-power, kind="stable")[:S]
    keep = np.sort(order)
    return dataclasses.replace(w, lmn=w.lmn[keep].copy(), amp=w.amp[:, keep, :].copy(),
                               amp_poly=w.amp_poly[keep].copy())


def uneven_instance(i: int, meta_seed: int = 3) -> Waveform:
    """One instance of the batched uneven workload.

    T ~ U[0.25, 2] yr, dt in {10, 15} s, K ~ U{50..150}, mode-subset size
    log-uniform in [10, 3843], modes = highest-power subset of the full set.
    """
    rng = np.random.default_rng([meta_seed, i])
    T = rng.uniform(0.25, 2.0) * YEAR_S
    dt = 10.0 if rng.uniform() < 0.5 else 15.0
    K = int(rng.integers(50, 151))
    S = int(round(math.exp(rng.uniform(math.log(10.0), math.log(3843.0)))))
    full = draw_waveform(rng, mode_list(2, 10, 30), T, K, dt)
    return top_modes(full, S)


def full_request(i: int, meta_seed: int = 4) -> Waveform:
    """A full-size served request: 3843 modes, 4 yr, dt 10 s, 100 knots."""
    rng = np.random.default_rng([meta_seed, 1_000_000 + i])
    return draw_waveform(rng, mode_list(2, 10, 30), 4.0 * YEAR_S, 100, 10.0)


def batch_config(n: int = 128, meta_seed: int = 3) -> List[Waveform]:
    return [uneven_instance(i, meta_seed) for i in range(n)]


@dataclasses.dataclass
class Arrival:
    t_arrival: float
    kind: str          # "small" or "full"
    index: int


def served_trace(rate: float = 20.0, duration: float = 60.0, p_full: float = 0.1,
                 seed: int = 4) -> List[Arrival]:
    """Poisson arrival times with a 10% share of full-size requests."""
    rng = np.random.default_rng(seed)
    out: List[Arrival] = []
    t = 0.0
    n_small = n_full = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        if rng.uniform() < p_full:
            out.append(Arrival(t, "full", n_full))
            n_full += 1
        else:
            out.append(Arrival(t, "small", n_small))
            n_small += 1
    return out


def served_request(a: Arrival, meta_seed: int = 4) -> Waveform:
    if a.kind == "full":
        return full_request(a.index, meta_seed)
    return uneven_instance(a.index, meta_seed * 1000 + 3)


def tiny_waveform(seed: int, K: int = 5, M: int = 4, n_samples: int = 40,
                  l_max: int = 3, n_max: int = 2, T: float = 1000.0,
                  phase_scale: float = 30.0) -> Waveform:
    """A small random instance with arbitrary (non-chirp) knot data.

    Knots are random increasing times on [0, T]; phases and amplitudes at the
    knots are independent random numbers; modes are drawn at random (with
    possible repeats) from l 2..l_max, m 0..l, |n| <= n_max.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.uniform(0.3, 1.0, K - 1)
    t = np.concatenate([[0.0], np.cumsum(gaps)])
    t = t / t[-1] * T
    t[-1] = T
    pp = np.cumsum(rng.uniform(0.0, phase_scale, K))
    pr = np.cumsum(rng.uniform(0.0, phase_scale * 0.7, K))
    modes = mode_list(2, l_max, n_max)
    pick = rng.integers(0, modes.shape[0], M)
    lmn = modes[pick]
    amp = rng.standard_normal((K, M, 2))
    dt = T / n_samples
    return Waveform(t_knots=t, phi_phi=pp, phi_r=pr, lmn=lmn, amp=amp,
                    theta=math.acos(rng.uniform(-1, 1)),
                    phi=rng.uniform(0, 2 * math.pi), dt=dt,
                    n_samples=n_samples_for(T, dt), T=T)
