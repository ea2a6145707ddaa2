"""GPU parity of the generic-Kerr spherical-projected sum (few_spline_fit_kerr +
few_mode_sum, through the C ABI) against the CPU oracle.

Bars as for the Schwarzschild sum: binary64 max relative error <= 1e-10; mixed
mismatch <= 1e-6 (max relative error <= 1e-4 as a sanity bound).
"""
import numpy as np
import pytest

import oracle
from paper_2104_04582_amd import synth

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_MISMATCH = 1e-6
MIXED_MAXREL = 1e-4


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2104_04582_amd import native
    native.load()
    assert torch.cuda.is_available()
    return native, torch, torch.device("cuda:0")


def dev(torch, a, d):
    return torch.from_numpy(np.ascontiguousarray(a)).to(d)


def run_kerr(env, w, prec, n=None):
    native, torch, d = env
    with native.Plan(0, prec) as plan:
        sp = plan.spline_fit_kerr(w.t_knots, dev(torch, w.phi_phi, d), dev(torch, w.phi_theta, d),
                                  dev(torch, w.phi_r, d), w.lmn, dev(torch, w.amp, d))
        out = plan.mode_sum(sp, w.theta, w.phi, w.dt, n or w.n_samples, t_start=w.t_start,
                            scale=w.scale)
        torch.cuda.synchronize()
        return out.cpu().numpy().astype(np.complex128)


def check(got, ref, prec):
    err = oracle.max_rel_error(got, ref)
    mm = oracle.mismatch(got, ref)
    log(f"    {prec}: max_rel_err={err:.3e} mismatch={mm:.3e}")
    if prec == "fp64":
        assert err <= FP64_TOL
    else:
        assert mm <= MIXED_MISMATCH
        assert err <= MIXED_MAXREL


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_kerr_small_full_output(env, prec):
    w = synth.kerr_small()
    log(f"[kerr] small M={w.M} K={w.K} N={w.n_samples} {prec}")
    check(run_kerr(env, w, prec), oracle.mode_sum_waveform(w), prec)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_kerr_tiny_random(env, prec, seed):
    w = synth.tiny_kerr(seed, K=6 + seed, M=5 + 7 * seed, n_samples=700 + 331 * seed,
                        l_max=5, k_max=3, n_max=4, phase_scale=80.0)
    log(f"[kerr] tiny seed={seed} M={w.M} N={w.n_samples} {prec}")
    check(run_kerr(env, w, prec), oracle.mode_sum_waveform(w), prec)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_kerr_full_sampled(env, prec):
    """34,587 modes over one year at sampled outputs (tile starts, interval
    edges, the last sample and a spread of interior points)."""
    w = synth.kerr_full()
    n = w.n_samples
    idx = np.unique(np.concatenate([np.linspace(0, n - 1, 160).astype(np.int64),
                                    np.arange(0, 4096, 511), [n - 2, n - 1]]))
    log(f"[kerr] full M={w.M} N={n} {prec}: {idx.size} sampled outputs")
    got = run_kerr(env, w, prec)
    ref = oracle.mode_sum_waveform(w, idx=idx)
    check(got[idx], ref, prec)


def test_kerr_with_k_zero_equals_schwarzschild(env):
    """All k = 0: the generic-Kerr path gives the Schwarzschild result bit for bit
    (Phi_theta drops out of every phase)."""
    native, torch, d = env
    w = synth.config0()
    lmkn = np.insert(w.lmn, 2, 0, axis=1)
    pt = 0.93 * w.phi_phi
    for prec in ("mixed", "fp64"):
        with native.Plan(0, prec) as plan:
            a = plan.spline_fit(w.t_knots, dev(torch, w.phi_phi, d), dev(torch, w.phi_r, d),
                                w.lmn, dev(torch, w.amp, d))
            ha = plan.mode_sum(a, w.theta, w.phi, w.dt, w.n_samples)
            b = plan.spline_fit_kerr(w.t_knots, dev(torch, w.phi_phi, d), dev(torch, pt, d),
                                     dev(torch, w.phi_r, d), lmkn, dev(torch, w.amp, d))
            hb = plan.mode_sum(b, w.theta, w.phi, w.dt, w.n_samples)
            torch.cuda.synchronize()
            assert np.array_equal(ha.cpu().numpy(), hb.cpu().numpy()), prec


def test_kerr_polar_phase_spline(env):
    """The third phase spline (Phi_theta) matches the oracle's spline."""
    native, torch, d = env
    w = synth.kerr_small()
    with native.Plan(0, "fp64") as plan:
        sp = plan.spline_fit_kerr(w.t_knots, dev(torch, w.phi_phi, d), dev(torch, w.phi_theta, d),
                                  dev(torch, w.phi_r, d), w.lmn, dev(torch, w.amp, d))
        pc = sp.coefs(1).cpu().numpy()                   # [K-1, 3, 4, 2]
    ref = oracle.spline_coefs(w.t_knots, w.phi_theta)      # [K-1, 4]
    got = pc[:, 2, :, 0] + pc[:, 2, :, 1]
    h = np.diff(w.t_knots)
    for p in (1, 2, 3):
        scale = np.abs(np.diff(w.phi_theta)) / h ** p
        assert np.all(np.abs(got[:, p] - ref[:, p]) <= 1e-12 * scale + 1e-300), p
    # p = 0: knot value reduced mod 2 pi
    red = np.angle(np.exp(1j * (got[:, 0] - w.phi_theta[:-1])))
    assert np.max(np.abs(red)) <= 1e-9


def test_kerr_rejects_bad_modes(env):
    native, torch, d = env
    w = synth.tiny_kerr(4)
    bad = w.lmn.copy()
    bad[0, 2] = 31
    with native.Plan(0, "mixed") as plan:
        with pytest.raises(native.FewError) as e:
            plan.spline_fit_kerr(w.t_knots, dev(torch, w.phi_phi, d), dev(torch, w.phi_theta, d),
                                 dev(torch, w.phi_r, d), bad, dev(torch, w.amp, d))
        assert e.value.code == native.FEW_E_MODES
