"""GPU tests of the fused inner products (few_inner_product): <d|h> and <h|h>
with a unit PSD (Sec. VI), formed without writing h, against the oracle's
inner_flat on the oracle's waveform, and against a reduction of the
materialised GPU waveform.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2104_04582_amd import synth

pytestmark = pytest.mark.gpu


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


def fit(plan, torch, d, w):
    if w.phi_theta is not None:
        return plan.spline_fit_kerr(w.t_knots, dev(torch, w.phi_phi, d),
                                    dev(torch, w.phi_theta, d), dev(torch, w.phi_r, d), w.lmn,
                                    dev(torch, w.amp, d))
    return plan.spline_fit(w.t_knots, dev(torch, w.phi_phi, d), dev(torch, w.phi_r, d), w.lmn,
                           dev(torch, w.amp, d))


def data_like(w, h_scale, seed):
    """Synthetic data: a noisy copy of a scaled waveform-sized random series."""
    rng = np.random.default_rng(seed)
    return h_scale * (rng.standard_normal(w.n_samples) + 1j * rng.standard_normal(w.n_samples))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["config0", "kerr_small"])
def test_inner_matches_oracle(env, prec, case):
    native, torch, d = env
    w = getattr(synth, case)()
    h = oracle.mode_sum_waveform(w)
    dat = h + data_like(w, 0.3 * np.std(np.abs(h)), 7)
    ref_dh = oracle.inner_flat(dat, h, w.dt)
    ref_hh = oracle.inner_flat(h, h, w.dt)
    norm = 2 * w.dt * np.linalg.norm(dat) * np.linalg.norm(h)
    with native.Plan(0, prec) as plan:
        sp = fit(plan, torch, d, w)
        ddev = torch.from_numpy(dat.astype(np.complex64 if prec == "mixed" else np.complex128)).to(d)
        got = plan.inner_product(sp, w.theta, w.phi, w.dt, w.n_samples, ddev,
                                 t_start=w.t_start, scale=w.scale).cpu().numpy()
    e_dh = abs(got[0] - ref_dh) / norm
    e_hh = abs(got[1] - ref_hh) / ref_hh
    log(f"[inner] {case} {prec}: <d|h> {got[0]:.6e} (err {e_dh:.2e}), <h|h> {got[1]:.6e} "
        f"(err {e_hh:.2e})")
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert e_dh <= tol and e_hh <= tol


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_inner_equals_reduction_of_materialised_waveform(env, prec):
    """Full one-year case: the fused products equal binary64 reductions of the
    stored waveform (same h values; only the summation order differs)."""
    native, torch, d = env
    w = synth.config1()
    cdt = torch.complex64 if prec == "mixed" else torch.complex128
    g = torch.Generator(device="cpu").manual_seed(11)
    dat = torch.complex(torch.randn(w.n_samples, generator=g, dtype=torch.float64),
                        torch.randn(w.n_samples, generator=g, dtype=torch.float64)).to(cdt).to(d)
    with native.Plan(0, prec) as plan:
        sp = fit(plan, torch, d, w)
        h = plan.mode_sum(sp, w.theta, w.phi, w.dt, w.n_samples)
        got = plan.inner_product(sp, w.theta, w.phi, w.dt, w.n_samples, dat).cpu().numpy()
        again = plan.inner_product(sp, w.theta, w.phi, w.dt, w.n_samples, dat).cpu().numpy()
        torch.cuda.synchronize()
    h64 = h.to(torch.complex128)
    d64 = dat.to(torch.complex128)
    ref_dh = 2 * w.dt * torch.real(torch.vdot(d64, h64)).item()
    ref_hh = 2 * w.dt * torch.real(torch.vdot(h64, h64)).item()
    norm = 2 * w.dt * torch.linalg.norm(d64).item() * torch.linalg.norm(h64).item()
    log(f"[inner] config1 {prec}: dh err {abs(got[0] - ref_dh) / norm:.2e}, "
        f"hh err {abs(got[1] - ref_hh) / ref_hh:.2e}")
    assert abs(got[0] - ref_dh) <= 1e-12 * norm
    assert abs(got[1] - ref_hh) <= 1e-12 * ref_hh
    assert np.array_equal(got, again)            # fixed reduction order


def test_inner_argument_errors(env):
    native, torch, d = env
    w = synth.config0()
    with native.Plan(0, "mixed") as plan:
        sp = fit(plan, torch, d, w)
        out2 = torch.empty(2, dtype=torch.float64, device=d)
        lib = native.load()
        rc = lib.few_inner_product(plan.handle, sp.handle, w.theta, w.phi, 1.0, 0.0, w.dt,
                                   w.n_samples, None, ctypes.c_void_p(out2.data_ptr()))
        assert rc == native.FEW_E_ARG
        dat = torch.zeros(w.n_samples, dtype=torch.complex64, device=d)
        rc = lib.few_inner_product(plan.handle, sp.handle, w.theta, w.phi, 1.0, 0.0, w.dt,
                                   w.n_samples, ctypes.c_void_p(dat.data_ptr()), None)
        assert rc == native.FEW_E_ARG
        with pytest.raises(native.FewError) as e:
            plan.inner_product(sp, w.theta, w.phi, w.dt, w.n_samples + 10 ** 6,
                               torch.zeros(w.n_samples + 10 ** 6, dtype=torch.complex64,
                                           device=d))
        assert e.value.code == native.FEW_E_RANGE
