"""GPU tests of the served path (few_submit / few_poll / few_wait).

Each request's result must be bitwise identical to the same request run alone
through the synchronous path: batching never changes tiling or reduction
order.  A few results are also checked against the oracle at sampled outputs.
"""
import time

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


def dev_inputs(torch, w, dev):
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev)
                 for a in (w.phi_phi, w.phi_r, w.amp))


def submit(plan, w, ins, out):
    pp, pr, amp = ins
    return plan.submit(w.t_knots, pp, pr, w.lmn, amp, w.theta, w.phi, w.dt, w.n_samples, out,
                       t_start=w.t_start, scale=w.scale)


def solo(native, torch, dev, w, prec):
    pp, pr, amp = dev_inputs(torch, w, dev)
    with native.Plan(0, prec) as plan:
        sp = plan.spline_fit(w.t_knots, pp, pr, w.lmn, amp)
        out = plan.mode_sum(sp, w.theta, w.phi, w.dt, w.n_samples, t_start=w.t_start,
                            scale=w.scale)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def shorten(w, max_samples):
    """Keep the first max_samples samples (same knots): smaller outputs."""
    w.n_samples = min(w.n_samples, max_samples)
    return w


def instances(n, max_samples=400_000):
    return [shorten(synth.uneven_instance(i), max_samples) for i in range(n)]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_batch_bitwise_equals_solo(env, prec):
    native, torch, dev = env
    ws = instances(10)
    log(f"[serve] batch of {len(ws)} {prec}: M={[w.M for w in ws]}")
    refs = [solo(native, torch, dev, w, prec) for w in ws]
    ins = [dev_inputs(torch, w, dev) for w in ws]
    dtype = torch.complex64 if prec == "mixed" else torch.complex128
    outs = [torch.empty(w.n_samples, dtype=dtype, device=dev) for w in ws]
    with native.Plan(0, prec, max_inflight=2) as plan:
        tickets = [submit(plan, w, ins[i], outs[i]) for i, w in enumerate(ws)]
        for tk in tickets:
            plan.wait(tk)
    for i, w in enumerate(ws):
        got = outs[i].cpu().numpy()
        assert np.array_equal(got, refs[i]), i
    # two of them against the oracle at sampled outputs
    for i in (0, 5):
        w = ws[i]
        idx = np.unique(np.linspace(0, w.n_samples - 1, 300).astype(np.int64))
        ref = oracle.mode_sum_waveform(w, idx=idx)
        got = refs[i][idx].astype(np.complex128)
        err = oracle.max_rel_error(got, ref)
        mm = oracle.mismatch(got, ref)
        log(f"    instance {i}: max_rel_err={err:.2e} mismatch={mm:.2e}")
        if prec == "fp64":
            assert err <= 1e-10
        else:
            assert mm <= 1e-6


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_one_launch_batch_bitwise_equals_solo(env, prec):
    """few_batch: uneven instances in one batched launch on the plan stream."""
    native, torch, dev = env
    ws = instances(16, max_samples=300_000)
    log(f"[batch] {len(ws)} {prec}")
    refs = [solo(native, torch, dev, w, prec) for w in ws]
    ins = [dev_inputs(torch, w, dev) for w in ws]
    dtype = torch.complex64 if prec == "mixed" else torch.complex128
    outs = [torch.empty(w.n_samples, dtype=dtype, device=dev) for w in ws]
    with native.Plan(0, prec) as plan:
        for rep in range(2):
            for o in outs:
                o.zero_()
            plan.batch([dict(t_knots=w.t_knots, phi_phi=ins[i][0], phi_r=ins[i][1],
                             lmn=w.lmn, amp=ins[i][2], theta=w.theta, phi=w.phi, dt=w.dt,
                             n_samples=w.n_samples, out=outs[i]) for i, w in enumerate(ws)])
            torch.cuda.synchronize()
            for i in range(len(ws)):
                assert np.array_equal(outs[i].cpu().numpy(), refs[i]), (rep, i)


@pytest.mark.parametrize("prec", ["mixed"])
def test_staggered_arrivals_same_as_alone(env, prec):
    """Requests submitted while earlier ones run are admitted into new
    batches; every result equals its solo run."""
    native, torch, dev = env
    ws = instances(8, max_samples=1_500_000)
    refs = [solo(native, torch, dev, w, prec) for w in ws]
    ins = [dev_inputs(torch, w, dev) for w in ws]
    outs = [torch.empty(w.n_samples, dtype=torch.complex64, device=dev) for w in ws]
    log(f"[serve] staggered {len(ws)}")
    with native.Plan(0, prec, max_inflight=3) as plan:
        tickets = []
        for i, w in enumerate(ws):
            tickets.append(submit(plan, w, ins[i], outs[i]))
            time.sleep(0.0007 * (i % 3))
        done = set()
        t0 = time.time()
        while len(done) < len(tickets):
            for tk in tickets:
                if tk not in done and plan.poll(tk):
                    done.add(tk)
            assert time.time() - t0 < 60, "served requests did not complete"
            time.sleep(0.0005)
    for i in range(len(ws)):
        assert np.array_equal(outs[i].cpu().numpy(), refs[i]), i


def test_admission_under_small_budget(env):
    """A budget that holds only a few requests at a time still completes every
    request (queued until memory frees); an oversized request is rejected."""
    native, torch, dev = env
    full = synth.config1()
    full.n_samples = 200_000
    ws = [full] + instances(5, max_samples=200_000)
    refs = [solo(native, torch, dev, w, "mixed") for w in ws]
    ins = [dev_inputs(torch, w, dev) for w in ws]
    outs = [torch.empty(w.n_samples, dtype=torch.complex64, device=dev) for w in ws]
    need = native.host_request_bytes("mixed", full.K, full.M, 1281)
    budget = int(need * 1.6)
    log(f"[serve] budget {budget / 1e6:.1f} MB, full request {need / 1e6:.1f} MB")
    with native.Plan(0, "mixed", hbm_budget_bytes=budget, max_inflight=2) as plan:
        tickets = [submit(plan, w, ins[i], outs[i]) for i, w in enumerate(ws)]
        for tk in tickets:
            plan.wait(tk)
    for i in range(len(ws)):
        assert np.array_equal(outs[i].cpu().numpy(), refs[i]), i
    with native.Plan(0, "mixed", hbm_budget_bytes=budget // 4) as small:
        big = ws[0]
        with pytest.raises(native.FewError) as e:
            submit(small, big, ins[0], outs[0])
        assert e.value.code == native.FEW_E_TOO_LARGE


def test_poll_unknown_ticket(env):
    native, torch, dev = env
    with native.Plan(0, "mixed") as plan:
        with pytest.raises(native.FewError) as e:
            plan.poll(12345)
        assert e.value.code == native.FEW_E_STATE
