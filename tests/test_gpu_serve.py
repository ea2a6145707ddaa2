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
def test_staggered_arrivals_same_as_alone(env, prec, tmp_path):
    """Requests submitted while earlier ones run are admitted into new
    batches; every result equals its solo run.  The request log holds one
    line per request with ordered arrival, admission and completion times."""
    import json
    native, torch, dev = env
    ws = instances(8, max_samples=1_500_000)
    refs = [solo(native, torch, dev, w, prec) for w in ws]
    ins = [dev_inputs(torch, w, dev) for w in ws]
    outs = [torch.empty(w.n_samples, dtype=torch.complex64, device=dev) for w in ws]
    log(f"[serve] staggered {len(ws)}")
    log_path = tmp_path / "requests.jsonl"
    with native.Plan(0, prec, max_inflight=3) as plan:
        plan.request_log(str(log_path))
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
    recs = {r["ticket"]: r for r in map(json.loads, log_path.read_text().splitlines())}
    assert sorted(recs) == sorted(tickets)
    for tk, w in zip(tickets, ws):
        r = recs[tk]
        assert r["status"] == 0 and r["samples"] == w.n_samples and r["modes"] == w.M
        assert r["knots"] == w.K and r["batch"] >= 0 and r["batch_size"] >= 1
        assert r["path"] in (("mfma", "vector") if prec == "mixed" else ("fp64",))
        assert 0.0 <= r["arrive_us"] <= r["admit_us"] <= r["done_us"]


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


def test_freed_spline_block_not_reused_while_queued_sums_read_it(env):
    """few_spline_free with summations of that spline still queued on the plan
    stream, then served requests that allocate from the same arena and run on
    the library's own streams: the freed block is handed out again only after
    the queued sums have run, so their output equals a solo run bit for bit."""
    native, torch, dev = env
    w = synth.config1()
    w.n_samples = 1_000_000
    ref = solo(native, torch, dev, w, "mixed")
    small = instances(6, max_samples=300_000)
    small_refs = [solo(native, torch, dev, s, "mixed") for s in small]
    pp, pr, amp = dev_inputs(torch, w, dev)
    ins = [dev_inputs(torch, s, dev) for s in small]
    outs = [torch.empty(s.n_samples, dtype=torch.complex64, device=dev) for s in small]
    sums = [torch.empty(w.n_samples, dtype=torch.complex64, device=dev) for _ in range(4)]
    log("[serve] free with queued sums, then served requests")
    with native.Plan(0, "mixed", max_inflight=2) as plan:
        sp = plan.spline_fit(w.t_knots, pp, pr, w.lmn, amp)
        for o in sums:
            plan.mode_sum(sp, w.theta, w.phi, w.dt, w.n_samples, out=o)
        sp.free()
        tickets = [submit(plan, s, ins[i], outs[i]) for i, s in enumerate(small)]
        for tk in tickets:
            plan.wait(tk)
        torch.cuda.synchronize()
    for o in sums:
        assert np.array_equal(o.cpu().numpy(), ref)
    for i in range(len(small)):
        assert np.array_equal(outs[i].cpu().numpy(), small_refs[i]), i


def test_served_inputs_produced_asynchronously_on_the_plan_stream(env):
    """Inputs written by work still queued on the plan's stream when
    few_submit is called (no host synchronisation): the served batch waits for
    that work, so it reads the final inputs, not the NaNs written before."""
    native, torch, dev = env
    ws = instances(3, max_samples=300_000)
    refs = [solo(native, torch, dev, w, "mixed") for w in ws]
    src = [dev_inputs(torch, w, dev) for w in ws]
    torch.cuda.synchronize()
    with native.Plan(0, "mixed", max_inflight=2) as plan:
        stream = torch.cuda.current_stream(dev)
        assert plan.stream == stream.cuda_stream
        ins = [tuple(torch.full_like(a, float("nan")) for a in s) for s in src]
        outs = [torch.full((w.n_samples,), float("nan"), dtype=torch.complex64, device=dev)
                for w in ws]
        # tens of milliseconds of queued work before the inputs are written
        x = torch.randn(4096, 4096, device=dev)
        for _ in range(16):
            x = torch.tanh(x @ x * 1e-3)
        for s, d in zip(src, ins):
            for a, b in zip(s, d):
                b.copy_(a)
        log("[serve] submitting with the input copies still queued")
        tickets = [submit(plan, w, ins[i], outs[i]) for i, w in enumerate(ws)]
        for tk in tickets:
            plan.wait(tk)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(x).all())
    for i in range(len(ws)):
        assert np.array_equal(outs[i].cpu().numpy(), refs[i]), i


def test_admission_fails_when_synchronous_memory_blocks_it(env):
    """With nothing in flight and the arena held by a synchronous-path spline,
    a served request that cannot fit fails with FEW_E_NOMEM instead of waiting
    forever; after the spline is freed the same request is served."""
    native, torch, dev = env
    full = synth.config1()
    full.n_samples = 200_000
    ref = solo(native, torch, dev, full, "mixed")
    need = native.host_request_bytes("mixed", full.K, full.M, 1281)
    pp, pr, amp = dev_inputs(torch, full, dev)
    out = torch.empty(full.n_samples, dtype=torch.complex64, device=dev)
    log(f"[serve] arena blocked by a synchronous spline ({need / 1e6:.1f} MB each)")
    with native.Plan(0, "mixed", hbm_budget_bytes=int(need * 1.5)) as plan:
        sp = plan.spline_fit(full.t_knots, pp, pr, full.lmn, amp)
        tk = submit(plan, full, (pp, pr, amp), out)
        with pytest.raises(native.FewError) as e:
            plan.wait(tk)
        assert e.value.code == native.FEW_E_NOMEM
        sp.free()
        torch.cuda.synchronize()
        plan.wait(submit(plan, full, (pp, pr, amp), out))
    assert np.array_equal(out.cpu().numpy(), ref)


def test_plan_destroy_with_queued_submissions(env):
    """few_plan_destroy while requests are still queued drains them: every
    output is complete and equal to its solo run."""
    native, torch, dev = env
    ws = instances(6, max_samples=400_000)
    refs = [solo(native, torch, dev, w, "mixed") for w in ws]
    ins = [dev_inputs(torch, w, dev) for w in ws]
    outs = [torch.empty(w.n_samples, dtype=torch.complex64, device=dev) for w in ws]
    log("[serve] destroy with queued submissions")
    plan = native.Plan(0, "mixed", max_inflight=1)
    for i, w in enumerate(ws):
        submit(plan, w, ins[i], outs[i])
    plan.close()
    torch.cuda.synchronize()
    for i in range(len(ws)):
        assert np.array_equal(outs[i].cpu().numpy(), refs[i]), i
