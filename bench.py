"""Benchmark of the interpolated harmonic-mode summation on one MI355X.

A step is one pass of the whole hot path over one resident batch of synthetic
input: few_spline_fit (not-a-knot splines of 2 phases + 7686 amplitude
series on 100 knots) followed by few_mode_sum (3843 modes x 3,155,760
samples, one year at dt = 10 s).  Inputs and the output buffer are resident in
HBM before timing starts.  The headline value is the mixed-precision path;
the binary64 path is timed the same way and reported beside it.

Also reported: the dominant kernel's roofline (the summation kernel, timed
with HIP events recorded by the library on the stream it launches on, around
the summation launches of the timed steps only; the per-stage breakdown comes
from a second, fully event-timed pass, since an event pair delays the launch
after it by several microseconds), the
served-stream latency (Poisson arrivals of uneven requests through
few_submit/few_poll) and the CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--serve-seconds S]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Published MI355X peaks used for the roofline (TFLOP/s, TB/s).
PEAK_FP32_VALU = 157.3
PEAK_FP64_VALU = 78.6
PEAK_FP16_MFMA = 2500.0   # dense
PEAK_HBM_TBS = 8.0


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def algorithmic_flops(n_terms: int, n_segs: int, n: int) -> float:
    """Flops of the summation kernel's algorithm per launch.

    Per folded (m, n) term and sample: the complex cubic C(u) with real u is
    3 complex-by-real FMAs (12 flop) and the Horner step S f + C is one complex
    multiply-add (8 flop): 20 flop.  Per segment and sample: the seed product
    (6 flop) and the accumulation (2 flop): 8 flop.
    """
    return float(n) * (20.0 * n_terms + 8.0 * n_segs)


def mfma_algorithmic_flops(n_terms: int, n_rows: int, n: int) -> float:
    """Flops of the matrix-core contraction per launch, counted once: per
    folded (m, n) term, power p of u and sample one complex multiply-add of the
    coefficient with u^p f^n (4 x 8 flop), and per signed m row and sample the
    complex multiply-add with e^{-i m Phi_phi} (8 flop).  The hi/lo split
    executes each product three times on the matrix cores; that is not
    counted here."""
    return float(n) * (32.0 * n_terms + 8.0 * n_rows)


def path_flops(native, lmn, n: int, precision: str) -> float:
    """Algorithmic flops of the summation path a request takes."""
    segs, tp, _ = native.host_terms(lmn)
    n_terms = tp.shape[0] - 1
    if precision == "mixed" and native.host_mfma_path(lmn):
        return mfma_algorithmic_flops(n_terms, len(set(int(x) for x in segs[:, 0])), n)
    return algorithmic_flops(n_terms, segs.shape[0], n)


def mfma_instructions(native, w, n_wg: int) -> int:
    """MFMA instructions of one matrix-core launch of request w: every
    workgroup takes an equal contiguous share of the samples and runs rounds
    (waves x tiles x 16 samples) inside each knot interval; in the last round
    of an interval only the waves with samples run."""
    sh = native.host_mfma_shape()
    per_wave = sh["tiles_per_wave"] * 16
    starts = [int(x) for x in native.host_interval_starts(w.t_knots, w.t_start, w.dt,
                                                          w.n_samples)]
    n = w.n_samples
    wave_rounds = 0
    for r in range(n_wg):
        lo, hi = n * r // n_wg, n * (r + 1) // n_wg
        for i in range(len(starts) - 1):
            a, e = max(lo, starts[i]), min(hi, starts[i + 1])
            if e > a:
                wave_rounds += (e - a + per_wave - 1) // per_wave
    return wave_rounds * sh["tiles_per_wave"] * sh["mfma_per_tile"]


def time_path(native, plan, w, dev, steps: int, warmup: int, settle_s: float = 0.0):
    """Mean wall time of `steps` fit + sum steps after at least `warmup` untimed
    steps and at least `settle_s` seconds of them (the shader clock takes a few
    milliseconds of load to settle), with the plan's kernel timings of the
    timed steps."""
    import torch
    pp = torch.from_numpy(np.ascontiguousarray(w.phi_phi)).to(dev)
    pr = torch.from_numpy(np.ascontiguousarray(w.phi_r)).to(dev)
    amp = torch.from_numpy(np.ascontiguousarray(w.amp)).to(dev)
    out = torch.empty(w.n_samples, dtype=plan.out_dtype, device=dev)

    def step():
        sp = plan.spline_fit(w.t_knots, pp, pr, w.lmn, amp)
        plan.mode_sum(sp, w.theta, w.phi, w.dt, w.n_samples, out=out)
        sp.free()

    t_w = time.perf_counter()
    done = 0
    while done < warmup or time.perf_counter() - t_w < settle_s:
        step()
        done += 1
        if done % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    plan.timing(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = plan.timing(reset=True)
    return elapsed / steps, tm, out, step


def step_spread(step, steps: int):
    """Median and min of single steps: a separate pass of `steps` steps, each
    between two events on the plan's stream (torch's current stream)."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return {"median_ms": float(np.median(ms)), "min_ms": float(ms.min()),
            "max_ms": float(ms.max()), "steps": steps}


def kerr_run(native, dev, steps: int = 5, warmup: int = 1):
    """Generic-Kerr sum (34,587 modes, 1 yr): fit + sum per step, both precisions."""
    import torch
    from paper_2104_04582_amd import synth
    w = synth.kerr_full()
    segs, tp, _ = native.host_terms(w.lmn)
    n_terms, n_segs = tp.shape[0] - 1, segs.shape[0]
    flops = algorithmic_flops(n_terms, n_segs, w.n_samples)
    ins = [torch.from_numpy(np.ascontiguousarray(a)).to(dev)
           for a in (w.phi_phi, w.phi_theta, w.phi_r, w.amp)]
    res = {"workload": "generic-Kerr spherical-projected sum, 34,587 modes (l 2..10, m 0..l, "
                       "k -4..4, n -30..30), 100 knots, 1 yr at dt 10 s",
           "modes": w.M, "samples": w.n_samples, "folded_terms": n_terms, "segments": n_segs}
    for prec in ("mixed", "fp64"):
        with native.Plan(0, prec, timing=True, hbm_budget_bytes=4 << 30) as plan:
            out = torch.empty(w.n_samples, dtype=plan.out_dtype, device=dev)

            def step():
                sp = plan.spline_fit_kerr(w.t_knots, *ins[:3], w.lmn, ins[3])
                plan.mode_sum(sp, w.theta, w.phi, w.dt, w.n_samples, out=out)
                sp.free()

            for _ in range(warmup):
                step()
            torch.cuda.synchronize()
            plan.timing(reset=True)
            t0 = time.perf_counter()
            for _ in range(steps):
                step()
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / steps
            tm = plan.timing(reset=True)
        sum_ms = tm["sum_ms"] / max(tm["sum_launches"], 1)
        res[prec] = {"value": w.mode_samples / sec, "ms_per_step": sec * 1e3,
                     "spline_ms": tm["spline_ms"] / max(tm["spline_launches"], 1),
                     "sum_ms": sum_ms, "sum_tflops": flops / (sum_ms * 1e-3) / 1e12}
    del ins
    torch.cuda.empty_cache()
    return res


def inner_timing(native, w, dev, reps: int = 20):
    """Fused <d|h>, <h|h> (few_inner_product) on the benchmark case: mean time
    per call after one warm-up, per precision (the spline is fitted once)."""
    import torch
    res = {}
    for prec in ("mixed", "fp64"):
        cdt = torch.complex64 if prec == "mixed" else torch.complex128
        pp, pr, amp = (torch.from_numpy(np.ascontiguousarray(a)).to(dev)
                       for a in (w.phi_phi, w.phi_r, w.amp))
        data = torch.ones(w.n_samples, dtype=cdt, device=dev)
        with native.Plan(0, prec) as plan:
            sp = plan.spline_fit(w.t_knots, pp, pr, w.lmn, amp)
            r = plan.inner_product(sp, w.theta, w.phi, w.dt, w.n_samples, data)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                plan.inner_product(sp, w.theta, w.phi, w.dt, w.n_samples, data, out2=r)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            res[prec] = {"ms": ms, "mode_samples_per_s": w.mode_samples / (ms * 1e-3),
                         "hh": float(r[1].item())}
    return res


def select_timing(native, w, dev, eps: float = 1e-5, reps: int = 20):
    """Mode selector on the benchmark amplitudes: kept modes and mean time."""
    import torch
    amp = torch.from_numpy(np.ascontiguousarray(w.amp)).to(dev)
    with native.Plan(0, "fp64") as plan:
        keep = plan.mode_select(amp, eps)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            plan.mode_select(amp, eps, keep=keep)
        b.record()
        torch.cuda.synchronize()
        return {"eps": eps, "kept": int(keep.sum().item()), "of": w.M,
                "ms": a.elapsed_time(b) / reps}


def batch_run(native, precision: str, dev, n: int, budget: int, reps: int = 3):
    """n uneven instances in one few_batch launch; best of reps after a warmup."""
    import torch
    from paper_2104_04582_amd import synth
    ws = synth.batch_config(n)
    dtype = torch.complex64 if precision == "mixed" else torch.complex128
    reqs = []
    for w in ws:
        reqs.append(dict(t_knots=w.t_knots,
                         phi_phi=torch.from_numpy(np.ascontiguousarray(w.phi_phi)).to(dev),
                         phi_r=torch.from_numpy(np.ascontiguousarray(w.phi_r)).to(dev),
                         lmn=w.lmn,
                         amp=torch.from_numpy(np.ascontiguousarray(w.amp)).to(dev),
                         theta=w.theta, phi=w.phi, dt=w.dt, n_samples=w.n_samples,
                         out=torch.empty(w.n_samples, dtype=dtype, device=dev)))
    ms = sum(w.mode_samples for w in ws)
    flops = sum(path_flops(native, w.lmn, w.n_samples, precision) for w in ws)
    best = None
    with native.Plan(0, precision, hbm_budget_bytes=budget) as plan:
        plan.batch(reqs)
        torch.cuda.synchronize()
        for _ in range(reps):
            t0 = time.perf_counter()
            plan.batch(reqs)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
    del reqs
    torch.cuda.empty_cache()
    # the folded work rate over the whole batch (fit, fold and sum, host enqueue
    # included): subsets of few modes fold less than the full basis, so
    # mode-samples/s alone understates how busy the launch keeps the ALUs
    return {"precision": precision, "waveforms": n, "seconds": best,
            "waveforms_per_s": n / best, "mode_samples": ms, "mode_samples_per_s": ms / best,
            "algorithmic_flop": flops, "algorithmic_tflops": flops / best / 1e12}


def host_threads() -> int:
    """Cores this process may use (affinity mask), at most the 16-core share of
    one GPU on the measurement host."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


CSRC = os.path.join(ROOT, "paper_2104_04582_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sum_mfma_kernel_traffic.txt")


def sources_digest() -> str:
    """sha256 over the kernel sources: kernels.hip and the headers it includes
    (file names and contents, sorted).  The host runtime (*.cpp) does not
    change what a kernel reads or writes."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the summation kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when that summary was
    taken on different native sources than the ones built now."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("sources_sha256") != sources_digest():
        return None
    try:
        return float(fields["fetch_bytes_per_launch"]) + float(fields["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def accuracy(got: np.ndarray, ref: np.ndarray) -> dict:
    """Max relative error (max |got - ref| / max |ref|) and mismatch (unit
    PSD, both polarisations) of a GPU output against the oracle."""
    import oracle
    g = got.astype(np.complex128)
    return {"max_rel_error": float(oracle.max_rel_error(g, ref)),
            "mismatch": float(oracle.mismatch(g, ref)), "samples": int(ref.size)}


def spread_indices(native, w, n_random: int = 3000, seed: int = 1) -> np.ndarray:
    """Both ends, both sides of every interior knot and n_random random
    samples over the whole waveform."""
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(w.n_samples, n_random, replace=False).tolist())
    idx.update([0, 1, w.n_samples - 2, w.n_samples - 1])
    for s in native.host_interval_starts(w.t_knots, w.t_start, w.dt, w.n_samples)[1:-1]:
        idx.update([int(s) - 1, int(s), int(s) + 1])
    return np.array(sorted(i for i in idx if 0 <= i < w.n_samples), dtype=np.int64)


def cpu_baseline(w, target_s: float = 12.0):
    """The oracle as it stands on the host cores, on a contiguous sample slice
    sized (from two short probes, which separate the fixed spline setup from
    the per-sample cost) to take about target_s seconds.  Also returns the
    oracle's output on that slice (the bench compares the GPU outputs with
    it)."""
    import oracle
    threads = host_threads()

    def run(n):
        t0 = time.perf_counter()
        oracle.mode_sum_waveform(w, idx=np.arange(n, dtype=np.int64), n_threads=threads)
        return time.perf_counter() - t0

    a, b = 512, 4096
    ta, tb = run(a), run(b)
    per = max((tb - ta) / (b - a), 1e-9)
    setup = max(ta - a * per, 0.0)
    n_s = int(min(w.n_samples, max(b, (target_s - setup) / per)))
    idx = np.arange(n_s, dtype=np.int64)
    t0 = time.perf_counter()
    ref = oracle.mode_sum_waveform(w, idx=idx, n_threads=threads)
    dt = time.perf_counter() - t0
    return {"value": w.M * n_s / dt, "unit": "mode-samples/s", "cores": threads,
            "kind": "oracle", "cpu_model": host_cpu_model(),
            "sample": f"first {n_s} of {w.n_samples} samples of the 3843-mode 1-yr case, "
                      f"all {w.M} modes, x87 extended precision, {dt:.1f} s wall"}, ref


def cpu_one_core_slice(w, frac: float = 0.01):
    """The oracle on one host core over a contiguous slice of `frac` of the
    one-year case's samples; the whole-waveform time is extrapolated from it
    (the work is linear in the sample count)."""
    import oracle
    n_s = max(1, int(w.n_samples * frac))
    t0 = time.perf_counter()
    oracle.mode_sum_waveform(w, idx=np.arange(n_s, dtype=np.int64), n_threads=1)
    dt = time.perf_counter() - t0
    return {"value": w.M * n_s / dt, "unit": "mode-samples/s", "cores": 1,
            "sample": f"first {n_s} samples ({frac:.0%}) of the 3843-mode 1-yr case",
            "slice_s": dt, "whole_waveform_s_extrapolated": dt / frac,
            "extrapolation": f"x{1 / frac:.0f} (work is linear in samples)"}


def cpu_served_requests(threads: int, n_req: int = 8, max_samples: int = 20000):
    """The oracle on the first n_req requests of the served trace (uneven and
    full requests), first max_samples samples of each, on `threads` cores."""
    import oracle
    from paper_2104_04582_amd import synth
    trace = synth.served_trace(rate=20.0, duration=60.0, p_full=0.1, seed=4)[:n_req]
    work = 0
    sec = 0.0
    kinds = []
    for a in trace:
        w = synth.served_request(a)
        n_s = min(w.n_samples, max_samples)
        t0 = time.perf_counter()
        oracle.mode_sum_waveform(w, idx=np.arange(n_s, dtype=np.int64), n_threads=threads)
        sec += time.perf_counter() - t0
        work += w.M * n_s
        kinds.append(f"{a.kind}:{w.M}")
    return {"value": work / sec, "unit": "mode-samples/s", "cores": threads,
            "sample": f"first {n_req} served requests ({', '.join(kinds)} modes), first "
                      f"{max_samples} samples of each", "seconds": sec}


def cpu_small(threads: int):
    """The oracle on the whole one-day, 132-mode case (8640 samples), on one
    host core and on `threads` cores: a reported context figure beside the
    bounded baseline above."""
    import oracle
    from paper_2104_04582_amd import synth
    w = synth.config0()
    res = {"workload": f"{w.M} modes x {w.n_samples} samples (1 day at dt = 10 s), whole "
                       "waveform, x87 extended precision", "unit": "mode-samples/s"}
    for key, n in (("one_core", 1), ("all_cores", threads)):
        t0 = time.perf_counter()
        oracle.mode_sum_waveform(w, n_threads=n)
        res[key] = w.mode_samples / (time.perf_counter() - t0)
    res["cores"] = threads
    return res


def served(native, precision: str, seconds: float, dev, budget: int,
           check_oracle: bool = True, request_log=None):
    """Replay a Poisson trace (20 req/s, 10% full 4-yr requests) through
    few_submit/few_poll; latency = arrival -> completion seen by the host.
    The client submits at the arrival time (it sleeps until shortly before an
    arrival, then spins) and, while requests are pending, polls them back to
    back, so that its own sleeps add no latency."""
    import torch
    from paper_2104_04582_amd import synth
    trace = synth.served_trace(rate=20.0, duration=seconds, p_full=0.1, seed=4)
    reqs = []
    for a in trace:
        w = synth.served_request(a)
        reqs.append((a, w,
                     torch.from_numpy(np.ascontiguousarray(w.phi_phi)).to(dev),
                     torch.from_numpy(np.ascontiguousarray(w.phi_r)).to(dev),
                     torch.from_numpy(np.ascontiguousarray(w.amp)).to(dev)))
    out_dtype = torch.complex64 if precision == "mixed" else torch.complex128
    torch.cuda.synchronize()
    lat = []
    kinds = []
    mode_samples = 0
    first_full = None   # (waveform, output) of the first full request served
    with native.Plan(0, precision, hbm_budget_bytes=budget, max_inflight=4) as plan:
        if request_log:
            plan.request_log(f"{request_log}.{precision}.jsonl")
        pending = {}
        t_start = time.perf_counter()
        nxt = 0
        while nxt < len(reqs) or pending:
            now = time.perf_counter() - t_start
            while nxt < len(reqs) and reqs[nxt][0].t_arrival <= now:
                a, w, pp, pr, amp = reqs[nxt]
                out = torch.empty(w.n_samples, dtype=out_dtype, device=dev)
                tk = plan.submit(w.t_knots, pp, pr, w.lmn, amp, w.theta, w.phi, w.dt,
                                 w.n_samples, out)
                pending[tk] = (a, w, out)
                nxt += 1
            done = [tk for tk in pending if plan.poll(tk)]
            t_done = time.perf_counter() - t_start
            for tk in done:
                a, w, out = pending.pop(tk)
                lat.append(t_done - a.t_arrival)
                kinds.append(a.kind)
                mode_samples += w.mode_samples
                if a.kind == "full" and first_full is None:
                    first_full = (w, out)
            if not done:
                if pending:
                    time.sleep(0)
                elif nxt < len(reqs):
                    wait = reqs[nxt][0].t_arrival - (time.perf_counter() - t_start)
                    if wait > 2e-3:
                        time.sleep(wait - 1e-3)
        wall = time.perf_counter() - t_start
    lat = np.array(lat) * 1e3
    kinds = np.array(kinds)

    def pct(x, q):
        return float(np.percentile(x, q)) if x.size else None

    vs_oracle = None
    if first_full is not None and check_oracle:
        import oracle
        w, out = first_full
        idx = spread_indices(native, w)
        ref = oracle.mode_sum_waveform(w, idx=idx, n_threads=host_threads())
        got = out[torch.from_numpy(idx).to(dev)].cpu().numpy()
        vs_oracle = dict(accuracy(got, ref), request=f"first full request ({w.M} modes, "
                         f"{w.n_samples} samples, 4 yr), ends, knots and random samples")
    return {"precision": precision, "requests": int(lat.size), "trace_s": seconds,
            "vs_oracle": vs_oracle,
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
            "p50_full_ms": pct(lat[kinds == "full"], 50),
            "p99_full_ms": pct(lat[kinds == "full"], 99),
            "p50_small_ms": pct(lat[kinds == "small"], 50),
            "p99_small_ms": pct(lat[kinds == "small"], 99),
            "mode_samples_per_s": mode_samples / wall, "waveforms_per_s": lat.size / wall}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-kerr", action="store_true", help="skip the generic-Kerr line")
    ap.add_argument("--batch", type=int, default=128, help="uneven instances in one launch")
    ap.add_argument("--request-log", default=None, metavar="PREFIX",
                    help="served replay: per-request JSON lines in PREFIX.<precision>.jsonl")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        x = torch.empty(args.copy_probe << 20, dtype=torch.uint8, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel(), "copies": 5}), flush=True)
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import torch
    from paper_2104_04582_amd import native, synth
    dev = torch.device("cuda:0")
    w = synth.config1()
    segs, tp, _ = native.host_terms(w.lmn)
    n_terms, n_segs = tp.shape[0] - 1, segs.shape[0]
    n_rows = len(set(int(x) for x in segs[:, 0]))
    mfma = native.host_mfma_path(w.lmn)
    flops_vec = algorithmic_flops(n_terms, n_segs, w.n_samples)
    flops_mf = mfma_algorithmic_flops(n_terms, n_rows, w.n_samples)
    canonical = 32.0 * w.M * w.n_samples
    n_wg = torch.cuda.get_device_properties(0).multi_processor_count
    mf_instr = mfma_instructions(native, w, n_wg) if mfma else 0
    log(f"[bench] workload K={w.K} M={w.M} N={w.n_samples} terms={n_terms} segs={n_segs} "
        f"matrix-core path={mfma} ({mf_instr} MFMA instructions per launch on {n_wg} CUs)")

    res = {}
    outs = {}
    # "mixed" is the headline (matrix-core summation for this mode list);
    # "mixed_vector" the same precision on the vector units only
    for prec in ("mixed", "fp64", "mixed_vector"):
        pp = "mixed" if prec == "mixed_vector" else prec
        vec = prec == "mixed_vector"
        log(f"[bench] {prec}: warmup {args.warmup} (and >= 0.2 s), steps {args.steps}")
        # Timed region: HIP events around every 8th summation launch only (an
        # event pair delays the launch after it; the other stages and the
        # other steps stay back to back).
        with native.Plan(0, pp, timing="sum_sparse", vector_only=vec) as plan:
            sec, tm, out, step = time_path(native, plan, w, dev, args.steps, args.warmup, 0.2)
            spread = step_spread(step, args.steps)
            if not vec:
                outs[prec] = out
            del out
        # Stage breakdown: the same steps with events around every launch.
        with native.Plan(0, pp, timing=True, vector_only=vec) as plan:
            _, tms, _, _ = time_path(native, plan, w, dev, 5, 2)
        if tm["sum_launches"] < 1:
            raise RuntimeError("no summation launch of the timed pass was timed")
        sum_ms = tm["sum_ms"] / tm["sum_launches"]
        flops = flops_mf if (prec == "mixed" and mfma) else flops_vec
        res[prec] = {
            "ms_per_step": sec * 1e3,
            "value": w.mode_samples / sec,
            "spline_ms": tms["spline_ms"] / max(tms["spline_launches"], 1),
            "prepare_ms": tms["prepare_ms"] / max(tms["prepare_launches"], 1),
            "sum_ms": sum_ms,
            "sum_tflops": flops / (sum_ms * 1e-3) / 1e12,
            "canonical_tflops": canonical / (sum_ms * 1e-3) / 1e12,
            "step_spread": spread,
        }
        log(f"[bench] {prec}: {json.dumps(res[prec])}")
    a = outs["fp64"]
    b = outs["mixed"].to(torch.complex128)
    num = torch.real(torch.vdot(a, b)).item()
    den = math.sqrt(torch.real(torch.vdot(a, a)).item() * torch.real(torch.vdot(b, b)).item())
    mm = 1.0 - num / den
    mx = (torch.max(torch.abs(a - b)) / torch.max(torch.abs(a))).item()
    host_out = {p: outs[p].cpu().numpy() for p in outs}
    del outs, a, b
    torch.cuda.empty_cache()

    # mode selector (the step before the path) on the same amplitudes
    sel = select_timing(native, w, dev)
    log(f"[bench] mode select: {json.dumps(sel)}")

    inner = inner_timing(native, w, dev)
    log(f"[bench] fused inner products: {json.dumps(inner)}")

    kerr = None
    if not args.no_kerr:
        log("[bench] generic-Kerr sum")
        kerr = kerr_run(native, dev)
        log(f"[bench] kerr: {json.dumps(kerr)}")

    batch = {}
    if args.batch > 0:
        for prec in ("mixed", "fp64"):
            log(f"[bench] batched launch of {args.batch} uneven instances, {prec}")
            batch[prec] = batch_run(native, prec, dev, args.batch, 16 << 30)
            log(f"[bench] batch {prec}: {json.dumps(batch[prec])}")

    serve = {}
    if args.serve_seconds > 0:
        for prec in ("mixed", "fp64"):
            log(f"[bench] served replay {prec}, {args.serve_seconds:.0f} s")
            serve[prec] = served(native, prec, args.serve_seconds, dev, 8 << 30,
                                 request_log=args.request_log)
            log(f"[bench] served {prec}: {json.dumps(serve[prec])}")

    cpu = None
    cpu_1day = cpu_1core = cpu_served = None
    vs_oracle = None
    if not args.no_cpu:
        import oracle
        log("[bench] cpu oracle baseline")
        cpu, ref_slice = cpu_baseline(w)
        log(f"[bench] cpu: {json.dumps(cpu)}")
        # accuracy of both GPU outputs against the oracle: on the baseline's
        # contiguous slice and on samples spread over the whole year
        idx = spread_indices(native, w)
        ref_spread = oracle.mode_sum_waveform(w, idx=idx, n_threads=cpu["cores"])
        n_s = ref_slice.size
        vs_oracle = {p: {"slice": accuracy(host_out[p][:n_s], ref_slice),
                         "spread": accuracy(host_out[p][idx], ref_spread)}
                     for p in host_out}
        vs_oracle["samples"] = {"slice": f"first {n_s} samples",
                                "spread": "both ends, both sides of every knot, 3000 random"}
        log(f"[bench] vs oracle: {json.dumps(vs_oracle)}")
        cpu_1day = cpu_small(cpu["cores"])
        log(f"[bench] cpu, one-day case: {json.dumps(cpu_1day)}")
        cpu_1core = cpu_one_core_slice(w)
        log(f"[bench] cpu, one core, 1% slice: {json.dumps(cpu_1core)}")
        cpu_served = cpu_served_requests(cpu["cores"])
        log(f"[bench] cpu, served requests: {json.dumps(cpu_served)}")

    m = res["mixed"]
    ach = m["sum_tflops"]
    line = {
        "metric": "mode-samples/s at 3843 modes x 1 yr (mixed vs FP64); p50/p99 served latency",
        "value": m["value"],
        "unit": "mode-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "step_ms": {"mean": m["ms_per_step"], "median": m["step_spread"]["median_ms"],
                    "min": m["step_spread"]["min_ms"],
                    "note": "median and min from a second pass with an event between steps"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16/f32" if mfma else "f32",
        "data": "synthetic",
        "config": {"workload": "interpolated mode sum, 3843 modes (l 2..10, m 0..l, n -30..30), "
                               "100 knots, 1 yr at dt 10 s (3,155,760 samples), mixed precision",
                   "modes": w.M, "knots": w.K, "samples": w.n_samples,
                   "folded_terms": n_terms, "segments": n_segs,
                   "summation": "matrix cores: fp16 hi/lo operands, fp32 accumulation" if mfma
                   else "vector units: binary32, Kahan-compensated"},
        "roofline": ({"bound": "mfma", "achieved": ach, "peak": PEAK_FP16_MFMA,
                      "unit": "TFLOP/s", "frac": ach / PEAK_FP16_MFMA,
                      "traffic": measured_traffic(),
                      "kernel": "sum_mfma_kernel<false>",
                      "flop_per_launch": flops_mf,
                      "flop_count": "folded contraction counted once: 32 flop per folded "
                                    "term and sample + 8 per signed-m row and sample",
                      "launch_ms": m["sum_ms"],
                      "executed_mfma_instructions": mf_instr,
                      "executed_mfma_tflops": mf_instr * 16384.0 / (m["sum_ms"] * 1e-3) / 1e12,
                      "executed_mfma_frac": mf_instr * 16384.0 / (m["sum_ms"] * 1e-3) / 1e12
                      / PEAK_FP16_MFMA,
                      "canonical_32flop_frac": m["canonical_tflops"] / PEAK_FP16_MFMA}
                     if mfma else
                     {"bound": "alu", "achieved": ach, "peak": PEAK_FP32_VALU,
                      "unit": "TFLOP/s", "frac": ach / PEAK_FP32_VALU,
                      "traffic": measured_traffic(),
                      "kernel": "sum_wg_kernel<float>",
                      "flop_per_launch": flops_vec, "launch_ms": m["sum_ms"]}),
        "mixed_vector": {"value": res["mixed_vector"]["value"],
                         "ms_per_step": res["mixed_vector"]["ms_per_step"],
                         "sum_ms": res["mixed_vector"]["sum_ms"],
                         "sum_tflops": res["mixed_vector"]["sum_tflops"],
                         "frac_fp32_peak": res["mixed_vector"]["sum_tflops"] / PEAK_FP32_VALU,
                         "note": "the same precision with FEW_FLAG_VECTOR_ONLY: binary32 "
                                 "vector-unit summation with Kahan-compensated accumulation"},
        "fp64": {"value": res["fp64"]["value"], "ms_per_step": res["fp64"]["ms_per_step"],
                 "sum_ms": res["fp64"]["sum_ms"], "sum_tflops": res["fp64"]["sum_tflops"],
                 "step_ms": {"median": res["fp64"]["step_spread"]["median_ms"],
                             "min": res["fp64"]["step_spread"]["min_ms"]},
                 "frac_fp64_peak": res["fp64"]["sum_tflops"] / PEAK_FP64_VALU},
        "stages_ms": {p: {k: res[p][k] for k in ("spline_ms", "prepare_ms", "sum_ms")}
                      for p in res},
        "canonical_32flop_tflops": {p: res[p]["canonical_tflops"] for p in res},
        "vs_oracle": vs_oracle,
        "mixed_vs_fp64": {"mismatch": mm, "max_rel_error": mx},
        "mode_select": sel,
        "fused_inner": inner,
        "kerr": kerr,
        "batched": batch or None,
        "served": serve or None,
        "cpu_baseline": cpu,
        "cpu_oracle_1day": cpu_1day,
        "cpu_oracle_1core": cpu_1core,
        "cpu_oracle_served": cpu_served,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
