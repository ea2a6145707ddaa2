"""CPU tests of libfew's host side: exported symbols and the host helpers
(term layout, interval starts, footprint).  No device work."""
import os
import re

import numpy as np
import pytest

from paper_2104_04582_amd import native, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "few.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(few_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = native.load()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(native.EXPORTED) == set(names)


def test_mode_counts_golden():
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "mode_counts.txt"))
            if l.strip() and not l.startswith("#")]
    got = {"schwarzschild_full": len(synth.mode_list(2, 10, 30)),
           "ff22": sum(1 for l, m, n in synth.mode_list(2, 2, 30) if m == 2)}
    for r in rows:
        assert got[r[0]] == int(r[5]), r


def check_layout(lmn, max_gap):
    segs, tp, src = native.host_terms(lmn, max_gap)
    n_terms = tp.shape[0] - 1
    # every listed mode once as itself and, for m > 0, once as its mirror
    seen = {}
    for s_idx, (m, n_lo, ln, first) in enumerate(segs):
        assert ln >= 1
        if s_idx + 1 < len(segs):
            assert segs[s_idx + 1][3] == first + ln
        for q in range(ln):
            term = first + q
            for e in range(tp[term], tp[term + 1]):
                k, packed = src[e]
                l, mm, mir = packed & 255, (packed >> 8) & 255, (packed >> 16) & 1
                L, Mm, N = lmn[k]
                assert (l, mm) == (L, Mm)
                if mir:
                    assert (m, n_lo + q) == (-Mm, -N)
                else:
                    assert (m, n_lo + q) == (Mm, N)
                seen[(k, mir)] = seen.get((k, mir), 0) + 1
    for k, (L, Mm, N) in enumerate(lmn):
        assert seen.get((k, 0)) == 1
        assert seen.get((k, 1), 0) == (1 if Mm > 0 else 0)
    # segments sorted by (m, n_lo); gaps inside a segment never exceed max_gap
    keys = [(m, n) for m, n, _, _ in segs]
    assert keys == sorted(keys)
    for m, n_lo, ln, first in segs:
        run = 0
        for q in range(ln):
            empty = tp[first + q] == tp[first + q + 1]
            run = run + 1 if empty else 0
            assert run <= max_gap
        assert tp[first] != tp[first + 1] and tp[first + ln - 1] != tp[first + ln]
    return segs, tp, src


def test_term_layout_full_mode_set():
    lmn = synth.mode_list(2, 10, 30)
    segs, tp, src = check_layout(lmn, 4)
    assert segs.shape[0] == 21            # m = -10..10
    assert tp.shape[0] - 1 == 21 * 61      # 671 listed (m, n) + 610 mirrored
    assert src.shape[0] == 3843 + 3294     # modes + mirrors of the m > 0 modes


@pytest.mark.parametrize("seed", range(6))
def test_term_layout_random_subsets(seed):
    rng = np.random.default_rng(seed)
    full = synth.mode_list(2, 8, 12)
    pick = rng.choice(full.shape[0], size=int(rng.integers(1, 60)), replace=True)
    lmn = full[pick]
    for gap in (0, 2, 4, 9):
        check_layout(lmn, gap)


def test_term_layout_rejects_bad_modes():
    with pytest.raises(native.FewError) as e:
        native.host_terms(np.array([[1, 0, 0]]))
    assert e.value.code == native.FEW_E_MODES
    with pytest.raises(native.FewError):
        native.host_terms(np.array([[3, 4, 0]]))
    with pytest.raises(native.FewError):
        native.host_terms(np.array([[31, 0, 0]]))


@pytest.mark.parametrize("cfg", ["c0", "c1", "tiny", "offset"])
def test_interval_starts_match_binary64_search(cfg):
    if cfg == "c0":
        w = synth.config0()
        t0, dt, n = 0.0, w.dt, w.n_samples
    elif cfg == "c1":
        w = synth.config1()
        t0, dt, n = 0.0, w.dt, w.n_samples
    elif cfg == "tiny":
        w = synth.tiny_waveform(3, K=7, n_samples=33)
        t0, dt, n = 0.0, w.dt, w.n_samples
    else:
        w = synth.tiny_waveform(4, K=9, n_samples=50)
        t0 = w.t_knots[1] * 0.5
        dt = (w.t_knots[-1] - t0) / 41.0
        n = 42
    got = native.host_interval_starts(w.t_knots, t0, dt, n)
    ts = t0 + np.arange(n, dtype=np.float64) * dt
    ref = np.searchsorted(ts, w.t_knots, side="left")
    ref[0] = 0
    ref[-1] = n
    np.testing.assert_array_equal(got, ref)


def test_interval_starts_on_knot_samples():
    """Samples that land exactly on a knot belong to the interval it starts."""
    t = np.array([0.0, 10.0, 20.0, 30.0, 40.0])
    got = native.host_interval_starts(t, 0.0, 5.0, 9)
    np.testing.assert_array_equal(got, [0, 2, 4, 6, 9])


def test_request_bytes():
    a = native.host_request_bytes("fp64", 100, 3843, 1281)
    b = native.host_request_bytes("mixed", 100, 3843, 1281)
    # a binary32 request long enough for the matrix-core path holds the fp16
    # operand table (99 intervals x 48 KiB) instead of a binary64 fold table
    # (99 x 1281 x 64 B)
    assert a > b > 99 * 3843 * 64
    # (plus the per-interval row scales and row list, a few KiB)
    assert abs((b - a) - (99 * 48 * 1024 - 99 * 1281 * 64)) <= 16384
    # shorter binary32 requests keep the binary32 fold table only
    c = native.host_request_bytes("fp64", 100, 300, 400)
    d = native.host_request_bytes("mixed", 100, 300, 400)
    assert c > d
    assert native.host_request_bytes("fp64", 3, 10, 10) == 0


def check_layout_kerr(lmkn, max_gap):
    """Generic-Kerr layout: every listed (l, m, k, n) once as itself and, for
    m > 0, once as its mirror (-m, -k, -n); segments of one signed (m, k) with
    contiguous n, in (m, k, n) order."""
    segs, tp, src = native.host_terms(lmkn, max_gap)
    seen = {}
    keys = []
    for s_idx, (x, n_lo, ln, first) in enumerate(segs):
        k = (int(x) + 128) >> 8
        m = int(x) - 256 * k
        keys.append((m, k, int(n_lo)))
        if s_idx + 1 < len(segs):
            assert segs[s_idx + 1][3] == first + ln
        for q in range(ln):
            for e in range(tp[first + q], tp[first + q + 1]):
                idx, packed = src[e]
                l, mm, mir = packed & 255, (packed >> 8) & 255, (packed >> 16) & 1
                kp = ((packed >> 17) & 127) - 64
                L, Mm, Kk, N = lmkn[idx]
                assert (l, mm) == (L, Mm)
                if mir:
                    assert (m, k, n_lo + q, kp) == (-Mm, -Kk, -N, -Kk)
                else:
                    assert (m, k, n_lo + q, kp) == (Mm, Kk, N, Kk)
                seen[(idx, mir)] = seen.get((idx, mir), 0) + 1
    for idx, (L, Mm, Kk, N) in enumerate(lmkn):
        assert seen.get((idx, 0)) == 1
        assert seen.get((idx, 1), 0) == (1 if Mm > 0 else 0)
    assert keys == sorted(keys)
    return segs, tp, src


def test_kerr_term_layout_full_mode_set():
    lmkn = synth.mode_list_kerr(2, 10, 4, 30)
    assert lmkn.shape[0] == 34587
    segs, tp, src = check_layout_kerr(lmkn, 4)
    assert segs.shape[0] == 21 * 9                   # signed (m, k)
    assert tp.shape[0] - 1 == 21 * 9 * 61            # signed (m, k, n)
    n_m0 = int(np.sum(lmkn[:, 1] == 0))
    assert src.shape[0] == 34587 + (34587 - n_m0)


@pytest.mark.parametrize("seed", range(4))
def test_kerr_term_layout_random_subsets(seed):
    rng = np.random.default_rng(100 + seed)
    full = synth.mode_list_kerr(2, 6, 3, 8)
    lmkn = full[rng.choice(full.shape[0], size=int(rng.integers(1, 80)), replace=True)]
    for gap in (0, 3):
        check_layout_kerr(lmkn, gap)


def test_kerr_k_zero_layout_equals_schwarzschild():
    """k = 0 everywhere: the same segments, terms and contributors as the
    (l, m, n) layout (contributor words carry k + 64 = 64 in both)."""
    lmn = synth.mode_list(2, 6, 7)
    a = native.host_terms(lmn)
    b = native.host_terms(np.insert(lmn, 2, 0, axis=1))
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_kerr_layout_rejects_bad_modes():
    with pytest.raises(native.FewError) as e:
        native.host_terms(np.array([[2, 1, 31, 0]]))
    assert e.value.code == native.FEW_E_MODES
    with pytest.raises(native.FewError):
        native.host_terms(np.array([[2, 3, 0, 0]]))


@pytest.mark.parametrize("seed", range(8))
def test_host_frame_matches_oracle(seed):
    import math
    from oracle.frame import frame_angles
    rng = np.random.default_rng(seed)
    ts, ps = math.acos(rng.uniform(-1, 1)), rng.uniform(0, 2 * math.pi)
    tk, pk = math.acos(rng.uniform(-1, 1)), rng.uniform(0, 2 * math.pi)
    th, ph, rot = native.host_frame(ts, ps, tk, pk)
    t_ref, p_ref, psi = frame_angles(ts, ps, tk, pk)
    assert abs(th - t_ref) < 1e-12 and ph == p_ref
    assert abs(rot - (-np.exp(-2j * psi))) < 1e-12


def test_host_frame_errors_and_degenerate():
    with pytest.raises(native.FewError) as e:
        native.host_frame(float("nan"), 0.0, 0.1, 0.2)
    assert e.value.code == native.FEW_E_ARG
    th, ph, rot = native.host_frame(0.4, 1.0, 0.4, 1.0)        # R = S
    assert abs(th - np.pi) < 1e-7 and rot == -1.0


def test_mfma_path_and_shape():
    """Which binary32 requests take the matrix-core summation: at most 24
    signed m values, |n| < 32 and at least 480 folded terms (Schwarzschild
    lists only)."""
    shape = native.host_mfma_shape()
    assert shape["max_rows"] == 24 and shape["abs_n_limit"] == 32
    assert shape["min_terms"] == 480
    # per 16-sample tile and round: 4 powers x row tiles x column steps x
    # 3 hi/lo products (the terms n and -n share one operand fragment)
    assert shape["mfma_per_tile"] == 4 * shape["row_tiles"] * shape["column_steps"] * 3
    full = synth.mode_list(2, 10, 30)                 # 21 signed m, |n| <= 30, 1281 terms
    assert native.host_mfma_path(full)
    assert not native.host_mfma_path(synth.mode_list(2, 4, 5))        # 99 terms
    assert native.host_mfma_path(synth.mode_list(2, 10, 31))          # |n| = 31
    assert not native.host_mfma_path(synth.mode_list(2, 10, 32))      # |n| = 32
    assert not native.host_mfma_path(synth.mode_list(2, 12, 20))      # 25 signed m
    with pytest.raises(native.FewError):
        native.host_mfma_path(np.array([[1, 0, 0]], dtype=np.int32))


def test_xcd_split_step_keeps_balanced_weights():
    """Equal finishing times leave weights of mean 1 unchanged."""
    w = np.array([1.2, 0.8, 1.0, 1.1, 0.9, 1.0, 1.05, 0.95])
    assert abs(w.mean() - 1.0) < 1e-15
    nxt = native.host_xcd_split_step(w, np.full(8, 3.0e4))
    np.testing.assert_allclose(nxt, w, rtol=0, atol=1e-15)


def test_xcd_split_step_moves_half_way_and_keeps_mean_one():
    """A slow XCD loses share, the others gain, by half a step of the
    proportional correction; the result has mean 1 when nothing is clamped."""
    t = np.full(8, 1.0)
    t[3] = 1.25
    nxt = native.host_xcd_split_step(np.ones(8), t)
    mean_t = t.mean()
    raw = 1.0 + 0.5 * (mean_t / t - 1.0)
    np.testing.assert_allclose(nxt, raw / raw.mean(), rtol=1e-14)
    assert nxt[3] < 1.0 and np.all(np.delete(nxt, 3) > 1.0)
    assert abs(nxt.mean() - 1.0) < 1e-14


def test_xcd_split_step_converges_to_equal_finishing_times():
    """With XCD x taking c_x per unit of work (time = weight x c_x), repeated
    steps reach the split w_x proportional to 1 / c_x, where every XCD
    finishes together."""
    c = np.array([1.00, 1.04, 0.97, 1.10, 1.00, 0.93, 1.02, 1.06])
    w = np.ones(8)
    for _ in range(60):
        w = native.host_xcd_split_step(w, w * c)
    target = (1.0 / c) / np.mean(1.0 / c)
    np.testing.assert_allclose(w, target, rtol=1e-9)
    t = w * c
    assert t.max() / t.min() - 1.0 < 1e-9


def test_xcd_split_step_clamps_and_rejects_bad_input():
    """Weights stay within [1/2, 2]; non-positive or non-finite times are an
    argument error."""
    t = np.ones(8)
    t[0] = 1e6                                   # one XCD far slower
    w = np.ones(8)
    for _ in range(20):
        w = native.host_xcd_split_step(w, t)
        assert np.all(w >= 0.5) and np.all(w <= 2.0)
    assert w[0] == 0.5
    for bad in (0.0, -1.0, np.inf, np.nan):
        t = np.ones(8)
        t[5] = bad
        with pytest.raises(native.FewError):
            native.host_xcd_split_step(np.ones(8), t)
