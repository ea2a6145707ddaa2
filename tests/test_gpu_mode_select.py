"""GPU mode selector against the oracle: the masks must be identical."""
import numpy as np
import pytest

from oracle.mode_select import mode_select
from paper_2104_04582_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2104_04582_amd import native
    native.load()
    return native, torch, torch.device("cuda:0")


def gpu_select(env, amp, eps, sorted_only=False):
    native, torch, dev = env
    a = torch.from_numpy(np.ascontiguousarray(amp, dtype=np.float64)).to(dev)
    with native.Plan(0, "fp64", select_sorted=sorted_only) as plan:
        keep = plan.mode_select(a, eps)
        torch.cuda.synchronize()
        return keep.cpu().numpy()


@pytest.mark.parametrize("sorted_only", [False, True], ids=["bounded", "sorted"])
@pytest.mark.parametrize("eps", [0.0, 1e-12, 1e-9, 1e-5, 1e-2, 0.5, 0.99])
def test_full_mode_set(env, eps, sorted_only):
    w = synth.config1()
    ref = mode_select(w.amp, eps)
    got = gpu_select(env, w.amp, eps, sorted_only)
    print(f"[select] eps={eps} sorted={sorted_only}: kept {int(ref.sum())} of {ref.size}",
          flush=True)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("sorted_only", [False, True], ids=["bounded", "sorted"])
@pytest.mark.parametrize("seed", range(5))
def test_random_with_ties_and_zeros(env, seed, sorted_only):
    rng = np.random.default_rng(seed)
    K, M = int(rng.integers(1, 9)), int(rng.integers(1, 300))
    amp = np.round(rng.standard_normal((K, M, 2)), 1)       # many exact ties
    amp[:, rng.random(M) < 0.2, :] = 0.0
    for eps in (0.0, 0.05, 0.4):
        np.testing.assert_array_equal(gpu_select(env, amp, eps, sorted_only),
                                      mode_select(amp, eps))


def test_bounded_stage_on_spread_and_tied_powers(env):
    """Powers over many binades (several radix levels), runs of equal powers
    at the cut (ranked by index), and comparisons that meet the threshold
    exactly (decided by the sorted stage)."""
    rng = np.random.default_rng(11)
    K, M = 6, 4000
    mag = np.exp(rng.uniform(-30.0, 0.0, size=(K, M)))
    amp = np.stack([mag, np.zeros_like(mag)], axis=-1)
    amp[:, 1000:1400, 0] = amp[:, 1000:1001, 0]                 # 400 equal powers
    amp[:, 3000:3010, :] = 0.0
    for eps in (1e-9, 1e-5, 1e-3, 0.1, 0.9):
        np.testing.assert_array_equal(gpu_select(env, amp, eps), mode_select(amp, eps))
    # two equal powers and eps = 1/2: the second mode's preceding sum equals
    # the threshold, so it is dropped
    two = np.array([[[1.0, 0.0], [1.0, 0.0]]])
    assert mode_select(two, 0.5).tolist() == [1, 0]
    np.testing.assert_array_equal(gpu_select(env, two, 0.5), [1, 0])
    # all powers equal: the lowest indices are kept
    flat = np.ones((2, 257, 2))
    np.testing.assert_array_equal(gpu_select(env, flat, 0.3), mode_select(flat, 0.3))


def test_limits(env):
    native, torch, dev = env
    amp = np.random.default_rng(7).standard_normal((2, 4096, 2))
    np.testing.assert_array_equal(gpu_select(env, amp, 1e-3), mode_select(amp, 1e-3))
    one = np.array([[[0.3, 0.4]]])
    np.testing.assert_array_equal(gpu_select(env, one, 0.5), [1])
    # no power at any knot: only the first mode (ties go to the lower index)
    zero = np.zeros((3, 65, 2))
    np.testing.assert_array_equal(gpu_select(env, zero, 0.1), mode_select(zero, 0.1))
    assert mode_select(zero, 0.1).tolist() == [1] + [0] * 64
    with native.Plan(0, "fp64") as plan:
        a = torch.zeros((2, 4097, 2), dtype=torch.float64, device=dev)
        with pytest.raises(native.FewError) as e:
            plan.mode_select(a, 0.1)
        assert e.value.code == native.FEW_E_MODES
        with pytest.raises(native.FewError) as e:
            plan.mode_select(a[:, :10].contiguous(), 1.0)
        assert e.value.code == native.FEW_E_ARG
