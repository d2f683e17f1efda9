"""The flagPermute entry point that allocates nothing
(qh_test_flag_permute_noalloc) against the one that allocates its scratch
(qh_test_flag_permute): the same permutation and head flags, bit for bit,
on consecutive calls that share the library's fixed scratch (the second one
smaller, so stale contents of the first would show), and its size limit."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qhm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1201_2936_amd import qh
    qh.load()
    return qh


def _inputs(seed, n, k, head_rate):
    rng = np.random.default_rng(seed)
    f = rng.integers(0, k, size=n).astype(np.int32)
    s = (rng.random(n) < head_rate).astype(np.uint8)
    s[0] = 1
    return torch.from_numpy(f).cuda(), torch.from_numpy(s).cuda()


def _both(qhm, f, s, k):
    p_ref, s_ref = qhm.qh_test_flag_permute(f, s, k)
    p_na, s_na = qhm.qh_test_flag_permute(f, s, k, noalloc=True)
    torch.cuda.synchronize()
    return p_ref.cpu().numpy(), s_ref.cpu().numpy(), p_na.cpu().numpy(), s_na.cpu().numpy()


def test_two_calls_match_the_allocating_call(qhm):
    # the larger call first (many heads, every state), then a smaller one with
    # fewer heads: its head flags must not keep any of the first call's
    cases = [(1, 700_000, 5, 0.01), (2, 40_000, 3, 0.0005)]
    for seed, n, k, rate in cases:
        f, s = _inputs(seed, n, k, rate)
        p_ref, s_ref, p_na, s_na = _both(qhm, f, s, k)
        assert np.array_equal(p_na, p_ref), (seed, n, k)
        assert np.array_equal(s_na, s_ref), (seed, n, k)
        assert np.array_equal(np.sort(p_na), np.arange(n))


def test_largest_size_and_ragged_tile(qhm):
    # 2 states: the largest n the fixed scratch takes (4,186,095), not a
    # multiple of the 1,024-element tile
    n = 4_186_095
    f, s = _inputs(3, n, 2, 0.001)
    p_ref, s_ref, p_na, s_na = _both(qhm, f, s, 2)
    assert np.array_equal(p_na, p_ref)
    assert np.array_equal(s_na, s_ref)


def test_limit_and_bad_state(qhm):
    lib = qhm.load()
    # beyond the fixed scratch: rejected before any device work
    n = 4_000_000
    f, s = _inputs(4, n, 16, 0.01)
    p = torch.empty(n, dtype=torch.int32, device="cuda")
    sn = torch.empty(n, dtype=torch.uint8, device="cuda")
    rc = lib.qh_test_flag_permute_noalloc(ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(s.data_ptr()), n, 16,
                                          ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(sn.data_ptr()), None)
    assert rc == qhm.QH_ECAPACITY
    # a state outside [0, k) is reported; the next call starts from a clear flag
    with pytest.raises(qhm.QhError) as ei:
        qhm.qh_test_flag_permute(torch.tensor([0, 1, 5], dtype=torch.int32, device="cuda"),
                                 torch.tensor([1, 0, 0], dtype=torch.uint8, device="cuda"), 3, noalloc=True)
    assert ei.value.status == qhm.QH_EINVAL
    f, s = _inputs(5, 5000, 3, 0.1)
    p_ref, s_ref, p_na, s_na = _both(qhm, f, s, 3)
    assert np.array_equal(p_na, p_ref) and np.array_equal(s_na, s_ref)
