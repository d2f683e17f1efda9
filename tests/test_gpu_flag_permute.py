"""Parity of the GPU flagPermute primitive with the oracle's (Figure 1).

The permutation and the new head flags are integer outputs: bit-exact.
"""
import os

import numpy as np
import pytest

from oracle import segmented

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "figure1_flagpermute.txt")


@pytest.fixture(scope="module")
def qhm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1201_2936_amd import qh
    qh.load()
    return qh


def _rows():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, *vals = line.split()
        rows[name] = [int(v) for v in vals]
    return rows


def _gpu(qhm, f, s, k):
    ft = torch.tensor(np.asarray(f, np.int32), device="cuda")
    st = torch.tensor(np.asarray(s, np.uint8), device="cuda")
    p, sn = qhm.qh_test_flag_permute(ft, st, k)
    return p.cpu().numpy(), sn.cpu().numpy()


def test_figure1(qhm):
    r = _rows()
    p, sn = _gpu(qhm, r["f"], r["s"], 3)
    assert p.tolist() == r["p"]
    assert sn.tolist() == r["s'"]


@pytest.mark.parametrize("seed", range(12))
def test_random_vs_oracle(qhm, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.choice([1, 2, 7, 1023, 1024, 1025, 5000, 40000]))
    k = int(rng.integers(1, 6))
    f = rng.integers(0, k, size=n)
    s = (rng.random(n) < rng.choice([0.0, 0.01, 0.3, 1.0])).astype(np.uint8)
    s[0] = 1
    want_p, want_s = segmented.flag_permute(f, s, k)
    p, sn = _gpu(qhm, f, s, k)
    assert p.tolist() == want_p.tolist()
    assert sn.tolist() == want_s.tolist()
    # properties at any size: a permutation, grouped by state inside every
    # segment, stable
    assert sorted(p.tolist()) == list(range(n))
    inv = np.empty(n, np.int64)
    inv[p] = np.arange(n)
    heads = np.flatnonzero(s)
    ends = np.append(heads[1:], n)
    for h, e in zip(heads, ends):
        assert (inv[h:e] >= h).all() and (inv[h:e] < e).all()
        states = f[inv[h:e]]
        assert (np.diff(states) >= 0).all()
        for c in range(k):
            idx = inv[h:e][states == c]
            assert (np.diff(idx) > 0).all()


def test_bad_state(qhm):
    with pytest.raises(qhm.QhError) as ei:
        _gpu(qhm, [0, 1, 5], [1, 0, 0], 3)
    assert ei.value.status == qhm.QH_EINVAL
