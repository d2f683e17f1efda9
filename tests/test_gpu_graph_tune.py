"""Graph replay (QH_FLAG_GRAPH) and the launch-configuration autotuner
(QH_FLAG_AUTOTUNE) of the 2D path: both must leave the output unchanged, bit
for bit, against the oracle.

Graph replays are checked one by one against the oracle, with the inputs'
contents changed in place between replays and eager device work and host
synchronisations in between (a captured graph must not depend on state that
only its first replay sees).
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qhm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1201_2936_amd import qh
    qh.load()
    return qh


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode", [0, 1])
def test_graph_replays_single(qhm, mode):
    n = 200_000
    inputs = [workloads.disk(workloads.rng_for(300 + j), n, 1 << 20) for j in range(3)]
    inputs.append(workloads.square(workloads.rng_for(310), n, 1 << 20))
    ctx = qhm.Context()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        buf = torch.empty((2, n), dtype=torch.int32, device="cuda")
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        scratch = torch.ones(1 << 20, device="cuda")
        launches = []
        for rep in range(8):
            p = inputs[rep % len(inputs)]
            _say(f"graph single mode={mode} replay={rep}")
            buf.copy_(torch.from_numpy(p))
            got, stats = qhm.qh_hull2d(buf, mode=mode, ctx=ctx, graph=True, out=out,
                                       stream=st.cuda_stream)
            assert got.cpu().tolist() == oracle.hull2d(p).tolist(), rep
            launches.append(stats["graph_launches"])
            # eager work and a host wait between replays
            scratch.mul_(1.0001)
            torch.cuda.synchronize()
        assert min(launches) >= 1
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_graph_replays_batched(qhm, mode):
    sizes = np.array([256, 5000, 70000, 2048, 1 << 17, 999, 0, 3], np.int64)
    base, off = workloads.batched_disks(len(sizes), sizes)
    # the same instance sizes, other contents: x and y swapped, mirrored
    sets = [(base, off), (np.ascontiguousarray(base[::-1]), off), (np.ascontiguousarray(-base), off)]
    ctx = qhm.Context()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        pts0, off0 = sets[0]
        buf = torch.empty(pts0.shape, dtype=torch.int32, device="cuda")
        offs = torch.from_numpy(off0).to("cuda")
        out = torch.empty(max(pts0.shape[1], 1), dtype=torch.int32, device="cuda")
        hoff = torch.empty(len(sizes) + 1, dtype=torch.int64, device="cuda")
        for rep in range(6):
            pts, off = sets[rep % len(sets)]
            assert off.tolist() == off0.tolist()
            _say(f"graph batched mode={mode} replay={rep}")
            buf.copy_(torch.from_numpy(pts))
            got, got_off, stats = qhm.qh_hull2d_batched(buf, offs, mode=mode, ctx=ctx, graph=True,
                                                        out=out, hull_offsets=hoff,
                                                        stream=st.cuda_stream)
            want, want_off = oracle.hull2d_batched(pts, off)
            assert got_off.cpu().tolist() == want_off.tolist(), rep
            assert got.cpu().tolist() == want.tolist(), rep
            assert stats["graph_launches"] >= 1
            torch.cuda.synchronize()
    ctx.close()


def test_graph_then_eager_and_new_buffers(qhm):
    """A graph call, an eager call and a graph call with other buffers on one
    context all give the oracle's hull."""
    ctx = qhm.Context()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for j, n in enumerate((50_000, 50_000, 120_000)):
            p = workloads.disk(workloads.rng_for(320 + j), n, 1 << 20)
            t = torch.from_numpy(p).to("cuda")
            want = oracle.hull2d(p).tolist()
            _say(f"graph/eager n={n}")
            got, _ = qhm.qh_hull2d(t, ctx=ctx, graph=True, stream=st.cuda_stream)
            assert got.cpu().tolist() == want
            got, _ = qhm.qh_hull2d(t, ctx=ctx, stream=st.cuda_stream)
            assert got.cpu().tolist() == want
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_autotune_keeps_output(qhm, mode):
    ctx = qhm.Context()
    p = workloads.disk(workloads.rng_for(330), 300_000, 1 << 20)
    t = torch.from_numpy(p).to("cuda")
    want = oracle.hull2d(p).tolist()
    _say(f"autotune single mode={mode}")
    got, stats = qhm.qh_hull2d(t, mode=mode, ctx=ctx, autotune=True)
    assert got.cpu().tolist() == want
    assert stats["tuned_configs"] == 12
    assert stats["multi_blocks"] > 0 and stats["finish_segments"] > 0
    got2, stats2 = qhm.qh_hull2d(t, mode=mode, ctx=ctx, autotune=True)
    assert got2.cpu().tolist() == want
    assert stats2["tuned_configs"] == 0
    assert (stats2["grid_blocks"], stats2["multi_blocks"], stats2["finish_segments"]) == \
        (stats["grid_blocks"], stats["multi_blocks"], stats["finish_segments"])
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_graph_replays_finish_runs(qhm, mode):
    """2,000 small disks: the last round finishes runs of small segments;
    replayed from graphs with the contents changed in place between calls."""
    rng = np.random.default_rng(606)
    sizes = np.floor(np.exp(rng.uniform(np.log(64), np.log(8000), size=2000))).astype(np.int64)
    base, off = workloads.batched_disks(len(sizes), sizes)
    sets = [base, np.ascontiguousarray(base[::-1]), np.ascontiguousarray(-base)]
    ctx = qhm.Context()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        buf = torch.empty(base.shape, dtype=torch.int32, device="cuda")
        offs = torch.from_numpy(off).to("cuda")
        out = torch.empty(base.shape[1], dtype=torch.int32, device="cuda")
        hoff = torch.empty(len(sizes) + 1, dtype=torch.int64, device="cuda")
        for rep in range(5):
            pts = sets[rep % len(sets)]
            _say(f"graph finish runs mode={mode} replay={rep}")
            buf.copy_(torch.from_numpy(pts))
            got, got_off, stats = qhm.qh_hull2d_batched(buf, offs, mode=mode, ctx=ctx, graph=True,
                                                        out=out, hull_offsets=hoff,
                                                        stream=st.cuda_stream)
            want, want_off = oracle.hull2d_batched(pts, off)
            assert got_off.cpu().tolist() == want_off.tolist(), rep
            assert got.cpu().tolist() == want.tolist(), rep
            assert stats["finish_runs"] == 1, rep
            torch.cuda.synchronize()
    ctx.close()


def test_autotune_batched_with_graph(qhm):
    sizes = np.array([256, 3000, 40000, 1 << 16, 777, 12345], np.int64)
    pts, off = workloads.batched_disks(len(sizes), sizes)
    want, want_off = oracle.hull2d_batched(pts, off)
    ctx = qhm.Context()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        t = torch.from_numpy(pts).to("cuda")
        offs = torch.from_numpy(off).to("cuda")
        out = torch.empty(pts.shape[1], dtype=torch.int32, device="cuda")
        hoff = torch.empty(len(sizes) + 1, dtype=torch.int64, device="cuda")
        for rep in range(3):
            _say(f"autotune batched graph rep={rep}")
            got, got_off, stats = qhm.qh_hull2d_batched(t, offs, mode=1, ctx=ctx, autotune=True,
                                                        graph=True, out=out, hull_offsets=hoff,
                                                        stream=st.cuda_stream)
            assert got_off.cpu().tolist() == want_off.tolist()
            assert got.cpu().tolist() == want.tolist()
            assert stats["tuned_configs"] == (12 if rep == 0 else 0)
            torch.cuda.synchronize()
    ctx.close()
