"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars (from the method's definition):
  - sampled terms (i, j, flags) bit-exact, recorded by the production layout
    kernel with the production launch shape;
  - one collision-free batch of updates within 1e-5 of the displacement of the
    pure-FP64 oracle, plus FP32 storage and evaluation rounding
    (batch_check.py), for the update kernel and for the layout kernels;
  - sampled path stress of the same layout: identical pair counts, sums within
    1e-9 relative (FP64 terms, different summation order);
  - full Hogwild layouts: sampled path stress within 3% of the oracle's (several
    layouts are correct, so only this statistic is compared; means over layout
    seeds where a single layout's spread would exceed the bar);
  - differentiable loss within 1e-5, gradient against the oracle's analytic
    FP64 gradient and FP64 finite differences.
"""
import ctypes
import glob
import json
import math
import os

import numpy as np
import pytest

import batch_check as B
import oracle as O
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2409_00876_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def P():
    return _P()


@pytest.fixture(scope="module")
def tiny(P):
    sg = synth.config_graph("tiny")
    return sg, O.Graph.from_synth(sg), P.Graph.from_synth(sg)


@pytest.fixture(scope="module")
def mid(P):
    sg = synth.config_graph("mid")
    return sg, O.Graph.from_synth(sg), P.Graph.from_synth(sg)


def _edge_synth():
    # a single-step path, an empty path, a path revisiting a node on both strands, a longer path
    node_len = np.array([5, 1, 3, 2, 7, 1, 4, 2, 9, 3], np.uint32)
    R = synth.REV_BIT
    paths = [[4], [], [0, 1, 2 | R, 1 | R, 3, 2], list(range(10)) + [9 | R, 8 | R, 7 | R] + list(range(3, 10))]
    off = np.cumsum([0] + [len(p) for p in paths]).astype(np.uint64)
    steps = np.array([s for p in paths for s in p], np.uint32)
    return synth.SynthGraph(node_len, off, steps, {}, "edge")


def _to_np_u64(t):
    return t.cpu().numpy().astype(np.uint64)


def _compare_terms(P, g, og, it, t0, count, **kw):
    kw.setdefault("schedule", 1)  # the plain enumeration (the others have their own checks)
    i, j, f = P.sample_terms(g, it, t0, count, **kw)
    oi, oj, of = O.sample_terms(og, it, t0, count, **{k: v for k, v in kw.items() if k in ("seed", "graph_id")})
    gi, gj, gf = _to_np_u64(i), _to_np_u64(j), f.cpu().numpy()
    bad = np.nonzero((gi != oi) | (gj != oj) | (gf != of))[0]
    assert bad.size == 0, f"iter {it} t0 {t0}: {bad.size} mismatches, first at t={t0 + bad[0]}: " \
                          f"gpu ({gi[bad[0]]},{gj[bad[0]]},{gf[bad[0]]}) oracle ({oi[bad[0]]},{oj[bad[0]]},{of[bad[0]]})"
    return gf


# ---------------------------------------------------------------------------
# graph upload and initial layout
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["tiny", "mid"])
def test_graph_info_and_init_coords(P, which, request):
    sg, og, g = request.getfixturevalue(which)
    assert (g.n_steps, g.n_nodes, g.n_paths, g.d_max) == (og.S, og.n_nodes, og.n_paths, og.d_max)
    c = g.new_coords()
    P.init_coords(g, c, seed=5, jitter=10.0)
    assert np.array_equal(c.cpu().numpy(), O.init_coords(og, seed=5, jitter=10.0))


def test_edge_graph_upload_and_sampling(P):
    sg = _edge_synth()
    og, g = O.Graph.from_synth(sg), P.Graph.from_synth(sg)
    assert (g.n_steps, g.d_max) == (og.S, og.d_max)
    c = g.new_coords()
    P.init_coords(g, c)
    assert np.array_equal(c.cpu().numpy(), O.init_coords(og))
    T = 10 * og.S
    for it in (0, 7, 15, 29):
        f = _compare_terms(P, g, og, it, 0, T)
        assert f.size == T
    # the single-step path is always skipped when cooling
    i, j, f = O.sample_terms(og, 20, 0, T)
    assert np.all((f[i == 0] >> 3) & 1)


# ---------------------------------------------------------------------------
# T1-T3: bit-exact sampling
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("it", [0, 14, 15, 29])
@pytest.mark.parametrize("graph_id", [0, 7])
def test_sampling_bitexact_tiny(P, tiny, it, graph_id):
    sg, og, g = tiny
    T = 10 * og.S  # whole iteration, ragged last group
    _compare_terms(P, g, og, it, 0, T, graph_id=graph_id)
    _compare_terms(P, g, og, it, 1000 + 7, 1 << 16, graph_id=graph_id, seed=99)


@pytest.mark.parametrize("it", [0, 14, 15, 29])
def test_sampling_bitexact_mid(P, mid, it):
    sg, og, g = mid
    T = 10 * og.S
    _compare_terms(P, g, og, it, 0, 1 << 20)
    _compare_terms(P, g, og, it, T // 2 + 5, 1 << 20, graph_id=7)
    _compare_terms(P, g, og, it, T - (1 << 18) - 3, (1 << 18) + 3)  # the ragged end


def test_sampling_bitexact_across_counter_carry(P, tiny, mid):
    for sg, og, g in (tiny, mid):
        _compare_terms(P, g, og, 3, (1 << 32) - (1 << 19) - 11, 1 << 20)


def test_sampling_bitexact_large_range(P, mid):
    sg, og, g = mid
    _compare_terms(P, g, og, 0, 123456789, 1 << 22)


@pytest.fixture(scope="module")
def chromosome(P):
    sg = synth.config_graph("chromosome")
    return sg, O.Graph.from_synth(sg), P.Graph.from_synth(sg)


# ---------------------------------------------------------------------------
# The windowed schedule: window-major slots (reading R18), recorded by its kernels
# ---------------------------------------------------------------------------
def _compare_windowed(P, g, og, it, s0, count, offsets=None, **kw):
    i, j, f = P.sample_terms(g, it, s0, count, schedule=3, **kw)
    okw = {k: v for k, v in kw.items() if k in ("seed", "graph_id")}
    oi, oj, of = O.sample_terms_windowed(og, it, s0, count, offsets=offsets, threads=16, **okw)
    gi, gj, gf = _to_np_u64(i), _to_np_u64(j), f.cpu().numpy()
    assert not np.any(gf == 255), "a slot was not processed"
    bad = np.nonzero((gi != oi) | (gj != oj) | (gf != of))[0]
    assert bad.size == 0, f"iter {it} s0 {s0}: {bad.size} mismatches, first at s={s0 + bad[0]}: " \
                          f"gpu ({gi[bad[0]]},{gj[bad[0]]},{gf[bad[0]]}) oracle ({oi[bad[0]]},{oj[bad[0]]},{of[bad[0]]})"


@pytest.mark.parametrize("it", [0, 14, 15, 29])
def test_windowed_sampling_bitexact_tiny(P, tiny, it):
    sg, og, g = tiny
    T = 10 * og.S  # whole iteration
    for waves in (0, 1, 37, 4096):  # the terms do not depend on the launch shape
        _compare_windowed(P, g, og, it, 0, T, max_inflight_waves=waves)
    _compare_windowed(P, g, og, it, 1000 + 7, 1 << 16, graph_id=5, seed=99)


def test_windowed_sampling_edge_graph(P):
    sg = _edge_synth()
    og, g = O.Graph.from_synth(sg), P.Graph.from_synth(sg)
    for it in (0, 15, 29):
        _compare_windowed(P, g, og, it, 0, 10 * og.S)


def test_windowed_split_run_equals_full_run(P, tiny):
    # one wave (automatic cap on tiny) makes the windowed layout deterministic: iterations
    # [0, 7) + [7, 19) + [19, 30) in three calls (each counting ahead on the second stream)
    # must give exactly the coordinates of one call over [0, 30)
    import torch
    sg, og, g = tiny
    c0 = O.init_coords(og)
    a = torch.from_numpy(c0).cuda()
    b = torch.from_numpy(c0).cuda()
    P.layout(g, a, schedule=3)
    for lo, hi in ((0, 7), (7, 19), (19, 30)):
        P.layout(g, b, schedule=3, first_iter=lo, last_iter=hi)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_windowed_count_ahead_equals_in_order(P, tiny):
    # one wave makes the windowed layout deterministic: counting each next iteration on the
    # graph's second stream must give exactly the coordinates of the in-order passes
    import torch
    sg, og, g = tiny
    c0 = O.init_coords(og)
    a = torch.from_numpy(c0).cuda()
    b = torch.from_numpy(c0).cuda()
    P.layout(g, a, schedule=3, max_inflight_waves=1, flags=P.FLAG_COUNT_AHEAD)
    P.layout(g, b, schedule=3, max_inflight_waves=1, flags=P.FLAG_COUNT_IN_ORDER)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert not torch.equal(a, torch.from_numpy(c0).cuda())
    for bad in (P.FLAG_COUNT_AHEAD | P.FLAG_COUNT_IN_ORDER, 4):
        with pytest.raises(P.PgsgdError):
            P.layout(g, a, schedule=3, flags=bad)


def test_windowed_sampling_many_short_paths(P):
    # 3,000 paths of 1-9 steps (windows of 2^8 steps span dozens of paths and take the
    # path search), plus empty paths, and S not a multiple of the window
    rng = np.random.default_rng(12)
    n_nodes = 5000
    lens = rng.integers(0, 10, size=3000)
    steps = [[int(x) | (synth.REV_BIT if rng.random() < 0.1 else 0) for x in rng.integers(0, n_nodes, size=k)]
             for k in lens]
    off = np.cumsum([0] + [len(p_) for p_ in steps]).astype(np.uint64)
    node_len = rng.integers(1, 30, size=n_nodes).astype(np.uint32)
    sg = synth.SynthGraph(node_len, off, np.array([x for p_ in steps for x in p_], np.uint32), {}, "short")
    og, g = O.Graph.from_synth(sg), P.Graph.from_synth(sg)
    assert og.S % (1 << O.window_shift(og.S)) != 0
    for it in (0, 20):
        _compare_windowed(P, g, og, it, 0, 10 * og.S)


@pytest.mark.parametrize("it", [0, 15])
def test_windowed_sampling_bitexact_mid(P, mid, it):
    sg, og, g = mid
    T = 10 * og.S
    off = O.window_offsets(og, it, threads=16)
    for s0, n in ((0, 1 << 20), (T // 3 + 17, 1 << 18), (T - (1 << 18) - 3, (1 << 18) + 3)):
        _compare_windowed(P, g, og, it, s0, n, offsets=off)


@pytest.mark.parametrize("it", [0, 29])
def test_windowed_sampling_bitexact_chromosome(P, chromosome, it):
    # full size, in the launch shape the benchmark times: start, middle and ragged end of the slots
    sg, og, g = chromosome
    T = 10 * og.S
    off = O.window_offsets(og, it, threads=16)
    for s0, n in ((0, 1 << 20), (T // 2 + 12345, 1 << 20), (T - (1 << 20) - 5, (1 << 20) + 5)):
        _compare_windowed(P, g, og, it, s0, n, offsets=off)


# ---------------------------------------------------------------------------
# Data-reuse variant (DRF, SRF)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("it", [0, 20])
@pytest.mark.parametrize("which", ["tiny", "mid"])
def test_reuse_sampling_bitexact(P, which, it, request):
    sg, og, g = request.getfixturevalue(which)
    n = 1 << 16
    i, j, f, o = P.sample_terms_reuse(g, it, 64 * 37, n, reuse_factor=4, step_reduction=2, graph_id=3, schedule=1)
    oi, oj, of = O.sample_terms_reuse(og, it, 64 * 37, n, graph_id=3)
    assert np.array_equal(_to_np_u64(i), oi) and np.array_equal(_to_np_u64(j), oj)
    assert np.array_equal(f.cpu().numpy(), of)
    go = o.cpu().numpy().reshape(-1, 3)
    for k in range(0, go.shape[0], 97):
        assert list(go[k]) == O.reuse_offsets(it, 37 + k, 4, graph_id=3)
    # a group shares one path
    path = np.searchsorted(og.path_off, oi, side="right") - 1
    assert np.all(path.reshape(-1, 64) == path.reshape(-1, 64)[:, :1])


def test_reuse_off_is_the_plain_layout(P, tiny):
    import torch
    sg, og, g = tiny
    c0 = O.init_coords(og)
    a = torch.from_numpy(c0).cuda()
    b = torch.from_numpy(c0).cuda()
    P.layout(g, a, max_inflight_waves=1, first_iter=0, last_iter=3, schedule=1)
    P.layout(g, b, max_inflight_waves=1, first_iter=0, last_iter=3, reuse_factor=1, step_reduction=1, schedule=1)
    assert torch.equal(a, b)


@pytest.mark.parametrize("schedule", [1, 3])
@pytest.mark.parametrize("drf,srf", [(2, 1), (2, 2), (4, 4)])
def test_reuse_layout_quality_matches_oracle_variant(P, tiny, drf, srf, schedule):
    import torch
    sg, og, g = tiny
    c0 = O.init_coords(og)
    gpu, ora = [], []
    for sd in (101, 102, 103, 104):
        c = torch.from_numpy(c0).cuda()
        P.layout(g, c, seed=sd, max_inflight_waves=1, reuse_factor=drf, step_reduction=srf, schedule=schedule)
        gpu.append(O.sps_expectation(og, c.cpu().numpy())[0])
        co = c0.copy()
        if schedule == 1:
            O.layout_reuse(og, co, drf, srf, seed=sd)
        else:
            O.layout_windowed(og, co, seed=sd, reuse_factor=drf, step_reduction=srf)
        ora.append(O.sps_expectation(og, co)[0])
    ratio = np.mean(gpu) / np.mean(ora)
    print(f"reuse ({drf},{srf}) schedule {schedule}: GPU {np.mean(gpu):.6f} oracle {np.mean(ora):.6f} "
          f"ratio {ratio:.4f}")
    assert abs(ratio - 1) <= 0.03


@pytest.mark.parametrize("it", [0, 20])
@pytest.mark.parametrize("which", ["tiny", "mid"])
def test_windowed_reuse_sampling_bitexact(P, which, it, request):
    # slots of the window-major enumeration with step reduction, and every slot's group offsets
    sg, og, g = request.getfixturevalue(which)
    T = O.window_slots(og, 10, 2)
    s0 = 1000 + 5 if which == "tiny" else T // 3 + 11
    n = min(1 << 16, T - s0)
    i, j, f, o = P.sample_terms_reuse(g, it, s0, n, reuse_factor=4, step_reduction=2, graph_id=3, schedule=3)
    off = O.window_offsets(og, it, graph_id=3, threads=16, step_reduction=2)
    oi, oj, of = O.sample_terms_windowed(og, it, s0, n, graph_id=3, offsets=off)
    assert np.array_equal(_to_np_u64(i), oi) and np.array_equal(_to_np_u64(j), oj)
    assert np.array_equal(f.cpu().numpy(), of)
    go = o.cpu().numpy().reshape(-1, 3)
    for k in range(0, n, 331):
        s = s0 + k
        w = int(np.searchsorted(off, s, side="right") - 1)
        lead = int(off[w]) + ((s - int(off[w])) // 64) * 64
        assert list(go[k]) == O.reuse_offsets(it, lead, 4, graph_id=3)


# ---------------------------------------------------------------------------
# T6b: one collision-free deterministic batch
# ---------------------------------------------------------------------------
def _batch_and_check(og, it, i, j, f, got_fn):
    """Keeps a collision-free subset of the sampled terms (i, j, f), lets
    got_fn(keep, start, eta) apply it on the GPU and checks the result against
    the oracle's FP64 batch (batch_check.check)."""
    keep = B.collision_free(og, i, j, f)
    assert keep.size > 2000
    eta = float(O.schedule(30, float(og.d_max) ** 2, 0.01).astype(np.float32)[it])
    start = B.start_coords(og, it)
    got = got_fn(keep, start, eta)
    ref, applied = B.fp64_result(og, eta, i[keep], j[keep], f[keep], start)
    assert applied == keep.size
    worst, untouched = B.check(og, og.pos, i[keep], j[keep], f[keep], eta, start, got, ref)
    assert worst <= 1.0, f"worst error / bound = {worst:.3f}"
    assert untouched, "a coordinate outside the batch changed"
    assert np.count_nonzero(got != start.astype(np.float64)) >= keep.size  # the batch really moved points


@pytest.mark.parametrize("which", ["tiny", "mid"])
@pytest.mark.parametrize("it", [0, 25])
def test_collision_free_batch_matches_fp64(P, which, it, request):
    # the update kernel on given terms (k_apply_terms)
    import torch
    sg, og, g = request.getfixturevalue(which)
    i, j, f = P.sample_terms(g, it, 0, B.K_TERMS, schedule=1)
    gi, gj, gf = _to_np_u64(i), _to_np_u64(j), f.cpu().numpy()
    oi, oj, of = O.sample_terms(og, it, 0, B.K_TERMS)
    assert np.array_equal(gi, oi) and np.array_equal(gj, oj) and np.array_equal(gf, of)

    def run(keep, start, eta):
        c = torch.from_numpy(start).cuda()
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
        P.apply_terms(g, c, eta, dev(gi[keep].astype(np.int64)), dev(gj[keep].astype(np.int64)), dev(gf[keep]))
        return c.cpu().numpy().astype(np.float64)

    _batch_and_check(og, it, gi, gj, gf, run)


@pytest.mark.parametrize("which", ["tiny", "mid"])
@pytest.mark.parametrize("it", [0, 25])
@pytest.mark.parametrize("schedule", [1, 3])
def test_collision_free_batch_in_the_layout_kernel(P, which, it, schedule, request):
    # the layout kernels themselves (plain k_layout_iter, windowed k_layout_local with
    # its far-first loads), in the layout's launch shape, applying only the batch
    import torch
    sg, og, g = request.getfixturevalue(which)
    i, j, f = P.sample_terms(g, it, 0, B.K_TERMS, schedule=schedule)
    gi, gj, gf = _to_np_u64(i), _to_np_u64(j), f.cpu().numpy()

    def run(keep, start, eta):
        c = torch.from_numpy(start).cuda()
        mask = np.zeros(B.K_TERMS, np.uint8)
        mask[keep] = 1
        P.apply_slots(g, c, it, 0, torch.from_numpy(mask).cuda(), schedule=schedule)
        return c.cpu().numpy().astype(np.float64)

    _batch_and_check(og, it, gi, gj, gf, run)


# ---------------------------------------------------------------------------
# T9: sampled path stress of the same layout
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("pairs", ["uniform", "power_law", "uniform_windowed"])
@pytest.mark.parametrize("which,m", [("tiny", 100), ("mid", 1)])
def test_sps_equals_oracle_on_same_layout(P, which, m, pairs, request):
    import torch
    sg, og, g = request.getfixturevalue(which)
    rng = np.random.default_rng(1)
    c0 = O.init_coords(og)
    c0 = (c0 + rng.normal(scale=50.0, size=c0.shape)).astype(np.float32)
    r = P.path_stress(g, torch.from_numpy(c0).cuda(), m, 7, pairs=pairs)
    o = O.sampled_path_stress(og, c0, m, 7, pairs=pairs)
    assert r["n_valid"] == o["n_valid"] and r["n_skipped"] == o["n_skipped"]
    assert r["n_valid"] + r["n_skipped"] == m * og.S
    assert abs(r["sum"] - o["sum"]) <= 1e-9 * abs(o["sum"])
    assert abs(r["sumsq_dev"] - o["sumsq_dev"]) <= 1e-9 * abs(o["sumsq_dev"])
    assert abs(r["ci_hi"] - o["ci_hi"]) <= 1e-9 * abs(o["ci_hi"])


def _short_paths_synth():
    # 3,000 paths of 0-9 steps: windows hold dozens of segments
    rng = np.random.default_rng(12)
    n_nodes = 5000
    lens = rng.integers(0, 10, size=3000)
    steps = [[int(x) | (synth.REV_BIT if rng.random() < 0.1 else 0) for x in rng.integers(0, n_nodes, size=k)]
             for k in lens]
    off = np.cumsum([0] + [len(p_) for p_ in steps]).astype(np.uint64)
    node_len = rng.integers(1, 30, size=n_nodes).astype(np.uint32)
    return synth.SynthGraph(node_len, off, np.array([x for p_ in steps for x in p_], np.uint32), {}, "short")


@pytest.mark.parametrize("which", ["edge", "short_paths"])
def test_sps_windowed_equals_oracle_on_edge_graphs(P, which):
    import torch
    sg = _edge_synth() if which == "edge" else _short_paths_synth()
    og, g = O.Graph.from_synth(sg), P.Graph.from_synth(sg)
    rng = np.random.default_rng(3)
    c0 = (O.init_coords(og) + rng.normal(scale=20.0, size=4 * og.n_nodes)).astype(np.float32)
    for m, seed in ((1, 7), (13, 9)):
        r = P.path_stress(g, torch.from_numpy(c0).cuda(), m, seed, pairs="uniform_windowed")
        o = O.sampled_path_stress(og, c0, m, seed, pairs="uniform_windowed")
        assert r["n_valid"] == o["n_valid"] and r["n_skipped"] == o["n_skipped"]
        assert r["n_valid"] + r["n_skipped"] == m * og.S
        assert abs(r["sum"] - o["sum"]) <= 1e-9 * abs(o["sum"])
        assert abs(r["sumsq_dev"] - o["sumsq_dev"]) <= 1e-9 * abs(o["sumsq_dev"])


def test_graph_without_steps(P):
    # two nodes and two empty paths: every call succeeds and leaves the coordinates alone
    import torch
    sg = synth.SynthGraph(np.array([3, 4], np.uint32), np.zeros(3, np.uint64), np.zeros(0, np.uint32), {}, "empty")
    g = P.Graph.from_synth(sg)
    assert g.n_steps == 0
    c = torch.arange(8, dtype=torch.float32, device="cuda")
    before = c.clone()
    for sched in (0, 1, 3):
        P.layout(g, c, schedule=sched)
    for pairs in ("uniform", "uniform_windowed", "power_law"):
        r = P.path_stress(g, c, 10, 7, pairs=pairs)
        assert r["n_valid"] == 0 and r["n_skipped"] == 0 and r["mean"] == 0.0
    assert P.path_stress_exact(g, c) == (0.0, 0)
    loss, nv = P.stress_forward(g, c, 1000, 1)
    assert float(loss) == 0.0 and int(nv) == 0
    torch.cuda.synchronize()
    assert torch.equal(c, before)


def test_device_byte_cap_on_lazy_scratch(P, tiny_synth, monkeypatch):
    """PGSGD_MAX_DEVICE_BYTES just above a graph's creation footprint: the
    windowed layout's first-use tables no longer fit (OOM, coordinates
    untouched), the plain layout and the allocation-free entry point still
    run."""
    import torch
    g0 = P.Graph.from_synth(tiny_synth)
    need = g0.device_bytes
    g0.close()
    monkeypatch.setenv("PGSGD_MAX_DEVICE_BYTES", str(need + 64))
    g = P.Graph.from_synth(tiny_synth)
    assert g.device_bytes == need
    c = g.new_coords()
    P.init_coords(g, c)
    before = c.clone()
    with pytest.raises(P.PgsgdError) as e:
        P.layout(g, c, schedule=3)
    assert e.value.status == -3 and "PGSGD_MAX_DEVICE_BYTES" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(c, before)
    P.layout(g, c, schedule=1, max_inflight_waves=1)
    P.layout_noalloc(g, before, max_inflight_waves=1)
    torch.cuda.synchronize()
    assert not torch.equal(c, before)


def test_sps_mode_and_size_errors(P, tiny):
    import torch
    from paper_2409_00876_amd import _lib
    sg, og, g = tiny
    c = torch.from_numpy(O.init_coords(og)).cuda()
    r = _lib.StressResult()
    st = P.lib().pgsgd_path_stress_pairs(g.handle, ctypes.c_void_p(c.data_ptr()), 10, 7, 0, 3, 0.99, 1000,
                                         ctypes.byref(r), None)
    assert st == _lib.ERR_INVALID_ARG and "pair mode" in P.lib().pgsgd_last_error().decode()
    # 32-bit segment counts: pairs_per_step * 2^(h + 1) must stay below 2^32
    with pytest.raises(P.PgsgdError, match="32-bit"):
        P.path_stress(g, c, 1 << 23, 7, pairs="uniform_windowed")
    # 16,000 two-step paths: the path table fits the LDS of the uniform order, the segment
    # histogram beside it does not
    n_paths = 16000
    sg2 = synth.SynthGraph(np.full(100, 5, np.uint32), (2 * np.arange(n_paths + 1)).astype(np.uint64),
                           (np.arange(2 * n_paths) % 100).astype(np.uint32), {}, "many-paths")
    og2, g2 = O.Graph.from_synth(sg2), P.Graph.from_synth(sg2)
    c2 = torch.from_numpy(O.init_coords(og2)).cuda()
    r2 = P.path_stress(g2, c2, 3, 7)
    o2 = O.sampled_path_stress(og2, c2.cpu().numpy(), 3, 7)
    assert r2["n_valid"] == o2["n_valid"] and r2["n_skipped"] == o2["n_skipped"]
    with pytest.raises(P.PgsgdError, match="segment histogram"):
        P.path_stress(g2, c2, 3, 7, pairs="uniform_windowed")


def test_sps_windowed_agrees_with_uniform_order_on_chromosome(P, chromosome):
    # full size, the benchmark's call: the two orders sample the same law, so on one layout
    # their means agree within the combined standard error; pair counts are exact
    import torch
    sg, og, g = chromosome
    c = g.new_coords()
    P.init_coords(g, c)
    P.layout(g, c, first_iter=0, last_iter=3)
    a = P.path_stress(g, c, 1, 7, pairs="uniform")
    b = P.path_stress(g, c, 1, 7, pairs="uniform_windowed")
    b2 = P.path_stress(g, c, 1, 7, pairs="uniform_windowed")
    # the same pairs again; only the order of the FP64 block sums may differ
    assert b["n_valid"] == b2["n_valid"] and b["n_skipped"] == b2["n_skipped"]
    assert abs(b["sum"] - b2["sum"]) <= 1e-12 * abs(b["sum"])
    for r in (a, b):
        assert r["n_valid"] + r["n_skipped"] == og.S
    se = math.sqrt(a["stddev"] ** 2 / a["n_valid"] + b["stddev"] ** 2 / b["n_valid"])
    assert abs(a["mean"] - b["mean"]) < 4.5 * se
    assert abs(a["n_skipped"] - b["n_skipped"]) < 6 * math.sqrt(a["n_skipped"] + 1) + 10


# ---------------------------------------------------------------------------
# Path stress (Eq. 1) and its relation to the sampled metric
# ---------------------------------------------------------------------------
def test_exact_path_stress_equals_oracle(P, tiny):
    import torch
    sg, og, g = tiny
    c0 = O.init_coords(og)
    c1 = c0.copy()
    O.layout(og, c1)
    for c in (c0, c1):
        ps, pairs = P.path_stress_exact(g, torch.from_numpy(c).cuda())
        ref, ref_pairs = O.path_stress_exact(og, c)
        assert pairs == ref_pairs
        assert abs(ps - ref) <= 1e-9 * abs(ref)


def test_exact_path_stress_edge_graph(P):
    import torch
    sg = _edge_synth()
    og, g = O.Graph.from_synth(sg), P.Graph.from_synth(sg)
    c = (O.init_coords(og) + np.random.default_rng(2).normal(scale=3, size=4 * og.n_nodes)).astype(np.float32)
    ps, pairs = P.path_stress_exact(g, torch.from_numpy(c).cuda())
    ref, ref_pairs = O.path_stress_exact(og, c)
    assert pairs == ref_pairs and abs(ps - ref) <= 1e-9 * abs(ref)


def test_sampled_path_stress_tracks_exact_path_stress(P):
    import math
    import bench
    rows = bench.sps_vs_ps_layouts(n_graphs=6, stages=(0, 2, 7, 30))
    xs = [math.log(r["sps"]) for r in rows]
    ys = [math.log(r["ps"]) for r in rows]
    r = np.corrcoef(xs, ys)[0, 1]
    print(f"log-space correlation of SPS and PS over {len(rows)} layouts: {r:.4f}")
    assert r > 0.95


# ---------------------------------------------------------------------------
# T7 + T10: full layouts
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("schedule", [1, 3])
def test_linear_path_converges_on_gpu(P, schedule):
    import torch
    sg = synth.linear_path(2000)
    og, g = O.Graph.from_synth(sg), P.Graph.from_synth(sg)
    c0 = O.init_coords(og)
    c = torch.from_numpy(c0).cuda()
    P.layout(g, c, schedule=schedule)
    s_gpu = P.path_stress(g, c, 100, 7)["mean"]
    co = c0.copy()
    O.layout(og, co)
    s_ora = O.sampled_path_stress(og, co, 100, 7)["mean"]
    assert s_gpu < 1e-3 and s_gpu <= max(1.5 * s_ora, 1e-3)


@pytest.mark.parametrize("schedule", [1, 3])
def test_full_layout_sps_parity_tiny(P, tiny, schedule):
    import torch
    sg, og, g = tiny
    c0 = O.init_coords(og)
    seeds = [101, 102, 103, 104, 105, 106]
    gpu, ora, gpu_sps = [], [], []
    for sd in seeds:
        c = torch.from_numpy(c0).cuda()
        P.layout(g, c, seed=sd, schedule=schedule)
        cg = c.cpu().numpy()
        gpu.append(O.sps_expectation(og, cg)[0])
        gpu_sps.append(P.path_stress(g, c, 100, 7)["mean"])
        co = c0.copy()
        O.layout(og, co, seed=sd)
        ora.append(O.sps_expectation(og, co)[0])
    ratio = np.mean(gpu) / np.mean(ora)
    print(f"tiny schedule {schedule}: GPU {np.mean(gpu):.6f} oracle {np.mean(ora):.6f} ratio {ratio:.4f} "
          f"(oracle seed spread {np.std(ora) / np.mean(ora):.4f}); GPU SPS(m=100) {np.mean(gpu_sps):.6f}")
    assert abs(ratio - 1) <= 0.03


def _mid_goldens():
    out = []
    for fn in sorted(glob.glob(os.path.join(GOLDEN, "oracle_sps_mid_seed*_t1.json"))):
        with open(fn) as f:
            out.append(json.load(f))
    return out


@pytest.mark.parametrize("schedule", [1, 3])
def test_full_layout_sps_parity_mid(P, mid, schedule):
    import torch
    goldens = _mid_goldens()
    if not goldens:
        pytest.skip("no stored oracle result for mid (tests/golden/make_golden.py writes it)")
    sg, og, g = mid
    c0 = O.init_coords(og)
    gpu, ora = [], []
    for rec in goldens:
        assert rec["graph"]["n_steps"] == og.S and rec["graph"]["n_nodes"] == og.n_nodes
        c = torch.from_numpy(c0).cuda()
        P.layout(g, c, seed=rec["layout_seed"], schedule=schedule)
        s = P.path_stress(g, c, rec["sps_m"], rec["sps_seed"])
        gpu.append(s["mean"])
        ora.append(rec["sps_mean"])
        print(f"mid seed {rec['layout_seed']} schedule {schedule}: GPU SPS {s['mean']:.5f} [{s['ci_lo']:.5f}, {s['ci_hi']:.5f}] "
              f"oracle {rec['sps_mean']:.5f} [{rec['sps_ci_lo']:.5f}, {rec['sps_ci_hi']:.5f}]")
    ratio = np.mean(gpu) / np.mean(ora)
    assert abs(ratio - 1) <= 0.03, f"GPU/oracle SPS ratio {ratio:.4f}"


# ---------------------------------------------------------------------------
# T12: differentiable form
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_diff(P):
    sg = synth.generate(500, 0.2, 32, 2)  # the mid model on a 500-node backbone
    og, g = O.Graph.from_synth(sg), P.Graph.from_synth(sg)
    rng = np.random.default_rng(7)
    c = O.init_coords(og)
    c = (c + rng.normal(scale=5.0, size=c.shape)).astype(np.float32)
    return sg, og, g, c


# the loss's pair order: plain enumeration (schedule 1) and window-major (reading R22, schedule 3, the default)
LOSS_ORDERS = [(1, O.stress_loss_grad), (3, O.stress_loss_grad_windowed)]


@pytest.mark.parametrize("schedule,ref", LOSS_ORDERS)
def test_loss_and_gradient_match_oracle(P, small_diff, schedule, ref):
    import torch
    sg, og, g, c0 = small_diff
    n_pairs, step = 200_000, 3
    c = torch.from_numpy(c0).cuda()
    loss, nv = P.stress_forward(g, c, n_pairs, step, seed=11, schedule=schedule)
    L_ref, n_ref, grad_ref = ref(og, c0, n_pairs, seed=11, step=step)
    assert int(nv.item()) == n_ref
    assert abs(float(loss.item()) - L_ref) <= 1e-5 * abs(L_ref)
    grad = torch.zeros_like(c)
    P.stress_backward(g, c, n_pairs, step, torch.ones(1, device="cuda"), nv, grad, seed=11, schedule=schedule)
    gg = grad.cpu().numpy().astype(np.float64)
    gmax = np.abs(grad_ref).max()
    sel = np.abs(grad_ref) > 1e-6 * gmax
    err = np.abs(gg - grad_ref)
    assert np.all(err[sel] <= 1e-4 * np.abs(grad_ref[sel]) + 1e-6 * gmax), \
        f"max rel err {np.max(err[sel] / np.abs(grad_ref[sel])):.3e}"
    assert np.all(err[~sel] <= 1e-6 * gmax)


@pytest.mark.parametrize("schedule,ref", LOSS_ORDERS)
def test_gradient_matches_fp64_finite_differences(P, small_diff, schedule, ref):
    import torch
    sg, og, g, c0 = small_diff
    n_pairs, step = 50_000, 1
    c = torch.from_numpy(c0).cuda()
    loss, nv = P.stress_forward(g, c, n_pairs, step, seed=11, schedule=schedule)
    grad = torch.zeros_like(c)
    P.stress_backward(g, c, n_pairs, step, torch.ones(1, device="cuda"), nv, grad, seed=11, schedule=schedule)
    gg = grad.cpu().numpy().astype(np.float64)
    gmax = np.abs(gg).max()
    rng = np.random.default_rng(3)
    cand = np.nonzero(np.abs(gg) > 1e-3 * gmax)[0]
    for k in rng.choice(cand, size=min(40, cand.size), replace=False):
        h = np.float32(2.0 ** (np.floor(np.log2(max(1.0, abs(float(c0[k]))))) - 14))
        cp, cm = c0.copy(), c0.copy()
        cp[k] += h
        cm[k] -= h
        Lp = ref(og, cp, n_pairs, seed=11, step=step, want_grad=False)[0]
        Lm = ref(og, cm, n_pairs, seed=11, step=step, want_grad=False)[0]
        fd = (Lp - Lm) / (float(cp[k]) - float(cm[k]))
        assert abs(fd - gg[k]) <= 1e-3 * abs(fd) + 1e-6 * gmax, (k, fd, gg[k])


def test_windowed_loss_on_the_mid_graph_matches_oracle(P, mid):
    """The window-major loss (reading R22) at the differentiable workload's
    size: 1e7 pairs on the mid graph, loss and valid-pair count against the
    oracle, the gradient against the oracle's on a sample of entries."""
    import torch
    sg, og, g = mid
    c0 = O.init_coords(og)
    c = torch.from_numpy(c0).cuda()
    n_pairs, step = 10_000_000, 7
    loss, nv = P.stress_forward(g, c, n_pairs, step, seed=11)
    L_ref, n_ref, grad_ref = O.stress_loss_grad_windowed(og, c0, n_pairs, seed=11, step=step)
    assert int(nv.item()) == n_ref
    assert abs(float(loss.item()) - L_ref) <= 1e-5 * abs(L_ref)
    grad = torch.zeros_like(c)
    P.stress_backward(g, c, n_pairs, step, torch.ones(1, device="cuda"), nv, grad, seed=11)
    gg = grad.cpu().numpy().astype(np.float64)
    gmax = np.abs(grad_ref).max()
    sel = np.abs(grad_ref) > 1e-4 * gmax
    err = np.abs(gg - grad_ref)
    assert np.all(err[sel] <= 1e-4 * np.abs(grad_ref[sel]) + 1e-6 * gmax)


def test_autograd_function_and_adam_reduce_loss(P, small_diff):
    import torch
    sg, og, g, c0 = small_diff
    x = torch.from_numpy(c0).cuda().requires_grad_(True)
    loss = P.SampledPathStress.apply(x, g, 100_000, 0, P.LayoutParams(seed=11))
    loss.backward()
    ref = torch.zeros_like(x)
    l2, nv = P.stress_forward(g, x.detach(), 100_000, 0, seed=11)
    P.stress_backward(g, x.detach(), 100_000, 0, torch.ones(1, device="cuda"), nv, ref, seed=11)
    assert torch.allclose(x.grad, ref, rtol=1e-5, atol=1e-7 * float(ref.abs().max()))
    # a few Adam steps on resampled pairs lower the loss
    xs = torch.from_numpy(c0).cuda()
    m, v = torch.zeros_like(xs), torch.zeros_like(xs)
    first = None
    for t in range(1, 41):
        loss, nv = P.stress_forward(g, xs, 100_000, t, seed=11)
        first = float(loss.item()) if first is None else first
        gr = torch.zeros_like(xs)
        P.stress_backward(g, xs, 100_000, t, torch.ones(1, device="cuda"), nv, gr, seed=11)
        P.adam_step(xs, gr, m, v, t, lr=1.0)
    last = float(P.stress_forward(g, xs, 100_000, 999, seed=11)[0].item())
    assert last < 0.7 * first


def test_adam_matches_pytorch_fp32_reference(P):
    import torch
    n = 10_000
    gen = torch.Generator().manual_seed(0)
    x0 = torch.randn(n, generator=gen)
    x, m, v = x0.clone().cuda(), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    xr, mr, vr = x0.clone(), torch.zeros(n), torch.zeros(n)
    b1, b2, eps, lr = 0.9, 0.999, 1e-8, 0.5
    for t in range(1, 6):
        gcpu = torch.randn(n, generator=gen)
        P.adam_step(x, gcpu.cuda(), m, v, t, lr=lr, beta1=b1, beta2=b2, eps=eps)
        mr = b1 * mr + (1 - b1) * gcpu
        vr = b2 * vr + (1 - b2) * gcpu * gcpu
        xr = xr - lr * (mr / (1 - b1 ** t)) / (torch.sqrt(vr / (1 - b2 ** t)) + eps)
    assert torch.allclose(x.cpu(), xr, rtol=1e-5, atol=1e-5)


# ---------------------------------------------------------------------------
# T11: batched form
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_batch(P):
    sgs = synth.batched_graphs(4, scale=0.0008)
    return sgs, [O.Graph.from_synth(s) for s in sgs], [P.Graph.from_synth(s) for s in sgs]


@pytest.mark.parametrize("it", [0, 15])
def test_batched_sampling_bitexact(P, small_batch, it):
    # the persistent plain-order kernel
    sgs, ogs, gs = small_batch
    # default order, graph-major with small items, 7 interleaved phases with large items and a capped grid
    tunes = [None, {"block_threads": 256, "groups_per_item": 1, "blocks_per_cu": 1},
             {"block_threads": 1024, "groups_per_item": 16, "blocks_per_cu": 2, "max_blocks": 3, "phases": 7},
             {"block_threads": 512, "groups_per_item": 4, "blocks_per_cu": 1, "phases": 64}]
    outs = [P.batch_sample_terms(gs, it, tune=t, graph_id=5, schedule=1) for t in tunes]
    for k, og in enumerate(ogs):
        oi, oj, of = O.sample_terms(og, it, 0, 10 * og.S, graph_id=5 + k)
        for out in outs:
            i, j, f = out[k]
            assert np.array_equal(_to_np_u64(i), oi), f"graph {k}: i differs"
            assert np.array_equal(_to_np_u64(j), oj), f"graph {k}: j differs"
            assert np.array_equal(f.cpu().numpy(), of), f"graph {k}: flags differ"


def test_batched_layout_matches_plain_quality(P, small_batch):
    import torch
    sgs, ogs, gs = small_batch
    init = [O.init_coords(og) for og in ogs]
    cb = [torch.from_numpy(c).cuda() for c in init]
    # one wave: these graphs have only 1.6K-3.9K nodes (see the automatic cap of layout())
    tune = {"block_threads": 64, "groups_per_item": 1, "blocks_per_cu": 1, "max_blocks": 1}
    P.layout_batched(gs, cb, tune=tune, graph_id=0, schedule=1)
    ratios = []
    for k, (og, g) in enumerate(zip(ogs, gs)):
        co = init[k].copy()
        O.layout(og, co, graph_id=k)
        s_b = O.sps_expectation(og, cb[k].cpu().numpy())[0]
        s_o = O.sps_expectation(og, co)[0]
        ratios.append(s_b / s_o)
    print("batched/oracle exact-SPS ratios:", [round(r, 4) for r in ratios])
    assert abs(np.mean(ratios) - 1) <= 0.03


@pytest.mark.parametrize("it", [0, 15])
def test_windowed_batch_sampling_bitexact(P, small_batch, it):
    sgs, ogs, gs = small_batch
    for t in (None, {"block_threads": 256, "groups_per_item": 1, "blocks_per_cu": 1, "branches": 3}):
        out = P.batch_sample_terms(gs, it, tune=t, graph_id=5)
        for k, og in enumerate(ogs):
            oi, oj, of = O.sample_terms_windowed(og, it, 0, 10 * og.S, graph_id=5 + k)
            i, j, f = out[k]
            assert np.array_equal(_to_np_u64(i), oi), f"graph {k}: i differs"
            assert np.array_equal(_to_np_u64(j), oj), f"graph {k}: j differs"
            assert np.array_equal(f.cpu().numpy(), of), f"graph {k}: flags differ"


@pytest.mark.parametrize("branches", [1, 3])
def test_windowed_batch_equals_single_layouts(P, small_batch, branches):
    # these graphs run one wave each (automatic cap), so every graph's layout is
    # deterministic: the batch must reproduce the single-graph layouts exactly
    import torch
    sgs, ogs, gs = small_batch
    init = [O.init_coords(og) for og in ogs]
    cb = [torch.from_numpy(c).cuda() for c in init]
    P.layout_batched(gs, cb, tune={"block_threads": 256, "groups_per_item": 1, "blocks_per_cu": 1,
                                   "branches": branches}, graph_id=3)
    for k, g in enumerate(gs):
        c = torch.from_numpy(init[k]).cuda()
        P.layout(g, c, graph_id=3 + k)
        assert torch.equal(c, cb[k]), f"graph {k} differs from its single layout"


def test_batch_handle_runs_and_autotune_keeps_coords(P, small_batch):
    import torch
    sgs, ogs, gs = small_batch
    cs = [g.new_coords() for g in gs]
    for g, c in zip(gs, cs):
        P.init_coords(g, c)
    before = [c.clone() for c in cs]
    res = P.autotune(gs, cs, use_cache=False, max_blocks=4, schedule=1)
    assert res["block_threads"] % 64 == 0 and res["groups_per_item"] >= 1 and res["max_blocks"] == 4
    assert res["phases"] in (1, 4)
    resw = P.autotune(gs, cs, use_cache=False)
    assert resw["branches"] in (1, 2, 3, 4)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(before, cs))
    bw = P.Batch(gs, cs, tune=resw, first_iter=0, last_iter=2)
    bw.run()
    torch.cuda.synchronize()
    assert any(not torch.equal(a, c) for a, c in zip(before, cs))
    bw.close()
    for g, c in zip(gs, cs):
        P.init_coords(g, c)
    b = P.Batch(gs, cs, tune=res, first_iter=0, last_iter=2, schedule=1)
    b.run()
    torch.cuda.synchronize()
    assert any(not torch.equal(a, c) for a, c in zip(before, cs))
    b.close()


def _scrambled(sg, seed):
    """The same graph with node ids permuted at random (caller id of original node k: q[k])."""
    rng = np.random.default_rng(seed)
    q = rng.permutation(sg.n_nodes).astype(np.uint32)
    node_len = np.empty_like(sg.node_len)
    node_len[q] = sg.node_len
    steps = q[sg.step_node & 0x7FFFFFFF] | (sg.step_node & 0x80000000)
    return synth.SynthGraph(node_len, sg.path_off, steps, dict(sg.stats), sg.name + "-scrambled"), q


def test_renumbered_graph_is_invisible_to_the_caller(P, tiny_synth):
    """The path-guided device order against the caller's own: the same initial
    layout, sampled terms, one-wave layouts (both schedules) bit for bit, the
    same sampled path stress, loss and (to float32 atomics' rounding) gradient,
    all in the caller's node order."""
    import torch
    sg, _ = _scrambled(tiny_synth, 5)
    a = P.Graph.from_synth(sg, renumber="never")
    b = P.Graph.from_synth(sg, renumber="always")
    assert not a.renumbered and b.renumbered
    perm = b.order()
    assert sorted(perm.tolist()) == list(range(sg.n_nodes)) and not np.array_equal(perm, np.arange(sg.n_nodes))
    ca, cb = a.new_coords(), b.new_coords()
    P.init_coords(a, ca)
    P.init_coords(b, cb)
    assert torch.equal(ca, cb)
    for it in (0, 20):
        for x, y in zip(P.sample_terms(a, it, 0, 4096), P.sample_terms(b, it, 0, 4096)):
            assert torch.equal(x, y)
    c0 = ca.clone()
    for sched in (3, 1):
        ca.copy_(c0)
        cb.copy_(c0)
        P.layout(a, ca, schedule=sched, max_inflight_waves=1)
        P.layout(b, cb, schedule=sched, max_inflight_waves=1)
        torch.cuda.synchronize()
        assert torch.equal(ca, cb), f"schedule {sched}: coordinates differ"
    # the same pairs; the window-major orders take work from counters, so their sums agree to rounding
    for pairs in ("uniform", "uniform_windowed", "power_law"):
        ra, rb = P.path_stress(a, ca, 10, 7, pairs=pairs), P.path_stress(b, cb, 10, 7, pairs=pairs)
        assert ra["n_valid"] == rb["n_valid"] and abs(ra["sum"] - rb["sum"]) <= 1e-12 * abs(ra["sum"]), pairs
    assert P.path_stress_exact(a, ca) == P.path_stress_exact(b, cb)
    la, na = P.stress_forward(a, c0, 100_000, 3)
    lb, nb = P.stress_forward(b, c0, 100_000, 3)
    assert abs(float(la) - float(lb)) <= 1e-6 * abs(float(la)) and int(na) == int(nb)
    one = torch.ones(1, device="cuda")
    ga, gb = torch.zeros_like(c0), torch.zeros_like(c0)
    P.stress_backward(a, c0, 100_000, 3, one, na, ga)
    P.stress_backward(b, c0, 100_000, 3, one, nb, gb)
    torch.cuda.synchronize()
    assert torch.allclose(ga, gb, rtol=1e-5, atol=1e-6 * float(ga.abs().max()))


def test_scrambled_ids_lay_out_at_the_ordered_rate(P):
    """A mid-size graph with random node ids: the automatic choice renumbers
    it, and its layout runs at >= 90% of the locality-ordered graph's rate with
    the same sampled path stress (5%); without renumbering it is slower."""
    import time
    import torch
    base = synth.generate(400_000, 0.2, 32, 2)
    sg, q = _scrambled(base, 9)
    res = {}
    for name, s_, mode in (("ordered", base, "auto"), ("scrambled", sg, "auto"), ("scrambled-never", sg, "never")):
        g = P.Graph.from_synth(s_, renumber=mode)
        if name == "scrambled":
            assert g.renumbered
        if name == "ordered":
            assert not g.renumbered
        c = g.new_coords()
        P.init_coords(g, c)
        P.layout(g, c, seed=3)  # warm-up
        best = 1e9
        for rep in range(3):
            P.init_coords(g, c)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P.layout(g, c)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        res[name] = (best, P.path_stress(g, c, 10, 7)["mean"])
        print(f"[renumber] {name}: {best:.4f} s, SPS {res[name][1]:.5g}", flush=True)
        g.close()
    assert res["ordered"][0] / res["scrambled"][0] >= 0.9
    assert abs(res["scrambled"][1] / res["ordered"][1] - 1) < 0.05


@pytest.mark.parametrize("pairs", ["uniform", "power_law", "uniform_windowed"])
def test_sps_outliers_equal_oracle(P, tiny, pairs):
    """The pairs above a stress threshold (the top 1% of Eq. 2's pairs on a
    partly converged tiny layout): the same set of pairs as the oracle's, with
    the same stress, and the same estimate."""
    import torch
    sg, og, g = tiny
    c0 = O.init_coords(og)
    O.layout(og, c0, first_iter=0, last_iter=8)
    n_all, i, j, e, st = O.sps_outliers(og, c0, 10, -1.0, max_out=10 * og.S + 1, seed=7, pairs=pairs)
    thr = float(np.quantile(st, 0.99))
    n_ref, i_ref, j_ref, e_ref, s_ref = O.sps_outliers(og, c0, 10, thr, seed=7, pairs=pairs)
    c = torch.from_numpy(c0).cuda()
    n, gi, gj, ge, gs, res = P.path_stress_outliers(g, c, 10, thr, max_out=4096, seed=7, pairs=pairs)
    assert n == n_ref and res["n_valid"] == n_all
    got = sorted(zip(gi.cpu().numpy().tolist(), gj.cpu().numpy().tolist(), ge.cpu().numpy().tolist(),
                     gs.cpu().numpy().tolist()))
    ref = sorted(zip(i_ref.tolist(), j_ref.tolist(), e_ref.tolist(), s_ref.tolist()))
    assert [x[:3] for x in got] == [x[:3] for x in ref]
    assert all(abs(a[3] - b[3]) <= 1e-12 * abs(b[3]) for a, b in zip(got, ref))
    # max_out below the count: the count stays exact, max_out pairs are written
    n2, gi2, *_ = P.path_stress_outliers(g, c, 10, thr, max_out=7, seed=7, pairs=pairs)
    assert n2 == n_ref and gi2.numel() == 7


def test_windowed_batch_keeps_its_power_law_table(P, small_batch):
    """A batch captured with W = 1000 keeps its own power-law table: calls on
    its graphs with another window and exponent (which rewrite each graph's own
    table) in between do not change what the batch samples, so its one-wave
    layouts still equal the single-graph layouts with W = 1000."""
    import torch
    sgs, ogs, gs = small_batch
    init = [O.init_coords(og) for og in ogs]
    cb = [torch.from_numpy(c).cuda() for c in init]
    b = P.Batch(gs, cb, tune={"block_threads": 256, "groups_per_item": 1, "blocks_per_cu": 1, "branches": 1},
                graph_id=3)
    for g, c in zip(gs, cb):
        P.stress_forward(g, c, 10_000, 1, zipf_window=100, zipf_theta=0.5)
    b.run()
    torch.cuda.synchronize()
    b.close()
    for k, g in enumerate(gs):
        c = torch.from_numpy(init[k]).cuda()
        P.layout(g, c, graph_id=3 + k)
        assert torch.equal(c, cb[k]), f"graph {k} differs from its single layout"


def test_batch_rejects_the_data_reuse_variant(P, small_batch):
    sgs, ogs, gs = small_batch
    cs = [g.new_coords() for g in gs]
    for kw in ({"reuse_factor": 2}, {"step_reduction": 2}):
        with pytest.raises(P.PgsgdError):
            P.Batch(gs, cs, **kw)


@pytest.mark.parametrize("pairs", ["uniform", "power_law", "uniform_windowed"])
def test_sps_compare_equals_oracle(P, tiny, pairs):
    """Two layouts on the same pairs: means, ratio and spreads as the oracle's
    paired evaluation (sums of FP64 terms in another order: 1e-9)."""
    import torch
    sg, og, g = tiny
    ca = O.init_coords(og)
    O.layout(og, ca, first_iter=0, last_iter=8)
    cb = ca.copy()
    O.layout(og, cb, first_iter=8, last_iter=30)
    ref = O.sps_compare(og, ca, cb, m=10, seed=7, pairs=pairs)
    r = P.path_stress_compare(g, torch.from_numpy(ca).cuda(), torch.from_numpy(cb).cuda(), 10, 7, pairs=pairs)
    assert r["n_valid"] == ref["n_valid"] and r["n_skipped"] == ref["n_skipped"]
    for k in ("sum_a", "sum_b", "ratio", "ratio_ci_lo", "ratio_ci_hi", "sd_a", "sd_b", "sd_diff"):
        assert abs(r[k] - ref[k]) <= 1e-9 * abs(ref[k]), k
    same = P.path_stress_compare(g, torch.from_numpy(ca).cuda(), torch.from_numpy(ca).cuda(), 10, 7, pairs=pairs)
    assert same["ratio"] == 1.0 and same["sd_diff"] == 0.0
