"""The allocation-free layout entry point (pgsgd_layout_noalloc) against
pgsgd_layout, through the C ABI: the same coordinates bit for bit where the
layout is deterministic (one wave), several calls in a row on graphs of
decreasing size (the shared scratch keeps the previous call's contents), the
graph's device memory unchanged by the call, and the sampled path stress of a
multi-wave layout within 3% of the allocating entry point's."""
import ctypes

import pytest

import synth
import paper_2409_00876_amd as P
from paper_2409_00876_amd import _lib

pytestmark = pytest.mark.gpu


def _call(name, g, c, params):
    import torch
    p = params.to_c()
    fn = getattr(P.lib(), name)
    st = fn(g.handle, ctypes.byref(p), ctypes.c_void_p(c.data_ptr()),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def _device_bytes(g):
    info = _lib.GraphInfo()
    _lib.check(P.lib().pgsgd_graph_get_info(g.handle, ctypes.byref(info)))
    return int(info.device_bytes)


def _pair(sg, params, label):
    """Lays sg out with both entry points from the same initial layout."""
    import torch
    print(f"[no_alloc] {label}: {sg.n_steps} steps", flush=True)
    g = P.Graph.from_synth(sg)
    a = g.new_coords()
    P.init_coords(g, a)
    b = a.clone()
    before = _device_bytes(g)
    _lib.check(_call("pgsgd_layout_noalloc", g, b, params))
    torch.cuda.synchronize()
    assert _device_bytes(g) == before, "the allocation-free call changed the graph's device memory"
    _lib.check(_call("pgsgd_layout", g, a, params))
    torch.cuda.synchronize()
    return g, a, b


@pytest.mark.parametrize("schedule", [3, 1])
def test_noalloc_equals_layout_on_shrinking_graphs(schedule):
    import torch
    graphs = [synth.config_graph("tiny"), synth.generate(600, 0.2, 4, 17), synth.generate(120, 0.2, 2, 18)]
    for k, sg in enumerate(graphs):
        params = P.LayoutParams(max_inflight_waves=1, schedule=schedule)
        g, a, b = _pair(sg, params, f"schedule {schedule}, graph {k}")
        assert torch.equal(a, b), f"graph {k}: coordinates differ"
        g.close()


def test_noalloc_data_reuse_equals_layout():
    import torch
    for k, sg in enumerate([synth.config_graph("tiny"), synth.generate(500, 0.2, 3, 19)]):
        params = P.LayoutParams(max_inflight_waves=1, reuse_factor=2, step_reduction=2)
        g, a, b = _pair(sg, params, f"data reuse, graph {k}")
        assert torch.equal(a, b), f"graph {k}: coordinates differ"
        g.close()


def test_noalloc_multiwave_stress_matches():
    """Automatic wave count (Hogwild races make the coordinates differ): the
    two layouts compared on the same pairs of Eq. 2 (the estimate's heavy tail
    cancels), within 3% or within the paired CI95; then a smaller graph
    follows on the same scratch."""
    for k, sg in enumerate([synth.generate(150_000, 0.2, 16, 5), synth.generate(40_000, 0.2, 8, 6)]):
        g, a, b = _pair(sg, P.LayoutParams(), f"automatic waves, graph {k}")
        r = P.path_stress_compare(g, b, a, 100, 7, pairs="uniform_windowed")
        print(f"[no_alloc] graph {k}: SPS noalloc / layout {r['ratio']:.4f} [{r['ratio_ci_lo']:.4f}, "
              f"{r['ratio_ci_hi']:.4f}]", flush=True)
        assert abs(r["ratio"] - 1) < 0.03 or r["ratio_ci_lo"] <= 1.0 <= r["ratio_ci_hi"]
        g.close()


def test_noalloc_rejects_count_ahead():
    sg = synth.config_graph("tiny")
    g = P.Graph.from_synth(sg)
    c = g.new_coords()
    P.init_coords(g, c)
    st = _call("pgsgd_layout_noalloc", g, c, P.LayoutParams(flags=_lib.FLAG_COUNT_AHEAD))
    assert st == _lib.ERR_INVALID_ARG
    assert "COUNT_AHEAD" in P.lib().pgsgd_last_error().decode()
