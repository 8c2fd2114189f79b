"""What the collision-free batch check of the update can resolve (no GPU).

The GPU tests apply one collision-free batch of sampled terms with the HIP
kernels and compare it with the oracle's FP64 result through
batch_check.check.  Here the same batches (tiny and mid graphs, iterations 0
and 25, the first 65,536 sampled terms thinned to distinct slots, start
coordinates near the origin) are checked against results the check must accept
(the FP64 result stored in FP32; the oracle's own FP32-storage update) and
against planted errors it must reject: the update's r scaled by 1 + eps, where
the smallest rejected eps on a quarter-decade grid is the check's resolution.
"""
import numpy as np
import pytest

import batch_check as B
import oracle as O
import synth


@pytest.fixture(scope="module", params=["tiny", "mid"])
def graph(request):
    og = O.Graph.from_synth(synth.config_graph(request.param))
    return request.param, og, og.pos


def _batch(og, it):
    eta = float(O.schedule(30, float(og.d_max) ** 2, 0.01).astype(np.float32)[it])
    i, j, f = O.sample_terms(og, it, 0, B.K_TERMS)
    keep = B.collision_free(og, i, j, f)
    return eta, i[keep], j[keep], f[keep], B.start_coords(og, it)


@pytest.mark.parametrize("it", [0, 25])
def test_batch_check_accepts_fp32_results(graph, it):
    name, og, pos = graph
    eta, i, j, f, start = _batch(og, it)
    assert i.size > 2000
    ref, applied = B.fp64_result(og, eta, i, j, f, start)
    assert applied == i.size  # no coincident points in a random start
    worst, untouched = B.check(og, pos, i, j, f, eta, start, ref.astype(np.float32).astype(np.float64), ref)
    assert worst <= 1.0 and untouched
    c32 = start.copy()
    O.apply_terms_f32(og, eta, i, j, f, c32)
    worst, untouched = B.check(og, pos, i, j, f, eta, start, c32.astype(np.float64), ref)
    assert worst <= 1.0 and untouched


@pytest.mark.parametrize("it", [0, 25])
def test_batch_check_resolves_the_update(graph, it):
    # measured: 1.8e-5 in all four cases (the first grid point above the 1e-5 bar)
    name, og, pos = graph
    eta, i, j, f, start = _batch(og, it)
    eps = B.resolution(og, pos, i, j, f, eta, start)
    print(f"{name} iteration {it}: smallest rejected relative error of r = {eps}")
    assert eps is not None and eps <= 1e-4


@pytest.mark.parametrize("it", [0, 25])
def test_batch_check_rejects_a_moved_untouched_coordinate(graph, it):
    name, og, pos = graph
    eta, i, j, f, start = _batch(og, it)
    ref, _ = B.fp64_result(og, eta, i, j, f, start)
    got = ref.astype(np.float32).astype(np.float64)
    a, b = B.slots(og, i, j, f)
    free = np.setdiff1d(np.arange(2 * og.n_nodes), np.concatenate([a, b]))
    got[free[0]] += 1.0
    assert not B.check(og, pos, i, j, f, eta, start, got, ref)[1]
