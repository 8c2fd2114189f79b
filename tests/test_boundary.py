"""CPU tests of the C ABI: the library loads and exports every declared symbol,
the host-only entry points agree with the oracle, and every validation error is
reported before any device work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2409_00876_amd as P
from paper_2409_00876_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pgsgd.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pgsgd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = P.lib()
    names = _declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), f"{n} declared in pgsgd.h but not exported"
        assert n in _lib.SIGNATURES, f"{n} has no ctypes signature"
    assert P.lib().pgsgd_version().startswith(b"pgsgd-gfx950")


def test_binding_constants_match_the_header():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    declared = {name: int(val) for name, val in re.findall(r"\b(PGSGD_[A-Z_]+)\s*=\s*(-?\d+)", text)}
    binding = {"PGSGD_OK": _lib.OK, "PGSGD_ERR_INVALID_ARG": _lib.ERR_INVALID_ARG, "PGSGD_ERR_RANGE": _lib.ERR_RANGE,
               "PGSGD_ERR_OOM": _lib.ERR_OOM, "PGSGD_ERR_DEVICE": _lib.ERR_DEVICE,
               "PGSGD_ERR_UNSUPPORTED": _lib.ERR_UNSUPPORTED,
               "PGSGD_SCHEDULE_AUTO": _lib.SCHEDULE_AUTO, "PGSGD_SCHEDULE_PLAIN": _lib.SCHEDULE_PLAIN,
               "PGSGD_SCHEDULE_WINDOWED": _lib.SCHEDULE_WINDOWED,
               "PGSGD_PAIRS_UNIFORM": _lib.PAIRS_UNIFORM, "PGSGD_PAIRS_POWER_LAW": _lib.PAIRS_POWER_LAW,
               "PGSGD_PAIRS_UNIFORM_WINDOWED": _lib.PAIRS_UNIFORM_WINDOWED,
               "PGSGD_FLAG_COUNT_AHEAD": _lib.FLAG_COUNT_AHEAD, "PGSGD_FLAG_COUNT_IN_ORDER": _lib.FLAG_COUNT_IN_ORDER,
               "PGSGD_RENUMBER_AUTO": _lib.RENUMBER_AUTO, "PGSGD_RENUMBER_NEVER": _lib.RENUMBER_NEVER,
               "PGSGD_RENUMBER_ALWAYS": _lib.RENUMBER_ALWAYS}
    for name, val in declared.items():
        assert name in binding, f"{name} declared in pgsgd.h but missing from the binding"
        assert binding[name] == val, f"{name}: header {val}, binding {binding[name]}"


def test_params_default_matches_paper_settings():
    p = _lib.Params()
    P.lib().pgsgd_params_default(ctypes.byref(p))
    assert (p.n_iters, p.terms_per_step, p.zipf_window, p.seed) == (30, 10, 1000, 24301)
    assert p.eta_max == 0.0 and p.eta_min == 0.01 and p.zipf_theta == 0.99 and p.flags == 0


@pytest.mark.parametrize("theta,W", [(0.99, 1000), (1.0, 60), (0.0, 37), (0.5, 1), (1.5, 4096)])
def test_zipf_table_equals_oracle_table(theta, W):
    assert np.array_equal(P.zipf_table(theta, W), O.zipf_table(theta, W))


@pytest.mark.parametrize("n_iters,dmax", [(30, 8973), (30, 4_300_000), (1, 50), (7, 2)])
def test_schedule_equals_oracle_schedule_in_float32(n_iters, dmax):
    eta = P.schedule(n_iters=n_iters, d_max=dmax)
    ref = O.schedule(n_iters, float(dmax) ** 2, 0.01).astype(np.float32)
    assert np.array_equal(eta, ref)


def _create(n_nodes, node_len, path_off, step_node, step_pos=None):
    node_len = np.ascontiguousarray(node_len, np.uint32)
    path_off = np.ascontiguousarray(path_off, np.uint64)
    step_node = np.ascontiguousarray(step_node, np.uint32)
    h = ctypes.c_void_p()
    sp = None if step_pos is None else np.ascontiguousarray(step_pos, np.int64)
    st = P.lib().pgsgd_graph_create(
        n_nodes, node_len.ctypes.data if node_len.size else None, len(path_off) - 1,
        path_off.ctypes.data if path_off.size else None, step_node.ctypes.data if step_node.size else None,
        sp.ctypes.data if sp is not None else None, 0, ctypes.byref(h))
    return st, h


GOOD = dict(n_nodes=3, node_len=[3, 2, 4], path_off=[0, 3], step_node=[0, 1 | 0x80000000, 2])


@pytest.mark.parametrize("change,status,needle", [
    (dict(node_len=[3, 0, 4]), _lib.ERR_INVALID_ARG, "length 0"),
    (dict(step_node=[0, 7, 2]), _lib.ERR_INVALID_ARG, "node 7"),
    (dict(path_off=[1, 3]), _lib.ERR_INVALID_ARG, "path_offsets[0]"),
    (dict(path_off=[0, 3, 2], step_node=[0, 1, 2]), _lib.ERR_INVALID_ARG, "monotone"),
    (dict(step_pos=[0, 3, 6]), _lib.ERR_INVALID_ARG, "step_pos"),
    (dict(path_off=[0]), _lib.ERR_INVALID_ARG, "n_paths"),
    (dict(n_nodes=2 ** 31), _lib.ERR_RANGE, "2^31"),
])
def test_graph_create_validation_errors(change, status, needle):
    args = dict(GOOD, **change)
    st, h = _create(**args)
    assert st == status and not h.value
    assert needle in P.lib().pgsgd_last_error().decode()


def test_graph_create_step_pos_accepted_when_correct():
    # valid input gets past validation; without a GPU it then fails at the device
    st, h = _create(**dict(GOOD, step_pos=[0, 3, 5]))
    assert st in (_lib.OK, _lib.ERR_DEVICE)
    if st == _lib.OK:
        P.lib().pgsgd_graph_destroy(h)


def test_null_pointers_are_rejected():
    L = P.lib()
    assert L.pgsgd_graph_create(1, None, 1, None, None, None, 0, None) == _lib.ERR_INVALID_ARG
    assert L.pgsgd_layout(None, None, None, None) == _lib.ERR_INVALID_ARG
    assert L.pgsgd_path_stress(None, None, 100, 7, 0, None, None) == _lib.ERR_INVALID_ARG
    assert L.pgsgd_schedule(None, 1, None) == _lib.ERR_INVALID_ARG
    assert L.pgsgd_zipf_table(0.99, 0, None) == _lib.ERR_INVALID_ARG
    assert L.pgsgd_adam_step(None, None, None, None, 1, 1.0, 0.9, 0.999, 1e-8, 1, None) == _lib.ERR_INVALID_ARG
    assert L.pgsgd_layout_batched(None, 0, None, None, None, None) == _lib.ERR_INVALID_ARG
    L.pgsgd_graph_destroy(None)
    L.pgsgd_batch_destroy(None)


def test_zipf_window_limits():
    out = np.zeros(70000, np.uint32)
    assert P.lib().pgsgd_zipf_table(0.99, 65536, out.ctypes.data) == _lib.ERR_INVALID_ARG
    assert P.lib().pgsgd_zipf_table(float("nan"), 10, out.ctypes.data) == _lib.ERR_INVALID_ARG
    assert P.lib().pgsgd_zipf_table(0.99, 65535, out.ctypes.data) == _lib.OK


def test_python_binding_rejects_cpu_tensors():
    import torch
    with pytest.raises((ValueError, TypeError)):
        P._check_tensor(torch.zeros(4), torch.float32, 4, "coords")


def test_device_byte_cap_forces_oom_before_device_work(monkeypatch, tiny_synth):
    """PGSGD_MAX_DEVICE_BYTES below what a graph needs: OOM, reported before
    any device work (so it shows without a GPU); a cap above it (or no cap)
    gets past the check."""
    sg = tiny_synth
    monkeypatch.setenv("PGSGD_MAX_DEVICE_BYTES", "100000")  # the records alone need 16 B x 14,416 steps
    st, h = _create(sg.n_nodes, sg.node_len, sg.path_off, sg.step_node)
    assert st == _lib.ERR_OOM and not h.value
    msg = P.lib().pgsgd_last_error().decode()
    assert "PGSGD_MAX_DEVICE_BYTES = 100000" in msg and "needs" in msg
    for cap in ("1000000000", "0", "garbage"):
        monkeypatch.setenv("PGSGD_MAX_DEVICE_BYTES", cap)
        st, h = _create(sg.n_nodes, sg.node_len, sg.path_off, sg.step_node)
        assert st in (_lib.OK, _lib.ERR_DEVICE)
        if st == _lib.OK:
            P.lib().pgsgd_graph_destroy(h)


def test_path_order_by_hand():
    """Progressive linearization: path 0 gives 0 1 2; path 1 (0, 3, 2) inserts
    node 3 right after 0; node 4 (on no path) goes last."""
    perm, fb, fa = P.path_order([1, 1, 1, 1, 1], [0, 3, 6], [0, 1, 2, 0, 3 | 0x80000000, 2])
    assert perm.tolist() == [0, 2, 3, 1, 4]
    # consecutive steps 0-1, 1-2, 0-3, 3-2: no jump is above 32 ids in either order
    assert fb == 0.0 and fa == 0.0


def test_path_order_restores_locality_of_scrambled_ids(tiny_synth):
    sg = tiny_synth
    rng = np.random.default_rng(3)
    q = rng.permutation(sg.n_nodes).astype(np.uint32)   # caller id of every original node
    node_len = np.empty_like(sg.node_len)
    node_len[q] = sg.node_len
    steps = q[sg.step_node & 0x7FFFFFFF] | (sg.step_node & 0x80000000)
    perm, fb, fa = P.path_order(node_len, sg.path_off, steps)
    assert sorted(perm.tolist()) == list(range(sg.n_nodes))       # a permutation
    assert fb > 0.9 and fa < 0.01
    # the order depends on the graph only, not on the caller's ids
    perm0, _, _ = P.path_order(sg.node_len, sg.path_off, sg.step_node)
    assert np.array_equal(perm[q], perm0)


def test_graph_create_ex_rejects_unknown_renumber_mode():
    st = P.lib().pgsgd_graph_create_ex(3, np.array([1, 1, 1], np.uint32).ctypes.data, 1,
                                       np.array([0, 3], np.uint64).ctypes.data,
                                       np.array([0, 1, 2], np.uint32).ctypes.data, None, 0, 3,
                                       ctypes.byref(ctypes.c_void_p()))
    assert st == _lib.ERR_INVALID_ARG and "renumber" in P.lib().pgsgd_last_error().decode()
