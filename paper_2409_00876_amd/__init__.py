"""PG-SGD pangenome graph layout on MI355X (gfx950).

A thin Python binding over ``libpgsgd.so``: it checks torch tensors (device,
dtype, contiguity), passes their device pointers and the current HIP stream to
the C ABI, and wraps the differentiable sampled stress as a
``torch.autograd.Function``.  Every step of the computation runs in the
library's HIP kernels; torch only supplies device memory and streams.

Method: "Rapid GPU-Based Pangenome Graph Layout" (SC24), Alg. 1 (layout loop)
and Eq. 2 (sampled path stress).
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass

import numpy as np
import torch

from ._lib import (CompareResult, GfaView, FLAG_COUNT_AHEAD, FLAG_COUNT_IN_ORDER, SCHEDULE_AUTO, SCHEDULE_WINDOWED, GraphInfo, Params, PgsgdError, StressResult, Tune,  # noqa: F401
                   check, lib)

__all__ = ["Graph", "GfaGraph", "read_gfa", "parse_gfa", "path_order", "LayoutParams", "layout", "layout_noalloc", "layout_timed", "init_coords", "path_stress", "path_stress_compare", "path_stress_outliers", "path_stress_exact", "schedule", "zipf_table",
           "sample_terms", "sample_terms_reuse", "apply_terms", "apply_slots", "stress_forward", "stress_backward", "SampledPathStress", "adam_step",
           "Batch", "layout_batched", "batch_sample_terms", "autotune", "PgsgdError"]


def _stream(torch, device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _np_ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _check_tensor(t, dtype, numel=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


@dataclass
class LayoutParams:
    """Alg. 1 inputs; defaults follow the paper (30 iterations, 10 terms per step)."""
    n_iters: int = 30
    terms_per_step: int = 10
    eta_max: float = 0.0        # <= 0: d_max^2
    eta_min: float = 0.01
    zipf_theta: float = 0.99
    zipf_window: int = 1000
    graph_id: int = 0
    seed: int = 24301
    first_iter: int = 0
    last_iter: int = 0
    max_inflight_waves: int = 0
    flags: int = 0
    schedule: int = 0           # 0 auto (= 3), 1 plain, 3 windowed
    reuse_factor: int = 1       # data-reuse variant: updates per sampled term (DRF)
    step_reduction: int = 1     # data-reuse variant: sampled terms divided by SRF

    def to_c(self) -> Params:
        p = Params()
        for f in Params._fields_:
            setattr(p, f[0], getattr(self, f[0]))
        return p


def _params(params, kw) -> Params:
    if params is None:
        params = LayoutParams(**kw)
    elif kw:
        params = LayoutParams(**{**params.__dict__, **kw})
    return params.to_c()


@dataclass
class GfaGraph:
    """The lean structure of a GFA file (the arrays Graph takes), with names.

    node_len  : uint32[n_nodes]; node k is the k-th S line
    path_off  : uint64[n_paths+1]; path p is the p-th P or W line
    step_node : uint32[S]; bit 31 = reverse-strand step
    """
    node_len: np.ndarray
    path_off: np.ndarray
    step_node: np.ndarray
    path_names: list
    n_links: int
    _node_names: bytes
    _node_name_off: np.ndarray

    @property
    def n_nodes(self) -> int:
        return int(self.node_len.shape[0])

    @property
    def n_paths(self) -> int:
        return int(self.path_off.shape[0]) - 1

    @property
    def n_steps(self) -> int:
        return int(self.path_off[-1])

    def node_name(self, k: int) -> str:
        return self._node_names[int(self._node_name_off[k]):int(self._node_name_off[k + 1]) - 1].decode()


def _gfa_from_handle(h) -> GfaGraph:
    try:
        v = GfaView()
        check(lib().pgsgd_gfa_get_view(h, ctypes.byref(v)))

        def arr(ptr, n, ctype, dtype):
            if n == 0:
                return np.zeros(0, dtype=dtype)
            return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctype)), shape=(n,)).astype(dtype, copy=True)

        nn, npth, ns = int(v.n_nodes), int(v.n_paths), int(v.n_steps)
        node_len = arr(v.node_len, nn, ctypes.c_uint32, np.uint32)
        path_off = arr(v.path_offsets, npth + 1, ctypes.c_uint64, np.uint64)
        step_node = arr(v.step_node, ns, ctypes.c_uint32, np.uint32)
        noff = arr(v.node_name_offsets, nn + 1, ctypes.c_uint64, np.uint64)
        poff = arr(v.path_name_offsets, npth + 1, ctypes.c_uint64, np.uint64)
        nnames = ctypes.string_at(v.node_names, int(noff[-1])) if nn else b""
        pblob = ctypes.string_at(v.path_names, int(poff[-1])) if npth else b""
        pnames = [pblob[int(poff[k]):int(poff[k + 1]) - 1].decode() for k in range(npth)]
        return GfaGraph(node_len, path_off, step_node, pnames, int(v.n_links), nnames, noff)
    finally:
        lib().pgsgd_gfa_free(h)


def path_order(node_len, path_off, step_node):
    """The path-guided node order (host only): (perm, far_before, far_after),
    perm[n] = new id of node n."""
    node_len = np.ascontiguousarray(node_len, dtype=np.uint32)
    path_off = np.ascontiguousarray(path_off, dtype=np.uint64)
    step_node = np.ascontiguousarray(step_node, dtype=np.uint32)
    perm = np.empty(len(node_len), dtype=np.uint32)
    fb, fa = ctypes.c_double(), ctypes.c_double()
    check(lib().pgsgd_path_order(len(node_len), _np_ptr(node_len), len(path_off) - 1, _np_ptr(path_off),
                                 _np_ptr(step_node) if step_node.size else None, _np_ptr(perm), ctypes.byref(fb),
                                 ctypes.byref(fa)))
    return perm, fb.value, fa.value


def read_gfa(path: str) -> GfaGraph:
    """Reads a GFA 1.0/1.1 file (S, P and W lines) into the lean structure."""
    h = ctypes.c_void_p()
    check(lib().pgsgd_gfa_read(os.fsencode(path), ctypes.byref(h)))
    return _gfa_from_handle(h)


def parse_gfa(text) -> GfaGraph:
    """The same as read_gfa for GFA text held in memory (str or bytes)."""
    data = text.encode() if isinstance(text, str) else bytes(text)
    h = ctypes.c_void_p()
    check(lib().pgsgd_gfa_parse(data, len(data), ctypes.byref(h)))
    return _gfa_from_handle(h)


class Graph:
    """A variation graph resident on one GPU (node lengths and path steps)."""

    RENUMBER = {"auto": 0, "never": 1, "always": 2}

    def __init__(self, node_len, path_off, step_node, step_pos=None, device: int = 0, renumber: str = "auto"):
        node_len = np.ascontiguousarray(node_len, dtype=np.uint32)
        path_off = np.ascontiguousarray(path_off, dtype=np.uint64)
        step_node = np.ascontiguousarray(step_node, dtype=np.uint32)
        pos = None if step_pos is None else np.ascontiguousarray(step_pos, dtype=np.int64)
        h = ctypes.c_void_p()
        check(lib().pgsgd_graph_create_ex(len(node_len), _np_ptr(node_len), len(path_off) - 1, _np_ptr(path_off),
                                          _np_ptr(step_node) if step_node.size else None,
                                          _np_ptr(pos) if pos is not None else None, int(device),
                                          self.RENUMBER[renumber], ctypes.byref(h)))
        self._h = h
        self.device = int(device)
        info = GraphInfo()
        check(lib().pgsgd_graph_get_info(h, ctypes.byref(info)))
        self.n_nodes = int(info.n_nodes)
        self.n_paths = int(info.n_paths)
        self.n_steps = int(info.n_steps)
        self.d_max = int(info.d_max)
        self.device_bytes = int(info.device_bytes)
        self.renumbered = bool(info.renumbered)

    @classmethod
    def from_synth(cls, sg, device: int = 0, renumber: str = "auto"):
        return cls(sg.node_len, sg.path_off, sg.step_node, device=device, renumber=renumber)

    def order(self) -> np.ndarray:
        """Device node id of every caller node id (the identity unless renumbered)."""
        perm = np.empty(self.n_nodes, dtype=np.uint32)
        check(lib().pgsgd_graph_get_order(self._h, _np_ptr(perm)))
        return perm

    @classmethod
    def from_gfa(cls, path: str, device: int = 0):
        """Reads a GFA file and copies its paths and node lengths to the device."""
        gg = read_gfa(path)
        return cls(gg.node_len, gg.path_off, gg.step_node, device=device)

    @property
    def handle(self):
        return self._h

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            lib().pgsgd_graph_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_coords(self):
        import torch
        return torch.empty(4 * self.n_nodes, dtype=torch.float32, device=f"cuda:{self.device}")


def schedule(params: LayoutParams | None = None, d_max: int = 1, **kw) -> np.ndarray:
    p = _params(params, kw)
    out = np.zeros(max(1, p.n_iters), dtype=np.float32)
    check(lib().pgsgd_schedule(ctypes.byref(p), int(d_max), _np_ptr(out)))
    return out[: p.n_iters]


def zipf_table(theta: float = 0.99, window: int = 1000) -> np.ndarray:
    out = np.zeros(window + 1, dtype=np.uint32)
    check(lib().pgsgd_zipf_table(float(theta), int(window), _np_ptr(out)))
    return out


def init_coords(g: Graph, coords, seed: int = 5, jitter: float = 10.0, graph_id: int = 0):
    import torch
    _check_tensor(coords, torch.float32, 4 * g.n_nodes, "coords")
    check(lib().pgsgd_init_coords(g.handle, int(seed), int(graph_id), float(jitter), ctypes.c_void_p(coords.data_ptr()),
                                  _stream(torch, coords.device)))
    return coords


def layout(g: Graph, coords, params: LayoutParams | None = None, **kw):
    """Runs Alg. 1 in place on coords (float32 [2][n_nodes][2] on the GPU), async on the current stream."""
    import torch
    _check_tensor(coords, torch.float32, 4 * g.n_nodes, "coords")
    p = _params(params, kw)
    check(lib().pgsgd_layout(g.handle, ctypes.byref(p), ctypes.c_void_p(coords.data_ptr()),
                             _stream(torch, coords.device)))
    return coords


def layout_noalloc(g: Graph, coords, params: LayoutParams | None = None, **kw):
    """layout() without device allocation: the windowed schedule's tables live
    in the library's per-device scratch array (calls on one device must not
    overlap); async on the current stream."""
    import torch
    _check_tensor(coords, torch.float32, 4 * g.n_nodes, "coords")
    p = _params(params, kw)
    check(lib().pgsgd_layout_noalloc(g.handle, ctypes.byref(p), ctypes.c_void_p(coords.data_ptr()),
                                     _stream(torch, coords.device)))
    return coords


def layout_timed(g: Graph, coords, params: LayoutParams | None = None, **kw):
    """layout() with HIP-event timing on the current stream; synchronises.
    Returns (iter_ms, main_ms, main_launches): each iteration's duration, the
    summed duration of its dominant-kernel launches, and that kernel's launches
    per iteration."""
    _check_tensor(coords, torch.float32, 4 * g.n_nodes, "coords")
    p = _params(params, kw)
    last = p.last_iter or p.n_iters
    n = max(1, last - p.first_iter)
    it_ms = np.zeros(n, dtype=np.float32)
    main_ms = np.zeros(n, dtype=np.float32)
    launches = ctypes.c_uint32()
    check(lib().pgsgd_layout_timed(g.handle, ctypes.byref(p), ctypes.c_void_p(coords.data_ptr()), _np_ptr(it_ms),
                                   _np_ptr(main_ms), ctypes.byref(launches), _stream(torch, coords.device)))
    return it_ms[: last - p.first_iter], main_ms[: last - p.first_iter], int(launches.value)


def path_stress(g: Graph, coords, pairs_per_step: int = 100, seed: int = 7, graph_id: int = 0,
                pairs: str = "uniform", zipf_theta: float = 0.99, zipf_window: int = 1000) -> dict:
    """Sampled path stress (Eq. 2) with CI95; synchronises the current stream.
    pairs="power_law" takes the cooling phase's power-law partner instead of a
    uniform one (a measure of local structure); pairs="uniform_windowed"
    samples the uniform law in window-major order (faster on large graphs)."""
    import torch
    _check_tensor(coords, torch.float32, 4 * g.n_nodes, "coords")
    modes = {"uniform": 0, "power_law": 1, "uniform_windowed": 2}
    if pairs not in modes:
        raise ValueError(f"pairs must be one of {sorted(modes)}")
    r = StressResult()
    check(lib().pgsgd_path_stress_pairs(g.handle, ctypes.c_void_p(coords.data_ptr()), int(pairs_per_step),
                                        int(seed), int(graph_id), modes[pairs], float(zipf_theta), int(zipf_window),
                                        ctypes.byref(r), _stream(torch, coords.device)))
    return {f[0]: getattr(r, f[0]) for f in StressResult._fields_}


def path_stress_compare(g: Graph, coords_a, coords_b, pairs_per_step: int = 10, seed: int = 7, graph_id: int = 0,
                        pairs: str = "uniform", zipf_theta: float = 0.99, zipf_window: int = 1000) -> dict:
    """Two layouts on the same pairs of Eq. 2: means, the ratio of the sums
    with its paired (delta-method) CI95; synchronises the current stream."""
    import torch
    _check_tensor(coords_a, torch.float32, 4 * g.n_nodes, "coords_a")
    _check_tensor(coords_b, torch.float32, 4 * g.n_nodes, "coords_b")
    modes = {"uniform": 0, "power_law": 1, "uniform_windowed": 2}
    r = CompareResult()
    check(lib().pgsgd_path_stress_compare(g.handle, ctypes.c_void_p(coords_a.data_ptr()),
                                          ctypes.c_void_p(coords_b.data_ptr()), int(pairs_per_step), int(seed),
                                          int(graph_id), modes[pairs], float(zipf_theta), int(zipf_window),
                                          ctypes.byref(r), _stream(torch, coords_a.device)))
    return {f[0]: getattr(r, f[0]) for f in CompareResult._fields_}


def path_stress_outliers(g: Graph, coords, pairs_per_step: int, threshold: float, max_out: int = 1 << 20,
                         seed: int = 7, graph_id: int = 0, pairs: str = "uniform", zipf_theta: float = 0.99,
                         zipf_window: int = 1000):
    """The pairs of path_stress() whose stress exceeds threshold: (count, i, j,
    e, stress, result) with i, j, e, stress device tensors of the first
    min(count, max_out) pairs found (in no particular order)."""
    import torch
    _check_tensor(coords, torch.float32, 4 * g.n_nodes, "coords")
    modes = {"uniform": 0, "power_law": 1, "uniform_windowed": 2}
    dev = coords.device
    i = torch.empty(max(1, max_out), dtype=torch.int64, device=dev)
    j = torch.empty_like(i)
    e = torch.empty(max(1, max_out), dtype=torch.uint8, device=dev)
    s = torch.empty(max(1, max_out), dtype=torch.float64, device=dev)
    n = ctypes.c_uint64()
    r = StressResult()
    check(lib().pgsgd_path_stress_outliers(g.handle, ctypes.c_void_p(coords.data_ptr()), int(pairs_per_step),
                                           int(seed), int(graph_id), modes[pairs], float(zipf_theta),
                                           int(zipf_window), float(threshold), int(max_out),
                                           ctypes.c_void_p(i.data_ptr()), ctypes.c_void_p(j.data_ptr()),
                                           ctypes.c_void_p(e.data_ptr()), ctypes.c_void_p(s.data_ptr()),
                                           ctypes.byref(n), ctypes.byref(r), _stream(torch, dev)))
    k = min(int(n.value), max_out)
    return int(n.value), i[:k], j[:k], e[:k], s[:k], {f[0]: getattr(r, f[0]) for f in StressResult._fields_}


def path_stress_exact(g: Graph, coords):
    """Path stress (Eq. 1) over all same-path step pairs; returns (mean, pairs). Synchronises."""
    _check_tensor(coords, torch.float32, 4 * g.n_nodes, "coords")
    mean = ctypes.c_double()
    pairs = ctypes.c_uint64()
    check(lib().pgsgd_path_stress_exact(g.handle, ctypes.c_void_p(coords.data_ptr()), ctypes.byref(mean),
                                        ctypes.byref(pairs), _stream(torch, coords.device)))
    return mean.value, int(pairs.value)


def sample_terms(g: Graph, iter: int, t_begin: int, count: int, params: LayoutParams | None = None, **kw):
    """The terms layout() samples: (i, j, flags) as device tensors (uint64 as int64, uint8)."""
    import torch
    p = _params(params, kw)
    dev = f"cuda:{g.device}"
    i = torch.empty(count, dtype=torch.int64, device=dev)
    j = torch.empty(count, dtype=torch.int64, device=dev)
    f = torch.full((count,), 255, dtype=torch.uint8, device=dev)  # 255 marks a term never recorded
    check(lib().pgsgd_sample_terms(g.handle, ctypes.byref(p), int(iter), int(t_begin), int(count),
                                   ctypes.c_void_p(i.data_ptr()), ctypes.c_void_p(j.data_ptr()),
                                   ctypes.c_void_p(f.data_ptr()), _stream(torch, dev)))
    return i, j, f


def sample_terms_reuse(g: Graph, iter: int, t_begin: int, count: int, params: LayoutParams | None = None, **kw):
    """The data-reuse variant's terms (i, j, flags) and reuse offsets (uint8,
    reuse_factor - 1 per 64-term group with the plain schedule, per slot with
    the windowed one), recorded by its kernel."""
    p = _params(params, kw)
    dev = f"cuda:{g.device}"
    i = torch.empty(count, dtype=torch.int64, device=dev)
    j = torch.empty(count, dtype=torch.int64, device=dev)
    f = torch.full((count,), 255, dtype=torch.uint8, device=dev)
    n_groups = (t_begin + count + 63) // 64 - t_begin // 64
    per = max(0, p.reuse_factor - 1)
    windowed = p.schedule in (SCHEDULE_AUTO, SCHEDULE_WINDOWED)
    o = torch.zeros(max(1, (count if windowed else n_groups) * per), dtype=torch.uint8, device=dev)
    check(lib().pgsgd_sample_terms_reuse(g.handle, ctypes.byref(p), int(iter), int(t_begin), int(count),
                                         ctypes.c_void_p(i.data_ptr()), ctypes.c_void_p(j.data_ptr()),
                                         ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(o.data_ptr()),
                                         _stream(torch, dev)))
    return i, j, f, o


def apply_terms(g: Graph, coords, eta: float, i, j, f):
    import torch
    _check_tensor(coords, torch.float32, 4 * g.n_nodes, "coords")
    _check_tensor(i, torch.int64, None, "i")
    _check_tensor(j, torch.int64, i.numel(), "j")
    _check_tensor(f, torch.uint8, i.numel(), "flags")
    check(lib().pgsgd_apply_terms(g.handle, float(eta), ctypes.c_void_p(i.data_ptr()), ctypes.c_void_p(j.data_ptr()),
                                  ctypes.c_void_p(f.data_ptr()), int(i.numel()), ctypes.c_void_p(coords.data_ptr()),
                                  _stream(torch, coords.device)))
    return coords


def apply_slots(g: Graph, coords, iter: int, t_begin: int, mask, params: LayoutParams | None = None, **kw):
    """Iteration `iter` of layout() with its own kernels and launch shape, applying only the terms
    (windowed: slots) t_begin + k with mask[k] != 0 (mask: uint8 device tensor)."""
    import torch
    _check_tensor(coords, torch.float32, 4 * g.n_nodes, "coords")
    _check_tensor(mask, torch.uint8, None, "mask")
    p = _params(params, kw)
    check(lib().pgsgd_apply_slots(g.handle, ctypes.byref(p), int(iter), int(t_begin), int(mask.numel()),
                                  ctypes.c_void_p(mask.data_ptr()), ctypes.c_void_p(coords.data_ptr()),
                                  _stream(torch, coords.device)))
    return coords


# ---------------------------------------------------------------------------
# Differentiable form
# ---------------------------------------------------------------------------
def stress_forward(g: Graph, coords, n_pairs: int, step: int = 0, params: LayoutParams | None = None, **kw):
    """Returns (loss float32 device scalar, n_valid int64 device scalar)."""
    import torch
    _check_tensor(coords, torch.float32, 4 * g.n_nodes, "coords")
    p = _params(params, kw)
    loss = torch.empty(1, dtype=torch.float32, device=coords.device)
    nv = torch.empty(1, dtype=torch.int64, device=coords.device)
    check(lib().pgsgd_stress_forward(g.handle, ctypes.byref(p), ctypes.c_void_p(coords.data_ptr()), int(n_pairs),
                                     int(step), ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(nv.data_ptr()),
                                     _stream(torch, coords.device)))
    return loss, nv


def stress_backward(g: Graph, coords, n_pairs: int, step: int, grad_out, n_valid, grad_coords,
                    params: LayoutParams | None = None, **kw):
    """Adds grad_out * dL/dcoords into grad_coords."""
    import torch
    _check_tensor(coords, torch.float32, 4 * g.n_nodes, "coords")
    _check_tensor(grad_coords, torch.float32, 4 * g.n_nodes, "grad_coords")
    _check_tensor(grad_out, torch.float32, 1, "grad_out")
    _check_tensor(n_valid, torch.int64, 1, "n_valid")
    p = _params(params, kw)
    check(lib().pgsgd_stress_backward(g.handle, ctypes.byref(p), ctypes.c_void_p(coords.data_ptr()), int(n_pairs),
                                      int(step), ctypes.c_void_p(grad_out.data_ptr()),
                                      ctypes.c_void_p(n_valid.data_ptr()), ctypes.c_void_p(grad_coords.data_ptr()),
                                      _stream(torch, coords.device)))
    return grad_coords


class SampledPathStress(torch.autograd.Function):
    """Sampled stress over power-law pairs as a differentiable loss.

    ``SampledPathStress.apply(coords, graph, n_pairs, step, params)`` returns a
    scalar loss.  The backward regenerates the same pairs from their Philox
    counters (no pair buffer) and scatters the adjoint with float32 atomics.
    """

    @staticmethod
    def forward(ctx, coords, graph, n_pairs, step, params=None):
        loss, nv = stress_forward(graph, coords.detach(), n_pairs, step, params)
        ctx.save_for_backward(coords.detach(), nv)
        ctx.graph, ctx.n_pairs, ctx.step, ctx.params = graph, n_pairs, step, params
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        coords, nv = ctx.saved_tensors
        grad = torch.zeros_like(coords)
        go = grad_out.reshape(1).to(torch.float32).contiguous()
        stress_backward(ctx.graph, coords, ctx.n_pairs, ctx.step, go, nv, grad, ctx.params)
        return grad, None, None, None, None


def adam_step(x, grad, m, v, t: int, lr: float = 1.0, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step in place on x (all float32 device tensors of the same size)."""
    import torch
    n = x.numel()
    for name, tt in (("x", x), ("grad", grad), ("m", m), ("v", v)):
        _check_tensor(tt, torch.float32, n, name)
    check(lib().pgsgd_adam_step(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                                ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), n, float(lr),
                                float(beta1), float(beta2), float(eps), int(t), _stream(torch, x.device)))
    return x


# ---------------------------------------------------------------------------
# Batched form
# ---------------------------------------------------------------------------
def _tune_c(tune) -> Tune | None:
    if tune is None:
        return None
    if isinstance(tune, Tune):
        return tune
    return Tune(int(tune["block_threads"]), int(tune["groups_per_item"]), int(tune["blocks_per_cu"]),
                int(tune.get("max_blocks", 0)), int(tune.get("phases", 1)), int(tune.get("branches", 0)))


def _graph_arrays(graphs, coords_list):
    import torch
    if len(graphs) != len(coords_list) or not graphs:
        raise ValueError("need one coords tensor per graph")
    for g, c in zip(graphs, coords_list):
        _check_tensor(c, torch.float32, 4 * g.n_nodes, "coords")
    gh = (ctypes.c_void_p * len(graphs))(*[g.handle.value for g in graphs])
    ch = (ctypes.c_void_p * len(graphs))(*[c.data_ptr() for c in coords_list])
    return gh, ch


class Batch:
    """Many graphs laid out together: one persistent launch per iteration, the
    iterations captured in one HIP graph.  Graph k uses graph_id = params.graph_id + k."""

    def __init__(self, graphs, coords_list, params: LayoutParams | None = None, tune=None, **kw):
        gh, ch = _graph_arrays(graphs, coords_list)
        p = _params(params, kw)
        t = _tune_c(tune)
        h = ctypes.c_void_p()
        check(lib().pgsgd_batch_create(gh, len(graphs), ctypes.byref(p), ch,
                                       ctypes.byref(t) if t is not None else None, ctypes.byref(h)))
        self._h = h
        self.graphs, self.coords = list(graphs), list(coords_list)
        self.device = graphs[0].device

    def run(self):
        import torch
        check(lib().pgsgd_batch_run(self._h, _stream(torch, f"cuda:{self.device}")))

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            lib().pgsgd_batch_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def layout_batched(graphs, coords_list, params: LayoutParams | None = None, tune=None, **kw):
    import torch
    gh, ch = _graph_arrays(graphs, coords_list)
    p = _params(params, kw)
    t = _tune_c(tune)
    check(lib().pgsgd_layout_batched(gh, len(graphs), ctypes.byref(p), ch,
                                     ctypes.byref(t) if t is not None else None,
                                     _stream(torch, f"cuda:{graphs[0].device}")))


def batch_sample_terms(graphs, iter: int, params: LayoutParams | None = None, tune=None, **kw):
    """The terms the batched kernel samples in iteration ``iter``, per graph: a
    list of (i, j, flags) device tensors of length terms_per_step * S_k."""
    p = _params(params, kw)
    dev = f"cuda:{graphs[0].device}"
    outs = []
    for g in graphs:
        T = p.terms_per_step * g.n_steps
        outs.append((torch.empty(T, dtype=torch.int64, device=dev), torch.empty(T, dtype=torch.int64, device=dev),
                     torch.empty(T, dtype=torch.uint8, device=dev)))
    n = len(graphs)
    gh = (ctypes.c_void_p * n)(*[g.handle.value for g in graphs])
    ih = (ctypes.c_void_p * n)(*[o[0].data_ptr() for o in outs])
    jh = (ctypes.c_void_p * n)(*[o[1].data_ptr() for o in outs])
    fh = (ctypes.c_void_p * n)(*[o[2].data_ptr() for o in outs])
    t = _tune_c(tune)
    check(lib().pgsgd_batch_sample_terms(gh, n, ctypes.byref(p), int(iter), ctypes.byref(t) if t is not None else None,
                                         ih, jh, fh, _stream(torch, dev)))
    return outs


def _tune_cache_path() -> str:
    return os.environ.get("PGSGD_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "pgsgd_tune.json"))


def autotune(graphs, coords_list, params: LayoutParams | None = None, use_cache: bool = True, max_blocks: int = 0,
             **kw) -> dict:
    """Picks block shape and work per wave for a batch by timing candidates
    (native tuner); results are cached per workload signature in a JSON file
    (PGSGD_TUNE_CACHE)."""
    import torch
    p = _params(params, kw)
    sig = "|".join([torch.cuda.get_device_name(graphs[0].device), str(len(graphs)),
                    str(sum(g.n_steps for g in graphs)), str(max(g.n_paths for g in graphs)),
                    str(p.terms_per_step), str(p.zipf_window), str(max_blocks), str(p.schedule)])
    path = _tune_cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        if sig in cache:
            return dict(cache[sig], cached=True)
    gh, ch = _graph_arrays(graphs, coords_list)
    best = Tune(0, 0, 0, int(max_blocks), 1, 0)
    ms = ctypes.c_float()
    check(lib().pgsgd_autotune_batched(gh, len(graphs), ctypes.byref(p), ch, ctypes.byref(best), ctypes.byref(ms),
                                       _stream(torch, f"cuda:{graphs[0].device}")))
    res = {"block_threads": best.block_threads, "groups_per_item": best.groups_per_item,
           "blocks_per_cu": best.blocks_per_cu, "max_blocks": best.max_blocks, "phases": best.phases,
           "branches": best.branches,
           "ms": ms.value}
    if use_cache:
        cache[sig] = res
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return dict(res, cached=False)
