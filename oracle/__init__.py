"""CPU oracle for PG-SGD layout — TEST INFRASTRUCTURE ONLY.

Plain single-threaded C (``oracle.c``, built with gcc into ``liboracle.so``)
written from the paper: the layout loop of Alg. 1, the path stress of Eq. 1
and the sampled path stress of Eq. 2 with its 95% confidence interval.  It
shares no code with the GPU library.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does.

Every function states the passage it follows; see ``oracle.c`` for the
readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# PGSGD_SANITIZED=1 loads the AddressSanitizer/UndefinedBehaviorSanitizer
# build (tests run it in a child process with the sanitizer runtimes preloaded)
SANITIZED = os.environ.get("PGSGD_SANITIZED") == "1"
_LIB_PATH = os.path.join(_HERE, "liboracle_san.so" if SANITIZED else "liboracle.so")
_lib = None
SAN_FLAGS = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]

# Compiled without FMA contraction or fast-math so each FP64 expression is
# evaluated exactly as written.
CFLAGS = ["-O2", "-fPIC", "-shared", "-std=gnu11", "-Wall", "-ffp-contract=off", "-fno-fast-math", "-pthread"]


def build(force: bool = True, sanitized: bool = None) -> str:
    """Compiles liboracle.so (or, sanitized, liboracle_san.so) with gcc."""
    san = SANITIZED if sanitized is None else sanitized
    path = os.path.join(_HERE, "liboracle_san.so" if san else "liboracle.so")
    if force or not os.path.exists(path):
        flags = [f for f in CFLAGS if f != "-O2"] + SAN_FLAGS if san else CFLAGS
        subprocess.check_call(["gcc", *flags, "-o", path, _SRC, "-lm"])
    return path


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    u32, u64, f64, f32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_float
    sig = {
        "or_philox4x32_10": ([P, P, P], None),
        "or_zipf_table": ([f64, u32, P], None),
        "or_zipf_draw": ([P, u32, u32], u32),
        "or_schedule": ([u32, f64, f64, P], None),
        "or_graph_new": ([u32, P, u32, P, P], P),
        "or_graph_free": ([P], None),
        "or_graph_pos": ([P], P),
        "or_graph_path_nt": ([P], P),
        "or_graph_d_max": ([P], ctypes.c_int64),
        "or_endpoint_pos": ([P, u64, u32], ctypes.c_int64),
        "or_sample_terms": ([P, u32, f64, u32, u64, u32, u32, u64, u64, P, P, P], None),
        "or_layout": ([P, u32, u32, f64, f64, f64, u32, u64, u32, u32, u32, P], u64),
        "or_layout_threaded": ([P, u32, u32, f64, f64, f64, u32, u64, u32, u32, u32, P, u32, u64], u64),
        "or_apply_terms_f64": ([P, f64, P, P, P, u64, P], u64),
        "or_sample_terms_reuse": ([P, u32, f64, u32, u64, u32, u32, u64, u64, P, P, P], None),
        "or_reuse_offsets": ([u64, u32, u32, u64, u32, P], None),
        "or_layout_reuse": ([P, u32, u32, u32, u32, f64, f64, f64, u32, u64, u32, u32, u32, P], u64),
        "or_apply_terms_f32": ([P, f64, P, P, P, u64, P], u64),
        "or_apply_terms_f64_scaled": ([P, f64, f64, P, P, P, u64, P], u64),
        "or_sampled_path_stress_threaded": ([P, P, u32, u64, u32, u32, u32, P, P], None),
        "or_window_shift": ([u64], u32),
        "or_window_counts": ([P, u64, u32, u32, u64, P, u32], None),
        "or_sample_terms_windowed": ([P, u32, f64, u32, u64, u32, u32, P, u64, u64, P, P, P], None),
        "or_layout_windowed": ([P, u32, u32, u32, u32, f64, f64, f64, u32, u64, u32, u32, u32, P], u64),
        "or_sampled_path_stress": ([P, P, u32, u64, u32, P, P], None),
        "or_sampled_path_stress_pairs": ([P, P, u32, u64, u32, u32, f64, u32, P, P], None),
        "or_sps_segments": ([P, P, P], u64),
        "or_loss_shift": ([u64], u32),
        "or_loss_segments": ([P, P, P], u64),
        "or_sps_segment_counts": ([P, u32, u64, u32, P, u64, P], None),
        "or_sps_windowed_pairs": ([P, u32, u64, u32, u64, u64, P, P, P], None),
        "or_sampled_path_stress_windowed": ([P, P, u32, u64, u32, P, P], None),
        "or_sps_expectation": ([P, P, P], None),
        "or_path_stress_exact": ([P, P, P], None),
        "or_init_coords": ([P, u64, u32, f32, P], None),
        "or_stress_loss_grad": ([P, P, u64, f64, u32, u64, u32, u32, P, P], None),
        "or_loss_segment_counts": ([P, u64, u64, u32, u32, P, u64, P], None),
        "or_sps_outliers": ([P, P, u32, u64, u32, u32, f64, u32, f64, u64, P, P, P, P], u64),
        "or_sps_compare": ([P, P, P, u32, u64, u32, u32, f64, u32, P, P], None),
        "or_loss_windowed_pairs": ([P, u64, f64, u32, u64, u32, u32, u64, u64, P, P, P], None),
        "or_stress_loss_grad_windowed": ([P, P, u64, f64, u32, u64, u32, u32, P, P], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


# ---------------------------------------------------------------------------
# Counter-based random numbers (Philox4x32-10, Salmon et al. SC'11)
# ---------------------------------------------------------------------------
def philox(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def zipf_table(theta: float = 0.99, window: int = 1000) -> np.ndarray:
    C = np.zeros(window + 1, dtype=np.uint32)
    _load().or_zipf_table(float(theta), int(window), _p(C))
    return C


def zipf_draw(C: np.ndarray, n: int, r: int) -> int:
    C = np.ascontiguousarray(C, dtype=np.uint32)
    return int(_load().or_zipf_draw(_p(C), int(n), int(r)))


def schedule(n_iters: int, eta_max: float, eta_min: float = 0.01) -> np.ndarray:
    eta = np.zeros(max(1, n_iters), dtype=np.float64)
    _load().or_schedule(int(n_iters), float(eta_max), float(eta_min), _p(eta))
    return eta[:n_iters]


# ---------------------------------------------------------------------------
# Graph + layout (Alg. 1)
# ---------------------------------------------------------------------------
class Graph:
    """Oracle view of a variation graph: node lengths and path step lists."""

    def __init__(self, node_len, path_off, step_node):
        self.node_len = np.ascontiguousarray(node_len, dtype=np.uint32)
        self.path_off = np.ascontiguousarray(path_off, dtype=np.uint64)
        self.step_node = np.ascontiguousarray(step_node, dtype=np.uint32)
        self.n_nodes = int(self.node_len.shape[0])
        self.n_paths = int(self.path_off.shape[0]) - 1
        self.S = int(self.path_off[-1])
        self._h = _load().or_graph_new(self.n_nodes, _p(self.node_len), self.n_paths, _p(self.path_off),
                                       _p(self.step_node))

    @classmethod
    def from_synth(cls, sg):
        return cls(sg.node_len, sg.path_off, sg.step_node)

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _lib is not None:
            _lib.or_graph_free(h)

    @property
    def pos(self) -> np.ndarray:
        addr = _load().or_graph_pos(self._h)
        return np.ctypeslib.as_array(ctypes.cast(addr, ctypes.POINTER(ctypes.c_int64)), shape=(max(1, self.S),))[
            : self.S].copy()

    @property
    def path_nt(self) -> np.ndarray:
        addr = _load().or_graph_path_nt(self._h)
        return np.ctypeslib.as_array(ctypes.cast(addr, ctypes.POINTER(ctypes.c_int64)),
                                     shape=(max(1, self.n_paths),))[: self.n_paths].copy()

    @property
    def d_max(self) -> int:
        return int(_load().or_graph_d_max(self._h))

    def endpoint_pos(self, s: int, e: int) -> int:
        return int(_load().or_endpoint_pos(self._h, int(s), int(e)))


DEFAULTS = dict(n_iters=30, terms_per_step=10, eta_max=0.0, eta_min=0.01, theta=0.99, window=1000, seed=24301,
                graph_id=0)


def sample_terms(g: Graph, iter: int, t_begin: int, count: int, n_iters=30, theta=0.99, window=1000, seed=24301,
                 graph_id=0):
    i = np.zeros(count, dtype=np.uint64)
    j = np.zeros(count, dtype=np.uint64)
    f = np.zeros(count, dtype=np.uint8)
    _load().or_sample_terms(g._h, int(n_iters), float(theta), int(window), int(seed), int(graph_id), int(iter),
                            int(t_begin), int(count), _p(i), _p(j), _p(f))
    return i, j, f


def layout(g: Graph, coords: np.ndarray, n_iters=30, terms_per_step=10, eta_max=0.0, eta_min=0.01, theta=0.99,
           window=1000, seed=24301, graph_id=0, first_iter=0, last_iter=0, threads=1, term_limit=0) -> int:
    """Runs Alg. 1 in place on float32 coords [2][n_nodes][2]; returns applied updates."""
    assert coords.dtype == np.float32 and coords.flags.c_contiguous and coords.size == 4 * g.n_nodes
    L = _load()
    if threads <= 1 and term_limit == 0:
        return int(L.or_layout(g._h, int(n_iters), int(terms_per_step), float(eta_max), float(eta_min),
                               float(theta), int(window), int(seed), int(graph_id), int(first_iter),
                               int(last_iter), _p(coords)))
    return int(L.or_layout_threaded(g._h, int(n_iters), int(terms_per_step), float(eta_max), float(eta_min),
                                    float(theta), int(window), int(seed), int(graph_id), int(first_iter),
                                    int(last_iter), _p(coords), int(threads), int(term_limit)))


def sample_terms_reuse(g: Graph, iter: int, t_begin: int, count: int, n_iters=30, theta=0.99, window=1000,
                       seed=24301, graph_id=0):
    """Terms of the data-reuse variant: group-shared paths (see oracle.c)."""
    i = np.zeros(count, dtype=np.uint64)
    j = np.zeros(count, dtype=np.uint64)
    f = np.zeros(count, dtype=np.uint8)
    _load().or_sample_terms_reuse(g._h, int(n_iters), float(theta), int(window), int(seed), int(graph_id),
                                  int(iter), int(t_begin), int(count), _p(i), _p(j), _p(f))
    return i, j, f


def reuse_offsets(iter: int, group: int, drf: int, seed=24301, graph_id=0) -> list:
    o = np.zeros(17, dtype=np.uint32)
    _load().or_reuse_offsets(int(seed), int(graph_id), int(iter), int(group), int(drf), _p(o))
    return [int(x) for x in o[1:drf]]


def layout_reuse(g: Graph, coords: np.ndarray, drf: int, srf: int, n_iters=30, terms_per_step=10, eta_max=0.0,
                 eta_min=0.01, theta=0.99, window=1000, seed=24301, graph_id=0, first_iter=0, last_iter=0) -> int:
    """The data-reuse variant of the layout loop, sequentially (see oracle.c)."""
    assert coords.dtype == np.float32 and coords.flags.c_contiguous and coords.size == 4 * g.n_nodes
    return int(_load().or_layout_reuse(g._h, int(n_iters), int(terms_per_step), int(drf), int(srf), float(eta_max),
                                       float(eta_min), float(theta), int(window), int(seed), int(graph_id),
                                       int(first_iter), int(last_iter), _p(coords)))


def window_shift(S: int) -> int:
    """log2 of the window length of the window-major enumeration (reading R18)."""
    return int(_load().or_window_shift(int(S)))


def window_slots(g: Graph, terms_per_step=10, step_reduction=1) -> int:
    """Slots of an iteration: ceil(terms_per_step * S / step_reduction)."""
    return (terms_per_step * g.S + step_reduction - 1) // step_reduction


def window_counts(g: Graph, iter: int, terms_per_step=10, seed=24301, graph_id=0, threads=1,
                  step_reduction=1) -> np.ndarray:
    """Slots of iteration `iter` per window: the plain step draws t < window_slots()
    counted by window (`threads` host threads count disjoint term ranges; the sum is exact)."""
    sh = window_shift(g.S)
    c = np.zeros((g.S + (1 << sh) - 1) >> sh, dtype=np.uint64)
    _load().or_window_counts(g._h, int(seed), int(graph_id), int(iter),
                             int(window_slots(g, terms_per_step, step_reduction)), _p(c), int(threads))
    return c


def window_offsets(g: Graph, iter: int, terms_per_step=10, seed=24301, graph_id=0, threads=1,
                   step_reduction=1) -> np.ndarray:
    """First slot of every window (and the slot count at the end)."""
    c = window_counts(g, iter, terms_per_step, seed, graph_id, threads, step_reduction)
    return np.concatenate([np.zeros(1, np.uint64), np.cumsum(c, dtype=np.uint64)])


def sample_terms_windowed(g: Graph, iter: int, s_begin: int, count: int, n_iters=30, terms_per_step=10, theta=0.99,
                          window=1000, seed=24301, graph_id=0, offsets=None, threads=1, step_reduction=1):
    """Terms of the window-major enumeration, slots [s_begin, s_begin + count) (below the slot
    count); `offsets` from window_offsets() for the same iteration, computed here if absent."""
    if offsets is None:
        offsets = window_offsets(g, iter, terms_per_step, seed, graph_id, threads, step_reduction)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    assert s_begin + count <= int(offsets[-1])
    i = np.zeros(count, dtype=np.uint64)
    j = np.zeros(count, dtype=np.uint64)
    f = np.zeros(count, dtype=np.uint8)
    _load().or_sample_terms_windowed(g._h, int(n_iters), float(theta), int(window), int(seed), int(graph_id),
                                     int(iter), _p(offsets), int(s_begin), int(count), _p(i), _p(j), _p(f))
    return i, j, f


def layout_windowed(g: Graph, coords: np.ndarray, n_iters=30, terms_per_step=10, eta_max=0.0, eta_min=0.01,
                    theta=0.99, window=1000, seed=24301, graph_id=0, first_iter=0, last_iter=0, reuse_factor=1,
                    step_reduction=1) -> int:
    """The layout loop with the window-major enumeration, sequentially (with
    reuse_factor > 1 or step_reduction > 1: the data-reuse variant on it)."""
    assert coords.dtype == np.float32 and coords.flags.c_contiguous and coords.size == 4 * g.n_nodes
    return int(_load().or_layout_windowed(g._h, int(n_iters), int(terms_per_step), int(reuse_factor),
                                          int(step_reduction), float(eta_max), float(eta_min), float(theta),
                                          int(window), int(seed), int(graph_id), int(first_iter), int(last_iter),
                                          _p(coords)))


def apply_terms_f64(g: Graph, eta: float, i, j, flags, coords64: np.ndarray) -> int:
    assert coords64.dtype == np.float64 and coords64.flags.c_contiguous
    i = np.ascontiguousarray(i, dtype=np.uint64)
    j = np.ascontiguousarray(j, dtype=np.uint64)
    flags = np.ascontiguousarray(flags, dtype=np.uint8)
    return int(_load().or_apply_terms_f64(g._h, float(eta), _p(i), _p(j), _p(flags), len(i), _p(coords64)))


def apply_terms_f64_scaled(g: Graph, eta: float, r_scale: float, i, j, flags, coords64: np.ndarray) -> int:
    """apply_terms_f64 with every update's r multiplied by r_scale: a planted error, used only to
    measure the resolution of the batch check."""
    assert coords64.dtype == np.float64 and coords64.flags.c_contiguous
    i = np.ascontiguousarray(i, dtype=np.uint64)
    j = np.ascontiguousarray(j, dtype=np.uint64)
    flags = np.ascontiguousarray(flags, dtype=np.uint8)
    return int(_load().or_apply_terms_f64_scaled(g._h, float(eta), float(r_scale), _p(i), _p(j), _p(flags), len(i),
                                                 _p(coords64)))


def apply_terms_f32(g: Graph, eta: float, i, j, flags, coords: np.ndarray) -> int:
    assert coords.dtype == np.float32 and coords.flags.c_contiguous
    i = np.ascontiguousarray(i, dtype=np.uint64)
    j = np.ascontiguousarray(j, dtype=np.uint64)
    flags = np.ascontiguousarray(flags, dtype=np.uint8)
    return int(_load().or_apply_terms_f32(g._h, float(eta), _p(i), _p(j), _p(flags), len(i), _p(coords)))


# ---------------------------------------------------------------------------
# Metrics (Eq. 1, Eq. 2)
# ---------------------------------------------------------------------------
def sampled_path_stress(g: Graph, coords: np.ndarray, m: int = 100, seed: int = 7, graph_id: int = 0,
                        pairs: str = "uniform", theta: float = 0.99, window: int = 1000, threads: int = 1) -> dict:
    """Eq. 2 with its CI95; pairs="power_law" takes the cooling phase's partner (reading R19),
    pairs="uniform_windowed" lists the uniform pairs' law window-major (reading R21).  threads > 1
    evaluates the uniform orders on that many host threads (the same pairs; sums in another order)."""
    coords = np.ascontiguousarray(coords, dtype=np.float32)
    out = np.zeros(6, dtype=np.float64)
    cnt = np.zeros(2, dtype=np.uint64)
    if threads > 1 and pairs in ("uniform", "uniform_windowed"):
        _load().or_sampled_path_stress_threaded(g._h, _p(coords), int(m), int(seed), int(graph_id),
                                                0 if pairs == "uniform" else 1, int(threads), _p(out), _p(cnt))
    elif pairs == "uniform":
        _load().or_sampled_path_stress(g._h, _p(coords), int(m), int(seed), int(graph_id), _p(out), _p(cnt))
    elif pairs == "power_law":
        _load().or_sampled_path_stress_pairs(g._h, _p(coords), int(m), int(seed), int(graph_id), 1, float(theta),
                                             int(window), _p(out), _p(cnt))
    elif pairs == "uniform_windowed":
        _load().or_sampled_path_stress_windowed(g._h, _p(coords), int(m), int(seed), int(graph_id), _p(out), _p(cnt))
    else:
        raise ValueError("pairs must be 'uniform', 'power_law' or 'uniform_windowed'")
    return dict(mean=out[0], ci_lo=out[1], ci_hi=out[2], stddev=out[3], sum=out[4], sumsq_dev=out[5],
                n_valid=int(cnt[0]), n_skipped=int(cnt[1]))


def sps_segments(g: Graph):
    """Segments of the window-major SPS order (reading R21): (start[n + 1], path[n])."""
    n = int(_load().or_sps_segments(g._h, None, None))
    start = np.zeros(n + 1, dtype=np.uint64)
    path = np.zeros(max(1, n), dtype=np.uint32)
    _load().or_sps_segments(g._h, _p(start), _p(path))
    return start, path[:n]


def sps_segment_counts(g: Graph, m: int = 100, seed: int = 7, graph_id: int = 0) -> np.ndarray:
    start, _ = sps_segments(g)
    n = len(start) - 1
    out = np.zeros(max(1, n), dtype=np.uint64)
    _load().or_sps_segment_counts(g._h, int(m), int(seed), int(graph_id), _p(start), n, _p(out))
    return out[:n]


def sps_windowed_pairs(g: Graph, m: int = 100, seed: int = 7, graph_id: int = 0, u_begin: int = 0, count=None):
    """Pairs of slots [u_begin, u_begin + count) of the window-major SPS order: (i, j, e_i | e_j << 1)."""
    if count is None:
        count = m * g.S - u_begin
    i = np.zeros(max(1, count), dtype=np.uint64)
    j = np.zeros(max(1, count), dtype=np.uint64)
    e = np.zeros(max(1, count), dtype=np.uint8)
    _load().or_sps_windowed_pairs(g._h, int(m), int(seed), int(graph_id), int(u_begin), int(count), _p(i), _p(j),
                                  _p(e))
    return i[:count], j[:count], e[:count]


def sps_expectation(g: Graph, coords: np.ndarray):
    coords = np.ascontiguousarray(coords, dtype=np.float32)
    out = np.zeros(2, dtype=np.float64)
    _load().or_sps_expectation(g._h, _p(coords), _p(out))
    return float(out[0]), float(out[1])


def path_stress_exact(g: Graph, coords: np.ndarray):
    coords = np.ascontiguousarray(coords, dtype=np.float32)
    out = np.zeros(2, dtype=np.float64)
    _load().or_path_stress_exact(g._h, _p(coords), _p(out))
    return float(out[0]), int(out[1])


def init_coords(g: Graph, seed: int = 5, jitter: float = 10.0, graph_id: int = 0) -> np.ndarray:
    coords = np.zeros(4 * g.n_nodes, dtype=np.float32)
    _load().or_init_coords(g._h, int(seed), int(graph_id), float(jitter), _p(coords))
    return coords


def stress_loss_grad(g: Graph, coords: np.ndarray, n_pairs: int, seed: int = 11, step: int = 0, theta=0.99,
                     window=1000, graph_id=0, want_grad=True):
    coords = np.ascontiguousarray(coords, dtype=np.float32)
    out = np.zeros(2, dtype=np.float64)
    grad = np.zeros(4 * g.n_nodes, dtype=np.float64) if want_grad else None
    _load().or_stress_loss_grad(g._h, _p(coords), int(n_pairs), float(theta), int(window), int(seed),
                                int(graph_id), int(step), _p(out), _p(grad))
    return float(out[0]), int(out[1]), grad


def loss_shift(S: int) -> int:
    """Window shift of the loss's segments (reading R22)."""
    return int(_load().or_loss_shift(int(S)))


def loss_segments(g: Graph):
    """Segments of the window-major loss pairs (reading R22): (start[n + 1], path[n])."""
    n = int(_load().or_loss_segments(g._h, None, None))
    start = np.zeros(n + 1, dtype=np.uint64)
    path = np.zeros(max(1, n), dtype=np.uint32)
    _load().or_loss_segments(g._h, _p(start), _p(path))
    return start, path[:n]


def loss_segment_counts(g: Graph, n_pairs: int, seed: int = 11, step: int = 0, graph_id: int = 0) -> np.ndarray:
    """Slots per segment of the window-major loss pairs (reading R22)."""
    start, _ = loss_segments(g)
    n = len(start) - 1
    out = np.zeros(max(1, n), dtype=np.uint64)
    _load().or_loss_segment_counts(g._h, int(n_pairs), int(seed), int(graph_id), int(step), _p(start), n, _p(out))
    return out[:n]


def loss_windowed_pairs(g: Graph, n_pairs: int, u_begin: int, count: int, seed: int = 11, step: int = 0,
                        theta=0.99, window=1000, graph_id=0):
    """Slots [u_begin, u_begin + count) of the window-major loss pairs: i, j,
    flags (e_i | e_j << 1 | skipped << 3)."""
    i = np.zeros(count, dtype=np.uint64)
    j = np.zeros(count, dtype=np.uint64)
    f = np.zeros(count, dtype=np.uint8)
    _load().or_loss_windowed_pairs(g._h, int(n_pairs), float(theta), int(window), int(seed), int(graph_id),
                                   int(step), int(u_begin), int(count), _p(i), _p(j), _p(f))
    return i, j, f


def stress_loss_grad_windowed(g: Graph, coords: np.ndarray, n_pairs: int, seed: int = 11, step: int = 0,
                              theta=0.99, window=1000, graph_id=0, want_grad=True):
    """The loss and its gradient over the window-major pairs (reading R22)."""
    coords = np.ascontiguousarray(coords, dtype=np.float32)
    out = np.zeros(2, dtype=np.float64)
    grad = np.zeros(4 * g.n_nodes, dtype=np.float64) if want_grad else None
    _load().or_stress_loss_grad_windowed(g._h, _p(coords), int(n_pairs), float(theta), int(window), int(seed),
                                         int(graph_id), int(step), _p(out), _p(grad))
    return float(out[0]), int(out[1]), grad


PAIR_MODES = {"uniform": 0, "power_law": 1, "uniform_windowed": 2}


def sps_outliers(g: Graph, coords: np.ndarray, m: int, threshold: float, max_out: int = 1 << 20, seed: int = 7,
                 graph_id: int = 0, pairs: str = "uniform", theta=0.99, window=1000):
    """The pairs of Eq. 2 (given order) with stress above threshold, in
    enumeration order: (count, i, j, e, stress) with the first max_out kept."""
    coords = np.ascontiguousarray(coords, dtype=np.float32)
    i = np.zeros(max_out, dtype=np.uint64)
    j = np.zeros(max_out, dtype=np.uint64)
    e = np.zeros(max_out, dtype=np.uint8)
    s = np.zeros(max_out, dtype=np.float64)
    n = int(_load().or_sps_outliers(g._h, _p(coords), int(m), int(seed), int(graph_id), PAIR_MODES[pairs],
                                    float(theta), int(window), float(threshold), int(max_out), _p(i), _p(j), _p(e),
                                    _p(s)))
    k = min(n, max_out)
    return n, i[:k], j[:k], e[:k], s[:k]


def sps_compare(g: Graph, coords_a: np.ndarray, coords_b: np.ndarray, m: int = 10, seed: int = 7, graph_id: int = 0,
                pairs: str = "uniform", theta=0.99, window=1000) -> dict:
    """Two layouts on the same pairs of Eq. 2: means, the ratio of the sums
    with its delta-method CI95, and the spreads (see oracle.c)."""
    a = np.ascontiguousarray(coords_a, dtype=np.float32)
    b = np.ascontiguousarray(coords_b, dtype=np.float32)
    out = np.zeros(10, dtype=np.float64)
    cnt = np.zeros(2, dtype=np.uint64)
    _load().or_sps_compare(g._h, _p(a), _p(b), int(m), int(seed), int(graph_id), PAIR_MODES[pairs], float(theta),
                           int(window), _p(out), _p(cnt))
    keys = ("mean_a", "mean_b", "ratio", "ratio_ci_lo", "ratio_ci_hi", "sd_a", "sd_b", "sd_diff", "sum_a", "sum_b")
    return {**dict(zip(keys, out.tolist())), "n_valid": int(cnt[0]), "n_skipped": int(cnt[1])}
