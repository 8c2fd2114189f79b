"""Seeded synthetic variation graphs: the inputs shared by the oracle and the GPU library.

This module only produces input data (node lengths, path step lists, initial
random coordinates); it contains none of the layout method's arithmetic.  The
generator itself is C (``synth.c``) for speed at chromosome scale; this file
loads it with ctypes and names the workload configurations.

The graph model stands in for the HPRC human chromosome graphs the paper
evaluates on (Section "Experiment Setup", Table "Properties of the human
pangenome graphs"), which are not available: a backbone chain with geometric
node lengths walked by haplotype paths with SNP bubbles, skips and inversions.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
# PGSGD_SANITIZED=1 loads the AddressSanitizer/UndefinedBehaviorSanitizer build
SANITIZED = os.environ.get("PGSGD_SANITIZED") == "1"
_LIB_PATH = os.path.join(_HERE, "libsynth_san.so" if SANITIZED else "libsynth.so")
_lib = None
SAN_FLAGS = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]

REV_BIT = 0x80000000


def build(force: bool = True, sanitized: bool = None) -> str:
    """Compile ``libsynth.so`` (or, sanitized, ``libsynth_san.so``) with gcc (host code only)."""
    san = SANITIZED if sanitized is None else sanitized
    path = os.path.join(_HERE, "libsynth_san.so" if san else "libsynth.so")
    if force or not os.path.exists(path):
        opt = SAN_FLAGS if san else ["-O2"]
        subprocess.check_call(["gcc", *opt, "-fPIC", "-shared", "-std=c11", "-Wall", "-o", path, _SRC])
    return path


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        p = ctypes.c_void_p
        lib.synth_generate.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint64,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_uint32,
                                       p, p, p, p, p, p]
        lib.synth_generate.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class SynthGraph:
    """A variation graph as plain arrays (the boundary's input form).

    node_len  : uint32[n_nodes], every entry >= 1
    path_off  : uint64[n_paths+1], CSR offsets into step_node
    step_node : uint32[S], node id with bit 31 set for a reverse-strand visit
    """
    node_len: np.ndarray
    path_off: np.ndarray
    step_node: np.ndarray
    stats: dict = field(default_factory=dict)
    name: str = ""

    @property
    def n_nodes(self) -> int:
        return int(self.node_len.shape[0])

    @property
    def n_paths(self) -> int:
        return int(self.path_off.shape[0]) - 1

    @property
    def n_steps(self) -> int:
        return int(self.path_off[-1])


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def generate(backbone: int, p_len: float, n_paths: int, seed: int, p_snp: float = 0.05,
             p_skip: float = 0.01, p_inv: float = 0.002, max_run: int = 20, name: str = "") -> SynthGraph:
    """Generate one synthetic graph; a pure function of its arguments."""
    lib = _load()
    backbone = int(backbone)
    node_len = np.empty(2 * backbone, dtype=np.uint32)
    path_off = np.empty(n_paths + 1, dtype=np.uint64)
    step_node = np.empty(max(1, n_paths * backbone), dtype=np.uint32)
    n_nodes = np.zeros(1, dtype=np.uint64)
    n_steps = np.zeros(1, dtype=np.uint64)
    stats = np.zeros(4, dtype=np.uint64)
    rc = lib.synth_generate(backbone, float(p_len), int(n_paths), int(seed), float(p_snp), float(p_skip),
                            float(p_inv), int(max_run), _ptr(node_len), _ptr(path_off), _ptr(step_node),
                            _ptr(n_nodes), _ptr(n_steps), _ptr(stats))
    if rc != 0:
        raise ValueError(f"synth_generate failed with code {rc}")
    nn, ns = int(n_nodes[0]), int(n_steps[0])
    node_len = np.ascontiguousarray(node_len[:nn])
    # keep the over-allocated buffer only when the tail is small; otherwise copy to free it
    step_node = step_node[:ns] if ns * 10 >= step_node.shape[0] * 9 else np.ascontiguousarray(step_node[:ns])
    st = {"snp_visits": int(stats[0]), "reverse_visits": int(stats[1]), "skipped_positions": int(stats[2]),
          "alt_nodes": int(stats[3]), "backbone": backbone, "n_nodes": nn, "n_steps": ns, "n_paths": n_paths}
    return SynthGraph(node_len, path_off, step_node, st, name)


# Workload configurations (the graph part; the layout parameters live with the callers).
CONFIGS = {
    # 2,000-node backbone, lengths 1+Geometric(0.2), 8 paths
    "tiny": dict(backbone=2000, p_len=0.2, n_paths=8, seed=1),
    # 1M-node backbone, same model, 32 paths
    "mid": dict(backbone=1_000_000, p_len=0.2, n_paths=32, seed=2),
    # 5M-node backbone, lengths 1+Geometric(0.05), 90 paths
    "chromosome": dict(backbone=5_000_000, p_len=0.05, n_paths=90, seed=3),
}


def config_graph(name: str) -> SynthGraph:
    return generate(name=name, **CONFIGS[name])


def batched_backbones(n_graphs: int = 24, lo: float = 2e5, hi: float = 5e6, seed: int = 999) -> list:
    """Backbone sizes log-uniform in [lo, hi] for the batched workload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(n_graphs)
    return [int(round(math.exp(math.log(lo) + x * (math.log(hi) - math.log(lo))))) for x in u]


def batched_graphs(n_graphs: int = 24, scale: float = 1.0, seed_base: int = 1000) -> list:
    """The uneven chromosome-like graphs of the batched workload (90 paths each,
    lengths 1+Geometric(0.05)); ``scale`` shrinks every backbone for tests."""
    sizes = batched_backbones(n_graphs)
    return [generate(max(2, int(b * scale)), 0.05, 90, seed_base + g, name=f"batched{g}")
            for g, b in enumerate(sizes)]


def linear_path(n_nodes: int, p_len: float = 0.2, seed: int = 0) -> SynthGraph:
    """One forward path through n_nodes nodes in id order (no variation)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    node_len = rng.geometric(p_len, size=n_nodes).astype(np.uint32)  # support 1.., mean 1/p
    path_off = np.array([0, n_nodes], dtype=np.uint64)
    step_node = np.arange(n_nodes, dtype=np.uint32)
    return SynthGraph(node_len, path_off, step_node, {"n_nodes": n_nodes}, "linear")


def random_coords(n_nodes: int, seed: int, scale: float) -> np.ndarray:
    """Random float32 coordinates in the boundary layout [2][n_nodes][2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.random((2, n_nodes, 2)) * scale).astype(np.float32)


def write_gfa(sg: SynthGraph, path: str, walks: bool = False, names: str = "numeric", sequence: bool = False,
              path_prefix: str = "hap") -> None:
    """Writes a graph as GFA 1.x text: one S line per node in id order (so the
    k-th S line is node k again when read back), then one P line per path, or
    one W line per path when ``walks`` (GFA 1.1).  ``names``: "numeric" gives
    segment k the name k+1, "text" the name "s<k>".  ``sequence`` writes a
    sequence of the node's length instead of '*' with an LN tag.  Output
    formatting only."""
    def seg(k: int) -> str:
        return str(k + 1) if names == "numeric" else f"s{k}"

    with open(path, "w") as f:
        f.write("H\tVN:Z:1.1\n" if walks else "H\tVN:Z:1.0\n")
        for k, ln in enumerate(sg.node_len.tolist()):
            if sequence:
                f.write(f"S\t{seg(k)}\t{'ACGT' * (ln // 4)}{'ACGT'[:ln % 4]}\n")
            else:
                f.write(f"S\t{seg(k)}\t*\tLN:i:{ln}\n")
        off = sg.path_off.tolist()
        steps = sg.step_node
        for p in range(sg.n_paths):
            s = steps[off[p]:off[p + 1]].tolist()
            if walks:
                body = "".join(("<" if v & REV_BIT else ">") + seg(v & (REV_BIT - 1)) for v in s) or "*"
                f.write(f"W\t{path_prefix}{p}\t0\tchr\t*\t*\t{body}\n")
            else:
                body = ",".join(seg(v & (REV_BIT - 1)) + ("-" if v & REV_BIT else "+") for v in s) or "*"
                f.write(f"P\t{path_prefix}{p}\t{body}\t*\n")
