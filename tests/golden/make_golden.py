"""Writes stored oracle results for configurations too large to run inside a test.

Calls only the oracle (and the seeded input generator).  Each run lays out a
synthetic configuration from the oracle's initial layout with the given layout
seed and stores the final sampled path stress (Eq. 2) with its CI95.

    python tests/golden/make_golden.py --config mid --seed 24301 --m 10 [--threads 1]

Single-threaded runs are deterministic; threaded runs are the Hogwild mode.
"""
import argparse
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import synth  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", required=True, choices=sorted(synth.CONFIGS))
    ap.add_argument("--seed", type=int, default=24301)
    ap.add_argument("--m", type=int, default=10)
    ap.add_argument("--sps-seed", type=int, default=7)
    ap.add_argument("--threads", type=int, default=1)
    ap.add_argument("--init-seed", type=int, default=5)
    ap.add_argument("--jitter", type=float, default=10.0)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()

    sg = synth.config_graph(a.config)
    g = O.Graph.from_synth(sg)
    c = O.init_coords(g, seed=a.init_seed, jitter=a.jitter)
    t0 = time.time()
    applied = O.layout(g, c, seed=a.seed, threads=a.threads, term_limit=0) if a.threads == 1 else \
        O.layout(g, c, seed=a.seed, threads=a.threads, term_limit=10 * g.S)
    t_layout = time.time() - t0
    s = O.sampled_path_stress(g, c, m=a.m, seed=a.sps_seed)
    rec = dict(config=a.config, graph=sg.stats, layout_seed=a.seed, init_seed=a.init_seed, jitter=a.jitter,
               n_iters=30, terms_per_step=10, eta_min=0.01, theta=0.99, window=1000,
               sps_m=a.m, sps_seed=a.sps_seed, sps_mean=s["mean"], sps_ci_lo=s["ci_lo"], sps_ci_hi=s["ci_hi"],
               sps_stddev=s["stddev"], sps_n_valid=s["n_valid"], sps_n_skipped=s["n_skipped"],
               applied_updates=applied, oracle_threads=a.threads,
               mode="sequential" if a.threads == 1 else "hogwild-threads",
               layout_seconds=round(t_layout, 1), host=platform.processor() or platform.machine())
    out = a.out or os.path.join(HERE, f"oracle_sps_{a.config}_seed{a.seed}_t{a.threads}.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1, default=int)
    print(json.dumps(rec, default=int))


if __name__ == "__main__":
    main()
