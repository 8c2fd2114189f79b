"""Writes stored oracle results for configurations too large to run inside a test.

Calls only the oracle (and the seeded input generator).  Each run lays out a
synthetic configuration from the oracle's initial layout with the given layout
seed and stores the final sampled path stress (Eq. 2) with its CI95, for one
or several pair counts m and pair orders (the uniform order of the pair
definition, and the window-major listing of the same law).

    python tests/golden/make_golden.py --config mid --seed 24301 --m 10 [--threads 1]
    python tests/golden/make_golden.py --config chromosome --threads 6 --save-layout L.f32
    python tests/golden/make_golden.py --config chromosome --threads 6 --load-layout L.f32 --m 10 100 \
        --orders uniform uniform_windowed --sps-threads 8

Single-threaded runs are deterministic; threaded runs are the Hogwild mode.
--save-layout keeps the final coordinates (raw float32, boundary layout) and a
small JSON beside them, so the stress at more pair counts can be evaluated
later with --load-layout without laying out again.  --sps-threads evaluates
Eq. 2 with the oracle's threaded evaluation (paths split over threads; the
same pairs, sums in another order).
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import synth  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", required=True, choices=sorted(synth.CONFIGS))
    ap.add_argument("--seed", type=int, default=24301)
    ap.add_argument("--m", type=int, nargs="+", default=[10])
    ap.add_argument("--orders", nargs="+", default=["uniform"], choices=["uniform", "uniform_windowed"])
    ap.add_argument("--sps-seed", type=int, default=7)
    ap.add_argument("--sps-threads", type=int, default=1)
    ap.add_argument("--threads", type=int, default=1)
    ap.add_argument("--init-seed", type=int, default=5)
    ap.add_argument("--jitter", type=float, default=10.0)
    ap.add_argument("--save-layout", default=None)
    ap.add_argument("--load-layout", default=None)
    ap.add_argument("--layout-only", action="store_true")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()

    sg = synth.config_graph(a.config)
    g = O.Graph.from_synth(sg)
    if a.load_layout:
        c = np.fromfile(a.load_layout, dtype=np.float32)
        assert c.size == 4 * g.n_nodes, "layout file does not match the graph"
        with open(a.load_layout + ".json") as f:
            meta = json.load(f)
        assert meta["config"] == a.config and meta["layout_seed"] == a.seed and meta["oracle_threads"] == a.threads
        applied, t_layout = meta["applied_updates"], meta["layout_seconds"]
    else:
        c = O.init_coords(g, seed=a.init_seed, jitter=a.jitter)
        t0 = time.time()
        applied = O.layout(g, c, seed=a.seed, threads=a.threads, term_limit=0) if a.threads == 1 else \
            O.layout(g, c, seed=a.seed, threads=a.threads, term_limit=10 * g.S)
        t_layout = round(time.time() - t0, 1)
        if a.save_layout:
            c.tofile(a.save_layout)
            with open(a.save_layout + ".json", "w") as f:
                json.dump(dict(config=a.config, layout_seed=a.seed, oracle_threads=a.threads, applied_updates=applied,
                               layout_seconds=t_layout, init_seed=a.init_seed, jitter=a.jitter), f, default=int)
        print(f"layout done in {t_layout} s, {applied} updates", flush=True)
    if a.layout_only:
        return
    evals = []
    for order in a.orders:
        for m in a.m:
            t0 = time.time()
            s = O.sampled_path_stress(g, c, m=m, seed=a.sps_seed, pairs=order, threads=a.sps_threads)
            evals.append(dict(order=order, m=m, mean=s["mean"], ci_lo=s["ci_lo"], ci_hi=s["ci_hi"],
                              stddev=s["stddev"], n_valid=s["n_valid"], n_skipped=s["n_skipped"],
                              seconds=round(time.time() - t0, 1)))
            print(json.dumps(evals[-1]), flush=True)
    first = evals[0]
    rec = dict(config=a.config, graph=sg.stats, layout_seed=a.seed, init_seed=a.init_seed, jitter=a.jitter,
               n_iters=30, terms_per_step=10, eta_min=0.01, theta=0.99, window=1000,
               sps_m=first["m"], sps_order=first["order"], sps_seed=a.sps_seed, sps_mean=first["mean"],
               sps_ci_lo=first["ci_lo"], sps_ci_hi=first["ci_hi"], sps_stddev=first["stddev"],
               sps_n_valid=first["n_valid"], sps_n_skipped=first["n_skipped"], sps=evals,
               applied_updates=applied, oracle_threads=a.threads,
               mode="sequential" if a.threads == 1 else "hogwild-threads",
               layout_seconds=t_layout, host=platform.processor() or platform.machine())
    out = a.out or os.path.join(HERE, f"oracle_sps_{a.config}_seed{a.seed}_t{a.threads}.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1, default=int)
    print(json.dumps(rec, default=int))


if __name__ == "__main__":
    main()
