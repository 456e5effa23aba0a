"""Writes the expected results of full-size IMM solves, computed by the CPU oracle only.

    python tests/golden/make_full_size.py [c2] [c3] [--threads N]

For each named workload (R-MAT scale 20 with weighted-cascade IC, k = 50, eps = 0.1; R-MAT
scale 22 with uniform-normalised LT weights, k = 100, eps = 0.1) this builds the seeded
synthetic inputs, runs the oracle's IMM (gIM Alg. 2 then Alg. 1) and stores, in
full_size_<name>.json next to this file: the seeds in selection order, theta, the number
of RR sets generated, the covered count, the phases, in-edges examined, total set members,
and LB / the spread estimate / lambda' / lambda* as exact hexadecimal doubles.  A SHA-256
of the input arrays is stored too, so a reader can tell whether its inputs are the same.
Nothing here touches the GPU library.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from synth import configs  # noqa: E402


def input_digest(w) -> str:
    h = hashlib.sha256()
    for a in (w.graph.in_off, w.graph.in_src, w.ic_p, w.lt_w):
        if a is not None:
            h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def solve(name: str, threads: int) -> dict:
    w = {"c2": configs.c2, "c3": configs.c3}[name]()
    model = oracle.IC if w.model == "IC" else oracle.LT
    t0 = time.perf_counter()
    r = oracle.imm_solve(w.graph, model, w.k, w.eps, w.ell, w.seed, ic_p=w.ic_p, lt_w=w.lt_w,
                         threads=threads)
    dt = time.perf_counter() - t0
    return {
        "workload": w.name, "n": w.graph.n, "m": w.graph.m, "model": w.model, "k": w.k,
        "eps": w.eps, "ell": w.ell, "pool_seed": w.seed, "fresh_final": False,
        "input_sha256": input_digest(w),
        "seeds": [int(s) for s in r["seeds"]],
        "theta": r["theta"], "num_rr": r["num_rr"], "covered": r["covered"],
        "phases": r["phases"], "edges_examined": r["edges"], "pool_ids": r["pool_ids"],
        "lb_hex": float(r["lb"]).hex(), "spread_est_hex": float(r["spread_est"]).hex(),
        "lambda_prime_hex": float(r["lambda_prime"]).hex(),
        "lambda_star_hex": float(r["lambda_star"]).hex(),
        "oracle_seconds": round(dt, 1), "oracle_threads": threads,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=["c2", "c3"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    for name in args.names:
        rec = solve(name, args.threads)
        path = os.path.join(HERE, f"full_size_{name}.json")
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
        print(f"{name}: theta={rec['theta']} num_rr={rec['num_rr']} "
              f"({rec['oracle_seconds']} s) -> {path}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
