"""Block error rates of the check rules and schedules -- TEST INFRASTRUCTURE
ONLY (context for the decoder's design; runs the CPU oracle alone).

Decodes the same seeded codewords with
  * int8 layered min-sum, beta = 3/4 (the decoder's own arithmetic),
  * double layered min-sum, beta = 3/4,
  * double layered sum-product (§III's exact check rule),
  * double flooding min-sum and flooding sum-product (§III's other schedule),
all at the same iteration limit with early exit, and prints one JSON line
per (Eb/N0, variant) with the block error rate against the transmitted
information bits and the mean iterations, then a markdown table.

  python -m oracle.bler_context --bg 2 --Z 16 --ebn0 1.5 2.0 2.5 --n 1000
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
from synth import make_batch_parallel, make_graph  # noqa: E402


def _bler(bits, u, K):
    got = oracle.unpack_bits(bits, K)
    return float((got != u).any(axis=1).mean())


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--bg", type=int, default=2)
    ap.add_argument("--Z", type=int, default=16)
    ap.add_argument("--rows", type=int, default=0, help="block rows kept (0: all)")
    ap.add_argument("--ebn0", type=float, nargs="+", default=[1.5, 2.0, 2.5])
    ap.add_argument("--n", type=int, default=1000)
    ap.add_argument("--max-iter", type=int, default=10)
    ap.add_argument("--seed", type=int, default=20)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args(argv)
    g = make_graph(a.bg, a.Z)
    if a.rows and a.rows != g.M:
        g = g.sub(a.rows)
    variants = [("int8 layered min-sum", None, None),
                ("layered min-sum", "minsum", "layered"),
                ("layered sum-product", "spa", "layered"),
                ("flooding min-sum", "minsum", "flooding"),
                ("flooding sum-product", "spa", "flooding")]
    table = {}
    for i, e in enumerate(a.ebn0):
        b = make_batch_parallel(g, a.n, e, data_seed=a.seed + i, workers=min(8, a.threads))
        for name, rule, sched in variants:
            if rule is None:
                bits, iters, _, _ = oracle.decode_i8(g, b.q, max_iter=a.max_iter,
                                                      n_threads=a.threads)
            else:
                # the double variants take the same quantised LLRs (units of 1/4)
                bits, iters, _, _ = oracle.decode_bp(g, b.q.astype(np.float64) / 4.0, rule=rule,
                                                     schedule=sched, max_iter=a.max_iter,
                                                     beta=0.75, n_threads=a.threads)
            rec = {"bg": a.bg, "Z": a.Z, "rows": g.M, "ebn0": e, "n": a.n, "variant": name,
                   "bler": _bler(bits, b.u, g.K), "mean_iters": float(iters.mean()),
                   "max_iter": a.max_iter, "seed": a.seed + i}
            table[(e, name)] = rec
            print(json.dumps(rec), flush=True)
    print()
    print("| variant | " + " | ".join(f"{e} dB" for e in a.ebn0) + " |")
    print("|---|" + "---|" * len(a.ebn0))
    for name, _, _ in variants:
        cells = [f"{table[(e, name)]['bler']:.3g} / {table[(e, name)]['mean_iters']:.2f}"
                 for e in a.ebn0]
        print(f"| {name} | " + " | ".join(cells) + " |")


if __name__ == "__main__":
    main()
