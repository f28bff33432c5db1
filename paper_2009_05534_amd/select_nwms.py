#!/usr/bin/env python3
"""Choose the learned weighted min-sum weights to ship, then report them on
held-out data.

Candidates are the trained checkpoints and their compositions: the rows of
one table for iterations t < t0 and another's (or plain beta = 3/4) from t0
on -- fast-converging weights early, weights without an error floor late.
Selection runs on validation codewords (data seed 11, disjoint from the
training seed 4 and the held-out seed 5): among the candidates that make no
more block errors than plain min-sum at any validation point, the one with
the fewest mean iterations. The chosen table is then evaluated on held-out
codewords (seed 5): 10^5 per Eb/N0 point at 0.5..2.0 dB and 10^6 at 1.75
and 2.0 dB, with 95 % Poisson intervals on the error counts.

  python -m paper_2009_05534_amd.select_nwms
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from synth import make_batch, make_graph  # noqa: E402

WDIR = os.path.join(ROOT, "paper_2009_05534_amd", "weights")
VALID_SEED, HELDOUT_SEED = 11, 5
PLAIN_Q = 96


def _chunk(args):
    bg, Z, ebn0, seed, start, n = args
    g = make_graph(bg, Z)
    b = make_batch(g, n, ebn0, seed, start=start)
    return b.q, b.u


def poisson_ci(k: int) -> tuple[float, float]:
    """95 % interval for a Poisson count (Wilson-Hilferty approximation of
    the exact chi-square bounds)."""
    def chi2_q(p, dof):
        from statistics import NormalDist
        z = NormalDist().inv_cdf(p)
        return dof * (1 - 2 / (9 * dof) + z * math.sqrt(2 / (9 * dof))) ** 3
    lo = 0.0 if k == 0 else chi2_q(0.025, 2 * k) / 2
    hi = chi2_q(0.975, 2 * (k + 1)) / 2
    return lo, hi


def candidates() -> dict[str, np.ndarray]:
    from paper_2009_05534_amd import nwms
    base = {}
    for name, fn in (("default", "nwms_bg1_z384.npz"), ("ramp", "nwms_bg1_z384_ramp.npz"),
                     ("wide", "nwms_bg1_z384_train0.5to2dB.npz")):
        wq, _ = nwms.load_weights(os.path.join(WDIR, fn))
        base[name] = np.asarray(wq, np.uint8)
    T, M = base["default"].shape
    plain = np.full((T, M), PLAIN_Q, np.uint8)
    out = dict(base)
    for a in ("default", "wide"):
        for b, tb in (("plain", plain), ("ramp", base["ramp"])):
            for t0 in range(3, 8):
                w = tb.copy()
                w[:t0] = base[a][:t0]
                out[f"{a}[:{t0}]+{b}"] = w
    return out


def decode_stats(pool, bg, Z, rows, tables: dict, ebn0, n, seed, chunk=8192):
    """errors / iterations / n of plain and every table on the same codewords."""
    import torch

    from paper_2009_05534_amd import ldpc
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in tables.items()}
    stats = {k: [0, 0, 0] for k in ["plain", *tables]}
    jobs = [(bg, Z, ebn0, seed, s, min(chunk, n - s)) for s in range(0, n, chunk)]
    for q, u in pool.map(_chunk, jobs):
        llr = torch.from_numpy(q).cuda()
        K = u.shape[1]
        for name in stats:
            w = None if name == "plain" else dev[name]
            bits, iters, _, _ = ldpc.decode(llr, bg, Z, rows, max_iter=10, weights=w)
            got = np.unpackbits(bits.cpu().numpy(), axis=1, bitorder="little")[:, :K]
            st = stats[name]
            st[0] += int((got != u).any(axis=1).sum())
            st[1] += int(iters.sum().item())
            st[2] += q.shape[0]
    return stats


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--valid-n", type=int, default=300_000)
    ap.add_argument("--valid-points", default="1.5,1.75,2.0")
    ap.add_argument("--heldout-n", type=int, default=100_000)
    ap.add_argument("--heldout-points", default="0.5,0.75,1.0,1.25,1.5,1.75,2.0")
    ap.add_argument("--floor-n", type=int, default=1_000_000)
    ap.add_argument("--floor-points", default="1.75,2.0")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--out", default=os.path.join(WDIR, "nwms_bg1_z384_select.npz"))
    args = ap.parse_args()
    pool = cf.ProcessPoolExecutor(max_workers=args.workers, mp_context=mp.get_context("fork"))
    import torch

    from paper_2009_05534_amd import ldpc, nwms
    bg, Z = 1, 384
    g = make_graph(bg, Z)
    torch.cuda.set_device(0)
    ldpc.register(g)
    rows = g.M
    cands = candidates()
    t0 = time.time()
    valid = {}
    for p in [float(x) for x in args.valid_points.split(",")]:
        valid[p] = decode_stats(pool, bg, Z, rows, cands, p, args.valid_n, VALID_SEED)
        print(f"[select] validation {p} dB: plain {valid[p]['plain'][0]} errors", flush=True)
    ok = []
    for name in cands:
        if all(valid[p][name][0] <= valid[p]["plain"][0] for p in valid):
            its = sum(valid[p][name][1] / valid[p][name][2] for p in valid)
            ok.append((its, name))
    table = {name: {str(p): {"errors": valid[p][name][0],
                             "mean_iters": valid[p][name][1] / valid[p][name][2]}
                    for p in valid} for name in ["plain", *cands]}
    print(json.dumps({"validation": table}), flush=True)
    if not ok:
        print("[select] no candidate matches plain's block errors at every validation point",
              flush=True)
        pool.shutdown()
        return
    ok.sort()
    chosen = ok[0][1]
    print(f"[select] chosen {chosen} ({time.time() - t0:.0f}s)", flush=True)
    w = cands[chosen]
    # held-out report
    heldout = {}
    for p in [float(x) for x in args.heldout_points.split(",")]:
        st = decode_stats(pool, bg, Z, rows, {"learned": w}, p, args.heldout_n, HELDOUT_SEED)
        heldout[str(p)] = {k: {"errors": v[0], "bler": v[0] / v[2], "mean_iters": v[1] / v[2],
                               "n": v[2], "errors_ci95": poisson_ci(v[0])}
                           for k, v in st.items()}
        print(json.dumps({str(p): heldout[str(p)]}), flush=True)
    floor = {}
    for p in [float(x) for x in args.floor_points.split(",")]:
        st = decode_stats(pool, bg, Z, rows, {"learned": w}, p, args.floor_n, HELDOUT_SEED)
        floor[str(p)] = {k: {"errors": v[0], "bler": v[0] / v[2], "mean_iters": v[1] / v[2],
                             "n": v[2], "errors_ci95": poisson_ci(v[0])}
                         for k, v in st.items()}
        print(json.dumps({"floor": {str(p): floor[str(p)]}}), flush=True)
    # save: the Q1.7 table (and w = wq / 128 as its real-valued form)
    meta = {"graph_digest": g.digest(), "bg": bg, "Z": Z, "rows": rows, "n_iter": int(w.shape[0]),
            "scale": 4.0,
            "composition": chosen, "selected_on": f"data seed {VALID_SEED}, "
            f"{args.valid_n} codewords at {args.valid_points} dB"}
    np.savez(args.out, w=w.astype(np.float64) / 128.0, wq=w)
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    with open(os.path.splitext(args.out)[0] + "_eval.json", "w") as f:
        json.dump({"checkpoint": os.path.basename(args.out), "composition": chosen,
                   "validation": table, "heldout_seed": HELDOUT_SEED, "heldout": heldout,
                   "floor": floor, "seconds": round(time.time() - t0, 1)}, f, indent=1)
    print(f"[select] wrote {args.out}", flush=True)
    pool.shutdown()


if __name__ == "__main__":
    main()
