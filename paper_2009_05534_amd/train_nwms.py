#!/usr/bin/env python3
"""Train the learned weighted min-sum weights on the GPU and compare the
quantised int8 decoder with plain normalised min-sum (beta = 3/4).

Training data: BG1-shaped Z = 384, all 46 rows, codewords from the seeded
encoder and BPSK/AWGN channel with Eb/N0 drawn uniformly from [0.5, 2.0] dB
per codeword (data seed 4), int8 LLRs used as fp32 inputs. Held-out data:
data seed 5 at fixed Eb/N0 points. Prints one progress line per report
interval and a final JSON summary; writes the checkpoint (.npz + .json).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from synth import make_batch, make_graph  # noqa: E402
from synth.prng import stream  # noqa: E402

TRAIN_SEED, HELDOUT_SEED = 4, 5


def _train_chunk(args):
    bg, Z, start, n, lo, hi = args
    g = make_graph(bg, Z)
    ebn0 = stream(TRAIN_SEED, 9, start).uniform(lo, hi, n)
    b = make_batch(g, n, ebn0, TRAIN_SEED, start=start)
    return b.q, b.c


def _heldout_chunk(args):
    bg, Z, rows, ebn0, start, n = args
    g = make_graph(bg, Z).sub(rows)
    b = make_batch(g, n, ebn0, HELDOUT_SEED, start=start)
    return b.q, b.u


def evaluate(pool, bg, Z, rows, wq, points, n_per_point, chunk, max_iter=10):
    """BLER and mean iterations of plain and learned int8 decoding."""
    import torch

    from paper_2009_05534_amd import ldpc
    wdev = torch.from_numpy(np.ascontiguousarray(wq)).cuda()
    out = {}
    for p in points:
        jobs = [(bg, Z, rows, p, s, min(chunk, n_per_point - s))
                for s in range(0, n_per_point, chunk)]
        stats = {"plain": [0, 0, 0], "learned": [0, 0, 0]}  # errors, iters, n
        for q, u in pool.map(_heldout_chunk, jobs):
            llr = torch.from_numpy(q).cuda()
            K = u.shape[1]
            for name, w in (("plain", None), ("learned", wdev)):
                bits, iters, _, _ = ldpc.decode(llr, bg, Z, rows, max_iter=max_iter, weights=w)
                got = np.unpackbits(bits.cpu().numpy(), axis=1, bitorder="little")[:, :K]
                st = stats[name]
                st[0] += int((got != u).any(axis=1).sum())
                st[1] += int(iters.sum().item())
                st[2] += q.shape[0]
        out[str(p)] = {k: {"bler": v[0] / v[2], "errors": v[0], "mean_iters": v[1] / v[2],
                           "n": v[2]} for k, v in stats.items()}
    return out


class _InProcess:
    """Executor stand-in that runs each job at once in this process
    (--workers 0: no child processes, e.g. under a profiler)."""

    class _Done:
        def __init__(self, value):
            self._value = value

        def result(self):
            return self._value

    def submit(self, fn, arg):
        return self._Done(fn(arg))

    def map(self, fn, args):
        return (fn(a) for a in args)

    def shutdown(self):
        pass


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--bg", type=int, default=1)
    ap.add_argument("--Z", type=int, default=384)
    ap.add_argument("--rows", type=int, default=46)
    ap.add_argument("--n-iter", type=int, default=10)
    ap.add_argument("--n-train", type=int, default=200_000)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--ebn0-lo", type=float, default=0.5, help="training Eb/N0 range (dB)")
    ap.add_argument("--ebn0-hi", type=float, default=2.0)
    ap.add_argument("--eval-n", type=int, default=20_000, help="held-out codewords per point")
    ap.add_argument("--eval-points", default="1.0,1.25,1.5,1.75,2.0")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="data-generation processes (0: generate in this process)")
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2009_05534_amd", "weights",
                                                  "nwms_bg1_z384.npz"))
    ap.add_argument("--report-every", type=int, default=20)
    ap.add_argument("--loss-iters", default="mean",
                    help="loss weight per iteration: 'mean' (1/n_iter each), 'ramp' "
                         "(proportional to the iteration number t) or 'pow:P' (to t**P)")
    ap.add_argument("--init", default="",
                    help="start from this checkpoint's weights (fresh optimiser state)")
    ap.add_argument("--data-start", type=int, default=0,
                    help="index of the first training codeword (fresh data when continuing)")
    ap.add_argument("--eval-only", default="",
                    help="evaluate this checkpoint (no training); results go to "
                         "<checkpoint>_eval<n>.json")
    args = ap.parse_args()

    # worker processes first, before the GPU is touched
    pool = (cf.ProcessPoolExecutor(max_workers=args.workers, mp_context=mp.get_context("fork"))
            if args.workers > 0 else _InProcess())
    if args.eval_only:
        import torch

        from paper_2009_05534_amd import ldpc, nwms
        g = make_graph(args.bg, args.Z)
        torch.cuda.set_device(0)
        ldpc.register(g)
        wq, meta = nwms.load_weights(args.eval_only)
        assert meta["graph_digest"] == g.digest(), "checkpoint of another graph"
        points = [float(x) for x in args.eval_points.split(",")]
        t1 = time.time()
        ev = {}
        for p in points:  # one point at a time, so progress shows
            ev.update(evaluate(pool, args.bg, args.Z, args.rows, wq, [p], args.eval_n, 8192))
            print(json.dumps({str(p): ev[str(p)]}), flush=True)
        summary = {"checkpoint": os.path.basename(args.eval_only), "eval_n": args.eval_n,
                   "eval_seconds": round(time.time() - t1, 1), "eval": ev}
        out = os.path.splitext(args.eval_only)[0] + f"_eval{args.eval_n}.json"
        with open(out, "w") as f:
            json.dump(summary, f, indent=1)
        print(f"[eval] wrote {out}", flush=True)
        pool.shutdown()
        return
    g = make_graph(args.bg, args.Z)
    assert args.rows == g.M, "training uses the full graph"

    import torch

    from paper_2009_05534_amd import ldpc, nwms
    torch.cuda.set_device(0)
    ldpc.register(g)
    iter_w = None
    if args.loss_iters != "mean":
        if args.loss_iters == "ramp":
            power = 1.0
        elif args.loss_iters.startswith("pow:"):
            power = float(args.loss_iters[4:])
        else:
            raise SystemExit(f"unknown --loss-iters {args.loss_iters}")
        iter_w = np.arange(1, args.n_iter + 1, dtype=np.float64) ** power
        iter_w /= iter_w.sum()
    tr = nwms.Trainer(args.bg, args.Z, args.rows, n_iter=args.n_iter, lr=args.lr, iter_w=iter_w)
    if args.init:
        _, meta0 = nwms.load_weights(args.init)
        assert meta0["graph_digest"] == g.digest(), "checkpoint of another graph"
        with np.load(args.init, allow_pickle=False) as f0:
            tr.w = np.array(f0["w"], dtype=np.float64)
    chunk = args.batch * 8
    end = args.data_start + args.n_train
    starts = list(range(args.data_start, end, chunk))
    t0 = time.time()
    rng_db = (args.ebn0_lo, args.ebn0_hi)
    futs = [pool.submit(_train_chunk, (args.bg, args.Z, s, min(chunk, end - s), *rng_db))
            for s in starts[:2]]
    nxt = 2
    seen = 0
    while futs:
        q, c = futs.pop(0).result()
        if nxt < len(starts):
            s = starts[nxt]
            futs.append(pool.submit(_train_chunk, (args.bg, args.Z, s,
                                                   min(chunk, end - s), *rng_db)))
            nxt += 1
        for i in range(0, q.shape[0], args.batch):
            loss = tr.step(q[i:i + args.batch], c[i:i + args.batch])
            seen += q[i:i + args.batch].shape[0]
            if tr.opt.t % args.report_every == 0:
                print(f"[train] step {tr.opt.t} codewords {seen} loss {loss:.5f} "
                      f"w[mean] {tr.w.mean():.4f} {time.time() - t0:.0f}s", flush=True)
    train_s = time.time() - t0
    tr.save(args.out, g.digest(), extra={"n_train": seen, "batch": args.batch,
                                          "train_seconds": train_s, "ebn0_db": list(rng_db),
                                          "init": os.path.basename(args.init) or None,
                                          "loss_iters": args.loss_iters,
                                          "data_start": args.data_start})
    print(f"[train] saved {args.out} after {seen} codewords in {train_s:.0f}s", flush=True)
    points = [float(x) for x in args.eval_points.split(",")]
    t1 = time.time()
    ev = evaluate(pool, args.bg, args.Z, args.rows, tr.wq, points, args.eval_n, 2048)
    summary = {"n_train": seen, "steps": tr.opt.t, "train_seconds": round(train_s, 1),
               "train_ebn0_db": list(rng_db), "lr": args.lr,
               "eval_seconds": round(time.time() - t1, 1), "eval": ev,
               "loss_first": tr.history[0]["loss"], "loss_last": tr.history[-1]["loss"]}
    with open(os.path.splitext(args.out)[0] + "_eval.json", "w") as f:
        json.dump(summary, f, indent=1)
    print(json.dumps(summary), flush=True)
    pool.shutdown()


if __name__ == "__main__":
    main()
