#!/usr/bin/env python3
"""Throughput benchmark of the MI355X layered min-sum LDPC decoder.

Workload: BG1-shaped QC-LDPC, Z = 384, all 46 block rows (rate 1/3,
K = 8448 information bits per codeword), 4096 codewords at each Eb/N0 of
0.5, 0.75, ..., 2.0 dB (seeded synthetic BPSK/AWGN, int8 LLRs), layered
normalised min-sum with beta = 3/4, at most 10 iterations, early exit on a
zero syndrome. One step decodes the 7 batches (28,672 codewords) with the
int8 kernel; inputs are resident in HBM before timing starts.

Prints one JSON line: decoded information Gbit/s, the roofline of the
dominant kernel (VALU-bound: 11 packed-16-bit element operations per
edge-update, peak 256 CU x 64 lanes x 2 x 2.4 GHz), the CPU oracle timed on
a bounded sample of the same workload, plus latency, BLER and the binary16
path as extra fields.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_ALU_TOPS = 256 * 64 * 2 * 2.4e9 / 1e12  # packed 16-bit element ops, Top/s
OPS_PER_EDGE_UPDATE = 11
EBN0_POINTS = (0.5, 0.75, 1.0, 1.25, 1.5, 1.75, 2.0)
# Channel data seeds of the Eb/N0 batches: DATA_SEED0 + point index, disjoint
# from the learned weights' training (4) and held-out evaluation (5) seeds.
DATA_SEED0 = 10
BG, Z, ROWS = 1, 384, 46


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


COUNTERS_FILE = os.path.join(ROOT, "profiles", "decode_i8_bg1_z384_counters.md")
KERNEL_SOURCES_F16 = ("decode_f16.hip", "ldpc_internal.h")
COUNTERS_FILE_F16 = os.path.join(ROOT, "profiles", "decode_f16_bg1_z384_counters.md")
KERNEL_SOURCES = ("decode_i8.hip", "ldpc_internal.h")
# the kernels the library runs for this workload by default: early-exit int8
# decodes go to the row-pair kernel (one codeword per workgroup at Z = 384)
KERNEL_I8 = "decode_i8_rp_kernel"
KERNEL_F16 = "decode_f16_kernel"


def kernel_source_sha(sources=KERNEL_SOURCES) -> str:
    """Hash of a kernel's sources (the int8 one by default) with comments
    and blank space removed (a comment edit does not change the measured
    kernel)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(ROOT, "paper_2009_05534_amd", "csrc", name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(counters_file=None, sources=None, kernel=None):
    """HBM bytes per launch of a decode kernel (the int8 one by default)
    from its committed counter summary (FETCH_SIZE and WRITE_SIZE, each
    scaled by what the counter reads for a plain copy of known size), or
    None when the summary is missing, names another kernel or was taken on
    other kernel sources."""
    try:
        text = open(counters_file or COUNTERS_FILE).read()
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("kernel_source_sha") != kernel_source_sha(sources or KERNEL_SOURCES):
        return None
    if rec.get("kernel") != (kernel or KERNEL_I8):
        return None
    return rec.get("traffic_bytes_per_launch")


def load_or_make_batches(g, n_cw, cache):
    """The seeded channel batches (one per Eb/N0 point); an npz cache keyed
    by the graph digest and batch size skips regenerating them."""
    from synth import make_batch_parallel
    from synth.channel import Batch
    key = f"{g.digest()}-{n_cw}-{','.join(map(str, EBN0_POINTS))}-seeds{DATA_SEED0}"
    if cache and os.path.exists(cache):
        with np.load(cache) as f:
            if str(f["key"]) == key:
                return [Batch(u=f[f"u{i}"], c=None, llr=None, q=f[f"q{i}"], ebn0=e)
                        for i, e in enumerate(EBN0_POINTS)]
    workers = max(1, min(16, os.cpu_count() or 1))
    batches = [make_batch_parallel(g, n_cw, e, data_seed=DATA_SEED0 + i, workers=workers)
               for i, e in enumerate(EBN0_POINTS)]
    if cache:
        arrays = {"key": np.array(key)}
        for i, b in enumerate(batches):
            arrays[f"u{i}"], arrays[f"q{i}"] = b.u, b.q
        np.savez(cache, **arrays)
    return batches


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-cw", type=int, default=4096)
    ap.add_argument("--max-iter", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target wall time of the CPU-oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the binary16, latency, fixed-iteration, batch and serving runs")
    ap.add_argument("--extras", default="fixed,f16,latency,batched,serving",
                    help="comma-separated subset of the extra runs to do")
    ap.add_argument("--data-cache", default="",
                    help="npz file holding the generated channel batches: loaded when present, "
                         "written otherwise (saves the generation time of repeated runs)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this many MiB before timing "
                         "(reference dispatch for calibrating memory counters)")
    args = ap.parse_args()

    extras = set() if args.no_extras else set(x for x in args.extras.split(",") if x)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the decoder has no multi-GPU path "
              "(codewords are independent, so a batch would shard by codeword ranges "
              "with no communication between GPUs)",
              file=sys.stderr)
        sys.exit(2)

    from synth import make_batch, make_graph
    g = make_graph(BG, Z)
    t0 = time.time()
    batches = load_or_make_batches(g, args.n_cw, args.data_cache)
    log(f"{len(batches)} x {args.n_cw} codewords ready in {time.time() - t0:.1f} s")

    import torch
    from paper_2009_05534_amd import ldpc

    torch.cuda.set_device(0)
    ldpc.register(g)
    K, T, Nc, E = ldpc.query(BG, Z, ROWS)
    U = E * Z  # edge-updates per iteration per codeword
    dev = torch.device("cuda:0")
    llr = [torch.from_numpy(b.q).to(dev) for b in batches]
    n = args.n_cw
    bits = [torch.empty((n, K // 8), dtype=torch.uint8, device=dev) for _ in batches]
    iters = [torch.empty(n, dtype=torch.int32, device=dev) for _ in batches]
    oks = [torch.empty(n, dtype=torch.uint8, device=dev) for _ in batches]
    stream = torch.cuda.current_stream()
    if args.copy_probe_mib:
        src = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    torch.cuda.synchronize()

    def run_step(precision="i8", early_exit=True, events=None):
        for i in range(len(batches)):
            if events is not None:
                events[i][0].record(stream)
            ldpc.decode_into(llr[i], BG, Z, ROWS, bits[i], iters[i], out_ok=oks[i],
                             max_iter=args.max_iter, precision=precision,
                             early_exit=early_exit, stream=stream)
            if events is not None:
                events[i][1].record(stream)

    def timed(precision, early_exit, steps, warmup):
        for _ in range(warmup):
            run_step(precision, early_exit)
        torch.cuda.synchronize()
        evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(2)]
                for _ in batches] for _ in range(steps)]
        edge_updates = 0
        t_start = time.perf_counter()
        for s in range(steps):
            run_step(precision, early_exit, evs[s])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        launch_ms = [evs[s][i][0].elapsed_time(evs[s][i][1])
                     for s in range(steps) for i in range(len(batches))]
        edge_updates = sum(int(it.sum().item()) for it in iters) * U * steps
        return wall, launch_ms, edge_updates

    log("timing int8, early exit")
    wall, launch_ms, eu = timed("i8", True, args.steps, args.warmup)
    info_bits = args.steps * len(batches) * n * K
    value = info_bits / wall / 1e9
    ms_per_step = wall / args.steps * 1e3
    kernel_s = sum(launch_ms) / 1e3
    achieved = OPS_PER_EDGE_UPDATE * eu / kernel_s / 1e12
    lat = np.array(launch_ms)

    # BLER and mean iterations per Eb/N0 from the last step's outputs
    bler, mean_it = {}, {}
    for i, b in enumerate(batches):
        got = np.unpackbits(bits[i].cpu().numpy(), axis=1, bitorder="little")[:, :K]
        bler[str(EBN0_POINTS[i])] = float(np.mean((got != b.u).any(axis=1)))
        mean_it[str(EBN0_POINTS[i])] = float(iters[i].float().mean().item())

    result = {
        "metric": "decoded info Gbit/s (BG1 Z=384, 10 it) + p99 latency; BLER vs plain min-sum",
        "value": round(value, 3),
        "unit": "Gbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {
            "workload": "BG1-shaped QC-LDPC Z=384, 46 rows (R=1/3), 4096 codewords x 7 Eb/N0 "
                        "points 0.5-2.0 dB, int8 layered min-sum beta=3/4, max 10 iterations, "
                        "early exit",
            "bg": BG, "Z": Z, "rows": ROWS, "n_cw_per_point": n, "ebn0_db": list(EBN0_POINTS),
            "max_iter": args.max_iter,
        },
        "roofline": {
            "bound": "alu",
            "kernel": KERNEL_I8,
            "achieved": round(achieved, 3),
            "peak": round(PEAK_ALU_TOPS, 2),
            "unit": "Top/s",
            "frac": round(achieved / PEAK_ALU_TOPS, 4),
            "traffic": measured_traffic(),
            "per_unit": f"{OPS_PER_EDGE_UPDATE} packed-16-bit element ops per edge-update",
            "units_per_launch": round(eu / len(launch_ms)),
            "avg_launch_ms": round(float(lat.mean()), 4),
        },
        "latency_ms": {"batch_p50": round(float(np.percentile(lat, 50)), 4),
                       "batch_p99": round(float(np.percentile(lat, 99)), 4)},
        "bler": bler,
        "mean_iters": mean_it,
    }

    # The learned weighted min-sum (default checkpoint, trained for this
    # shape) against plain min-sum on the same batches, outside the timing.
    wpath = os.path.join(ROOT, "paper_2009_05534_amd", "weights", "nwms_bg1_z384_select.npz")
    if os.path.exists(wpath):
        from paper_2009_05534_amd import nwms
        wq, _ = nwms.load_weights(wpath)
        wdev = torch.from_numpy(np.ascontiguousarray(wq)).to(dev)
        lb, li = {}, {}
        for i, b in enumerate(batches):
            ldpc.decode_into(llr[i], BG, Z, ROWS, bits[i], iters[i], max_iter=args.max_iter,
                             weights=wdev, out_ok=oks[i])
            torch.cuda.synchronize()
            got = np.unpackbits(bits[i].cpu().numpy(), axis=1, bitorder="little")[:, :K]
            lb[str(EBN0_POINTS[i])] = float(np.mean((got != b.u).any(axis=1)))
            li[str(EBN0_POINTS[i])] = float(iters[i].float().mean().item())
        result["learned"] = {"checkpoint": os.path.basename(wpath), "bler": lb, "mean_iters": li,
                             "note": "int8 decoder with the trained per-(iteration, row) weights; "
                                     "bler/mean_iters above are plain beta = 3/4"}

    if "fixed" in extras:
        log("timing int8, fixed 10 iterations")
        w10, l10, eu10 = timed("i8", False, 2, 1)
        result["fixed_iter"] = {
            "gbps": round(2 * len(batches) * n * K / w10 / 1e9, 3),
            "frac": round(OPS_PER_EDGE_UPDATE * eu10 / (sum(l10) / 1e3) / 1e12 / PEAK_ALU_TOPS, 4),
            "avg_launch_ms": round(float(np.mean(l10)), 4),
        }
    if "f16" in extras:
        log("timing binary16, early exit")
        w16, l16, eu16 = timed("f16", True, 2, 1)
        ach16 = OPS_PER_EDGE_UPDATE * eu16 / (sum(l16) / 1e3) / 1e12
        t16 = measured_traffic(COUNTERS_FILE_F16, KERNEL_SOURCES_F16, KERNEL_F16)
        result["f16"] = {
            "gbps": round(2 * len(batches) * n * K / w16 / 1e9, 3),
            "avg_launch_ms": round(float(np.mean(l16)), 4),
            "roofline": {
                "bound": "alu", "kernel": KERNEL_F16, "achieved": round(ach16, 3),
                "peak": round(PEAK_ALU_TOPS, 2), "unit": "Top/s",
                "frac": round(ach16 / PEAK_ALU_TOPS, 4), "traffic": t16,
                "hbm_tb_per_s": (round(t16 / (float(np.mean(l16)) / 1e3) / 1e12, 3)
                                 if t16 else None),
                "per_unit": f"{OPS_PER_EDGE_UPDATE} packed binary16 element ops per edge-update",
                "units_per_launch": round(eu16 / len(l16)),
            },
        }
    if "latency" in extras:
        # single-codeword latency per iteration (fixed 10 iterations), with
        # one lane per check row and with the low-latency mapping (alpha
        # lanes per check row), at Z = 384 and Z = 128
        def one_cw_us_per_iter(bg, Zx, rows, q1, alpha, precision="i8", pairing="auto"):
            b1 = torch.empty((1, bg_k(bg) * Zx // 8), dtype=torch.uint8, device=dev)
            i1 = torch.empty(1, dtype=torch.int32, device=dev)
            for _ in range(3):
                ldpc.decode_into(q1, bg, Zx, rows, b1, i1, max_iter=10, early_exit=False,
                                 lanes_per_row=alpha, precision=precision, pairing=pairing)
            torch.cuda.synchronize()
            ts = []
            for _ in range(50):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                ldpc.decode_into(q1, bg, Zx, rows, b1, i1, max_iter=10, early_exit=False,
                                 lanes_per_row=alpha, precision=precision, pairing=pairing)
                e1.record(stream)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1))
            return round(float(np.percentile(ts, 50)) * 1e3 / 10, 2)

        def bg_k(bg):
            return 22 if bg == 1 else 10

        one = llr[4][:1].contiguous()
        # one lane per row: check rows u and u + Z/2 of the codeword per lane
        # (the default for one codeword at lifts above 256) and codeword
        # pairs (the codeword in one half of every lane)
        lat1 = {"1": one_cw_us_per_iter(BG, Z, ROWS, one, 1, pairing="rows"),
                "1_codeword_pairs": one_cw_us_per_iter(BG, Z, ROWS, one, 1, pairing="codewords"),
                "2": one_cw_us_per_iter(BG, Z, ROWS, one, 2)}
        g128 = make_graph(BG, 128)
        ldpc.register(g128)
        q128 = torch.from_numpy(make_batch(g128, 1, EBN0_POINTS[4], data_seed=9).q).to(dev)
        lat128 = {str(al): one_cw_us_per_iter(BG, 128, ROWS, q128, al) for al in (1, 2, 4)}
        lat128["1_row_pairs"] = one_cw_us_per_iter(BG, 128, ROWS, q128, 1, pairing="rows")
        # BG2-shaped Z = 384, all 42 rows: by default one codeword takes row
        # pairs with its messages in LDS (no row weighs more than 10 blocks)
        g2 = make_graph(2, Z)
        ldpc.register(g2)
        q2 = torch.from_numpy(make_batch(g2, 1, EBN0_POINTS[4], data_seed=9).q).to(dev)
        lat_bg2 = {"1": one_cw_us_per_iter(2, Z, g2.M, q2, 1),
                   "1_codeword_pairs": one_cw_us_per_iter(2, Z, g2.M, q2, 1, pairing="codewords")}
        result["latency_ms"]["single_codeword_us_per_iter_p50"] = min(lat1.values())
        # binary16: one codeword on Z/2 lanes (two check rows per lane)
        lat16 = {f"Z{Z}": one_cw_us_per_iter(BG, Z, ROWS, one, 0, "f16"),
                 "Z128": one_cw_us_per_iter(BG, 128, ROWS, q128, 0, "f16")}
        result["latency_ms"]["single_codeword_us_per_iter"] = {
            "note": "one codeword, 10 iterations, p50 over 50 calls, by lanes per check row "
                    "(int8 '1': check rows u and u + Z/2 per lane at Z = 384 -- for the "
                    "BG2-shaped code with the messages in LDS -- and codeword pairs at "
                    "Z = 128; '1_codeword_pairs' / '1_row_pairs': the other pairing)",
            f"Z{Z}": lat1, "Z128": lat128, f"bg2_Z{Z}": lat_bg2, "f16": lat16}

    if "batched" in extras:
        # ldpc_tune on two single-shape batches (int8, early exit): the
        # default launch against the tuned one, which later default calls
        # of that shape and batch size take
        log("autotuning single-shape launches")

        def time_default(q, Zx, bb, ii, reps=10):
            ldpc.decode_into(q, BG, Zx, ROWS, bb, ii, max_iter=args.max_iter)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                ldpc.decode_into(q, BG, Zx, ROWS, bb, ii, max_iter=args.max_iter)
            e1.record(stream)
            e1.synchronize()
            return e0.elapsed_time(e1) / reps

        g_t = make_graph(BG, 128)
        ldpc.register(g_t)
        q_t = torch.from_numpy(make_batch(g_t, 64, EBN0_POINTS[4], data_seed=10).q).to(dev)
        tune_cases = [(128, q_t), (Z, llr[4])]
        result["tuned"] = {}
        for Zx, q in tune_cases:
            nq = int(q.shape[0])
            bb = torch.empty((nq, 22 * Zx // 8), dtype=torch.uint8, device=dev)
            ii = torch.empty(nq, dtype=torch.int32, device=dev)
            before = time_default(q, Zx, bb, ii)
            pick = ldpc.decode_into(q, BG, Zx, ROWS, bb, ii, max_iter=args.max_iter, tune=True)
            after = time_default(q, Zx, bb, ii)
            result["tuned"][f"bg{BG}_z{Zx}_n{nq}"] = {
                **{k: (round(v, 4) if isinstance(v, float) else v) for k, v in pick.items()},
                "default_ms": round(before, 4), "tuned_ms": round(after, 4)}
        # Mixed-shape batch: 2048 codewords, (bg, Z, rows) drawn per codeword,
        # one persistent launch, captured as a HIP graph with an autotuned grid.
        from synth.mixed import make_mixed
        from synth import LIFTS
        for bgx in (1, 2):
            for Zx in LIFTS:
                ldpc.register(make_graph(bgx, Zx))
        groups = make_mixed(2048, 1.5, seed=3)
        jobs = [ldpc.BatchJob(torch.from_numpy(gr.batch.q).to(dev), gr.bg, gr.Z, gr.rows)
                for gr in groups]
        plan = ldpc.Plan(jobs, graph=True, autotune=True)
        plan.launch()
        torch.cuda.synchronize()
        reps = 10
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            plan.launch(stream)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        kbits = sum(gr.batch.u.shape[0] * gr.batch.u.shape[1] for gr in groups)
        result["batched"] = {"workload": "2048 codewords, BG1/BG2-shaped, Z in {16..384}, "
                                         "rows 4..M, 1.5 dB, one persistent launch",
                             "gbps": round(kbits / (ms / 1e3) / 1e9, 3),
                             "ms_per_launch": round(ms, 4), "shapes": len(groups),
                             **plan.info()}
        plan.close()
    if "serving" in extras:
        log("serving sweep")
        from paper_2009_05534_amd import serve, nwms
        from synth import LIFTS
        for bgx in (1, 2):
            for Zx in LIFTS:
                ldpc.register(make_graph(bgx, Zx))
        wpath = os.path.join(ROOT, "paper_2009_05534_amd", "weights", "nwms_bg1_z384_select.npz")
        wq, shapes = None, None
        if os.path.exists(wpath):
            wq, meta = nwms.load_weights(wpath)
            shapes = [(meta["Z"], meta["rows"])]
        # a quarter of the blocks are full-rate BG1 Z = 384 blocks, which
        # take the learned weights and, for failing codewords, the fallback
        blocks = serve.make_trace(600, seed=6, embb_share=0.25)
        # one persistent batch launch per admission round, offered load
        # stepped up to saturation; each block's LLR upload is issued at its
        # arrival, on the stream of its launch, and counts in its latency
        srv = serve.Server(weights_bg1=wq, n_slots=8, mem_budget=256 << 20, learned_shapes=shapes)
        # warm-up over the whole trace: first uses of the fallback merge and
        # of larger admission rounds (kernel loading, allocator growth) cost
        # tens of milliseconds once and are not serving latency
        srv.run(serve.rescale(blocks, 5e3))
        result["serving"] = []
        for r in (1e3, 5e3, 2e4, 5e4, 1e5, 4e5):
            st = srv.run(serve.rescale(blocks, r))
            st["rate_blocks_per_s"] = r
            result["serving"].append(st)

    if not args.no_cpu_baseline:
        import tempfile
        import oracle
        nproc = os.cpu_count() or 1
        # the host share a GPU job gets here is 16 cores, whatever nproc says
        threads = max(1, min(16, nproc))
        tmpdir = tempfile.mkdtemp(prefix="oracle_native_")
        oracle.use_native_build(tmpdir)

        # A stratified sample: the first m codewords of every Eb/N0 batch, so
        # the iteration mix matches the timed workload.
        def cpu_run(m, nt):
            per = []
            for b in batches:
                t0 = time.perf_counter()
                oracle.decode_i8(g, b.q[:m], max_iter=args.max_iter, n_threads=nt)
                per.append(time.perf_counter() - t0)
            return per
        probe = 16
        dt = sum(cpu_run(probe, threads))
        m = int(min(n, max(probe, probe * args.cpu_seconds / max(dt, 1e-3))))
        log(f"CPU oracle baseline on {m} codewords per Eb/N0 point, {threads} threads")
        per = cpu_run(m, threads)
        dt = sum(per)
        # one thread on a sample a sixteenth that size (a few seconds)
        m1 = max(4, m // 16)
        log(f"CPU oracle baseline on {m1} codewords per Eb/N0 point, 1 thread")
        per1 = cpu_run(m1, 1)
        result["cpu_baseline"] = {
            "value": round(len(batches) * m * K / dt / 1e9, 6),
            "unit": "Gbit/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"first {m} codewords of each of the {len(batches)} Eb/N0 batches "
                      f"({len(batches) * m} codewords), int8 oracle (gcc -O3 -march=native), "
                      f"max {args.max_iter} iterations, early exit, {threads} threads, "
                      f"{dt:.1f} s",
            "host_nproc": nproc,
            "per_ebn0_gbps": {str(e): round(m * K / t / 1e9, 6)
                              for e, t in zip(EBN0_POINTS, per)},
            "one_thread": {"value": round(len(batches) * m1 * K / sum(per1) / 1e9, 6),
                           "sample": f"first {m1} codewords per Eb/N0 point, "
                                     f"{sum(per1):.1f} s",
                           "per_ebn0_gbps": {str(e): round(m1 * K / t / 1e9, 6)
                                             for e, t in zip(EBN0_POINTS, per1)}},
        }

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
