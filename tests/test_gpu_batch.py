"""Mixed-shape persistent batch decode, plans, graph replay and autotuning:
every job's results equal decoding it alone and the oracle."""
import numpy as np
import pytest

import oracle
from libgraph import library_graph
from synth import make_graph
from synth.mixed import make_mixed

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05534_amd import ldpc
    for bg in (1, 2):
        for Z in (16, 32, 64, 96, 128, 192, 256, 384):
            ldpc.register(make_graph(bg, Z))
    return ldpc


def _jobs(ldpc, groups):
    return [ldpc.BatchJob(torch.from_numpy(gr.batch.q).cuda(), gr.bg, gr.Z, gr.rows)
            for gr in groups]


def _alone(ldpc, gr, **kw):
    bits, iters, ok, _ = ldpc.decode(torch.from_numpy(gr.batch.q).cuda(), gr.bg, gr.Z, gr.rows,
                                     msg_placement="device", **kw)
    return bits.cpu().numpy(), iters.cpu().numpy(), ok.cpu().numpy()


def test_mixed_batch_equals_alone_and_oracle(lib):
    groups = make_mixed(300, 1.5, seed=3)
    assert len(groups) > 20
    jobs = _jobs(lib, groups)
    lib.decode_batch(jobs)
    for gr, jb in zip(groups, jobs):
        got = (jb.out_bits.cpu().numpy(), jb.out_iters.cpu().numpy(),
               jb.out_ok.cpu().numpy().astype(bool))
        alone = _alone(lib, gr)
        for a, b in zip(got, alone):
            assert (a == b).all(), (gr.bg, gr.Z, gr.rows)
        g = library_graph(gr.bg, gr.Z, gr.rows)
        ref = oracle.decode_i8(g, gr.batch.q, n_threads=4)
        for a, b in zip(got, ref[:3]):
            assert (a == b).all(), (gr.bg, gr.Z, gr.rows)


def _shape_jobs(ldpc, shapes, ebn0, seed, split=False):
    """Jobs of (bg, Z, rows, n) with seeded channel batches, and the batches."""
    from synth import make_batch
    jobs, batches = [], []
    for i, (bg, Z, rows, n) in enumerate(shapes):
        ldpc.register(make_graph(bg, Z))
        b = make_batch(make_graph(bg, Z, rows), n, ebn0, data_seed=seed + i)
        batches.append(b)
        jobs.append(ldpc.BatchJob(torch.from_numpy(b.q).cuda(), bg, Z, rows, split=split))
    return jobs, batches


SHAPES_A = [(1, 384, 46, 3), (2, 320, 20, 2), (1, 352, 10, 1), (2, 64, 42, 5), (1, 128, 30, 7),
            (2, 288, 42, 2), (2, 192, 20, 3)]


@pytest.mark.parametrize("shapes,ebn0,split", [
    # small tasks: one pair per task, lifts above 256 as one-codeword
    # row-pair tasks, next to wave tasks
    (SHAPES_A, 1.5, True),
    (SHAPES_A, 1.5, False),
    # many Z = 384 codewords, full codeword-pair tasks and small ones
    ([(2, 384, 6, 300), (1, 32, 20, 7)], 2.5, False),
    ([(2, 384, 6, 300), (1, 32, 20, 7)], 2.5, True),
])
def test_split_and_full_tasks_equal_oracle(lib, shapes, ebn0, split):
    jobs, batches = _shape_jobs(lib, shapes, ebn0, 900, split)
    print(f"[batch] shapes {shapes} split={split}", flush=True)
    lib.decode_batch(jobs)
    for (bg, Z, rows, n), jb, b in zip(shapes, jobs, batches):
        ref = oracle.decode_i8(library_graph(bg, Z, rows), b.q, n_threads=8)
        got = (jb.out_bits.cpu().numpy(), jb.out_iters.cpu().numpy(),
               jb.out_ok.cpu().numpy().astype(bool))
        for a, r in zip(got, ref[:3]):
            assert (a == r).all(), (bg, Z, rows, n)


def test_split_plan_graph_replays(lib):
    # small tasks (row-pair tasks included) captured in a graph and replayed
    jobs, batches = _shape_jobs(lib, SHAPES_A, 1.5, 950, split=True)
    plan = lib.Plan(jobs, graph=True, autotune=False)
    refs = [oracle.decode_i8(library_graph(bg, Z, rows), b.q, n_threads=8)
            for (bg, Z, rows, n), b in zip(SHAPES_A, batches)]
    for rep in range(3):
        for jb in jobs:
            jb.out_bits.zero_()
            jb.out_iters.zero_()
        plan.launch()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
        for (bg, Z, rows, n), jb, ref in zip(SHAPES_A, jobs, refs):
            assert (jb.out_bits.cpu().numpy() == ref[0]).all(), (rep, bg, Z, rows)
            assert (jb.out_iters.cpu().numpy() == ref[1]).all(), (rep, bg, Z, rows)
    plan.close()


def test_plan_graph_replays_match_eager(lib):
    from synth import make_batch
    groups = make_mixed(120, 1.75, seed=12)
    jobs = _jobs(lib, groups)
    plan = lib.Plan(jobs, graph=True, autotune=True)
    info = plan.info()
    # lifts above 64: one task per 2*floor(384/Z) codewords of a shape; lifts
    # up to 64: one wave task per 2*floor(64/Z), six wave tasks to a bundle
    big = sum(-(-len(gr.indices) // (2 * (384 // gr.Z))) for gr in groups if gr.Z > 64)
    small = sum(-(-len(gr.indices) // (2 * (64 // gr.Z))) for gr in groups if gr.Z <= 64)
    bundles = -(-small // 6)
    assert info["n_tasks"] == big + bundles, info
    assert info["grid"] >= 1 and info["tuned_ms"] > 0
    for rep in range(3):
        # refill every job's input buffer in place with fresh data of its shape
        qs = []
        for gr, jb in zip(groups, jobs):
            g = make_graph(gr.bg, gr.Z, gr.rows)
            q = make_batch(g, jb.n, 1.75, data_seed=100 + rep, indices=gr.indices).q
            jb.llr.copy_(torch.from_numpy(q))
            qs.append(q)
        plan.launch()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
        for gr, jb, q in zip(groups, jobs, qs):
            bits, iters, ok, _ = lib.decode(torch.from_numpy(q).cuda(), gr.bg, gr.Z, gr.rows)
            assert (jb.out_bits.cpu() == bits.cpu()).all(), (rep, gr.bg, gr.Z, gr.rows)
            assert (jb.out_iters.cpu() == iters.cpu()).all(), (rep, gr.bg, gr.Z, gr.rows)
    plan.close()


def test_batch_with_learned_weights(lib):
    groups = [g for g in make_mixed(200, 1.5, seed=15) if g.bg == 1][:6]
    rng = np.random.default_rng(9)
    jobs = []
    ws = []
    for gr in groups:
        w = rng.integers(64, 128, (3, gr.rows)).astype(np.uint8)
        ws.append(w)
        jobs.append(lib.BatchJob(torch.from_numpy(gr.batch.q).cuda(), gr.bg, gr.Z, gr.rows,
                                 weights=torch.from_numpy(w).cuda()))
    lib.decode_batch(jobs)
    for gr, jb, w in zip(groups, jobs, ws):
        g = library_graph(gr.bg, gr.Z, gr.rows)
        ref = oracle.decode_i8(g, gr.batch.q, wq=w, n_threads=4)
        assert (jb.out_bits.cpu().numpy() == ref[0]).all()
        assert (jb.out_iters.cpu().numpy() == ref[1]).all()


def test_small_lift_wave_tasks_random_lifts(lib):
    """Lifts up to 64 (one wave per task, six tasks of any shapes to a
    workgroup) mixed with larger ones, over lifts outside the standard set:
    every job equals decoding it alone, with and without early exit."""
    import random
    rng = random.Random(7)
    lifts = sorted({8 * rng.randint(1, 8) for _ in range(10)} | {8, 40, 56, 120, 200})
    for bg in (1, 2):
        for Z in lifts:
            lib.register(make_graph(bg, Z))
    groups = make_mixed(240, 1.25, seed=11, lifts=tuple(lifts))
    assert any(gr.Z <= 64 for gr in groups) and any(gr.Z > 64 for gr in groups)
    for ee in (True, False):
        jobs = _jobs(lib, groups)
        lib.decode_batch(jobs, early_exit=ee)
        for gr, jb in zip(groups, jobs):
            got = (jb.out_bits.cpu().numpy(), jb.out_iters.cpu().numpy(),
                   jb.out_ok.cpu().numpy().astype(bool))
            alone = _alone(lib, gr, early_exit=ee)
            for a, b in zip(got, alone):
                assert (a == b).all(), (ee, gr.bg, gr.Z, gr.rows)


def test_async_launches_reuse_stream_buffers(lib):
    # back-to-back asynchronous launches with no synchronisation between
    # them, on one stream and on two: launches of up to 32 MiB share a
    # per-stream buffer that grows (small, larger, small again), a larger
    # launch allocates its own; every result equals the oracle's
    small = [(2, 64, 42, 3), (1, 32, 20, 5)]
    larger = [(1, 384, 46, 6), (2, 128, 30, 9)]
    big = [(1, 384, 46, 2048)]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    plan = [(s1, small, 1000), (s1, larger, 1010), (s1, small, 1020), (s2, small, 1030),
            (s1, big, 1040), (s2, larger, 1050), (s1, larger, 1060), (s2, small, 1070)]
    launched = []
    for st, shapes, seed in plan:
        jobs, batches = _shape_jobs(lib, shapes, 1.5, seed)
        nbytes = lib.decode_batch_bytes(jobs)
        assert (nbytes > 32 << 20) == (shapes is big), (shapes, nbytes)
        torch.cuda.synchronize()  # inputs uploaded; the launches below do not wait
        launched.append((shapes, jobs, batches, nbytes))
    for (st, _, _), (shapes, jobs, _, nbytes) in zip(plan, launched):
        print(f"[batch async] {len(shapes)} shapes, {nbytes} bytes", flush=True)
        assert lib.decode_batch_async(jobs, stream=st) == nbytes
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    for shapes, jobs, batches, _ in launched:
        for (bg, Z, rows, n), jb, b in zip(shapes, jobs, batches):
            idx = np.arange(n) if n <= 16 else np.sort(rng.choice(n, 12, replace=False))
            ref = oracle.decode_i8(library_graph(bg, Z, rows), b.q[idx], n_threads=8)
            got = (jb.out_bits.cpu().numpy()[idx], jb.out_iters.cpu().numpy()[idx],
                   jb.out_ok.cpu().numpy().astype(bool)[idx])
            for a, r in zip(got, ref[:3]):
                assert (a == r).all(), (bg, Z, rows, n)
