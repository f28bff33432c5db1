"""Learned weighted min-sum on the GPU (fp32 forward and hand-written
backward kernels, through the C ABI) against the double-precision oracle."""
import numpy as np
import pytest

import oracle
from libgraph import library_graph
from synth import make_batch, make_graph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def assert_grad_close(got, ref):
    """Element by element: |got - ref| <= 1e-4 * max(|ref|, 1e-3 * max|ref|)
    (fp32 kernels against the double oracle; the floor covers weights whose
    gradient is a cancelling sum far below the largest one)."""
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    err = np.abs(got - ref) / scale
    worst = np.unravel_index(np.argmax(err), err.shape)
    assert err.max() <= 1e-4, f"gradient element {worst}: {got[worst]} vs {ref[worst]}"


@pytest.mark.parametrize("bg,Z,rows,T,n,ebn0,weighted", [
    (2, 16, 12, 3, 4, 1.0, False),
    (1, 32, 20, 4, 3, 1.5, False),
    (1, 384, 46, 2, 2, 1.5, False),
    (2, 16, 12, 3, 4, 1.0, True),
    (1, 32, 20, 4, 3, 1.5, True),
    # the unrolled depth the weights are trained with (10 iterations), at
    # the small shape and at the trained shape (BG1, Z = 384, all 46 rows)
    (2, 16, 42, 10, 6, 1.0, True),
    (1, 384, 46, 10, 2, 1.25, True),
])
def test_loss_grad_match_oracle(bg, Z, rows, T, n, ebn0, weighted):
    from paper_2009_05534_amd import ldpc
    ldpc.register(make_graph(bg, Z))
    g = library_graph(bg, Z, rows)
    b = make_batch(g, n, ebn0, data_seed=40 + Z)
    llr = b.q.astype(np.float32)  # training input: the int8 LLRs in units of 1/4
    w = np.random.default_rng(5).uniform(0.5, 1.0, (T, rows)).astype(np.float32)
    dl = torch.from_numpy(llr).cuda()
    dc = torch.from_numpy(b.c).cuda()
    dw = torch.from_numpy(w).cuda()
    # per-iteration loss weights (rising towards the last iteration), or the default
    lam = np.linspace(0.5, 1.5, T).astype(np.float32) / T if weighted else None
    dlam = torch.from_numpy(lam).cuda() if weighted else None
    loss, grad, post = ldpc.nwms_loss_grad(dl, dc, dw, bg, Z, rows, iter_w=dlam, want_llr=True)
    torch.cuda.synchronize()
    ref_loss, ref_grad = oracle.nwms_loss_grad(
        g, llr.astype(np.float64), b.c, w.astype(np.float64),
        iter_w=lam.astype(np.float64) if weighted else None)
    assert np.allclose(loss.cpu().numpy(), ref_loss, rtol=1e-5, atol=0)
    gg = grad.cpu().numpy().astype(np.float64)
    assert_grad_close(gg, ref_grad)
    # final posteriors equal the double decoder with the same weights
    _, _, _, ref_post = oracle.decode_f64(g, llr.astype(np.float64), max_iter=T,
                                          early_exit=False, w=w.astype(np.float64),
                                          want_llr=True)
    p = post.cpu().numpy().astype(np.float64)
    assert (np.abs(p - ref_post) <= 1e-4 * np.maximum(np.abs(ref_post), 1.0)).all()


def test_training_step_reduces_loss():
    # a few Adam steps on a fixed batch lower the loss (smoke test of the
    # trainer around the kernels)
    from paper_2009_05534_amd import ldpc, nwms
    full = make_graph(2, 64)
    ldpc.register(full)
    b = make_batch(full, 64, 1.0, data_seed=41)
    tr = nwms.Trainer(2, 64, full.M, n_iter=5, lr=0.05)
    first = tr.step(b.q, b.c)
    for _ in range(20):
        last = tr.step(b.q, b.c)
    assert last < first
    assert tr.wq.shape == (5, full.M) and tr.wq.dtype == np.uint8
