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


def assert_grad_close(got, ref, spread):
    """Element by element: |got - ref| <= 1e-4 * (|ref| + max|ref|) + 4 * spread.

    The kernels run in fp32 (unit roundoff u = 2^-24) through the whole
    unrolled layered recurrence; each gradient element is a sum over
    codewords, check rows and edges of terms whose errors scale with the
    gradient flowing through the recurrence, not with the element itself,
    which may cancel far below it (hence the max|ref| term). Min-sum's
    gradient also jumps where two magnitudes tie (the argmin edge takes the
    row's gradient), so near ties make the exact gradient itself move when
    the state moves by rounding: `spread` is how far the double oracle's
    gradient moves when only the inputs are perturbed by u (largest of
    three draws, per element), and the fp32 kernel, which rounds at every
    step, may differ by a few times that. The whole vector is also held to
    1e-4 in norm beyond the same allowance."""
    top = np.abs(ref).max()
    err = np.abs(got - ref)
    bound = 1e-4 * (np.abs(ref) + top) + 4.0 * spread
    worst = np.unravel_index(np.argmax(err / bound), err.shape)
    print(f"gradient: max |d|/max|g| = {err.max() / top:.3g}, "
          f"spread/max|g| = {spread.max() / top:.3g}", flush=True)
    assert (err <= bound).all(), f"gradient element {worst}: {got[worst]} vs {ref[worst]}"
    assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref) + 4.0 * np.linalg.norm(spread)


def oracle_spread(g, llr, c, w, lam):
    """Per element, the largest change of the double gradient over three
    relative perturbations of the inputs by 2^-24 (fp32's unit roundoff)."""
    ref = oracle.nwms_loss_grad(g, llr, c, w, iter_w=lam)[1]
    rng = np.random.default_rng(123)
    spread = np.zeros_like(ref)
    for _ in range(3):
        p = llr * (1.0 + 2.0 ** -24 * rng.standard_normal(llr.shape))
        spread = np.maximum(spread, np.abs(oracle.nwms_loss_grad(g, p, c, w, iter_w=lam)[1] - ref))
    return spread


@pytest.mark.parametrize("bg,Z,rows,T,n,ebn0,weighted", [
    (2, 16, 12, 3, 4, 1.0, False),
    (1, 32, 20, 4, 3, 1.5, False),
    (1, 384, 46, 2, 2, 1.5, False),
    (2, 16, 12, 3, 4, 1.0, True),
    (1, 32, 20, 4, 3, 1.5, True),
    # the unrolled depth the weights are trained with (10 iterations), at
    # the small shape and at the trained shape (BG1, Z = 384, all 46 rows)
    (2, 16, 42, 10, 6, 2.0, True),
    (1, 384, 46, 10, 2, 2.5, True),
])
def test_loss_grad_match_oracle(bg, Z, rows, T, n, ebn0, weighted):
    """At 10 unrolled iterations two things change. Only codewords that the
    decoder corrects are compared: on a codeword that does not converge the
    layered min-sum map keeps amplifying differences in its state, so after
    ten iterations the fp32 and the double trajectories are no longer the
    same trajectory (their losses differ by about 1 %). And the inputs are
    the unquantised channel LLRs (times 4, the int8 units): integer LLRs
    make exact and near-exact ties between magnitudes, where the min-sum
    gradient jumps (the argmin edge takes the row's gradient), and at this
    depth the exact gradient itself moves by about 7e-4 of its largest
    element when integer inputs move by 1e-7; real-valued inputs have ties
    with probability zero. At BG1 Z = 384 the sample is taken at 2.5 dB,
    where the gradient is well conditioned (near 1.75 dB fp32-size input
    changes move the exact gradient by 2 % of its largest element)."""
    from paper_2009_05534_amd import ldpc
    ldpc.register(make_graph(bg, Z))
    g = library_graph(bg, Z, rows)
    w = np.random.default_rng(5).uniform(0.5, 1.0, (T, rows)).astype(np.float32)
    b = make_batch(g, n if T < 8 else 4 * n, ebn0, data_seed=40 + Z)
    llr = b.q.astype(np.float32)  # training input: the int8 LLRs in units of 1/4
    c = b.c
    if T >= 8:
        llr = (4.0 * b.llr).astype(np.float32)
        _, _, ok, _ = oracle.decode_f64(g, llr.astype(np.float64), max_iter=T,
                                        early_exit=False, w=w.astype(np.float64))
        keep = np.nonzero(ok)[0][:n]
        assert len(keep) == n, "too few corrected codewords in the sample"
        llr, c = np.ascontiguousarray(llr[keep]), np.ascontiguousarray(c[keep])
    dl = torch.from_numpy(llr).cuda()
    dc = torch.from_numpy(c).cuda()
    dw = torch.from_numpy(w).cuda()
    # per-iteration loss weights (rising towards the last iteration), or the default
    lam = np.linspace(0.5, 1.5, T).astype(np.float32) / T if weighted else None
    dlam = torch.from_numpy(lam).cuda() if weighted else None
    loss, grad, post = ldpc.nwms_loss_grad(dl, dc, dw, bg, Z, rows, iter_w=dlam, want_llr=True)
    torch.cuda.synchronize()
    ref_loss, ref_grad = oracle.nwms_loss_grad(
        g, llr.astype(np.float64), c, w.astype(np.float64),
        iter_w=lam.astype(np.float64) if weighted else None)
    assert np.allclose(loss.cpu().numpy(), ref_loss, rtol=1e-5, atol=0)
    lam64 = lam.astype(np.float64) if weighted else None
    spread = oracle_spread(g, llr.astype(np.float64), c, w.astype(np.float64), lam64)
    # a sample whose gradient is this sensitive would make the check vacuous
    assert spread.max() <= 1e-3 * np.abs(ref_grad).max(), "ill-conditioned sample"
    gg = grad.cpu().numpy().astype(np.float64)
    assert_grad_close(gg, ref_grad, spread)
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
