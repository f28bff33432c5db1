"""The trained weighted min-sum against plain normalised min-sum (beta =
3/4) in the int8 decoder, with the committed weights of BG1 Z = 384:
held-out codewords (data seed 5, indices past the evaluation set) decode
with fewer iterations, and at 1.5 dB with fewer block errors."""
import os

import numpy as np
import pytest

from synth import make_batch, make_graph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_2009_05534_amd", "weights",
                       "nwms_bg1_z384_select.npz")
N = 1024


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_05534_amd import ldpc, nwms
    g = make_graph(1, 384)
    ldpc.register(g)
    wq, meta = nwms.load_weights(WEIGHTS)
    assert meta["graph_digest"] == g.digest() and wq.shape == (10, 46)
    return ldpc, g, torch.from_numpy(wq).cuda()


def _run(ldpc, g, w, ebn0):
    # generated in this process (no worker processes once the GPU is in use)
    b = make_batch(g, N, ebn0, data_seed=5, start=200_000)
    llr = torch.from_numpy(b.q).cuda()
    out = {}
    for name, wt in (("plain", None), ("learned", w)):
        bits, iters, ok, _ = ldpc.decode(llr, 1, 384, 46, max_iter=10, weights=wt)
        got = np.unpackbits(bits.cpu().numpy(), axis=1, bitorder="little")[:, :g.K]
        out[name] = (int((got != b.u).any(axis=1).sum()), float(iters.float().mean().item()))
    return out


def test_learned_gain_at_1p5db(setup):
    ldpc, g, w = setup
    r = _run(ldpc, g, w, 1.5)
    (e_p, it_p), (e_l, it_l) = r["plain"], r["learned"]
    # plain: about 9 % block errors; learned: almost none, ~2 iterations fewer
    assert e_l < e_p / 4, r
    assert it_l < it_p - 1.0, r


def test_learned_fewer_iterations_at_2db(setup):
    ldpc, g, w = setup
    r = _run(ldpc, g, w, 2.0)
    (e_p, it_p), (e_l, it_l) = r["plain"], r["learned"]
    assert e_l <= e_p + 2, r
    assert it_l < it_p - 0.1, r
