"""Pins of the learned weighted min-sum oracle: forward equals the (pinned)
double-precision decoder with constant weights, and the analytic gradient
equals central finite differences of the loss."""
import numpy as np
import pytest

import oracle
from synth import make_batch, make_graph


def _bce_loss(L_list, c, scale):
    # mean over iterations and bits of BCE(sigmoid(-L/scale), c)
    tot = 0.0
    for L in L_list:
        y = L / scale
        tot += np.mean(np.where(c == 1, np.logaddexp(0, y), np.logaddexp(0, -y)))
    return tot / len(L_list)


def test_forward_matches_double_decoder():
    g = make_graph(2, 16, 12)
    b = make_batch(g, 3, 1.0, data_seed=21)
    T = 4
    w = np.full((T, g.M), 0.75)
    loss, _ = oracle.nwms_loss_grad(g, b.llr, b.c, w, scale=4.0)
    for i in range(3):
        Ls = [oracle.decode_f64(g, b.llr[i:i + 1] * 1.0, max_iter=t, early_exit=False,
                                beta=0.75, want_llr=True)[3][0] for t in range(1, T + 1)]
        assert abs(loss[i] - _bce_loss(Ls, b.c[i], 4.0)) < 1e-12


@pytest.mark.parametrize("bg,Z,M,T", [(2, 8, 10, 3), (1, 8, 8, 2)])
def test_gradient_matches_finite_differences(bg, Z, M, T):
    g = make_graph(bg, Z, M)
    b = make_batch(g, 2, 1.0, data_seed=22 + Z)
    rng = np.random.default_rng(3)
    w = rng.uniform(0.5, 1.0, (T, g.M))
    _, grad = oracle.nwms_loss_grad(g, b.llr, b.c, w)
    h = 1e-6
    checked = 0
    for t in range(T):
        for r in range(g.M):
            wp, wm = w.copy(), w.copy()
            wp[t, r] += h
            wm[t, r] -= h
            lp = oracle.nwms_loss_grad(g, b.llr, b.c, wp)[0].sum()
            lm = oracle.nwms_loss_grad(g, b.llr, b.c, wm)[0].sum()
            l0 = oracle.nwms_loss_grad(g, b.llr, b.c, w)[0].sum()
            fwd, bwd = (lp - l0) / h, (l0 - lm) / h
            if abs(fwd - bwd) > 1e-4 * max(1e-3, abs(fwd)):
                continue  # an argmin switches inside +-h: not differentiable here
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad[t, r]) <= 1e-5 * max(1e-3, abs(fd)), (t, r, fd, grad[t, r])
            checked += 1
    assert checked >= 0.9 * T * g.M
    assert np.abs(grad).max() > 0


def test_iteration_weighted_loss():
    """Per-iteration loss weights: the loss is the weighted sum of the
    per-iteration BCE means of the double decoder's posteriors, and the
    analytic gradient still equals central finite differences."""
    g = make_graph(2, 8, 10)
    b = make_batch(g, 2, 1.0, data_seed=31)
    T = 3
    lam = np.array([0.1, 0.3, 0.6])
    rng = np.random.default_rng(5)
    w = rng.uniform(0.5, 1.0, (T, g.M))
    loss, grad = oracle.nwms_loss_grad(g, b.llr, b.c, w, iter_w=lam)
    # forward: constant weights reduce to the double decoder
    wc = np.full((T, g.M), 0.75)
    lc, _ = oracle.nwms_loss_grad(g, b.llr, b.c, wc, iter_w=lam)
    for i in range(2):
        Ls = [oracle.decode_f64(g, b.llr[i:i + 1] * 1.0, max_iter=t, early_exit=False,
                                beta=0.75, want_llr=True)[3][0] for t in range(1, T + 1)]
        per_t = [_bce_loss([L], b.c[i], 4.0) for L in Ls]
        assert abs(lc[i] - float(np.dot(lam, per_t))) < 1e-12
    # last-iteration-only weights differ from the uniform loss
    l_last, _ = oracle.nwms_loss_grad(g, b.llr, b.c, wc, iter_w=np.array([0.0, 0.0, 1.0]))
    l_uni, _ = oracle.nwms_loss_grad(g, b.llr, b.c, wc)
    assert not np.allclose(l_last, l_uni)
    h = 1e-6
    checked = 0
    for t in range(T):
        for r in range(g.M):
            wp, wm = w.copy(), w.copy()
            wp[t, r] += h
            wm[t, r] -= h
            lp = oracle.nwms_loss_grad(g, b.llr, b.c, wp, iter_w=lam)[0].sum()
            lm = oracle.nwms_loss_grad(g, b.llr, b.c, wm, iter_w=lam)[0].sum()
            l0 = loss.sum()
            fwd, bwd = (lp - l0) / h, (l0 - lm) / h
            if abs(fwd - bwd) > 1e-4 * max(1e-3, abs(fwd)):
                continue
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad[t, r]) <= 1e-5 * max(1e-3, abs(fd)), (t, r, fd, grad[t, r])
            checked += 1
    assert checked >= 0.9 * T * g.M
