"""BPSK over AWGN and the int8 LLR quantiser for the synthetic workloads.

Per codeword i (data seed d): information bits u ~ Bernoulli(1/2) i.i.d.,
codeword c = encode(u), BPSK x = 1 - 2c (bit 0 -> +1), y = x + sigma·n with
n ~ N(0, 1), sigma^2 = 1 / (2 R 10^(Eb/N0 / 10)), R = K_b / (N - 2) (the rate
over transmitted bits). The channel LLR log P(0|y)/P(1|y) = 2y/sigma^2 is the
decoder's L_b (paper §III); the int8 form is q = clamp(round_half_away(4·2y/
sigma^2), -127, 127), i.e. LLR units of 1/4. The first two (punctured)
columns are not transmitted.

Both the information bits and the noise of codeword i come from the keyed
stream (d, i), so any subset or split of a batch reproduces.
This module is an input generator: it holds none of the decoding arithmetic.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .encoder import ElimEncoder, encode
from .graph import BaseGraph
from .prng import stream

LLR_SCALE = 4.0  # int8 LLR units per natural-log unit
_TAG_DATA = 7


def sigma2(rate: float, ebn0_db: float) -> float:
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def quantize(llr: np.ndarray, scale: float = LLR_SCALE) -> np.ndarray:
    v = np.asarray(llr, dtype=np.float64) * scale
    r = np.sign(v) * np.floor(np.abs(v) + 0.5)
    return np.clip(r, -127, 127).astype(np.int8)


@dataclasses.dataclass
class Batch:
    u: np.ndarray  # uint8 [B, K] information bits
    c: np.ndarray  # uint8 [B, N*Z] codewords
    llr: np.ndarray  # float32 [B, T] channel LLRs 2y/sigma^2
    q: np.ndarray  # int8 [B, T] quantised LLRs
    ebn0: np.ndarray  # float64 [B]


def info_bits(g: BaseGraph, data_seed: int, idx: np.ndarray) -> np.ndarray:
    out = np.empty((len(idx), g.K), dtype=np.uint8)
    for j, i in enumerate(idx):
        out[j] = stream(data_seed, _TAG_DATA, int(i)).integers(0, 2, g.K, dtype=np.uint8)
    return out


def make_batch(g: BaseGraph, n_cw: int, ebn0_db, data_seed: int, start: int = 0,
               encoder: ElimEncoder | None = None, indices=None) -> Batch:
    """Codewords start..start+n_cw-1 (or the given ``indices``) of data seed
    ``data_seed``.

    ``ebn0_db`` is a scalar or one value per codeword. The information bits
    and the noise of codeword i are drawn, in that order, from stream i.
    """
    idx = np.arange(start, start + n_cw) if indices is None else np.asarray(indices)
    n_cw = len(idx)
    ebn0 = np.broadcast_to(np.asarray(ebn0_db, dtype=np.float64), (n_cw,)).copy()
    u = np.empty((n_cw, g.K), dtype=np.uint8)
    noise = np.empty((n_cw, g.T), dtype=np.float64)
    for j, i in enumerate(idx):
        s = stream(data_seed, _TAG_DATA, int(i))
        u[j] = s.integers(0, 2, g.K, dtype=np.uint8)
        noise[j] = s.standard_normal(g.T)
    c = encoder.encode(u) if encoder is not None else encode(g, u)
    tx = c[:, g.n_punct * g.Z:]
    sig2 = np.array([sigma2(g.rate, e) for e in ebn0])
    y = (1.0 - 2.0 * tx) + np.sqrt(sig2)[:, None] * noise
    llr = 2.0 * y / sig2[:, None]
    return Batch(u=u, c=c, llr=llr.astype(np.float32), q=quantize(llr), ebn0=ebn0)


def _chunk(args):
    g, n, ebn0, seed, start = args
    return make_batch(g, n, ebn0, seed, start=start)


def make_batch_parallel(g: BaseGraph, n_cw: int, ebn0_db, data_seed: int, start: int = 0,
                        workers: int = 8) -> Batch:
    """``make_batch`` split over worker processes; the result is identical
    because every codeword is keyed by its own index."""
    if workers <= 1 or n_cw < 64:
        return make_batch(g, n_cw, ebn0_db, data_seed, start=start)
    import concurrent.futures as cf
    import multiprocessing as mp
    ebn0 = np.broadcast_to(np.asarray(ebn0_db, dtype=np.float64), (n_cw,))
    bounds = np.linspace(0, n_cw, workers + 1).astype(int)
    jobs = [(g, int(b - a), ebn0[a:b].copy(), data_seed, start + int(a))
            for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        parts = list(ex.map(_chunk, jobs))
    return Batch(u=np.concatenate([p.u for p in parts]), c=np.concatenate([p.c for p in parts]),
                 llr=np.concatenate([p.llr for p in parts]), q=np.concatenate([p.q for p in parts]),
                 ebn0=np.concatenate([p.ebn0 for p in parts]))


def noiseless_q(c: np.ndarray, g: BaseGraph, mag: int = 8) -> np.ndarray:
    """int8 LLRs of magnitude ``mag`` with the sign of each transmitted bit."""
    tx = np.asarray(c, dtype=np.int16)[:, g.n_punct * g.Z:]
    return (mag * (1 - 2 * tx)).astype(np.int8)
