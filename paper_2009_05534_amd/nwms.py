"""Training and use of the learned (neural) weighted min-sum decoder.

The min-sum correction factor becomes one multiplier w[t][r] per iteration
t and block row r. The weights are trained in fp32 by the library's unrolled
forward and hand-written backward kernels (``ldpc.nwms_loss_grad``) with Adam
on the host, then quantised to Q1.7 (w_q = clamp(round(128 w), 0, 255)) for
the int8 decoder, where iteration t of the decode uses row min(t, iters) of
w_q. The plain normalised min-sum (beta = 3/4, w_q = 96) is both the starting
point and the reference the learned weights are judged against.
"""
from __future__ import annotations

import dataclasses
import json
import os

import numpy as np

W_MAX = 255 / 128  # largest multiplier the Q1.7 int8 path can represent


def quantize_weights(w: np.ndarray) -> np.ndarray:
    """Q1.7 multipliers for the int8 decoder."""
    return np.clip(np.round(np.asarray(w, np.float64) * 128.0), 0, 255).astype(np.uint8)


@dataclasses.dataclass
class Adam:
    """Adam (Kingma & Ba, 2015) on a small parameter array."""
    lr: float = 1e-2
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: np.ndarray | None = None
    v: np.ndarray | None = None

    def step(self, p: np.ndarray, g: np.ndarray) -> np.ndarray:
        if self.m is None:
            self.m = np.zeros_like(p)
            self.v = np.zeros_like(p)
        self.t += 1
        self.m = self.beta1 * self.m + (1 - self.beta1) * g
        self.v = self.beta2 * self.v + (1 - self.beta2) * g * g
        mh = self.m / (1 - self.beta1 ** self.t)
        vh = self.v / (1 - self.beta2 ** self.t)
        return p - self.lr * mh / (np.sqrt(vh) + self.eps)


class Trainer:
    """Trains w [n_iter, rows] on device-resident batches of int8 LLRs
    (used as fp32 in LLR units of 1/scale) and transmitted codewords."""

    def __init__(self, bg: int, Z: int, rows: int, n_iter: int = 10, lr: float = 1e-2,
                 beta0: float = 0.75, scale: float = 4.0, device="cuda:0", iter_w=None):
        self.bg, self.Z, self.rows, self.n_iter, self.scale = bg, Z, rows, n_iter, scale
        # per-iteration loss weights (None: the mean over iterations)
        self.iter_w = None if iter_w is None else np.asarray(iter_w, dtype=np.float32)
        self.w = np.full((n_iter, rows), beta0, dtype=np.float64)
        self.opt = Adam(lr=lr)
        self.device = device
        self.history: list[dict] = []

    def step(self, q: np.ndarray, c: np.ndarray) -> float:
        """One Adam step on a batch; returns the mean loss."""
        import torch

        from . import ldpc
        dev = torch.device(self.device)
        llr = torch.from_numpy(np.ascontiguousarray(q, dtype=np.float32)).to(dev)
        cb = torch.from_numpy(np.ascontiguousarray(c, dtype=np.uint8)).to(dev)
        w = torch.from_numpy(self.w.astype(np.float32)).to(dev)
        lam = None if self.iter_w is None else torch.from_numpy(self.iter_w).to(dev)
        loss, grad, _ = ldpc.nwms_loss_grad(llr, cb, w, self.bg, self.Z, self.rows,
                                            scale=self.scale, iter_w=lam)
        n = q.shape[0]
        g = grad.cpu().numpy().astype(np.float64) / n
        self.w = np.clip(self.opt.step(self.w, g), 0.0, W_MAX)
        lv = float(loss.mean().item())
        self.history.append({"step": self.opt.t, "loss": lv, "grad_norm": float(np.linalg.norm(g))})
        return lv

    @property
    def wq(self) -> np.ndarray:
        return quantize_weights(self.w)

    def save(self, path: str, graph_digest: str, extra: dict | None = None) -> None:
        """Checkpoint: weights (fp32 and Q1.7), Adam state and metadata."""
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        np.savez(path, w=self.w, wq=self.wq, adam_m=self.opt.m if self.opt.m is not None else 0,
                 adam_v=self.opt.v if self.opt.v is not None else 0, adam_t=self.opt.t)
        meta = {"bg": self.bg, "Z": self.Z, "rows": self.rows, "n_iter": self.n_iter,
                "scale": self.scale, "graph_digest": graph_digest, "adam_lr": self.opt.lr,
                "steps": self.opt.t}
        if extra:
            meta.update(extra)
        with open(os.path.splitext(path)[0] + ".json", "w") as f:
            json.dump(meta, f, indent=1)

    @classmethod
    def load(cls, path: str, device="cuda:0") -> "Trainer":
        with open(os.path.splitext(path)[0] + ".json") as f:
            meta = json.load(f)
        tr = cls(meta["bg"], meta["Z"], meta["rows"], meta["n_iter"], lr=meta["adam_lr"],
                 scale=meta["scale"], device=device)
        d = np.load(path, allow_pickle=False)
        tr.w = d["w"]
        tr.opt.t = int(d["adam_t"])
        if tr.opt.t:
            tr.opt.m, tr.opt.v = d["adam_m"], d["adam_v"]
        return tr


def load_weights(path: str) -> tuple[np.ndarray, dict]:
    """Q1.7 weights [n_iter, rows] and metadata of a checkpoint."""
    with open(os.path.splitext(path)[0] + ".json") as f:
        meta = json.load(f)
    return np.load(path, allow_pickle=False)["wq"], meta
