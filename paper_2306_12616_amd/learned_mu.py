"""Learned start for the chemical-potential search: data, training, checkpoints.

The network (64 inputs -> 256 -> 256 -> 1, ReLU, float32; the C ABI's
``chebdm_mlp_*``) maps a problem's Chebyshev trace moments, its electron
fraction and its scaled inverse temperature to the scaled chemical potential
mu~ at which the quadrature trace of the library's chemical-potential search
meets N_e (the search is the library's reading: the paper takes mu as an
input).  It is not in the paper either: it only supplies a guess g.  The
batched search takes Newton steps from g, growing a bracket from the points
it evaluates; a step that is undefined, leaves [-1, 1] or strays further than
delta from g, or no bracket after 8 evaluations, falls back to plain
bisection, so the result is always a point where the quadrature trace meets
N_e, never the network's output itself.

Everything numeric runs in the library's kernels: training targets and
inputs come from moments-only batched runs with bisection, and the forward,
backward and Adam passes are the library's.  This module only moves device
buffers (minibatch gathers), keeps the host-side loop and writes checkpoints
(a flat float32 file plus a JSON header).
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _binding as B

N_FEATURES = 64
FORMAT = "chebdm-mu-net-1"


def init_weights(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases; the output layer scaled by 0.1 (float32, host)."""
    rng = np.random.default_rng(seed)
    w1 = rng.uniform(-1, 1, (256, 64)) * np.sqrt(6.0 / 64)
    w2 = rng.uniform(-1, 1, (256, 256)) * np.sqrt(6.0 / 256)
    w3 = rng.uniform(-1, 1, 256) * np.sqrt(6.0 / 256) * 0.1
    flat = np.concatenate([w1.ravel(), np.zeros(256), w2.ravel(), np.zeros(256), w3, np.zeros(1)])
    assert flat.size == B.chebdm_mlp_num_params()
    return flat.astype(np.float32)


class MuNet:
    """Weights and Adam state of the network on one device."""

    def __init__(self, handle: B.Handle, weights: Optional[np.ndarray] = None, seed: int = 0):
        import torch

        self.handle = handle
        self.device = torch.device("cuda", handle.device)
        w = init_weights(seed) if weights is None else np.asarray(weights, dtype=np.float32)
        if w.size != B.chebdm_mlp_num_params():
            raise ValueError("wrong number of parameters")
        self.W = torch.from_numpy(w.copy()).to(self.device)
        self.M = torch.zeros_like(self.W)
        self.V = torch.zeros_like(self.W)
        self.G = torch.zeros_like(self.W)
        self.step = 0
        self.meta: Dict = {}

    # -- inference / training -------------------------------------------------------------------
    def predict(self, X):
        return B.chebdm_mlp_forward(self.handle, self.W, X)

    def loss(self, X, T) -> float:
        _, loss = B.chebdm_mlp_backward(self.handle, self.W, X, T, grad=self.G)
        return loss

    def train(self, X, T, epochs: int = 60, batch: int = 256, lr: float = 1e-3, seed: int = 0,
              lr_final: Optional[float] = None, log=None) -> List[float]:
        """Minibatch Adam on the mean squared error; returns the mean loss of every epoch.

        The learning rate decays geometrically from ``lr`` to ``lr_final``
        (default lr / 30) over the epochs.  Minibatches are drawn without
        replacement from a seeded permutation; the last partial one is kept.
        """
        import torch

        count = X.shape[0]
        rng = np.random.default_rng(seed)
        lr_final = lr / 30.0 if lr_final is None else lr_final
        history = []
        for ep in range(epochs):
            rate = lr * (lr_final / lr) ** (ep / max(1, epochs - 1))
            perm = torch.from_numpy(rng.permutation(count)).to(self.device)
            total, nb = 0.0, 0
            for s in range(0, count, batch):
                idx = perm[s:s + batch]
                xb = X.index_select(0, idx).contiguous()
                tb = T.index_select(0, idx).contiguous()
                _, loss = B.chebdm_mlp_backward(self.handle, self.W, xb, tb, grad=self.G,
                                                want_loss=(s + batch >= count))
                self.step += 1
                B.chebdm_mlp_adam(self.handle, self.W, self.G, self.M, self.V, self.step, lr=rate)
                if loss is not None:
                    total, nb = total + loss, nb + 1
            history.append(total / max(nb, 1))
            if log is not None:
                log(f"epoch {ep + 1}/{epochs} lr {rate:.2e} loss {history[-1]:.3e}")
        return history

    # -- checkpoints ----------------------------------------------------------------------------
    def save(self, path: str, **meta) -> None:
        """``path`` + '.bin' (W, M, V as float32) and ``path`` + '.json' (header)."""
        blob = np.concatenate([t.detach().cpu().numpy() for t in (self.W, self.M, self.V)]).astype("<f4")
        with open(path + ".bin", "wb") as f:
            f.write(blob.tobytes())
        head = {"format": FORMAT, "n_params": int(self.W.numel()), "step": int(self.step),
                "arrays": ["weights", "adam_m", "adam_v"], "dtype": "float32-le"}
        head.update(self.meta)
        head.update(meta)
        with open(path + ".json", "w") as f:
            json.dump(head, f, indent=1, sort_keys=True)

    @classmethod
    def load(cls, handle: B.Handle, path: str) -> "MuNet":
        import torch

        with open(path + ".json") as f:
            head = json.load(f)
        n = B.chebdm_mlp_num_params()
        if head.get("format") != FORMAT or head.get("n_params") != n:
            raise ValueError(f"{path}.json is not a checkpoint of this network")
        blob = np.fromfile(path + ".bin", dtype="<f4")
        if blob.size != 3 * n:
            raise ValueError(f"{path}.bin holds {blob.size} floats, expected {3 * n}")
        net = cls(handle, blob[:n])
        net.M.copy_(torch.from_numpy(blob[n:2 * n].copy()))
        net.V.copy_(torch.from_numpy(blob[2 * n:].copy()))
        net.step = int(head["step"])
        net.meta = {k: v for k, v in head.items() if k not in ("format", "n_params", "step", "arrays", "dtype")}
        return net


def make_samples(batch: B.Batch, Hs: Sequence, betas: Sequence[float], n_elecs: Sequence[float]):
    """One moments-only bisection run of ``batch``: (features, targets mu~, ok mask).

    Features are ``batch.features()`` (device, count x 64); targets are the
    scaled chemical potentials mu~ the bisection found (device float32);
    ``ok`` marks problems whose search converged (status 0).
    """
    import torch

    if batch.search_mode != 0:
        batch.set_search("bisection")
    mu, status, iters, t = batch.mu_only(Hs, betas, n_elecs, allow_errors=True)
    X = batch.features()
    _, _, mu_s, _ = batch.stats()
    T = torch.from_numpy(mu_s.astype(np.float32)).to(X.device)
    return X, T, status == 0


def collect_samples(plan: B.Batch, draw, chunks: int, log=None):
    """Training set from ``chunks`` moments-only bisection runs of one plan.

    ``draw(c)`` returns ``(Hs, betas, n_elecs)`` for chunk c, with the plan's
    sizes.  Problems whose search did not converge are dropped.  Returns
    device tensors (X: samples x 64, T: samples) in chunk order.
    """
    import torch

    Xs, Ts = [], []
    for c in range(chunks):
        Hs, betas, nes = draw(c)
        X, T, ok = make_samples(plan, Hs, betas, nes)
        keep = torch.from_numpy(np.nonzero(ok)[0]).to(X.device)
        Xs.append(X.index_select(0, keep))
        Ts.append(T.index_select(0, keep))
        del Hs
        if log is not None:
            log(f"chunk {c + 1}/{chunks}: {int(ok.sum())} of {len(ok)} samples")
    return torch.cat(Xs), torch.cat(Ts)


def search_report(batch: B.Batch, status, iters, trace, n_elecs) -> Dict:
    """Summary of one run: mean / max trace evaluations, learned-bracket share, worst |t - N_e|."""
    evals, learned, _, _ = batch.stats()
    ok = status == 0
    err = np.abs(np.asarray(trace) - np.asarray(n_elecs, dtype=np.float64))
    return {"mean_evals": float(evals.mean()), "max_evals": int(evals.max()),
            "learned_share": float(learned.mean()), "converged": int(ok.sum()),
            "max_count_err": float(err[ok].max()) if ok.any() else float("nan")}


def delta_from_residuals(residual: np.ndarray, quantile: float = 0.999, floor: float = 1e-4,
                         factor: float = 2.0) -> float:
    """How far the learned start's Newton steps may move from g before the search falls back:
    ``factor`` times a high quantile of the validation residuals |g - mu~|."""
    r = np.abs(np.asarray(residual, dtype=np.float64))
    return float(max(floor, factor * np.quantile(r, quantile)))


def load_or_none(handle: B.Handle, path: Optional[str]) -> Optional[MuNet]:
    if path and os.path.exists(path + ".json") and os.path.exists(path + ".bin"):
        return MuNet.load(handle, path)
    return None


__all__ = ["MuNet", "init_weights", "make_samples", "collect_samples", "search_report", "delta_from_residuals", "load_or_none",
           "N_FEATURES", "FORMAT"]
