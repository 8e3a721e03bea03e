"""The small network that proposes impact speeds for Q_RD* bracketing,
trained on the GPU by the library's own kernels (``sph_mlp_forward``,
``sph_mlp_backward``, ``sph_mlp_adam``).  Host code only standardises the
inputs, owns the device buffers and sequences the launches.
"""
from __future__ import annotations

import numpy as np
import torch

from . import sph

N_PARAMS = 4545


def glorot_params(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases, in the library's flat layout
    W1[64][4] b1[64] W2[64][64] b2[64] W3[64] b3."""
    rng = np.random.default_rng(seed)
    out = []
    for fan_out, fan_in in ((64, 4), (64, 64), (1, 64)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        out.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        out.append(np.zeros(fan_out))
    p = np.concatenate(out)
    assert p.size == N_PARAMS
    return p


class MlpProposer:
    def __init__(self, seed: int = 0, lr: float = 3e-3):
        self.P = torch.tensor(glorot_params(seed), dtype=torch.float32, device="cuda")
        self.M = torch.zeros_like(self.P)
        self.V = torch.zeros_like(self.P)
        self.G = torch.zeros_like(self.P)
        self.t = 0
        self.lr = lr
        self.mu = np.zeros(4)
        self.sd = np.ones(4)

    def _std(self, X):
        return (np.asarray(X, dtype=np.float64) - self.mu) / self.sd

    def fit(self, X, Y, epochs: int = 1500, refit_scaler: bool = True) -> float:
        """Full-batch Adam on the mean squared error; returns the final loss."""
        X = np.asarray(X, dtype=np.float64)
        if refit_scaler:
            self.mu = X.mean(0)
            self.sd = X.std(0)
            self.sd[self.sd == 0] = 1.0
        B = X.shape[0]
        Xd = torch.tensor(self._std(X), dtype=torch.float32, device="cuda").contiguous()
        Yd = torch.tensor(np.asarray(Y), dtype=torch.float32, device="cuda").contiguous()
        out = torch.empty(B, dtype=torch.float32, device="cuda")
        h1 = torch.empty((B, 64), dtype=torch.float32, device="cuda")
        h2 = torch.empty((B, 64), dtype=torch.float32, device="cuda")
        work = torch.empty(B * 129, dtype=torch.float32, device="cuda")
        for _ in range(epochs):
            self.t += 1
            sph.sph_mlp_forward(Xd, self.P, out, h1, h2)
            sph.sph_mlp_backward(Xd, Yd, self.P, out, h1, h2, work, self.G)
            sph.sph_mlp_adam(self.P, self.G, self.M, self.V, self.t, self.lr)
        sph.sph_mlp_forward(Xd, self.P, out, h1, h2)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        sph.sph_mlp_loss(out, Yd, loss)
        return float(loss.item())

    def predict(self, X) -> np.ndarray:
        Xd = torch.tensor(self._std(X), dtype=torch.float32, device="cuda").contiguous()
        out = torch.empty(Xd.shape[0], dtype=torch.float32, device="cuda")
        sph.sph_mlp_forward(Xd, self.P, out, None, None)
        return out.cpu().numpy().astype(np.float64)
