"""Rank predictor for learned-rank rounding: host-side driver of the MLP kernels.

The network (three hidden tanh layers of 64 units, FP32) is trained and
evaluated only by the library's own HIP kernels (qt_mlp_train_step,
qt_mlp_infer); this module marshals arguments and runs the epoch loop.
Training data are the rank logs written by the solver in SVD-truncated sketch
mode (features of bond k at step s of iteration t, label = the class of the
rank kept at that bond and step in iteration t + 1).  Classes stand for ranks
8 (c + 1), the coarse rank lattice of Sec. 5.1 with base rank 8.
"""
from __future__ import annotations

import numpy as np

from . import inputs, qtt

N_CLS = 8          # ranks 8 .. 64 (default: rank caps up to 64)


def n_classes(max_rank: int) -> int:
    """Class count whose top class (rank 8 n_cls) reaches the rank cap (at most
    32 classes, rank 256); with fewer classes the predictor could never ask for
    the capped rank and every capped learned rounding would fall back."""
    return max(2, min(32, -(-int(max_rank) // 8)))
LOSS_BETA = 1.0    # weight of the asymmetric cost term
LOSS_GAMMA = 2.0   # cost of predicting below the label


def flat_params(layers) -> np.ndarray:
    """[W0, b0, W1, b1, ...] -> the flat float32 layout of the kernels."""
    return np.concatenate([np.asarray(a, dtype=np.float32).ravel() for a in layers])


class RankPredictor:
    """MLP parameters and Adam state resident on the device."""

    def __init__(self, ctx: qtt.Context, n_cls: int = N_CLS, seed: int = 0):
        torch = qtt._torch()
        self.ctx = ctx
        self.n_cls = n_cls
        self.n_in = qtt.RANK_FEATURES
        flat = flat_params(inputs.mlp_init(self.n_in, n_cls, seed))
        assert flat.size == qtt.mlp_num_params(self.n_in, n_cls)
        self.params = torch.from_numpy(flat).to("cuda")
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.t = 0

    def train(self, X, Y, epochs: int = 300, lr: float = 3e-3, beta: float = LOSS_BETA,
              gamma: float = LOSS_GAMMA):
        """Full-batch Adam on device tensors X [n, 24] float32, Y [n] int32; returns the
        loss history (one value per epoch, read back once at the end)."""
        torch = qtt._torch()
        hist = torch.zeros(epochs, dtype=torch.float32, device="cuda")
        for e in range(epochs):
            self.t += 1
            qtt.mlp_train_step(self.ctx, self.params, self.m, self.v, self.t, X, Y, self.n_cls,
                               lr, beta, gamma, loss=hist[e:e + 1])
        self.ctx.sync()
        return hist.cpu().numpy()

    def infer(self, X, quantile: float = 0.9, rank_cap=None):
        return qtt.mlp_infer(self.ctx, self.params, X, self.n_cls, quantile, rank_cap)

    def install(self, quantile: float = 0.9, accept_factor: float = 1.0):
        """Makes QT_ROUND_LEARNED solves on this context use the predictor."""
        qtt.set_predictor(self.ctx, self.params, self.n_cls, quantile, accept_factor)
