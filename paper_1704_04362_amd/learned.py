"""Learned lateral-leverage proposal: training driver and sampling weights.

The network (17 -> 128 -> 128 -> 1, fp16 matrix cores) maps per-slice
features of a tensor to logits whose softmax over the lateral slices
predicts the tubal leverage distribution (eq. cur-col-prob); the labels are
the leverage scores of the randomized t-SVD of the same tensors. All
arithmetic runs in libtprod's kernels (features, forward, backward, Adam,
t-SVD); this module orders the calls, batches the data and keeps the state.

The proposal never replaces the exact scores as the reference: it is mixed with
the uniform distribution (alpha) so that no slice becomes unreachable, and
callers can always fall back to the exact leverage kind of tp_tcur.
"""
import numpy as np
import torch

from . import api

D_SKETCH = 16
N_FEATURES = 17


def sketch_matrix(n1, n3, seed=0, device="cuda"):
    """Gaussian (n1 n3) x 16 sketch with N(0, 1/16) entries (the scale
    cancels in the whitening)."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return torch.randn((n1 * n3, D_SKETCH), generator=g, device=device, dtype=torch.float32) / 4


def leverage_scores(A, r, p=10, q=1, seed=0, prec="f32"):
    """Unnormalised lateral tubal leverage scores (float64, length n2) from the
    randomized t-SVD: the training labels."""
    _, lev, _ = api.tsvd_rand(A, r, p=p, q=q, seed=seed, prec=prec)
    return lev


class Trainer:
    """Parameters (float32 master copy), Adam moments and step count of one
    network. state_dict()/load_state_dict() checkpoint all of it, so a run
    resumed from a checkpoint continues bit for bit."""

    def __init__(self, init=None, device="cuda"):
        if init is None:
            g = np.random.default_rng([1704, 4362])
            init = {
                "W1": g.standard_normal((N_FEATURES, 128)) * np.sqrt(2.0 / N_FEATURES),
                "b1": np.zeros(128),
                "W2": g.standard_normal((128, 128)) * np.sqrt(2.0 / 128),
                "b2": np.zeros(128),
                "w3": g.standard_normal(128) * np.sqrt(1.0 / 128),
                "b3": np.zeros(1),
            }
        self.params = api.mlp_pack(init, device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0

    def state_dict(self):
        return {"params": self.params.clone(), "m": self.m.clone(), "v": self.v.clone(), "step": self.step}

    def load_state_dict(self, st):
        self.params.copy_(st["params"])
        self.m.copy_(st["m"])
        self.v.copy_(st["v"])
        self.step = int(st["step"])

    def train_step(self, feat, target, lr):
        """One Adam step on a batch: feat ((T n) x 17), target (T x n)
        leverage scores. Returns the loss as a device tensor."""
        self.step += 1
        loss, _ = api.mlp_train_step(self.params, self.m, self.v, self.step, lr, feat, target)
        return loss

    def fit(self, feats, targets, epochs, batch=16, lr=2e-3, seed=0, log=None, log_every=1):
        """Epochs over a set of tensors: feats (T, n, 17) and targets (T, n),
        device tensors; each epoch visits the tensors in a seeded random order
        in batches of `batch` tensors. Returns the per-epoch mean losses."""
        T = feats.shape[0]
        g = torch.Generator()
        g.manual_seed(int(seed))
        history = []
        for ep in range(epochs):
            order = torch.randperm(T, generator=g).to(feats.device)
            losses = []
            for b0 in range(0, T, batch):
                idx = order[b0:b0 + batch]
                f = feats.index_select(0, idx).reshape(-1, N_FEATURES).contiguous()
                t = targets.index_select(0, idx).contiguous()
                losses.append(self.train_step(f, t, lr))
            history.append(float(torch.stack(losses).mean().item()))
            if log and (ep + 1) % log_every == 0:
                log(f"train epoch {ep + 1}/{epochs} loss {history[-1]:.4f}")
        return history

    def logits(self, feat):
        return api.mlp_forward(self.params, feat)

    def proposal(self, A, phi, alpha=0.4):
        """float64 sampling weights for A's lateral slices: (1 - alpha) times
        the network's softmax plus alpha / n2. The default weight was chosen
        on generated tensors outside the training and held-out sets (the
        largest share of them needing no more slices than uniform sampling
        for a 1e-3 t-CUR, among 0.1 ... 0.5)."""
        return api.mlp_proposal(self.params, A, phi, alpha)
