"""Learned tubal-leverage proposal (oracle; test infrastructure only).

Not in the paper: the paper estimates leverage scores with a randomized
routine it cites but does not describe. This proposal predicts the lateral
leverage distribution of a tensor from cheap per-slice features, and the
exact scores of eq. cur-col-prob remain its reference and fallback.

Definitions (float64):
* features(A, Phi): for lateral slice j, s_j = Phi^T vec(A_{:j:}) (Phi is
  (n1 n3) x 16, vec ordering (i, k) -> i n3 + k), whitened as
  z_j = G^{-1/2} s_j sqrt(n2) with G = sum_j s_j s_j^T, and
  f_j = log(n2 a_j / sum a) with a_j = ||A_{:j:}||_F^2; the feature row is
  [z_j, f_j] (17 values).
* forward: h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), o = h2 w3 + b3
  (17 -> 128 -> 128 -> 1).
* loss per tensor: p = softmax(o over its slices), KL(p* || p), where p*
  is the tensor's leverage scores divided by their sum.
* backward: analytic gradients of the mean KL over the tensors of a batch.
* adam: Kingma & Ba's update with bias correction.

Parity unpinned by the paper (it has no such component). Pins
(tests/test_oracle_mlp.py): central finite differences of the loss for
every parameter block, the closed form of the first Adam step, the
softmax/KL gradient identity dL/do = p - p*, whitened features having
identity second moment, and invariance of the features under scaling of A.
"""

import numpy as np

D_SKETCH = 16
D_IN = D_SKETCH + 1
HIDDEN = 128


def features(A, Phi):
    A = np.asarray(A, dtype=np.float64)
    n1, n2, n3 = A.shape
    X = np.transpose(A, (1, 0, 2)).reshape(n2, n1 * n3)  # row j = vec(A_{:j:})
    S = X @ np.asarray(Phi, dtype=np.float64)
    a = np.sum(X * X, axis=1)
    G = S.T @ S
    lam, Q = np.linalg.eigh(G)
    Gih = (Q / np.sqrt(lam)[None, :]) @ Q.T
    Z = (S @ Gih) * np.sqrt(n2)
    f = np.log(n2 * a / a.sum())
    return np.concatenate([Z, f[:, None]], axis=1)


def init_params(seed):
    """He-style initialisation (seeded)."""
    g = np.random.default_rng([int(seed), 99])
    return {
        "W1": g.standard_normal((D_IN, HIDDEN)) * np.sqrt(2.0 / D_IN),
        "b1": np.zeros(HIDDEN),
        "W2": g.standard_normal((HIDDEN, HIDDEN)) * np.sqrt(2.0 / HIDDEN),
        "b2": np.zeros(HIDDEN),
        "w3": g.standard_normal(HIDDEN) * np.sqrt(1.0 / HIDDEN),
        "b3": np.zeros(1),
    }


def forward(P, X):
    z1 = X @ P["W1"] + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"] + P["b2"]
    h2 = np.maximum(z2, 0.0)
    o = h2 @ P["w3"] + P["b3"][0]
    return o, (X, z1, h1, z2, h2)


def softmax(o):
    e = np.exp(o - np.max(o))
    return e / e.sum()


def kl(p_target, p):
    m = p_target > 0
    return float(np.sum(p_target[m] * (np.log(p_target[m]) - np.log(p[m]))))


def loss_and_grad(P, X, targets, nslices):
    """Mean over tensors of KL(p* || softmax(o)); X stacks the slices of
    len(targets) tensors, nslices each, in order. Returns (loss, grads, o)."""
    o, (X_, z1, h1, z2, h2) = forward(P, X)
    T = len(targets)
    do = np.zeros_like(o)
    loss = 0.0
    for t in range(T):
        sl = slice(t * nslices, (t + 1) * nslices)
        p = softmax(o[sl])
        tsum = np.sum(targets[t])
        q = np.asarray(targets[t], dtype=np.float64) / tsum if tsum > 0 else np.zeros(nslices)
        loss += kl(q, p)
        do[sl] = (p - q) / T
    loss /= T
    g = {}
    g["w3"] = h2.T @ do
    g["b3"] = np.array([do.sum()])
    dh2 = np.outer(do, P["w3"]) * (z2 > 0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ P["W2"].T) * (z1 > 0)
    g["W1"] = X_.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return loss, g, o


def adam_step(P, G, M, V, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (P, M, V)."""
    P2, M2, V2 = {}, {}, {}
    for k in P:
        M2[k] = beta1 * M[k] + (1 - beta1) * G[k]
        V2[k] = beta2 * V[k] + (1 - beta2) * G[k] ** 2
        mh = M2[k] / (1 - beta1 ** t)
        vh = V2[k] / (1 - beta2 ** t)
        P2[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return P2, M2, V2


def proposal(P, X, alpha=0.1):
    """Sampling probabilities (1 - alpha) softmax(o) + alpha / n, the
    network's distribution mixed with the uniform one; outputs that are not
    all finite give the uniform distribution (the defensive part alone)."""
    with np.errstate(invalid="ignore", over="ignore"):
        o, _ = forward(P, X)
    if not np.all(np.isfinite(o)):
        return np.full(o.size, 1.0 / o.size)
    return (1 - alpha) * softmax(o) + alpha / o.size
