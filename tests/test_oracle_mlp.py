"""Pins of the learned-proposal oracle (no paper definition exists; these
check the mathematics of the network, loss and optimiser)."""
import numpy as np
import pytest

from oracle import mlp as M

rs = np.random.default_rng(5)


def _batch(T=3, n=20):
    X = rs.standard_normal((T * n, M.D_IN))
    targets = [M.softmax(rs.standard_normal(n) * 2) for _ in range(T)]
    return X, targets, n


def test_finite_differences_every_block():
    P = M.init_params(1)
    P["b1"] = rs.standard_normal(M.HIDDEN) * 0.1
    P["b2"] = rs.standard_normal(M.HIDDEN) * 0.1
    X, targets, n = _batch()
    _, g, _ = M.loss_and_grad(P, X, targets, n)
    h = 1e-6
    for name in ["W1", "b1", "W2", "b2", "w3", "b3"]:
        flat = P[name].ravel()
        idx = rs.choice(flat.size, size=min(8, flat.size), replace=False)
        for i in idx:
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[name].ravel()[i] += h
            Pm[name].ravel()[i] -= h
            num = (M.loss_and_grad(Pp, X, targets, n)[0] - M.loss_and_grad(Pm, X, targets, n)[0]) / (2 * h)
            assert abs(num - g[name].ravel()[i]) < 1e-6 * max(1.0, abs(num)), (name, i)


def test_softmax_kl_gradient_identity():
    o = rs.standard_normal(7)
    pt = M.softmax(rs.standard_normal(7))
    h = 1e-6
    for j in range(7):
        op, om = o.copy(), o.copy()
        op[j] += h
        om[j] -= h
        num = (M.kl(pt, M.softmax(op)) - M.kl(pt, M.softmax(om))) / (2 * h)
        assert abs(num - (M.softmax(o)[j] - pt[j])) < 1e-8


def test_first_adam_step_closed_form():
    P = {"w": np.array([1.0, -2.0, 0.5])}
    G = {"w": np.array([0.3, -4.0, 1e-3])}
    Z = {"w": np.zeros(3)}
    P2, M2, V2 = M.adam_step(P, G, Z, Z, 1, lr=0.01)
    # bias-corrected moments equal g and g^2: the step is lr * g / (|g| + eps)
    np.testing.assert_allclose(P2["w"], P["w"] - 0.01 * G["w"] / (np.abs(G["w"]) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(M2["w"], 0.1 * G["w"])
    np.testing.assert_allclose(V2["w"], 0.001 * G["w"] ** 2)


def test_features_whitened_and_scale_invariant():
    A = rs.standard_normal((6, 40, 5)) * np.exp(rs.standard_normal(40))[None, :, None]
    Phi = rs.standard_normal((30, M.D_SKETCH)) / 4
    F = M.features(A, Phi)
    assert F.shape == (40, M.D_IN)
    Z = F[:, :M.D_SKETCH]
    np.testing.assert_allclose(Z.T @ Z / 40, np.eye(M.D_SKETCH), atol=1e-10)
    np.testing.assert_allclose(np.sum(np.exp(F[:, -1])), 40, rtol=1e-12)
    np.testing.assert_allclose(M.features(A * 7.5, Phi), F, atol=1e-10)


def test_proposal_is_a_distribution():
    P = M.init_params(3)
    X = rs.standard_normal((25, M.D_IN))
    p = M.proposal(P, X, alpha=0.1)
    assert abs(p.sum() - 1) < 1e-12 and np.all(p >= 0.1 / 25 - 1e-15)
    # alpha = 1 is the uniform distribution, alpha = 0 the network's softmax
    np.testing.assert_allclose(M.proposal(P, X, alpha=1.0), np.full(25, 1 / 25), rtol=1e-14)
    np.testing.assert_allclose(M.proposal(P, X, alpha=0.0), M.softmax(M.forward(P, X)[0]), rtol=1e-14)


def test_proposal_nonfinite_output_gives_uniform():
    """A network whose outputs are not finite (here an infinite and a NaN
    output bias) gives the uniform distribution, the defensive part of the
    mixture, instead of NaN weights; finite outputs are untouched."""
    P = M.init_params(4)
    X = rs.standard_normal((13, M.D_IN))
    for bad in (np.nan, np.inf):
        Q = dict(P)
        Q["b3"] = np.array([bad])
        np.testing.assert_array_equal(M.proposal(Q, X, alpha=0.3), np.full(13, 1 / 13))
    p = M.proposal(P, X, alpha=0.3)
    assert abs(p.sum() - 1) < 1e-12 and not np.allclose(p, 1 / 13)

