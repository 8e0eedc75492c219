"""GPU tests of the learned-proposal pipeline at a small scale: labels from
the randomized t-SVD against the oracle's exact leverage, bitwise
determinism and checkpoint/resume of training, and the held-out gain over
squared-norm sampling (KL to the exact distribution and t-CUR slices
needed for 1e-3 error)."""
import numpy as np
import pytest
import torch

from oracle import sampling as S

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1704_04362_amd.api")
from paper_1704_04362_amd import learned as LP  # noqa: E402
from workloads.device import learned_parts  # noqa: E402

SHAPE = (96, 128, 16)


def make(index, shape=SHAPE, rmin=3, rmax=8):
    n1, n2, n3 = shape
    G1, G2, N, r, sigma_c = learned_parts(index, n1=n1, n2=n2, n3=n3, rmin=rmin, rmax=rmax)
    A = api.tprod(G1, G2, prec="f32")
    rms = torch.linalg.vector_norm(A) / (A.numel() ** 0.5)
    A.add_(N, alpha=float(1e-4 * rms))
    return A, r, sigma_c


def dataset(indices, phi):
    feats, targets = [], []
    for t in indices:
        A, r, _ = make(t)
        feats.append(api.mlp_features(A, phi))
        targets.append(LP.leverage_scores(A, r).float())
    return torch.stack(feats), torch.stack(targets)


@pytest.fixture(scope="module")
def phi():
    return LP.sketch_matrix(SHAPE[0], SHAPE[2], seed=5)


def test_labels_match_oracle_exact_leverage():
    for t in range(4):
        A, r, _ = make(900 + t)
        lev = LP.leverage_scores(A, r).cpu().numpy()
        ref = S.weights_lateral_leverage(A.cpu().numpy().astype(np.float64), r)
        assert np.abs(lev / lev.sum() - ref / ref.sum()).sum() < 1e-3


def test_training_is_deterministic_and_resumable(phi):
    F, Tg = dataset(range(24), phi)
    a = LP.Trainer()
    a.fit(F, Tg, epochs=4, batch=8, lr=2e-3, seed=1)
    b = LP.Trainer()
    b.fit(F, Tg, epochs=4, batch=8, lr=2e-3, seed=1)
    assert torch.equal(a.params, b.params) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v)
    # resume: 3 steps, checkpoint, 3 more in a new trainer == 6 steps straight
    idx = [list(range(0, 8)), list(range(8, 16)), list(range(16, 24))] * 2
    c = LP.Trainer()
    for ids in idx:
        c.train_step(F[ids].reshape(-1, 17).contiguous(), Tg[ids].contiguous(), 1e-3)
    d = LP.Trainer()
    for ids in idx[:3]:
        d.train_step(F[ids].reshape(-1, 17).contiguous(), Tg[ids].contiguous(), 1e-3)
    ck = d.state_dict()
    e = LP.Trainer()
    e.load_state_dict(ck)
    for ids in idx[3:]:
        e.train_step(F[ids].reshape(-1, 17).contiguous(), Tg[ids].contiguous(), 1e-3)
    assert e.step == c.step == 6
    assert torch.equal(c.params, e.params) and torch.equal(c.m, e.m) and torch.equal(c.v, e.v)


def _kl(p, q):
    m = p > 0
    return float(np.sum(p[m] * (np.log(p[m]) - np.log(q[m]))))


def test_held_out_gain_over_norm_and_uniform_sampling(phi):
    """The trained network's proposal against the two cheap proposals it
    competes with: closer to the exact leverage distribution (KL) than
    squared norms and than uniform sampling, and no more slices needed for
    a 1e-3 t-CUR (median over held-out tensors)."""
    F, Tg = dataset(range(160), phi)
    tr = LP.Trainer()
    hist = tr.fit(F, Tg, epochs=30, batch=16, lr=2e-3, seed=2)
    assert hist[-1] < 0.7 * hist[0]
    kl_net, kl_nrm, kl_uni = [], [], []
    need = {"learned": [], "norm2": [], "uniform": []}
    grid = [16, 24, 32, 48, 64, 96]
    for t in range(1000, 1008):
        A, r, _ = make(t)
        lev = LP.leverage_scores(A, r).cpu().numpy()
        p = lev / lev.sum()
        o = tr.logits(api.mlp_features(A, phi)).double().cpu().numpy()
        q = np.exp(o - o.max())
        kl_net.append(_kl(p, q / q.sum()))
        nrm = api.slice_norms(A, "lateral").cpu().numpy()
        kl_nrm.append(_kl(p, nrm / nrm.sum()))
        kl_uni.append(_kl(p, np.full(p.size, 1.0 / p.size)))
        w = tr.proposal(A, phi)
        for kind in need:
            c_ok = None
            for c in grid:
                errs = []
                for s in range(5):
                    Z, _, _ = api.tcur(A, c, c, r, col_kind="user" if kind == "learned" else kind,
                                       col_w=w if kind == "learned" else None, seed=s, prec="f32")
                    errs.append(float(torch.linalg.vector_norm(Z - A) / torch.linalg.vector_norm(A)))
                if np.median(errs) <= 1e-3:
                    c_ok = c
                    break
            need[kind].append(c_ok if c_ok is not None else 10 ** 6)
    assert np.mean(kl_net) < np.mean(kl_nrm)
    assert np.mean(kl_net) < np.mean(kl_uni)
    assert np.median(need["learned"]) <= np.median(need["norm2"])
    assert np.median(need["learned"]) <= np.median(need["uniform"])
