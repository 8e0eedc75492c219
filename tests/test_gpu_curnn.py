"""GPU parity of robust tensor PCA (Algorithm 7 as stated, eq. tlow7) and
CUR t-NN (Algorithm 6) against the FP64 oracle, through the C ABI.

Inputs are low-tubal-rank tensors with sparse +-5 spikes (robust PCA) or
with a share of entries unobserved (completion), composed on the CPU by the
oracle's t-product from seeded factors and handed to both sides as the same
float32 bytes. CUR t-NN is compared on the picks the GPU drew (the oracle
takes them as inputs).

Tolerances: ADMM iterates 1e-4 relative Frobenius error (the float32 error
of each t-SVT, ~1e-6, carried through the iterations, as for completion);
recovered low-rank parts 1e-4 relative to the oracle's (which recovers L*
to ~1e-15 on these inputs); per-slice ranks exact (the recovered spectra
have a wide gap above the threshold).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import decomp as D
from oracle import sampling as picks_oracle
from oracle import tensor as T

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1704_04362_amd.api")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    a = a.cpu().numpy() if torch.is_tensor(a) else a
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def spiky(n1, n2, n3, r, frac=0.05, salt=0):
    G1, G2, S = W.rpca_problem(n1, n2, n3, r, spike_frac=frac, salt=salt)
    return T.tprod_fft(G1, G2), S


@pytest.mark.parametrize("shape", [(40, 36, 8, 3), (33, 50, 5, 2)])
def test_trpca_matches_oracle_iterates(shape):
    n1, n2, n3, r = shape
    Ls, S = spiky(n1, n2, n3, r, salt=1)
    X = (Ls + S + 0.05 * np.random.default_rng(3).standard_normal(Ls.shape)).astype(np.float32)
    lam = D.rpca_lambda(X.shape)
    L, E, Y, ranks = api.trpca(dev(X), lam, iters=30)
    Lr, Er, Yr, hist = D.admm_rpca(X.astype(np.float64), lam, iters=30)
    assert rel(L, Lr) < 1e-4
    assert rel(E, Er) < 1e-4
    assert rel(Y, Yr) < 1e-4
    np.testing.assert_array_equal(ranks.cpu().numpy(), hist[-1]["ranks"])


@pytest.mark.parametrize("shape", [(48, 40, 6, 2), (64, 64, 16, 4)])
def test_trpca_separates_low_rank_and_spikes(shape):
    n1, n2, n3, r = shape
    Ls, S = spiky(n1, n2, n3, r, salt=2)
    X = (Ls + S).astype(np.float32)
    L, E, Y, ranks = api.trpca(dev(X), iters=100)
    Lr = D.admm_rpca(X.astype(np.float64), D.rpca_lambda(X.shape), iters=100)[0]
    assert rel(L, Lr) < 1e-4
    assert rel(L, Ls) < 1e-4
    assert rel(E, S) < 1e-4
    assert np.all(ranks.cpu().numpy() == r)


@pytest.mark.parametrize("kinds", [("uniform", "uniform", "uniform"), ("lev", "lev", "iid"), ("norm2", "norm2", "iid")])
def test_tcur_nn_robust_pca_matches_oracle(kinds):
    n1, n2, n3, r = 48, 56, 6, 2
    Ls, S = spiky(n1, n2, n3, r, salt=3)
    X = (Ls + S).astype(np.float32)
    lam = D.rpca_lambda(X.shape)
    Lg, cols, rows = api.tcur_nn(dev(X), 24, 20, r, lam=lam, col_kind=kinds[0], row_kind=kinds[1],
                                 mode=kinds[2], seed=5, iters=100)
    ci, ri = cols.host()[0].numpy(), rows.host()[0].numpy()
    assert len(ci) == 24 and len(ri) == 20
    if kinds[2] == "uniform":
        assert len(set(ci.tolist())) == 24 and len(set(ri.tolist())) == 20
    # where both sides sample from identical weights the picks are the
    # oracle's bit for bit: no weights (uniform), and the squared norms of
    # X's slices (float64 sums of the same float32 values; equal up to
    # summation order, far from any bin edge at this seed)
    if kinds[0] == "uniform":
        np.testing.assert_array_equal(ci, picks_oracle.sample_uniform_norepl(n2, 24, seed=5, stream=0)[0])
        np.testing.assert_array_equal(ri, picks_oracle.sample_uniform_norepl(n1, 20, seed=5, stream=1)[0])
    if kinds[0] == "norm2":
        wc, wr = picks_oracle.weights_norm2(X), picks_oracle.horizontal_sq_norms(X)
        np.testing.assert_array_equal(ci, picks_oracle.sample_iid(wc, 24, seed=5, stream=0)[0])
        np.testing.assert_array_equal(ri, picks_oracle.sample_iid(wr, 20, seed=5, stream=1)[0])
    Lr, _, _ = D.cur_tnn(X.astype(np.float64), ci, ri, r=r, lam=lam, iters=100)
    assert rel(Lg, Lr) < 1e-4
    assert rel(Lg, Ls) < 1e-4


@pytest.mark.parametrize("n3", [6, 7])
def test_tcur_nn_completion_matches_oracle(n3):
    n1, n2, r = 40, 52, 2
    G1, G2, _, mask = W.completion_problem(n1, n2, n3, r, noise_var=0.0, p_obs=0.7, salt=4, dtype=np.float64)
    Ls = T.tprod_fft(G1, G2)
    X = (Ls * mask).astype(np.float32)
    Lg, cols, rows = api.tcur_nn(dev(X), 26, 22, r, mask=dev(mask), col_kind="uniform", row_kind="uniform",
                                 mode="uniform", seed=9, iters=120)
    ci, ri = cols.host()[0].numpy(), rows.host()[0].numpy()
    Lr, _, _ = D.cur_tnn(X.astype(np.float64), ci, ri, r=r, mask=mask, iters=120)
    assert rel(Lg, Lr) < 1e-4
    assert rel(Lr, Ls) < 1e-6


def test_tcur_nn_iid_picks_with_repeats():
    # IID picks may repeat a slice; W then has repeated rows and columns and
    # the pseudo-inverse handles them
    n1, n2, n3, r = 30, 34, 4, 2
    Ls, S = spiky(n1, n2, n3, r, salt=5)
    X = (Ls + S).astype(np.float32)
    lam = D.rpca_lambda(X.shape)
    Lg, cols, rows = api.tcur_nn(dev(X), 20, 18, r, lam=lam, col_kind="norm2", row_kind="norm2", mode="iid",
                                 seed=2, iters=100)
    ci, ri = cols.host()[0].numpy(), rows.host()[0].numpy()
    Lr, _, _ = D.cur_tnn(X.astype(np.float64), ci, ri, r=r, lam=lam, iters=100)
    assert rel(Lg, Lr) < 1e-4
