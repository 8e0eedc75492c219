"""GPU parity of t-project (Algorithm 3) and t-CX boosted by repetition
(Algorithm 4) against the FP64 oracle, through the C ABI.

Tolerances: float64 1e-10 relative Frobenius error (CholeskyQR2 against the
oracle's pseudo-inverse on well-conditioned slices); float32 1e-5 and split
bf16 products 5e-5, as for the other float32 paths. Exact-rank inputs are
reproduced to the same tolerances. t-CX is compared on the picks the GPU
drew (the oracle takes them as inputs).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import decomp as D
from oracle import sampling as S
from oracle import tensor as T

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1704_04362_amd.api")

CASES = [(np.float64, "f64", 1e-10), (np.float32, "f32", 1e-5), (np.float32, "bf16x3", 5e-5)]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    a = a.cpu().numpy() if torch.is_tensor(a) else a
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


@pytest.mark.parametrize("dtype,prec,tol", CASES)
@pytest.mark.parametrize("shape", [(40, 70, 8, 12), (65, 33, 7, 30), (70, 90, 1, 64)])
def test_tproject_matches_oracle(shape, dtype, prec, tol):
    n1, n2, n3, c = shape
    g = np.random.default_rng(sum(shape))
    X = g.standard_normal((n1, n2, n3)).astype(dtype)
    Cs = g.standard_normal((n1, c, n3)).astype(dtype)
    if c >= n1:
        pytest.skip("C of full row rank: the projector is the identity")
    Z = api.tproject(dev(X), dev(Cs), prec=prec)
    ref = D.tproject(X.astype(np.float64), Cs.astype(np.float64))
    assert rel(Z, ref) < tol


@pytest.mark.parametrize("dtype,prec,tol", CASES)
def test_tproject_repeated_and_zero_slices(dtype, prec, tol):
    # C = [B, B permuted, 0]: 12 lateral slices spanning the 5 of B (exact
    # duplicates stay exact through the transform); the projector is that
    # of B
    g = np.random.default_rng(5)
    X = g.standard_normal((36, 50, 6)).astype(dtype)
    B = g.standard_normal((36, 5, 6)).astype(dtype)
    Cs = np.concatenate([B, B[:, [3, 0, 4, 1, 2], :], B[:, :1, :], np.zeros((36, 1, 6), dtype)], axis=1)
    Z = api.tproject(dev(X), dev(Cs), prec=prec)
    ref = D.tproject(X.astype(np.float64), B.astype(np.float64))
    assert rel(Z, ref) < tol


@pytest.mark.parametrize("dtype,prec,tol", CASES)
@pytest.mark.parametrize("kind,mode,rounds", [("norm2", "iid", 1), ("uniform", "uniform", 3), ("lev", "iid", 2)])
def test_tcx_matches_oracle_on_same_picks(kind, mode, rounds, dtype, prec, tol):
    n1, n2, n3, r = 48, 80, 8, 4
    G1, G2, N = W.lowrank_factors(n1, n2, n3, r, noise_var=1e-2, salt=11, dtype=np.float64)
    A = (T.tprod_fft(G1, G2) + N).astype(dtype)
    Z, picks = api.tcx(dev(A), 8, rounds=rounds, r=r, col_kind=kind, mode=mode, seed=4, prec=prec)
    idx, _ = picks.host()
    assert len(idx) == 8 * rounds
    # round i draws from stream 16 i: the oracle's picks for identical
    # weights (none for uniform; the squared norms of the same values)
    for i in range(rounds):
        if kind == "uniform":
            want = S.sample_uniform_norepl(n2, 8, seed=4, stream=16 * i)[0]
        elif kind == "norm2":
            want = S.sample_iid(S.weights_norm2(A), 8, seed=4, stream=16 * i)[0]
        else:
            continue
        np.testing.assert_array_equal(idx.numpy()[8 * i:8 * (i + 1)], want)
    ref = D.tcx_union(A.astype(np.float64), [idx.numpy()[8 * i:8 * (i + 1)] for i in range(rounds)])
    assert rel(Z, ref) < tol


def test_tcx_exact_rank_reproduces_input():
    n1, n2, n3, r = 40, 60, 6, 3
    G1, G2, _ = W.lowrank_factors(n1, n2, n3, r, noise_var=1e-30, salt=12, dtype=np.float64)
    A = T.tprod_fft(G1, G2)
    Z, _ = api.tcx(dev(A), 6, rounds=2, r=r, col_kind="lev", mode="iid", seed=1, prec="f64")
    assert rel(Z, A) < 1e-10


def test_tcx_rounds_boost_and_picks_follow_weights():
    # the union of three rounds is never worse than its first round, and the
    # i.i.d. picks of every round equal the oracle's draws for the same
    # weights and stream
    n1, n2, n3, r = 32, 64, 4, 6
    g = np.random.default_rng(2)
    A = T.tprod_fft(g.standard_normal((n1, r, n3)), g.standard_normal((r, n2, n3))) + 0.3 * g.standard_normal(
        (n1, n2, n3))
    w = W.lognormal_weights(n2, seed=9)
    Z3, p3 = api.tcx(dev(A), 5, rounds=3, col_kind="user", col_w=dev(w), mode="iid", seed=7, prec="f64")
    Z1, p1 = api.tcx(dev(A), 5, rounds=1, col_kind="user", col_w=dev(w), mode="iid", seed=7, prec="f64")
    i3, i1 = p3.host()[0].numpy(), p1.host()[0].numpy()
    np.testing.assert_array_equal(i3[:5], i1)
    for i in range(3):
        ref, _ = S.sample(w, 5, "iid", seed=7, stream=16 * i)
        np.testing.assert_array_equal(i3[5 * i:5 * (i + 1)], ref)
    assert rel(Z3, A) <= rel(Z1, A) + 1e-12


# More than 64 lateral slices: the basis comes from the block Jacobi on the
# rows of Chat_k^H (float32 data). The Jacobi stops when every row inner
# product is below 1e-6 of the larger squared row norm, so the basis is
# orthonormal to ~1e-6 and the projection carries ~1e-5 relative error;
# split bf16 products add theirs.
WIDE = [(np.float32, "f32", 2e-5), (np.float32, "bf16x3", 5e-5)]


@pytest.mark.parametrize("dtype,prec,tol", WIDE)
@pytest.mark.parametrize("shape", [(300, 250, 8, 100), (150, 200, 5, 65), (130, 90, 1, 90)])
def test_tproject_wide_matches_oracle(shape, dtype, prec, tol):
    n1, n2, n3, c = shape
    g = np.random.default_rng(sum(shape) + 3)
    X = g.standard_normal((n1, n2, n3)).astype(dtype)
    Cs = g.standard_normal((n1, c, n3)).astype(dtype)
    Z = api.tproject(dev(X), dev(Cs), prec=prec)
    ref = D.tproject(X.astype(np.float64), Cs.astype(np.float64))
    assert rel(Z, ref) < tol


def test_tproject_wide_repeated_slices():
    # 96 lateral slices spanning 40: repeats and a zero slice project onto
    # the span of the 40 (their singular values are rounding residue, below
    # the cut)
    g = np.random.default_rng(6)
    X = g.standard_normal((120, 70, 6)).astype(np.float32)
    B = g.standard_normal((120, 40, 6)).astype(np.float32)
    Cs = np.concatenate([B, B[:, ::-1, :], B[:, :15, :], np.zeros((120, 1, 6), np.float32)], axis=1)
    Z = api.tproject(dev(X), dev(Cs), prec="f32")
    ref = D.tproject(X.astype(np.float64), B.astype(np.float64))
    assert rel(Z, ref) < 2e-5


@pytest.mark.parametrize("kind,mode,rounds", [("norm2", "iid", 2), ("uniform", "uniform", 1)])
def test_tcx_wide_matches_oracle(kind, mode, rounds):
    n1, n2, n3, r = 200, 240, 8, 6
    G1, G2, N = W.lowrank_factors(n1, n2, n3, r, noise_var=1e-2, salt=13, dtype=np.float64)
    A = (T.tprod_fft(G1, G2) + N).astype(np.float32)
    c = 80 if rounds == 1 else 45
    Z, picks = api.tcx(dev(A), c, rounds=rounds, r=r, col_kind=kind, mode=mode, seed=5, prec="f32")
    idx, _ = picks.host()
    assert len(idx) == c * rounds
    ref = D.tcx_union(A.astype(np.float64), [idx.numpy()[c * i:c * (i + 1)] for i in range(rounds)])
    assert rel(Z, ref) < 2e-5


def test_tcx_at_c200_on_the_tcur_workload_sampled_tubes():
    """t-CX with c = 200 uniform picks of the 1024x1024x128 tensor of tubal
    rank 20 plus N(0, 1e-3) noise, in float32 with split bf16 products: 64
    tubes of Z against the oracle's projection of the same tubes
    (Algorithm 3 on the picked slices), composed in float64 from the same
    factors.

    Tolerance: 180 of the 200 directions of every Chat_k are noise, with
    singular values ~1e-4 of the largest, the float32 resolution of the
    slices themselves (the input is float32). The part of Z along them is
    fixed only to within the noise, whose projection is ~2.5e-4 of ||A||
    (noise floor 6.25e-4 of ||A||, 180 of 1024 directions), so Z is checked
    to 1e-3, and the approximation error ||A - Z|| / ||A|| on the tubes, the
    quantity the method is judged by (~5e-4 here, at the noise floor), to
    5e-5 of the oracle's, the split bf16 bar."""
    n1, n2, n3, r, c = 1024, 1024, 128, 20, 200
    G1, G2, N = W.lowrank_factors(n1, n2, n3, r, noise_var=1e-3)
    Ag = api.tprod(dev(G1), dev(G2), prec="f32")
    Ag += dev(N)
    Z, picks = api.tcx(Ag, c, rounds=1, col_kind="uniform", mode="uniform", seed=3, prec="bf16x3")
    Zs = Z.cpu().numpy()
    del Ag, Z
    torch.cuda.empty_cache()
    idx = picks.host()[0].numpy()
    np.testing.assert_array_equal(idx, S.sample_uniform_norepl(n2, c, seed=3, stream=0)[0])
    rs = np.random.default_rng(1)
    ii, jj = rs.integers(0, n1, 64), rs.integers(0, n2, 64)
    jcols = np.unique(jj)
    G1d, G2d = G1.astype(np.float64), G2.astype(np.float64)
    Csl = T.tprod_fft(G1d, np.ascontiguousarray(G2d[:, idx, :])) + N[:, idx, :]
    Xcols = T.tprod_fft(G1d, np.ascontiguousarray(G2d[:, jcols, :])) + N[:, jcols, :]
    ref = D.tproject_tubes(Csl, Xcols, jcols, ii, jj)
    got = Zs[ii, jj, :]
    assert rel(got, ref) < 1e-3
    pos = {int(j): t for t, j in enumerate(jcols)}
    At = Xcols[ii, [pos[int(j)] for j in jj], :]
    e_gpu, e_ref = rel(got, At), rel(ref, At)
    assert abs(e_gpu - e_ref) < 5e-5, (e_gpu, e_ref)
