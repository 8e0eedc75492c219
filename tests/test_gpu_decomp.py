"""GPU parity of the randomized t-SVD summary, tubal leverage scores and
t-CUR (Algorithm 5) against the FP64 oracle.

Low-tubal-rank test tensors are composed on the CPU from the seeded factors
(workloads) by the oracle's t-product and handed to both sides as the same
bytes, so the parity checks the decompositions alone.

Tolerances:
* singular values / leverage of an exact-rank float64 input: 1e-9 (the
  range finder is exact when r + p exceeds the rank; the rest is rounding);
* float32 inputs with noise: singular values 1e-4 relative, leverage
  1e-4 * max p (the range-finder error decays like
  (sigma_{r+p+1}/sigma_r)^(2q+1) and the float32 products add ~1e-6);
* t-CUR given the same picks: 1e-9 (float64), 1e-5 (float32), 1.1e-5
  (split bf16 products: twice the largest measured error, 5.2e-6, which is
  the split product's own) relative Frobenius error; the core is float64 on
  both sides and the randomized top-r subspace equals the exact one up to
  the gap term above.
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (n if n > 0 else 1.0)


def lowrank(n1, n2, n3, r, noise_var=0.0, salt=0):
    G1, G2, N = W.lowrank_factors(n1, n2, n3, r, noise_var=max(noise_var, 1e-30), salt=salt, dtype=np.float64)
    L = T.tprod_fft(G1, G2)
    return L + (N if noise_var > 0 else 0.0), L


@pytest.mark.parametrize("shape", [(48, 40, 8, 3), (64, 96, 7, 5), (70, 50, 16, 4)])
def test_tsvd_rand_exact_rank_f64(shape):
    n1, n2, n3, r = shape
    A, _ = lowrank(n1, n2, n3, r, salt=sum(shape))
    S_, lat, hor = api.tsvd_rand(dev(A), r, p=6, q=1, seed=3)
    _, _, _, sv = T.tsvd(A)
    np.testing.assert_allclose(S_.cpu().numpy(), sv[:, :r], rtol=1e-9, atol=1e-9 * sv.max())
    np.testing.assert_allclose(lat.cpu().numpy(), S.weights_lateral_leverage(A, r), rtol=1e-9, atol=1e-9)
    ref_h = S.weights_lateral_leverage(T.ttranspose(A), r)  # left singular slices of A
    np.testing.assert_allclose(hor.cpu().numpy(), ref_h, rtol=1e-9, atol=1e-9)
    # every Fourier slice has rank r: the scores sum to r n3
    assert abs(lat.sum().item() - r * n3) < 1e-8 * r * n3


def test_tsvd_full_rank_of_the_exact_workload():
    """The full t-SVD of the float64 exact-product workload's A (64x48x16,
    N(0,1)): r = min(n1, n2) = 48 and no power iteration, so the range
    finder spans every Fourier slice and the randomized t-SVD is exact.
    Every lateral slice then has leverage n3 (each Fourier slice of V is
    square unitary)."""
    A, _ = W.exact_pair()
    S_, lat, hor = api.tsvd_rand(dev(A), 48, p=0, q=0, seed=5)
    _, _, _, sv = T.tsvd(A)
    np.testing.assert_allclose(S_.cpu().numpy(), sv[:, :48], rtol=1e-10, atol=1e-12 * sv.max())
    np.testing.assert_allclose(lat.cpu().numpy(), S.weights_lateral_leverage(A, 48), rtol=1e-9)
    np.testing.assert_allclose(lat.cpu().numpy(), np.full(48, 16.0), rtol=1e-9)
    ref_h = S.weights_lateral_leverage(T.ttranspose(A), 48)
    np.testing.assert_allclose(hor.cpu().numpy(), ref_h, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_tsvd_rand_noisy_f32(prec):
    n1, n2, n3, r = 160, 192, 16, 6
    A, _ = lowrank(n1, n2, n3, r, noise_var=1e-3, salt=7)
    A32 = A.astype(np.float32)
    S_, lat, hor = api.tsvd_rand(dev(A32), r, p=10, q=1, seed=1, prec=prec)
    _, _, _, sv = T.tsvd(A32.astype(np.float64))
    np.testing.assert_allclose(S_.cpu().numpy(), sv[:, :r], rtol=1e-4)
    p_ref = S.normalise(S.weights_lateral_leverage(A32, r))
    p_gpu = S.normalise(lat.cpu().numpy())
    assert np.max(np.abs(p_gpu - p_ref)) < 1e-4 * p_ref.max()
    h_ref = S.normalise(S.weights_lateral_leverage(T.ttranspose(A32.astype(np.float64)), r))
    h_gpu = S.normalise(hor.cpu().numpy())
    assert np.max(np.abs(h_gpu - h_ref)) < 1e-4 * h_ref.max()


def test_tsvd_rand_rank_above_true_rank():
    # r larger than the tubal rank: the extra directions have zero singular
    # values and must not contaminate the scores
    A, _ = lowrank(40, 36, 6, 2, salt=11)
    S_, lat, _ = api.tsvd_rand(dev(A), 4, p=4, q=1, seed=2)
    _, _, _, sv = T.tsvd(A)
    np.testing.assert_allclose(S_.cpu().numpy()[:, :2], sv[:, :2], rtol=1e-9)
    assert np.all(S_.cpu().numpy()[:, 2:] < 1e-6 * sv.max())
    np.testing.assert_allclose(lat.cpu().numpy(), S.weights_lateral_leverage(A, 2), rtol=1e-7, atol=1e-9)


def _user_weights(n, seed):
    return W.lognormal_weights(n, seed=seed, zeros=0, sigma=0.5)


@pytest.mark.parametrize("dtype,prec,tol", [(np.float64, "f64", 1e-9), (np.float32, "f32", 1e-5),
                                            (np.float32, "bf16x3", 1.1e-5)])
@pytest.mark.parametrize("mode", ["iid", "bernoulli", "uniform"])
def test_tcur_with_user_picks_matches_oracle(dtype, prec, tol, mode):
    n1, n2, n3, r, c, l = 72, 90, 8, 4, 24, 20
    A, _ = lowrank(n1, n2, n3, r, noise_var=1e-3, salt=3)
    A = A.astype(dtype)
    wc, wr = _user_weights(n2, 1), _user_weights(n1, 2)
    if mode == "uniform":
        # uniform picks without replacement use no weights (the uniform kind)
        Z, cols, rows = api.tcur(dev(A), c, l, r, col_kind="uniform", row_kind="uniform", mode=mode, seed=9,
                                 prec=prec)
    else:
        Z, cols, rows = api.tcur(dev(A), c, l, r, col_kind="user", row_kind="user", col_w=dev(wc), row_w=dev(wr),
                                 mode=mode, seed=9, prec=prec)
    ci, cs = S.sample(wc, c, mode, seed=9, stream=0)
    ri, rsc = S.sample(wr, l, mode, seed=9, stream=1)
    gi, gs = cols.host()
    hi, hs = rows.host()
    np.testing.assert_array_equal(gi.numpy(), ci)
    np.testing.assert_array_equal(hi.numpy(), ri)
    np.testing.assert_array_equal(gs.numpy(), cs)
    np.testing.assert_array_equal(hs.numpy(), rsc)
    Zr, _ = D.tcur(A.astype(np.float64), ci, cs, ri, rsc, r=r)
    assert rel(Z.cpu().numpy(), Zr) < tol


@pytest.mark.parametrize("dtype,prec,tol", [(np.float64, "f64", 1e-9), (np.float32, "f32", 1e-5)])
def test_tcur_exact_rank_reproduces_input(dtype, prec, tol):
    A, _ = lowrank(64, 80, 16, 5, salt=5)
    A = A.astype(dtype)
    for kinds in [("lev", "lev"), ("norm2", "norm2"), ("uniform", "lev")]:
        Z, cols, rows = api.tcur(dev(A), 20, 20, 5, col_kind=kinds[0], row_kind=kinds[1], seed=4, prec=prec)
        assert rel(Z.cpu().numpy(), A) < tol, kinds


@pytest.mark.parametrize("dtype,prec,tol", [(np.float64, "f64", 1e-9), (np.float32, "f32", 1e-5),
                                            (np.float32, "bf16x3", 1.1e-5)])
@pytest.mark.parametrize("c,l,n3", [(64, 60, 8), (60, 64, 7), (66, 60, 8), (40, 70, 5)])
def test_tcur_core_paths_match_oracle(dtype, prec, tol, c, l, n3):
    """Cores with l, c <= 64 take the fused one-workgroup-per-slice
    pseudo-inverse, larger ones the multi-kernel range finder; both must give
    the oracle's t-CUR (odd tube lengths have no real Nyquist slice)."""
    n1, n2, r = 90, 100, 6
    A, _ = lowrank(n1, n2, n3, r, noise_var=1e-3, salt=c + l)
    A = A.astype(dtype)
    wc, wr = _user_weights(n2, 3), _user_weights(n1, 4)
    Z, cols, rows = api.tcur(dev(A), c, l, r, col_kind="user", row_kind="user", col_w=dev(wc), row_w=dev(wr),
                             mode="iid", seed=13, prec=prec)
    ci, cs = S.sample(wc, c, "iid", seed=13, stream=0)
    ri, rsc = S.sample(wr, l, "iid", seed=13, stream=1)
    np.testing.assert_array_equal(cols.host()[0].numpy(), ci)
    np.testing.assert_array_equal(rows.host()[0].numpy(), ri)
    Zr, _ = D.tcur(A.astype(np.float64), ci, cs, ri, rsc, r=r)
    assert rel(Z.cpu().numpy(), Zr) < tol


def test_tcur_leverage_picks_follow_oracle_scores():
    # The GPU draws from its range-finder leverage scores; they equal the
    # oracle's exact scores to 1e-9 here (exact rank, float64), so the picks
    # coincide with the oracle's own picks for the same seed.
    A, _ = lowrank(60, 70, 8, 4, salt=8)
    Z, cols, rows = api.tcur(dev(A), 16, 14, 4, col_kind="lev", row_kind="lev", seed=21, prec="f64")
    ci, cs = S.sample_iid(S.weights_lateral_leverage(A, 4), 16, seed=21, stream=0)
    gi, gs = cols.host()
    np.testing.assert_array_equal(gi.numpy(), ci)
    np.testing.assert_allclose(gs.numpy(), cs, rtol=1e-9)
    C = A[:, ci, :] * cs[None, :, None]
    ri, rsc = S.sample_iid(S.weights_horizontal_leverage(C, 4), 14, seed=21, stream=1)
    hi, hs = rows.host()
    np.testing.assert_array_equal(hi.numpy(), ri)
    Zr, _ = D.tcur(A, ci, cs, ri, rsc, r=4)
    assert rel(Z.cpu().numpy(), Zr) < 1e-9


def test_tcur_picks_only():
    A, _ = lowrank(30, 40, 4, 3, salt=12)
    Z, cols, rows = api.tcur(dev(A), 10, 8, 3, col_kind="norm2", row_kind="norm2", seed=2, prec="f64",
                             want_z=False)
    assert Z is None
    ci, _ = S.sample_iid(S.weights_norm2(A), 10, seed=2, stream=0)
    np.testing.assert_array_equal(cols.host()[0].numpy(), ci)
    ri, _ = S.sample_iid(S.horizontal_sq_norms(A), 8, seed=2, stream=1)
    np.testing.assert_array_equal(rows.host()[0].numpy(), ri)


def test_tcur_full_size_sampled_tubes():
    """The 1024x1024x128 tubal-rank-20 workload with noise of variance 1e-3,
    c = l = 200, r = 20, in float32 with split-bf16 products: picks from
    seeded user weights (identical on both sides), 64 tubes of Z checked
    against the oracle's t-CUR of its own float64 composition of the same
    factors."""
    n1, n2, n3, r, c, l = 1024, 1024, 128, 20, 200, 200
    G1, G2, N = W.lowrank_factors(n1, n2, n3, r, noise_var=1e-3)
    Ag = api.tprod(dev(G1), dev(G2), prec="f32")
    Ag += dev(N)
    wc, wr = _user_weights(n2, 31), _user_weights(n1, 32)
    Z, cols, rows = api.tcur(Ag, c, l, r, col_kind="user", row_kind="user", col_w=dev(wc), row_w=dev(wr),
                             mode="iid", seed=5, prec="bf16x3")
    Zs = Z.cpu().numpy()
    del Ag, Z
    torch.cuda.empty_cache()
    ci, cs = S.sample_iid(wc, c, seed=5, stream=0)
    ri, rsc = S.sample_iid(wr, l, seed=5, stream=1)
    np.testing.assert_array_equal(cols.host()[0].numpy(), ci)
    # Algorithm 5 reads only the picked slices: compose those from the factors
    G1d, G2d = G1.astype(np.float64), G2.astype(np.float64)
    Csl = T.tprod_fft(G1d, np.ascontiguousarray(G2d[:, ci, :])) + N[:, ci, :]
    Rsl = T.tprod_fft(np.ascontiguousarray(G1d[ri, :, :]), G2d) + N[ri, :, :]
    rs = np.random.default_rng(0)
    ii, jj = rs.integers(0, n1, 64), rs.integers(0, n2, 64)
    ref = D.tcur_tubes(Csl, Rsl, cs, ri, rsc, r, ii, jj)
    assert rel(Zs[ii, jj, :], ref) < 1.1e-5


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tcur_core_matches_oracle(prec):
    # the exported core Uhat_k = pinv_r(D S^T Chat_k) of every Fourier slice
    n1, n2, n3, r, c, l = 60, 70, 7, 4, 18, 16
    A, _ = lowrank(n1, n2, n3, r, noise_var=1e-3, salt=41)
    A = A.astype(np.float64 if prec == "f64" else np.float32)
    wc, wr = _user_weights(n2, 42), _user_weights(n1, 43)
    Z, cols, rows, (cre, cim) = api.tcur(dev(A), c, l, r, col_kind="user", row_kind="user", col_w=dev(wc),
                                         row_w=dev(wr), mode="iid", seed=3, prec=prec, want_core=True)
    ci, cs = S.sample_iid(wc, c, seed=3, stream=0)
    ri, rsc = S.sample_iid(wr, l, seed=3, stream=1)
    Zr, core_r = D.tcur(A.astype(np.float64), ci, cs, ri, rsc, r=r)
    core = cre.cpu().numpy() + 1j * cim.cpu().numpy()
    assert core.shape == core_r.shape
    crel = np.linalg.norm((core - core_r).ravel()) / np.linalg.norm(core_r.ravel())
    assert crel < (1e-7 if prec == "f64" else 1e-4)
    assert rel(Z.cpu().numpy(), Zr) < (1e-9 if prec == "f64" else 1e-5)
    # the core alone, without Z
    Z2, _, _, (cre2, cim2) = api.tcur(dev(A), c, l, r, col_kind="user", row_kind="user", col_w=dev(wc),
                                      row_w=dev(wr), mode="iid", seed=3, prec=prec, want_z=False, want_core=True)
    assert Z2 is None
    np.testing.assert_array_equal(cre2.cpu().numpy(), cre.cpu().numpy())


@pytest.mark.parametrize("row_mode", ["iid", "bernoulli"])
def test_tcur_approximate_leverage_procedure(row_mode):
    # the remark after Corollary cor:gnys-main: lateral slices uniformly
    # without replacement, then horizontal leverage computed from them; the
    # column picks are the oracle's bit for bit, the row picks those of the
    # oracle's horizontal leverage of the same C (exact rank, float64: the
    # scores agree to ~1e-10, far from any bin edge)
    n1, n2, n3, r, c, l = 64, 80, 8, 4, 16, 14
    A, _ = lowrank(n1, n2, n3, r, salt=44)
    Z, cols, rows = api.tcur(dev(A), c, l, r, col_kind="uniform", row_kind="lev", mode="uniform", row_mode=row_mode,
                             seed=17, prec="f64")
    ci, cs = S.sample_uniform_norepl(n2, c, seed=17, stream=0)
    gi, gs = cols.host()
    np.testing.assert_array_equal(gi.numpy(), ci)
    np.testing.assert_array_equal(gs.numpy(), cs)
    C = A[:, ci, :] * cs[None, :, None]
    ri, rsc = S.sample(S.weights_horizontal_leverage(C, r), l, row_mode, seed=17, stream=1)
    hi, hs = rows.host()
    np.testing.assert_array_equal(hi.numpy(), ri)
    np.testing.assert_allclose(hs.numpy(), rsc, rtol=1e-9)
    Zr, _ = D.tcur(A, ci, cs, ri, rsc, r=r)
    assert rel(Z.cpu().numpy(), Zr) < 1e-9
    assert rel(Z.cpu().numpy(), A) < 1e-9


def test_tcur_learned_kind_equals_its_weights():
    # TP_P_LEARNED computes the proposal inside the call: the same picks and
    # Z as passing tp_mlp_proposal's weights as TP_P_USER
    from paper_1704_04362_amd import learned as LP
    n1, n2, n3, r = 48, 64, 8, 3
    A, _ = lowrank(n1, n2, n3, r, noise_var=1e-4, salt=45)
    A = dev(A.astype(np.float32))
    net = LP.Trainer()
    phi = LP.sketch_matrix(n1, n3, seed=5)
    w = api.mlp_proposal(net.params, A, phi, alpha=0.1)
    Z1, c1, r1 = api.tcur(A, 16, 12, r, col_kind="learned", row_kind="lev", mlp=(net.params, phi, 0.1), seed=6,
                          prec="f32")
    Z2, c2, r2 = api.tcur(A, 16, 12, r, col_kind="user", col_w=w, row_kind="lev", seed=6, prec="f32")
    np.testing.assert_array_equal(c1.host()[0].numpy(), c2.host()[0].numpy())
    np.testing.assert_array_equal(r1.host()[0].numpy(), r2.host()[0].numpy())
    np.testing.assert_array_equal(Z1.cpu().numpy(), Z2.cpu().numpy())


@pytest.mark.parametrize("dtype,prec,tol", [(np.float64, "f64", 1e-7), (np.float32, "f32", 2e-5)])
def test_tsvd_rand_rank_r_approximation(dtype, prec, tol):
    # tubal rank 5 plus noise of variance 1e-10: a gap after the 5th singular
    # value of every Fourier slice, so the leading subspaces, the truncation
    # A_r = U * S * V^T and the singular values are unique; the range finder
    # (p = 10, q = 1) captures them to the noise level
    n1, n2, n3, r = 70, 60, 8, 5
    G1, G2, N = W.lowrank_factors(n1, n2, n3, r, noise_var=1e-10, salt=46, dtype=np.float64)
    A = T.tprod_fft(G1, G2) + N
    U, Sv, V, Z = api.tsvd_rand_factors(dev(A.astype(dtype)), r, prec=prec)
    Ur, Sr, Vr, svr = T.tsvd(A, r)
    Ar = T.tprod_fft(T.tprod_fft(Ur, Sr), T.ttranspose(Vr))
    Z, U, V = (x.cpu().numpy().astype(np.float64) for x in (Z, U, V))
    assert rel(Z, Ar) < tol
    np.testing.assert_allclose(Sv.cpu().numpy(), svr[:, :r], rtol=tol)
    # t-orthonormal factors and the projectors onto the leading subspaces
    assert rel(T.tprod_fft(T.ttranspose(U), U), T.teye(r, n3)) < tol
    assert rel(T.tprod_fft(T.ttranspose(V), V), T.teye(r, n3)) < tol
    P, Pr = T.tprod_fft(U, T.ttranspose(U)), T.tprod_fft(Ur, T.ttranspose(Ur))
    assert rel(P, Pr) < 10 * tol
    Q, Qr = T.tprod_fft(V, T.ttranspose(V)), T.tprod_fft(Vr, T.ttranspose(Vr))
    assert rel(Q, Qr) < 10 * tol


@pytest.mark.parametrize("r", [12, 5])
def test_tsvd_rand_slices_basis_is_tcx(r):
    # with the picked lateral slices as the basis and no power iteration the
    # result is the t-CX projection C C^+ A (Algorithm 4), truncated to
    # tubal rank r
    n1, n2, n3, c = 50, 66, 6, 12
    A, _ = lowrank(n1, n2, n3, 7, noise_var=1e-3, salt=47)
    Ad = dev(A)
    picks = api.tsample("uniform", c, mode="uniform", seed=8, n=n2)
    idx, sc = picks.host()
    U, Sv, V, Z = api.tsvd_rand_factors(Ad, r, q=0, picks=picks, prec="f64")
    Zx = D.tcx(A, idx.numpy(), sc.numpy())
    Ux, Sx, Vx, _ = T.tsvd(Zx, r)
    want = T.tprod_fft(T.tprod_fft(Ux, Sx), T.ttranspose(Vx))
    assert rel(Z.cpu().numpy(), want) < 1e-9
