"""Pins of the oracle's randomized decompositions."""
import numpy as np
import pytest

from oracle import decomp as D
from oracle import sampling as S
from oracle import tensor as T

rs = np.random.default_rng(4242)


def _lowrank(n1, n2, n3, r, seed=0):
    g = np.random.default_rng(seed)
    return T.tprod_bcirc(g.standard_normal((n1, r, n3)), g.standard_normal((r, n2, n3)))


def test_rtprod_full_budget_is_exact():
    A = rs.standard_normal((6, 9, 5))
    B = rs.standard_normal((9, 4, 5))
    idx, sc = S.sample_bernoulli(np.ones(9), 9, seed=0)
    assert T.rel_fro(D.rtprod(A, B, idx, sc), T.tprod_bcirc(A, B)) < 1e-13


def test_rtprod_empty_pick_is_zero():
    A = rs.standard_normal((3, 4, 2))
    B = rs.standard_normal((4, 5, 2))
    Z = D.rtprod(A, B, np.array([], dtype=np.int64), np.array([]))
    assert Z.shape == (3, 5, 2) and not Z.any()


def _gammas(A, B):
    return np.array([np.sum(T.tprod_bcirc(A[:, j:j + 1, :], B[j:j + 1, :, :]) ** 2) for j in range(A.shape[1])])


@pytest.mark.parametrize("mode", ["bernoulli", "iid"])
def test_rtprod_unbiased_with_exact_second_moment(mode):
    # Z - A*B is a sum of independent (Bernoulli) or i.i.d. (IID) terms, so its
    # mean is 0 and its expected squared norm has a closed form in
    # gamma_j = ||A_{:j:} * B_{j::}||_F^2.
    n1, n2, n4, n3, c, reps = 4, 10, 3, 4, 4, 1500
    A = rs.standard_normal((n1, n2, n3)) * np.exp(rs.standard_normal(n2))[None, :, None]
    B = rs.standard_normal((n2, n4, n3))
    w = S.weights_norm2(A)
    AB = T.tprod_bcirc(A, B)
    gam = _gammas(A, B)
    q, Ssum = S.quantize(w)
    p = np.array(q, dtype=float) / Ssum
    if mode == "bernoulli":
        pi = np.minimum(1.0, c * p)
        m = pi < 1
        expect = float(np.sum((1.0 / pi[m] - 1.0) * gam[m]))
    else:
        expect = float((np.sum(gam / p) - np.sum(AB ** 2)) / c)
    acc = np.zeros_like(AB)
    errs = []
    for seed in range(reps):
        idx, sc = S.sample(w, c, mode, seed=seed, stream=2)
        Z = D.rtprod(A, B, idx, sc)
        acc += Z
        errs.append(np.sum((Z - AB) ** 2))
    errs = np.array(errs)
    mean_err = np.mean(errs)
    assert abs(mean_err - expect) < 5 * np.std(errs) / np.sqrt(reps)
    bias = acc / reps - AB
    assert np.sum(bias ** 2) < 10 * expect / reps


def test_rtprod_meets_paper_bound_on_white_inputs():
    # Theorem theorem:matmult-main-exact with norm-squared probabilities
    # (beta = 1): E||AB - CR||_F <= ||A||_F ||B||_F / sqrt(c). Gaussian tubes
    # are spectrally flat in expectation, where the bound's proof applies.
    A = rs.standard_normal((8, 40, 6))
    B = rs.standard_normal((40, 7, 6))
    c = 10
    AB = T.tprod_bcirc(A, B)
    w = S.weights_norm2(A)
    errs = [np.linalg.norm((D.rtprod(A, B, *S.sample_bernoulli(w, c, seed=s)) - AB).ravel()) for s in range(100)]
    assert np.mean(errs) <= np.linalg.norm(A.ravel()) * np.linalg.norm(B.ravel()) / np.sqrt(c)


def test_tcx_reproduces_exact_rank():
    A = _lowrank(12, 15, 6, 3)
    w = S.weights_lateral_leverage(A, 3)
    idx, sc = S.sample_iid(w, 6, seed=1)
    assert T.rel_fro(D.tcx(A, idx, sc), A) < 1e-10


def test_tcx_is_least_squares_optimal():
    # eq. ell2reg: C * C^+ * X minimises ||X - C * Y||_F; compare with a
    # per-Fourier-slice least-squares solve and with random perturbations
    A = rs.standard_normal((8, 10, 5))
    idx = np.array([1, 4, 7])
    Z = D.tcx(A, idx, np.ones(3))
    Ah = T.fft3(A)
    Ch = Ah[:, idx, :]
    Zh = np.zeros_like(Ah)
    for k in range(5):
        Y, *_ = np.linalg.lstsq(Ch[:, :, k], Ah[:, :, k], rcond=None)
        Zh[:, :, k] = Ch[:, :, k] @ Y
    assert T.rel_fro(Z, np.real(T.ifft3(Zh))) < 1e-12
    base = np.linalg.norm((A - Z).ravel())
    C = A[:, idx, :]
    for _ in range(5):
        Yp = rs.standard_normal((3, 10, 5))
        assert np.linalg.norm((A - T.tprod_bcirc(C, Yp)).ravel()) >= base - 1e-12


def test_tcx_scale_cancels():
    A = rs.standard_normal((7, 9, 4))
    idx = np.array([0, 2, 5])
    Z1 = D.tcx(A, idx, np.ones(3))
    Z2 = D.tcx(A, idx, np.array([0.3, 5.0, 2.0]))
    assert T.rel_fro(Z2, Z1) < 1e-12


def test_tcur_reproduces_exact_rank():
    n1, n2, n3, r = 14, 16, 6, 3
    A = _lowrank(n1, n2, n3, r, seed=5)
    ci, cs = S.sample_iid(S.weights_lateral_leverage(A, r), 7, seed=2)
    C = A[:, ci, :] * cs[None, :, None]
    ri, rsc = S.sample_iid(S.weights_horizontal_leverage(C, r), 7, seed=3, stream=1)
    Z, core = D.tcur(A, ci, cs, ri, rsc, r=r)
    assert T.rel_fro(Z, A) < 1e-9
    assert core.shape == (4, 7, 7)


def test_tcur_n3_one_is_matrix_cur():
    M = rs.standard_normal((9, 3)) @ rs.standard_normal((3, 11)) + 1e-3 * rs.standard_normal((9, 11))
    ci, ri = np.array([0, 3, 5, 8]), np.array([1, 2, 6, 7])
    cs, rsc = np.array([1.0, 2.0, 0.5, 1.5]), np.array([1.0, 0.7, 1.3, 2.0])
    Z, _ = D.tcur(M[:, :, None], ci, cs, ri, rsc, r=3)
    Cm = M[:, ci] * cs
    Wm = rsc[:, None] * Cm[ri, :]
    u, s, vh = np.linalg.svd(Wm)
    Wp = vh[:3].T @ np.diag(1 / s[:3]) @ u[:, :3].T
    ref = Cm @ Wp @ (rsc[:, None] * M[ri, :])
    np.testing.assert_allclose(Z[:, :, 0], ref, atol=1e-12)


def test_pinv_r_properties():
    W = rs.standard_normal((6, 5)) + 1j * rs.standard_normal((6, 5))
    P = D.pinv_r(W)
    np.testing.assert_allclose(P, np.linalg.pinv(W), atol=1e-12)
    P2 = D.pinv_r(W, 2)
    u, s, vh = np.linalg.svd(W)
    np.testing.assert_allclose(P2, vh[:2].conj().T @ np.diag(1 / s[:2]) @ u[:, :2].conj().T, atol=1e-12)


def test_tsvt_matches_matrix_svt_of_circ():
    # the t-SVT with threshold tau is the matrix SVT of circ(M) with the same
    # tau: the DFT block-diagonalisation (eq. circ1) is a unitary similarity
    # once scaled by 1/sqrt(n3)
    M = rs.standard_normal((5, 4, 6))
    tau = 1.3
    L, ranks = D.tsvt(M, tau)
    ref, _ = D.svt_matrix(T.circ(M), tau)
    np.testing.assert_allclose(T.circ(L), ref, atol=1e-12)
    assert ranks.shape == (4,)


def test_tsvt_zero_threshold_and_large_threshold():
    M = rs.standard_normal((4, 6, 5))
    L, ranks = D.tsvt(M, 0.0)
    assert T.rel_fro(L, M) < 1e-13
    assert np.all(ranks == 4)
    L2, r2 = D.tsvt(M, 1e6)
    assert not np.any(np.abs(L2) > 1e-12) and np.all(r2 == 0)


def test_tsvt_is_the_tnn_prox():
    # L minimises ||L||_TNN + 1/(2 tau) ||L - M||_F^2
    M = rs.standard_normal((4, 5, 4))
    tau = 0.8
    L, _ = D.tsvt(M, tau)

    def obj(X):
        return T.tnn(X) + np.sum((X - M) ** 2) / (2 * tau)

    base = obj(L)
    for _ in range(20):
        assert obj(L + 1e-3 * rs.standard_normal(M.shape)) >= base - 1e-12


def test_admm_completion_recovers_low_rank():
    n1, n2, n3, r = 20, 20, 6, 2
    Ls = _lowrank(n1, n2, n3, r, seed=8)
    mask = (rs.random(Ls.shape) < 0.6).astype(np.uint8)
    X = Ls * mask
    L, E, Y, hist = D.admm_complete(X, mask, iters=80, L_true=Ls)
    assert hist[-1]["rse"] < 1e-2
    assert hist[-1]["rse"] < 0.1 * hist[5]["rse"]
    # E stays on the unobserved entries
    assert not np.any(E[mask == 1])
    assert hist[-1]["res"] < hist[20]["res"]


def test_tcur_tubes_match_full_tcur():
    A = rs.standard_normal((9, 11, 6)) + _lowrank(9, 11, 6, 2, seed=3)
    ci, cs = np.array([0, 2, 5, 9]), np.array([1.0, 0.5, 2.0, 1.5])
    ri, rsc = np.array([1, 4, 8]), np.array([0.7, 1.1, 1.9])
    Z, _ = D.tcur(A, ci, cs, ri, rsc, r=2)
    ii, jj = np.array([0, 3, 8, 5]), np.array([10, 0, 4, 5])
    got = D.tcur_tubes(A[:, ci, :], A[ri, :, :], cs, ri, rsc, 2, ii, jj)
    np.testing.assert_allclose(got, Z[ii, jj, :], atol=1e-12)


def _spiky(n1, n2, n3, r, frac, seed):
    """Low tubal rank r plus sparse +-5 spikes on a fraction of the entries."""
    g = np.random.default_rng(seed)
    Ls = _lowrank(n1, n2, n3, r, seed=seed)
    S = np.zeros(Ls.shape)
    hit = g.random(Ls.shape) < frac
    S[hit] = 5.0 * g.choice([-1.0, 1.0], int(hit.sum()))
    return Ls, S


def test_completion_e_update_optimality_every_iteration():
    # E-update of the completion loop: Y vanishes off the observed entries
    Ls = _lowrank(12, 10, 5, 2, seed=21)
    mask = (rs.random(Ls.shape) < 0.5).astype(np.uint8)
    for iters in (1, 4, 15):
        L, E, Y, _ = D.admm_complete(Ls * mask, mask, iters=iters)
        assert np.max(np.abs(Y[mask == 0])) <= 1e-12 * max(1.0, np.max(np.abs(Y)))


def test_soft_threshold_is_the_l1_prox():
    V = rs.standard_normal((5, 4, 3))
    t = 0.4
    E = D.soft_threshold(V, t)

    def obj(Z):
        return t * np.sum(np.abs(Z)) + 0.5 * np.sum((Z - V) ** 2)

    base = obj(E)
    for _ in range(30):
        assert obj(E + 1e-3 * rs.standard_normal(V.shape)) >= base - 1e-12
    np.testing.assert_array_equal(D.soft_threshold(V, 0.0), V)
    assert not np.any(D.soft_threshold(V, 10.0))


def test_rpca_e_update_optimality_every_iteration():
    # 0 in lam d||E||_1 + Y_{k+1}: |Y| <= lam everywhere, Y = -lam sign(E) on supp(E)
    Ls, S = _spiky(14, 12, 4, 2, 0.1, seed=22)
    X = Ls + S
    lam = D.rpca_lambda(X.shape)
    for iters in (2, 40, 100):
        L, E, Y, _ = D.admm_rpca(X, lam, iters=iters)
        assert np.max(np.abs(Y)) <= lam * (1 + 1e-9)
        on = np.abs(E) > 0
        assert on.any() or iters < 100
        np.testing.assert_allclose(Y[on], -lam * np.sign(E[on]), rtol=0, atol=1e-9 * lam)


def test_rpca_l_update_optimality_every_iteration():
    # the L-update is the exact prox of the TNN (eq. tnuc): with
    # G = -Y_{k+1} - mu_k (E_k - E_{k+1}), G is a subgradient of ||.||_TNN at
    # L_{k+1}: its tensor spectral norm (the dual norm) is <= 1 and
    # <G, L_{k+1}> = ||L_{k+1}||_TNN
    Ls, S = _spiky(20, 16, 5, 2, 0.05, seed=23)
    X = Ls + S + 0.05 * rs.standard_normal(Ls.shape)
    lam = D.rpca_lambda(X.shape)
    for iters in (30, 60, 100):
        L, E, Y, hist = D.admm_rpca(X, lam, iters=iters)
        Ep = D.admm_rpca(X, lam, iters=iters - 1)[1]
        G = -Y - hist[-1]["mu"] * (Ep - E)
        assert T.tspec(G) <= 1 + 1e-10
        assert abs(np.sum(G * L) - T.tnn(L)) <= 1e-10 * T.tnn(L)
        assert T.tnn(L) > 0


def test_rpca_converges_to_a_feasible_split():
    Ls, S = _spiky(20, 16, 5, 2, 0.05, seed=23)
    X = Ls + S + 0.05 * rs.standard_normal(Ls.shape)
    L, E, Y, hist = D.admm_rpca(X, D.rpca_lambda(X.shape), iters=250)
    assert hist[-1]["res"] < 1e-10 and hist[-1]["dL"] < 1e-8
    assert np.count_nonzero(E) > 0 and np.all(hist[-1]["ranks"] < 16)


def test_rpca_unbounded_lambda_is_full_completion():
    X = rs.standard_normal((9, 7, 4))
    a = D.admm_rpca(X, 1e300, iters=25)
    b = D.admm_complete(X, np.ones(X.shape, np.uint8), iters=25)
    for u, v in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(u, v)


def test_rpca_separates_low_rank_and_spikes():
    Ls, S = _spiky(30, 30, 5, 2, 0.05, seed=1)
    L, E, Y, hist = D.admm_rpca(Ls + S, D.rpca_lambda(Ls.shape), iters=200, L_true=Ls)
    assert hist[-1]["rse"] < 1e-10
    assert T.rel_fro(E, S) < 1e-10


def test_cur_tnn_reproduces_exact_rank_observed_in_full():
    Ls = _lowrank(30, 36, 5, 2, seed=3)
    ci, ri = np.array([0, 3, 7, 11, 20, 35]), np.array([1, 2, 9, 17, 29])
    L, Ct, Rt = D.cur_tnn(Ls, ci, ri, mask=np.ones(Ls.shape, np.uint8), iters=100)
    assert T.rel_fro(Ct, Ls[:, ci, :]) < 1e-12
    assert T.rel_fro(L, Ls) < 1e-12


def test_cur_tnn_robust_pca_recovers_low_rank():
    Ls, S = _spiky(30, 36, 5, 2, 0.05, seed=3)
    g = np.random.default_rng(2)
    ci, ri = np.sort(g.choice(36, 18, replace=False)), np.sort(g.choice(30, 16, replace=False))
    L, Ct, Rt = D.cur_tnn(Ls + S, ci, ri, lam=D.rpca_lambda(Ls.shape), iters=200)
    assert T.rel_fro(Rt, Ls[ri]) < 1e-10
    assert T.rel_fro(L, Ls) < 1e-10


def test_cur_tnn_structure_on_noisy_data():
    # L = Ct * W^+ * Rt with W = Ct[ri]: every lateral slice of L lies in the
    # t-range of Ct, and with l >= c = rank(W) the picked rows of L are the
    # projection of Rt onto the t-range of W
    X = _lowrank(16, 18, 4, 2, seed=5) + 0.2 * rs.standard_normal((16, 18, 4))
    ci, ri = np.array([1, 4, 6, 13]), np.array([0, 2, 3, 8, 10, 15])
    L, Ct, Rt = D.cur_tnn(X, ci, ri, lam=0.2, iters=30)
    assert T.rel_fro(D.tproject(L, Ct), L) < 1e-10
    assert T.rel_fro(L[ri], D.tproject(Rt, Ct[ri])) < 1e-10
    assert T.rel_fro(L[ri], Rt) > 1e-3


def test_cur_tnn_with_every_slice_is_the_admm():
    X = _lowrank(12, 14, 5, 2, seed=6) + 0.3 * rs.standard_normal((12, 14, 5))
    lam = D.rpca_lambda(X.shape)
    L, Ct, _ = D.cur_tnn(X, np.arange(14), np.arange(12), lam=lam, iters=40)
    La = D.admm_rpca(X, lam, iters=40)[0]
    np.testing.assert_array_equal(Ct, La)
    assert T.rel_fro(L, La) < 1e-12


def test_tcx_union_never_worse_than_a_round():
    A = _lowrank(16, 30, 5, 4, seed=9) + 0.3 * rs.standard_normal((16, 30, 5))
    g = np.random.default_rng(3)
    rounds = [g.choice(30, 5, replace=False) for _ in range(3)]
    Zu = D.tcx_union(A, rounds)
    errs = [T.rel_fro(D.tcx(A, r, np.ones(5)), A) for r in rounds]
    assert T.rel_fro(Zu, A) <= min(errs) + 1e-12
    # a single round is plain t-CX; the union of all slices reproduces A
    np.testing.assert_allclose(D.tcx_union(A, rounds[:1]), D.tcx(A, rounds[0], np.ones(5)), atol=1e-12)
    assert T.rel_fro(D.tcx_union(A, [np.arange(30)]), A) < 1e-12


@pytest.mark.parametrize("variant", ["complete", "rpca"])
def test_admm_stops_at_the_first_iteration_meeting_the_check(variant):
    # Algorithm 7 ends the loop once ||L_{k+1} - L_k||_inf, ||E_{k+1} -
    # E_k||_inf and ||L_{k+1} + E_{k+1} - X||_inf are all at most eps. The
    # stopped run must equal the unstopped run cut at that first iteration,
    # and no earlier iteration may meet the check.
    Ls = _lowrank(10, 9, 4, 2, seed=31)
    if variant == "complete":
        mask = (np.random.default_rng(32).random(Ls.shape) < 0.7).astype(np.uint8)

        def run(**kw):
            return D.admm_complete(Ls * mask, mask, **kw)
    else:
        lam = D.rpca_lambda(Ls.shape)

        def run(**kw):
            return D.admm_rpca(Ls, lam, **kw)

    _, _, _, full = run(iters=300)
    q = np.array([max(h["dL"], h["dE"], h["res"]) for h in full])
    tol = float(np.quantile(q[q > 0], 0.2))
    first = int(np.argmax(q <= tol))
    assert q[first] <= tol and np.all(q[:first] > tol)
    L, E, Y, hist = run(iters=300, tol=tol)
    assert len(hist) == first + 1
    L2, E2, Y2, _ = run(iters=first + 1)
    np.testing.assert_array_equal(L, L2)
    np.testing.assert_array_equal(E, E2)
    np.testing.assert_array_equal(Y, Y2)
    # an unreachable tolerance runs the whole budget
    assert len(run(iters=7, tol=0.0)[3]) == 7


def test_tproject_tubes_match_full_tproject():
    X = rs.standard_normal((12, 9, 6)) + _lowrank(12, 9, 6, 2, seed=51)
    C = X[:, [1, 4, 7], :] + 0.1 * rs.standard_normal((12, 3, 6))
    Z = D.tproject(X, C)
    jcols = np.array([8, 0, 3])
    ii, jj = np.array([0, 5, 11, 7]), np.array([3, 8, 0, 3])
    got = D.tproject_tubes(C, X[:, jcols, :], jcols, ii, jj)
    np.testing.assert_allclose(got, Z[ii, jj, :], atol=1e-12)
