"""Pins of the oracle's generator, probabilities and pick procedure."""
import math

import numpy as np
import pytest

from oracle import philox, sampling as S
from oracle import tensor as T

rs = np.random.default_rng(99)


@pytest.mark.parametrize("key", [(0, 0), (5, 7), (2 ** 63 + 11, 123456789), (17040436, 3)])
def test_philox_matches_numpy(key):
    # numpy's Philox advances its counter before each block, so block j of its
    # raw stream is the block at counter j + 1.
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.zeros(4, dtype=np.uint64))
    raw = [int(x) for x in bg.random_raw(12)]
    for j in range(3):
        mine = philox.philox4x64_10((j + 1, 0, 0, 0), key)
        assert list(mine) == raw[4 * j:4 * j + 4]


def test_philox_high_counter_words():
    ctr = np.array([2 ** 64 - 1, 5, 0, 0], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([9, 10], dtype=np.uint64), counter=ctr)
    raw = [int(x) for x in bg.random_raw(4)]
    # counter (2^64-1) + 1 wraps into the next word: (0, 6, 0, 0)
    assert list(philox.philox4x64_10((0, 6, 0, 0), (9, 10))) == raw


def test_quantize_power_of_two_invariance_and_range():
    w = rs.exponential(size=37)
    q, s = S.quantize(w)
    q2, s2 = S.quantize(w * 2.0 ** 17)
    assert q == q2 and s == s2
    B = 62 - (37 - 1).bit_length()
    assert max(q) < 2 ** B and max(q) >= 2 ** (B - 1)
    assert s < 2 ** 62


def test_quantize_rejects_bad_weights():
    for bad in ([0.0, 0.0], [1.0, -1.0], [1.0, float("nan")], [float("inf"), 1.0], []):
        with pytest.raises(ValueError):
            S.quantize(bad)


def test_bernoulli_full_budget_keeps_everything():
    n = 12
    idx, sc = S.sample_bernoulli(np.ones(n), n, seed=3)
    np.testing.assert_array_equal(idx, np.arange(n))
    np.testing.assert_array_equal(sc, np.ones(n))


def test_bernoulli_inclusion_frequencies():
    n, c, reps = 16, 5, 3000
    w = rs.exponential(size=n) ** 2
    w[3] = 0.0
    w[7] = 40.0  # c p_7 > 1: always kept
    p = w / w.sum()
    pi = np.minimum(1.0, c * p)
    counts = np.zeros(n)
    sizes = []
    for seed in range(reps):
        idx, sc = S.sample_bernoulli(w, c, seed=seed, stream=1)
        assert np.all(np.diff(idx) > 0)
        np.testing.assert_allclose(sc, 1.0 / np.sqrt(pi[idx]), rtol=1e-12)
        counts[idx] += 1
        sizes.append(len(idx))
    assert counts[3] == 0 and counts[7] == reps
    inner = (pi > 0) & (pi < 1)
    z = (counts[inner] - reps * pi[inner]) / np.sqrt(reps * pi[inner] * (1 - pi[inner]))
    assert np.max(np.abs(z)) < 4.5
    chi2 = float(np.sum(z ** 2))
    dof = int(inner.sum())
    assert chi2 < dof + 6 * math.sqrt(2 * dof)
    assert abs(np.mean(sizes) - pi.sum()) < 5 * np.sqrt(np.sum(pi * (1 - pi)) / reps)


def test_iid_frequencies_follow_quantised_weights():
    n, c, reps = 10, 8, 1500
    w = rs.exponential(size=n)
    q, s = S.quantize(w)
    p = np.array(q, dtype=float) / s
    counts = np.zeros(n)
    for seed in range(reps):
        idx, sc = S.sample_iid(w, c, seed=seed)
        assert len(idx) == c
        np.testing.assert_allclose(sc, 1.0 / np.sqrt(c * p[idx]), rtol=1e-12)
        np.add.at(counts, idx, 1)
    N = reps * c
    z = (counts - N * p) / np.sqrt(N * p * (1 - p))
    assert np.max(np.abs(z)) < 4.5


def test_iid_never_draws_zero_weight():
    w = np.array([0.0, 1.0, 0.0, 3.0, 0.0])
    for seed in range(200):
        idx, _ = S.sample_iid(w, 4, seed=seed)
        assert set(idx.tolist()) <= {1, 3}


def test_uniform_without_replacement():
    n, c, reps = 12, 4, 2000
    counts = np.zeros(n)
    for seed in range(reps):
        idx, sc = S.sample_uniform_norepl(n, c, seed=seed)
        assert len(idx) == c and len(set(idx.tolist())) == c
        assert np.all(np.diff(idx) > 0)
        np.testing.assert_allclose(sc, math.sqrt(n / c))
        counts[idx] += 1
    p = c / n
    z = (counts - reps * p) / math.sqrt(reps * p * (1 - p))
    assert np.max(np.abs(z)) < 4.5


def test_norm_probabilities():
    A = rs.standard_normal((5, 7, 4))
    B = rs.standard_normal((7, 3, 4))
    a = S.lateral_sq_norms(A)
    b = S.horizontal_sq_norms(B)
    for j in range(7):
        assert abs(a[j] - np.sum(A[:, j, :] ** 2)) < 1e-12 * a[j]
        assert abs(b[j] - np.sum(B[j, :, :] ** 2)) < 1e-12 * b[j]
    assert abs(S.weights_norm2(A).sum() - np.sum(A ** 2)) < 1e-12 * np.sum(A ** 2)
    np.testing.assert_allclose(S.weights_normprod(A, B), np.sqrt(a) * np.sqrt(b), rtol=1e-13)


def test_lateral_leverage_identities():
    n1, n2, n3, r = 9, 12, 6, 3
    A = rs.standard_normal((n1, n2, n3))
    lev = S.weights_lateral_leverage(A, r)
    # every Fourier slice has rank >= r, so the squared norms sum to r n3
    assert abs(lev.sum() - r * n3) < 1e-10
    # ||Vhat_{j::}||_F^2 = n3 ||V_{j::}||_F^2 (Parseval, used in the proof of
    # Theorem thm:regress-main)
    _, _, V, _ = T.tsvd(A, r=r)
    np.testing.assert_allclose(lev, n3 * np.sum(V ** 2, axis=(1, 2)), rtol=1e-10)
    p = lev / (r * n3)
    assert np.all(p >= -1e-15) and np.all(p <= 1 + 1e-12)
    # a tensor whose right singular slices are the first r lateral basis
    # slices puts all leverage on those slices
    G = np.zeros((n1, n2, n3))
    G[:r, :r, 0] = np.diag([3.0, 2.0, 1.0])
    lev2 = S.weights_lateral_leverage(G, r)
    np.testing.assert_allclose(lev2[:r], n3, rtol=1e-12)
    assert np.all(lev2[r:] < 1e-20)


def test_horizontal_leverage_of_lateral_subtensor():
    C = rs.standard_normal((10, 4, 5))
    lev = S.weights_horizontal_leverage(C, 2)
    assert abs(lev.sum() - 2 * 5) < 1e-10


def test_horizontal_leverage_follows_left_singular_slices():
    # eq. colprob_rows_exact indexes horizontal slices, so its scores come
    # from the LEFT singular slices of C (one value per row of C). Build C
    # (n1 x c x n3, n1 != c) whose column space in every Fourier slice is
    # spanned by the horizontal basis slices in `rows`: its top-r left
    # singular slices are supported on exactly those rows, each with
    # ||Uhat_{i::}||_F^2 = n3, and every other row scores 0.
    n1, c, n3 = 11, 5, 6
    rows = [2, 5, 9]
    r = len(rows)
    G = rs.standard_normal((r, c, n3))
    C = np.zeros((n1, c, n3))
    C[rows] = G
    lev = S.weights_horizontal_leverage(C, r)
    assert lev.shape == (n1,)
    np.testing.assert_allclose(lev[rows], n3, rtol=1e-10)
    others = [i for i in range(n1) if i not in rows]
    assert np.all(np.abs(lev[others]) < 1e-20)
    # the right singular slices of this C are spread over its c columns:
    # their lateral scores are not an indicator, so a left/right mix-up
    # fails here as well as on the length
    lat = S.weights_lateral_leverage(C, r)
    assert lat.shape == (c,) and np.max(lat) < n3 * (1 - 1e-3)


def test_horizontal_leverage_is_lateral_leverage_of_the_t_transpose():
    # the t-transpose swaps left and right singular slices (Definition
    # t-transpose with the t-SVD theorem): U of C is V of C^T, so the
    # horizontal scores of C are the lateral scores of C^T
    C = rs.standard_normal((9, 4, 7))
    for r in (1, 2, 3):
        h = S.weights_horizontal_leverage(C, r)
        v = S.weights_lateral_leverage(T.ttranspose(C), r)
        assert h.shape == (9,)
        np.testing.assert_allclose(h, v, rtol=1e-10, atol=1e-12)
        assert abs(h.sum() - r * 7) < 1e-9
