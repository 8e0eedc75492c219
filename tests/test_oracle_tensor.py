"""Pins of the oracle's t-product algebra against facts fixed by the paper's
definitions and by linear algebra (not against the oracle itself)."""
import os

import numpy as np
import pytest

from oracle import tensor as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
rs = np.random.default_rng(1234)


def _read_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_golden_circular_convolution():
    rows = {r[0]: np.array([float(x) for x in r[1:]]) for r in _read_rows("circconv_tube3.txt")}
    a = rows["a"].reshape(1, 1, 3)
    b = rows["b"].reshape(1, 1, 3)
    np.testing.assert_array_equal(T.tprod_bcirc(a, b).ravel(), rows["c"])
    np.testing.assert_allclose(T.tprod_fft(a, b).ravel(), rows["c"], rtol=0, atol=1e-12)


def test_golden_2x2x2():
    mats = {}
    for r in _read_rows("tprod_2x2x2.txt"):
        mats[(r[0], int(r[1]) - 1)] = np.array([float(x) for x in r[2:]]).reshape(2, 2)
    A = np.stack([mats[("A", 0)], mats[("A", 1)]], axis=2)
    B = np.stack([mats[("B", 0)], mats[("B", 1)]], axis=2)
    C = np.stack([mats[("C", 0)], mats[("C", 1)]], axis=2)
    np.testing.assert_array_equal(T.tprod_bcirc(A, B), C)
    np.testing.assert_allclose(T.tprod_fft(A, B), C, atol=1e-12)


def test_circ_layout_first_block_row():
    # first block row of circ(Z) is Z_1, Z_n3, ..., Z_2
    Z = rs.standard_normal((2, 3, 4))
    M = T.circ(Z)
    for t, k in enumerate([0, 3, 2, 1]):
        np.testing.assert_array_equal(M[0:2, 3 * t:3 * t + 3], Z[:, :, k])


@pytest.mark.parametrize("shape", [(3, 4, 5, 1), (4, 3, 2, 2), (5, 6, 4, 7), (6, 5, 3, 8), (3, 7, 2, 16)])
def test_bcirc_and_fft_routes_agree(shape):
    n1, n2, n4, n3 = shape
    A = rs.standard_normal((n1, n2, n3))
    B = rs.standard_normal((n2, n4, n3))
    C1 = T.tprod_bcirc(A, B)
    C2 = T.tprod_fft(A, B)
    assert T.rel_fro(C2, C1) < 1e-13


def test_bcirc_direct_sum_branch_matches_materialised():
    A = rs.standard_normal((40, 30, 12))
    B = rs.standard_normal((30, 20, 12))
    big = T.tprod_bcirc(A, B)                    # small: circ(A) is materialised
    # force the direct-sum branch by a shape over the threshold
    A2 = rs.standard_normal((120, 200, 14))
    B2 = rs.standard_normal((200, 10, 14))
    assert A2.shape[0] * 14 * A2.shape[1] * 14 > 4_000_000
    C2 = T.tprod_bcirc(A2, B2)
    assert T.rel_fro(C2, T.fold(T.circ(A2) @ T.unfold(B2), 14)) < 1e-13
    assert T.rel_fro(big, T.tprod_fft(A, B)) < 1e-13


def test_n3_one_is_matrix_product():
    A = rs.standard_normal((5, 4, 1))
    B = rs.standard_normal((4, 3, 1))
    np.testing.assert_allclose(T.tprod_bcirc(A, B)[:, :, 0], A[:, :, 0] @ B[:, :, 0], atol=1e-14)


def test_identity_tensor():
    A = rs.standard_normal((4, 5, 6))
    np.testing.assert_allclose(T.tprod_bcirc(T.teye(4, 6), A), A, atol=1e-14)
    np.testing.assert_allclose(T.tprod_bcirc(A, T.teye(5, 6)), A, atol=1e-14)


def test_transpose_reverses_products():
    A = rs.standard_normal((4, 5, 6))
    B = rs.standard_normal((5, 3, 6))
    lhs = T.ttranspose(T.tprod_bcirc(A, B))
    rhs = T.tprod_bcirc(T.ttranspose(B), T.ttranspose(A))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)
    # circ of the t-transpose is the transpose of circ
    np.testing.assert_array_equal(T.circ(T.ttranspose(A)), T.circ(A).T)


def test_associativity():
    A = rs.standard_normal((3, 4, 5))
    B = rs.standard_normal((4, 2, 5))
    C = rs.standard_normal((2, 3, 5))
    np.testing.assert_allclose(T.tprod_bcirc(T.tprod_bcirc(A, B), C),
                               T.tprod_bcirc(A, T.tprod_bcirc(B, C)), atol=1e-12)


@pytest.mark.parametrize("n3", [1, 4, 7])
def test_tube_basis_is_circular_shift(n3):
    a = rs.standard_normal((1, 1, n3))
    for i in range(n3):
        np.testing.assert_allclose(T.tprod_bcirc(T.tube_basis(n3, i), a).ravel(), np.roll(a.ravel(), i),
                                   atol=1e-15)


def test_parseval():
    X = rs.standard_normal((4, 6, 9))
    lhs = np.sum(X ** 2)
    rhs = np.sum(np.abs(T.fft3(X)) ** 2) / 9
    assert abs(lhs - rhs) < 1e-12 * lhs


def test_dft_block_diagonalises_circ():
    # eq. circ1: (F kron I_n1) circ(X) (F^-1 kron I_n2) = bdiag(Xhat)
    n1, n2, n3 = 3, 2, 5
    X = rs.standard_normal((n1, n2, n3))
    F = np.fft.fft(np.eye(n3), axis=0)
    lhs = np.kron(F, np.eye(n1)) @ T.circ(X) @ np.kron(np.linalg.inv(F), np.eye(n2))
    Xh = T.fft3(X)
    rhs = np.zeros((n1 * n3, n2 * n3), dtype=complex)
    for k in range(n3):
        rhs[k * n1:(k + 1) * n1, k * n2:(k + 1) * n2] = Xh[:, :, k]
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("shape", [(6, 4, 5), (4, 6, 8), (5, 5, 1)])
def test_tsvd_reconstructs_and_is_orthogonal(shape):
    X = rs.standard_normal(shape)
    U, S, V, sv = T.tsvd(X)
    rec = T.tprod_bcirc(T.tprod_bcirc(U, S), T.ttranspose(V))
    assert T.rel_fro(rec, X) < 1e-12
    m = U.shape[1]
    np.testing.assert_allclose(T.tprod_bcirc(T.ttranspose(U), U), T.teye(m, shape[2]), atol=1e-12)
    np.testing.assert_allclose(T.tprod_bcirc(T.ttranspose(V), V), T.teye(m, shape[2]), atol=1e-12)
    # f-diagonal: every frontal slice of S is diagonal
    off = S.copy()
    for k in range(shape[2]):
        off[:, :, k] -= np.diag(np.diag(S[:, :, k]))
    assert np.max(np.abs(off)) < 1e-13
    assert np.all(np.diff(sv, axis=1) <= 1e-12)


def test_eckart_young_per_slice():
    X = rs.standard_normal((7, 6, 6))
    r = 2
    U, S, V, _ = T.tsvd(X, r=r)
    Xr = T.tprod_bcirc(T.tprod_bcirc(U, S), T.ttranspose(V))
    Xh = T.fft3(X)
    tail = sum(np.sum(np.linalg.svd(Xh[:, :, k], compute_uv=False)[r:] ** 2) for k in range(6)) / 6
    assert abs(np.sum((X - Xr) ** 2) - tail) < 1e-10 * tail


def test_tnn_and_spectral_norm_via_circ():
    X = rs.standard_normal((4, 3, 5))
    s = np.linalg.svd(T.circ(X), compute_uv=False)
    assert abs(T.tnn(X) - s.sum() / 5) < 1e-12 * s.sum()
    assert abs(T.tspec(X) - s[0]) < 1e-12 * s[0]


def test_tubal_rank_of_factor_product():
    G1 = rs.standard_normal((8, 3, 6))
    G2 = rs.standard_normal((3, 9, 6))
    ranks = T.tubal_multirank(T.tprod_bcirc(G1, G2))
    assert max(ranks) == 3


@pytest.mark.parametrize("n3", [1, 2, 5, 8])
def test_half_spectrum_roundtrip_and_conjugate_symmetry(n3):
    X = rs.standard_normal((3, 4, n3))
    H = T.half_spectrum(X)
    full = T.fft3(X)
    for k in range(n3):
        ref = H[k] if k < H.shape[0] else np.conj(H[n3 - k])
        np.testing.assert_allclose(full[:, :, k], ref, atol=1e-12)
    np.testing.assert_allclose(T.from_half_spectrum(H, n3), X, atol=1e-13)
    # imaginary parts of the real slices are ignored by the inverse
    H2 = H.copy()
    H2[0] += 1j
    if n3 % 2 == 0:
        H2[-1] -= 2j
    np.testing.assert_allclose(T.from_half_spectrum(H2, n3), X, atol=1e-13)


def test_tprod_entries_match_definition():
    A = rs.standard_normal((5, 6, 7))
    B = rs.standard_normal((6, 4, 7))
    Cref = T.tprod_bcirc(A, B)
    ii, jj, kk = rs.integers(0, 5, 20), rs.integers(0, 4, 20), rs.integers(0, 7, 20)
    np.testing.assert_allclose(T.tprod_entries(A, B, ii, jj, kk), Cref[ii, jj, kk], atol=1e-12)


def test_tprod_slices_match_definition():
    A = rs.standard_normal((4, 6, 5))
    B = rs.standard_normal((6, 3, 5))
    np.testing.assert_allclose(T.tprod_slices(A, B, [0, 3]), T.tprod_bcirc(A, B)[:, :, [0, 3]], atol=1e-12)
