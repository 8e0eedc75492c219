"""Numerical evidence behind the precision of the thresholding's block
Jacobi (CPU, emulated rounding): which matrix-core precision its Gram
matrices and rotations could use.

A pair step computes the Gram matrix of 32 float32 rows and declares the
pair converged when max |G_st| / max(G_ss, G_tt) < 1e-6; it then rotates
the rows of X and of the accumulated U^H by a 32 x 32 unitary. bf16 values
are emulated by rounding float32 to the nearest 8-bit mantissa (ties to
even), the split products as hi*hi + hi*lo + lo*hi accumulated in float32,
as the matrix cores do."""
import numpy as np

TOL = 1e-6


def bf16(x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def mm32(A, B):
    """A @ B with float32 accumulation in contraction order."""
    out = np.zeros((A.shape[0], B.shape[1]), np.float32)
    for k in range(A.shape[1]):
        out = (out + np.outer(A[:, k], B[k, :]).astype(np.float32)).astype(np.float32)
    return out


def split3(A, B):
    ah, bh = bf16(A), bf16(B)
    al, bl = bf16(A - ah), bf16(B - bh)
    return mm32(ah, bh) + mm32(ah, bl) + mm32(al, bh)


def stop_ratio(G):
    d = np.diag(G)
    return float((np.abs(G - np.diag(d)) / np.maximum.outer(d, d)).max())


def orthogonal_rows(seed, n=256, m=32):
    """m mutually orthogonal float32 rows of length n whose norms span two
    decades: a converged pair as the stop test sees it."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, m)))
    return (Q.T * (10.0 ** rng.uniform(-1, 1, m))[:, None]).astype(np.float32)


def test_gram_precision_against_the_stop_test():
    for seed in range(2):
        X = orthogonal_rows(seed)
        X64 = X.astype(np.float64)
        f64 = stop_ratio(X64 @ X64.T)
        x3 = stop_ratio(split3(X, X.T).astype(np.float64))
        x1 = stop_ratio(mm32(bf16(X), bf16(X).T).astype(np.float64))
        # float64 products certify convergence with two orders to spare;
        # one bf16 term cannot reach the tolerance; three terms sit just
        # under it (0.2-0.7 of it in these runs)
        assert f64 < 1e-2 * TOL
        assert x1 > 100 * TOL
        assert x3 < TOL


def test_rotation_precision():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((32, 256)).astype(np.float32)
    V, _ = np.linalg.qr(rng.standard_normal((32, 32)))
    Y = V.T @ X.astype(np.float64)
    e_f64 = np.linalg.norm(Y.astype(np.float32) - Y) / np.linalg.norm(Y)
    e_x3 = np.linalg.norm(split3(V.T.astype(np.float32), X).astype(np.float64) - Y) / np.linalg.norm(Y)
    # float64 products rounded once to float32 storage: ~eps_32 / 2; split
    # bf16 products: two orders of magnitude more per rotation, which the
    # thousands of rotations an ADMM run applies to U^H would accumulate
    assert e_f64 < 6e-8
    assert e_x3 > 50 * e_f64
