"""t-product algebra in float64 (oracle; test infrastructure only).

Indices are 0-based: the paper's frontal slice ``k`` (1-based) is ``[:, :, k-1]``
here. Tensors are numpy arrays of shape (n1, n2, n3).

Pins (tests/test_oracle_tensor.py): brute-force circular convolution on a
hand-worked golden case; two independent routes (block-circulant product and
the convolution theorem) agree; identity, t-transpose, associativity and
tube-basis shift invariants; n3=1 reduces to a matrix product; Parseval;
t-SVD reconstruction, orthogonality and Eckart-Young; the nuclear-norm
identity of the circulant form.
"""

import numpy as np


# ---------------------------------------------------------------------------
# Definition of the t-product (Section 2.2, Definition "Tensor product", eq.
# tprod): C = fold(circ(Z) . unfold(X)).
# ---------------------------------------------------------------------------

def unfold(X):
    """Stack the frontal slices X_{::1}, ..., X_{::n3} vertically
    (an (n1*n3) x n2 matrix)."""
    n1, n2, n3 = X.shape
    return np.concatenate([X[:, :, k] for k in range(n3)], axis=0)


def fold(M, n3):
    """Inverse of unfold: split the rows into n3 blocks of equal height."""
    rows = M.shape[0] // n3
    return np.stack([M[k * rows:(k + 1) * rows, :] for k in range(n3)], axis=2)


def circ(Z):
    """Block-circulant matrix of Z: block row k, block column t holds the
    frontal slice Z_{::((k - t) mod n3)} (0-based), so the first block column
    is Z_1, Z_2, ..., Z_n3 and each block row is the previous one shifted
    right by one block."""
    n1, n2, n3 = Z.shape
    M = np.zeros((n1 * n3, n2 * n3), dtype=np.result_type(Z, np.float64))
    for k in range(n3):
        for t in range(n3):
            M[k * n1:(k + 1) * n1, t * n2:(t + 1) * n2] = Z[:, :, (k - t) % n3]
    return M


def tprod_bcirc(Z, X):
    """t-product by its definition, fold(circ(Z) unfold(X)).

    For inputs whose circulant matrix would be large, the same sum is
    evaluated block row by block row without materialising circ(Z):
    C_{::k} = sum_t Z_{::(k-t) mod n3} X_{::t}. No FFT is used on either
    branch.
    """
    n1, n2, n3 = Z.shape
    n2b, n4, n3b = X.shape
    if n2 != n2b or n3 != n3b:
        raise ValueError("t-product needs Z n1 x n2 x n3 and X n2 x n4 x n3")
    Z = np.asarray(Z, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    if n1 * n3 * n2 * n3 <= 4_000_000:
        return fold(circ(Z) @ unfold(X), n3)
    Zs = [np.ascontiguousarray(Z[:, :, t]) for t in range(n3)]
    Xs = [np.ascontiguousarray(X[:, :, t]) for t in range(n3)]
    C = np.zeros((n1, n4, n3))
    for k in range(n3):
        acc = np.zeros((n1, n4))
        for t in range(n3):
            acc += Zs[(k - t) % n3] @ Xs[t]
        C[:, :, k] = acc
    return C


def fft3(X):
    """fft along the third mode, MATLAB convention (forward unscaled)."""
    return np.fft.fft(np.asarray(X, dtype=np.float64), axis=2)


def ifft3(Xh):
    """ifft along the third mode (inverse carries the 1/n3 factor)."""
    return np.fft.ifft(Xh, axis=2)


def _real_part_checked(Y):
    scale = max(1.0, float(np.max(np.abs(Y))) if Y.size else 1.0)
    if Y.size and np.max(np.abs(Y.imag)) > 1e-10 * scale:
        raise AssertionError("inverse transform of a conjugate-symmetric "
                             "spectrum should be real")
    return np.ascontiguousarray(Y.real)


def slice_matmul(Ah, Bh):
    """Per-frontal-slice matrix product of two spectra:
    out[:, :, k] = Ah[:, :, k] @ Bh[:, :, k]."""
    prod = np.matmul(np.ascontiguousarray(np.moveaxis(Ah, 2, 0)), np.ascontiguousarray(np.moveaxis(Bh, 2, 0)))
    return np.moveaxis(prod, 0, 2)


def tprod_fft(Z, X):
    """Algorithm 1: fft both operands along the tubes, multiply every
    frontal slice pair, then ifft (a second, independent route)."""
    if Z.shape[1] != X.shape[0] or Z.shape[2] != X.shape[2]:
        raise ValueError("t-product needs Z n1 x n2 x n3 and X n2 x n4 x n3")
    return _real_part_checked(ifft3(slice_matmul(fft3(Z), fft3(X))))


# ---------------------------------------------------------------------------
# Definitions of Section 2.2: conjugate transpose, identity, basis.
# ---------------------------------------------------------------------------

def ttranspose(X):
    """Transpose every frontal slice, then reverse the order of slices
    2 through n3 (Definition "Conjugate transpose"; X is real)."""
    n3 = X.shape[2]
    T = np.transpose(X, (1, 0, 2))
    order = [0] + list(range(n3 - 1, 0, -1))
    return np.ascontiguousarray(T[:, :, order])


def teye(n, n3):
    """Identity tensor: first frontal slice is I_n, the others are zero."""
    I = np.zeros((n, n, n3))
    I[:, :, 0] = np.eye(n)
    return I


def tube_basis(n3, i):
    """Tube basis element of length n3 with a 1 at (0-based) position i."""
    e = np.zeros((1, 1, n3))
    e[0, 0, i] = 1.0
    return e


# ---------------------------------------------------------------------------
# t-SVD (Theorem "t-SVD" and eq. circ1: the DFT block-diagonalises circ).
# ---------------------------------------------------------------------------

def half_spectrum_count(n3):
    """Number of Fourier slices that are not conjugates of another one."""
    return n3 // 2 + 1


def spectral_weights(n3):
    """Weight of each non-redundant Fourier slice when a sum over all n3
    slices is folded onto the half spectrum: 1 for the DC slice and (n3
    even) the Nyquist slice, 2 for the others, whose mirror is their
    conjugate."""
    K = half_spectrum_count(n3)
    w = np.full(K, 2.0)
    w[0] = 1.0
    if n3 % 2 == 0:
        w[K - 1] = 1.0
    return w


def tsvd(X, r=None):
    """t-SVD X = U * S * V^T from SVDs of the Fourier slices.

    Slices k = 0..floor(n3/2) get a full SVD; the remaining slices are set to
    the conjugates of their mirrors, so U, S, V are real after ifft. With
    ``r`` the factors are truncated to the first r singular triplets of every
    slice (the tubal rank-r approximation).

    Returns (U, S, V, sv) with U n1 x m x n3, S m x m x n3 f-diagonal,
    V n2 x m x n3 (m = min(n1, n2) or r) and sv the (K, m) singular values of
    the non-redundant Fourier slices.
    """
    n1, n2, n3 = X.shape
    m = min(n1, n2) if r is None else int(r)
    Xh = fft3(X)
    K = half_spectrum_count(n3)
    Uh = np.zeros((n1, m, n3), dtype=complex)
    Sh = np.zeros((m, m, n3), dtype=complex)
    Vh = np.zeros((n2, m, n3), dtype=complex)
    sv = np.zeros((K, m))
    for k in range(K):
        Mk = Xh[:, :, k]
        if k == 0 or (n3 % 2 == 0 and k == n3 // 2):
            Mk = Mk.real  # exactly real slices: keep real factors
        u, s, vh = np.linalg.svd(Mk, full_matrices=False)
        Uh[:, :, k] = u[:, :m]
        Sh[:, :, k] = np.diag(s[:m])
        Vh[:, :, k] = vh.conj().T[:, :m]
        sv[k] = s[:m]
    for k in range(K, n3):
        Uh[:, :, k] = Uh[:, :, n3 - k].conj()
        Sh[:, :, k] = Sh[:, :, n3 - k]
        Vh[:, :, k] = Vh[:, :, n3 - k].conj()
    U = _real_part_checked(ifft3(Uh))
    S = _real_part_checked(ifft3(Sh))
    V = _real_part_checked(ifft3(Vh))
    return U, S, V, sv


def tubal_multirank(X, tol=None):
    """Rank of every Fourier slice (Definition "Tensor multi and tubal
    rank"); the tubal rank is the maximum."""
    Xh = fft3(X)
    ranks = []
    for k in range(X.shape[2]):
        s = np.linalg.svd(Xh[:, :, k], compute_uv=False)
        t = tol if tol is not None else max(X.shape[:2]) * np.finfo(float).eps * (s[0] if s.size else 0)
        ranks.append(int(np.sum(s > t)))
    return ranks


def tnn(X):
    """Tensor nuclear norm, eq. tnuc: mean of the nuclear norms of all n3
    Fourier slices."""
    Xh = fft3(X)
    n3 = X.shape[2]
    return sum(np.linalg.svd(Xh[:, :, k], compute_uv=False).sum() for k in range(n3)) / n3


def tspec(X):
    """Tensor spectral norm (Definition def:spec:ten): largest spectral norm
    of the Fourier slices."""
    Xh = fft3(X)
    return max(np.linalg.svd(Xh[:, :, k], compute_uv=False)[0] for k in range(X.shape[2]))


def rel_fro(X, Y):
    """||X - Y||_F / ||Y||_F (Y is the reference)."""
    den = np.linalg.norm(np.asarray(Y, dtype=np.float64).ravel())
    num = np.linalg.norm((np.asarray(X, dtype=np.float64) - np.asarray(Y, dtype=np.float64)).ravel())
    return num / den if den > 0 else num


# ---------------------------------------------------------------------------
# Views used to check the Fourier engine and full-size products.
# ---------------------------------------------------------------------------

def half_spectrum(X):
    """The K = floor(n3/2)+1 non-redundant Fourier slices of X as a
    (K, n1, n2) complex array (slice-major)."""
    K = X.shape[2] // 2 + 1
    return np.ascontiguousarray(np.transpose(fft3(X)[:, :, :K], (2, 0, 1)))


def from_half_spectrum(H, n3):
    """Real tensor whose Fourier slices k <= n3/2 are H[k] and whose other
    slices are their conjugates (the imaginary parts of slice 0 and, for
    even n3, slice n3/2 do not belong to a real signal and are dropped)."""
    H = np.asarray(H)
    return np.ascontiguousarray(np.fft.irfft(np.transpose(H, (1, 2, 0)), n=n3, axis=2))


def tprod_entries(A, B, ii, jj, kk):
    """Selected entries C[i, j, k] of C = A * B straight from eq. tprod:
    C_{ij k} = sum_t sum_s A_{i s (k-t) mod n3} B_{s j t}."""
    n3 = A.shape[2]
    out = np.empty(len(ii))
    for e, (i, j, k) in enumerate(zip(ii, jj, kk)):
        acc = 0.0
        for t in range(n3):
            acc += float(np.dot(A[i, :, (k - t) % n3].astype(np.float64), B[:, j, t].astype(np.float64)))
        out[e] = acc
    return out


def tprod_slices(A, B, ks):
    """Frontal slices C_{::k}, k in ks, of C = A * B by the block-row sum of
    eq. tprod: C_{::k} = sum_t A_{::(k-t) mod n3} B_{::t}."""
    n3 = A.shape[2]
    As = [np.ascontiguousarray(A[:, :, t], dtype=np.float64) for t in range(n3)]
    Bs = [np.ascontiguousarray(B[:, :, t], dtype=np.float64) for t in range(n3)]
    out = []
    for k in ks:
        acc = np.zeros((A.shape[0], B.shape[1]))
        for t in range(n3):
            acc += As[(k - t) % n3] @ Bs[t]
        out.append(acc)
    return np.stack(out, axis=2)
