"""Randomized t-product decompositions in float64 (oracle; test
infrastructure only).

* rtprod      Algorithm 2 given the picked slices and their scales.
* tproject    Algorithm 3, t-CX (Algorithm 4) given picked lateral slices.
* tpinv_r     per-Fourier-slice rank-r truncated pseudo-inverse.
* tcx_union   t-CX boosted by repetition (the union of the rounds' picks).
* tcur        Algorithm 5 given picked lateral and horizontal slices.
* tsvt        singular value thresholding of every Fourier slice, the
              closed-form L-update of Algorithm 7 with the tensor nuclear norm.
* admm_complete  Algorithm 7 adapted to the completion problem (eq. tlow6).
* admm_rpca   Algorithm 7 as stated, robust tensor PCA (eq. tlow7).
* cur_tnn     Algorithm 6 (CUR t-NN) given its picks.

Readings where the paper is silent or garbled:
* S and D carry their entries in the first frontal slice only and are zero
  elsewhere, so in the Fourier domain every slice uses the same selection
  and the same diagonal scaling (Algorithms 4-5 state "defined in the
  Fourier domain" and set slices 2..n3 to zero; taken literally that would
  zero every Fourier slice but the first).
* Algorithm 5 takes a rank parameter r but never uses it; here the core is
  the rank-r truncated pseudo-inverse of every Fourier slice of D S^T C,
  additionally dropping singular values at or below max(l, c) eps sigma_1.
* The completion variant of Algorithm 7 ("with a small modification") keeps
  X = L + E exactly with E supported on the unobserved entries; the L-update
  is the tensor-nuclear-norm prox, i.e. a per-Fourier-slice threshold of
  exactly 1/mu (both the nuclear norm and the squared Frobenius norm carry
  the same 1/n3 factor in the Fourier domain).
* Algorithm 6 picks C and R by the probabilities of eqs. cur-col-prob and
  colprob_rows_exact but, unlike Algorithms 2-5, does not rescale them: the
  picked slices are cleaned by the ADMM as they are, and W is the matching
  rows of the cleaned C, unscaled.
* The weight lambda of eq. tlow7 is not given; rpca_lambda returns the usual
  1 / sqrt(max(n1, n2) n3).

Pins (tests/test_oracle_decomp.py): c = n2 with uniform weights gives the
exact product; unbiasedness and the exact second moment of the estimator by
Monte Carlo; exact-rank inputs are reproduced exactly by t-CX and t-CUR;
t-CX is the least-squares optimum (eq. ell2reg) and its union over rounds
is never worse than any round; n3 = 1 reduces to matrix
CX/CUR; circ(tsvt(M, tau)) equals the matrix SVT of circ(M) with the same
tau; tau = 0 is the identity; prox optimality under random perturbations;
ADMM residuals shrink; every ADMM iterate satisfies the optimality
condition of its E-update exactly (Y = 0 off the observed entries for
completion, |Y| <= lambda with Y = -lambda sign(E) on the support of E for
robust PCA) and the converged robust-PCA iterate satisfies the optimality
conditions of eq. tlow7 (-Y a subgradient of the tensor nuclear norm at L);
robust PCA with an unbounded lambda is completion with every entry observed;
low-rank plus sparse spikes are separated; CUR t-NN reproduces an exact-rank
tensor observed in full, and with every slice picked equals the ADMM of the
whole tensor.
"""

import numpy as np

from . import tensor as T


def _is_real_slice(k, n3):
    return k == 0 or (n3 % 2 == 0 and k == n3 // 2)


def _mirror(Zh, K, n3):
    for k in range(K, n3):
        Zh[:, :, k] = Zh[:, :, n3 - k].conj()
    return Zh


def rtprod(A, B, idx, scale):
    """Algorithm 2 given its picks: C = A*S*D (picked lateral slices of A,
    each times its scale), R = D*S^T*B (the matching horizontal slices of B)
    and Z = C*R, the latter by the t-product definition."""
    idx = np.asarray(idx, dtype=np.int64)
    scale = np.asarray(scale, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if idx.size == 0:
        return np.zeros((A.shape[0], B.shape[1], A.shape[2]))
    C = A[:, idx, :] * scale[None, :, None]
    R = B[idx, :, :] * scale[:, None, None]
    return T.tprod_bcirc(C, R)


def pinv_r(W, r=None):
    """Rank-r truncated Moore-Penrose pseudo-inverse of one matrix."""
    u, s, vh = np.linalg.svd(W, full_matrices=False)
    if s.size == 0:
        return np.zeros((W.shape[1], W.shape[0]), dtype=W.dtype)
    keep = s > max(W.shape) * np.finfo(float).eps * s[0]
    if r is not None:
        keep[int(r):] = False
    inv = np.zeros_like(s)
    inv[keep] = 1.0 / s[keep]
    return (vh.conj().T * inv[None, :]) @ u.conj().T


def tproject(X, C):
    """Algorithm 3: Zhat_k = Chat_k Chat_k^+ Xhat_k for every Fourier slice."""
    n3 = X.shape[2]
    K = T.half_spectrum_count(n3)
    Xh, Ch = T.fft3(X), T.fft3(C)
    Zh = np.zeros(Xh.shape, dtype=complex)
    for k in range(K):
        Ck = Ch[:, :, k].real if _is_real_slice(k, n3) else Ch[:, :, k]
        Xk = Xh[:, :, k].real if _is_real_slice(k, n3) else Xh[:, :, k]
        Zh[:, :, k] = Ck @ (np.linalg.pinv(Ck) @ Xk)
    return T._real_part_checked(T.ifft3(_mirror(Zh, K, n3)))


def tcx(A, idx, scale):
    """Algorithm 4 given its picks: Chat_k = Ahat_k S D, Zhat_k = Chat_k
    Chat_k^+ Ahat_k."""
    idx = np.asarray(idx, dtype=np.int64)
    C = np.asarray(A, dtype=np.float64)[:, idx, :] * np.asarray(scale)[None, :, None]
    return tproject(A, C)


def tcx_union(A, rounds):
    """t-CX boosted by repetition: Algorithm 4 repeated with independent
    picks, keeping the projection onto the union of all picked lateral
    slices, C * C^+ * A with C = A[:, concatenation of the rounds' picks, :].
    By the least-squares property of eq. ell2reg it is never worse than the
    best single round (the argument that boosts the success probability)."""
    idx = np.concatenate([np.asarray(r, dtype=np.int64) for r in rounds])
    return tproject(A, np.asarray(A, dtype=np.float64)[:, idx, :])


def tcur(A, cidx, cscale, ridx, rscale, r=None):
    """Algorithm 5 given its picks. Returns (Z, core) where core[k] is the
    (c x l) matrix Uhat_k for the non-redundant Fourier slices k."""
    A = np.asarray(A, dtype=np.float64)
    n1, n2, n3 = A.shape
    cidx = np.asarray(cidx, dtype=np.int64)
    ridx = np.asarray(ridx, dtype=np.int64)
    cscale = np.asarray(cscale, dtype=np.float64)
    rscale = np.asarray(rscale, dtype=np.float64)
    K = T.half_spectrum_count(n3)
    Ah = T.fft3(A)
    Zh = np.zeros((n1, n2, n3), dtype=complex)
    core = np.zeros((K, cidx.size, ridx.size), dtype=complex)
    for k in range(K):
        Ak = Ah[:, :, k].real if _is_real_slice(k, n3) else Ah[:, :, k]
        Ck = Ak[:, cidx] * cscale[None, :]          # Chat_k = Ahat_k S D
        Rk = rscale[:, None] * Ak[ridx, :]          # Rhat_k = D S^T Ahat_k
        Wk = rscale[:, None] * Ck[ridx, :]          # D S^T Chat_k
        Uk = pinv_r(Wk, r)
        core[k] = Uk
        Zh[:, :, k] = Ck @ Uk @ Rk
    Z = T._real_part_checked(T.ifft3(_mirror(Zh, K, n3)))
    return Z, core


def svt_matrix(M, tau):
    """Matrix singular value thresholding U max(S - tau, 0) V^H and the
    number of singular values above tau."""
    u, s, vh = np.linalg.svd(M, full_matrices=False)
    st = np.maximum(s - tau, 0.0)
    return (u * st[None, :]) @ vh, int(np.sum(s > tau))


def tsvt(M, tau):
    """Per-Fourier-slice SVT with threshold tau. Returns (L, ranks) with
    ranks[k] the number of singular values above tau in Fourier slice k for
    the non-redundant slices."""
    M = np.asarray(M, dtype=np.float64)
    n3 = M.shape[2]
    K = T.half_spectrum_count(n3)
    Mh = T.fft3(M)
    Lh = np.zeros(Mh.shape, dtype=complex)
    ranks = np.zeros(K, dtype=np.int64)
    for k in range(K):
        Mk = Mh[:, :, k].real if _is_real_slice(k, n3) else Mh[:, :, k]
        Lh[:, :, k], ranks[k] = svt_matrix(Mk, tau)
    L = T._real_part_checked(T.ifft3(_mirror(Lh, K, n3)))
    return L, ranks


def _stopped(rec, tol):
    """Algorithm 7's convergence check: every one of the three
    infinity-norm quantities is at most tol."""
    return tol is not None and rec["dL"] <= tol and rec["dE"] <= tol and rec["res"] <= tol


def admm_complete(X, mask, iters=100, rho=1.1, mu0=1e-3, mu_max=1e10, L_true=None, tol=None):
    """Algorithm 7 for the completion problem: minimise ||L||_TNN subject to
    X = L + E with E zero on the observed entries.

    X holds the observed values and zeros elsewhere; mask is 1 where
    observed. Starting from L = E = Y = 0 each iteration does
        L <- tsvt(X - E - Y/mu, 1/mu)
        E <- P_unobserved(X - L - Y/mu)
        Y <- Y + mu (L + E - X)
        mu <- min(rho mu, mu_max)
    and then Algorithm 7's check: with tol given, the loop ends after the
    first iteration whose changes ||L_{k+1} - L_k||_inf, ||E_{k+1} - E_k||_inf
    and residual ||L_{k+1} + E_{k+1} - X||_inf are all at most tol; at most
    `iters` iterations run either way. Returns (L, E, Y, history) where
    history holds, per iteration run, the three stop quantities, the
    per-slice ranks, and the relative error against L_true when given.
    """
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(mask, dtype=np.float64)
    L = np.zeros_like(X)
    E = np.zeros_like(X)
    Y = np.zeros_like(X)
    mu = float(mu0)
    hist = []
    for _ in range(int(iters)):
        Lprev, Eprev = L, E
        L, ranks = tsvt(X - E - Y / mu, 1.0 / mu)
        E = (1.0 - W) * (X - L - Y / mu)
        Y = Y + mu * (L + E - X)
        rec = {
            "dL": float(np.max(np.abs(L - Lprev))),
            "dE": float(np.max(np.abs(E - Eprev))),
            "res": float(np.max(np.abs(L + E - X))),
            "ranks": ranks,
            "mu": mu,
        }
        if L_true is not None:
            rec["rse"] = T.rel_fro(L, L_true)
        hist.append(rec)
        mu = min(rho * mu, mu_max)
        if _stopped(rec, tol):
            break
    return L, E, Y, hist


def tcur_tubes(Csl, Rsl, cscale, ridx, rscale, r, ii, jj):
    """Selected tubes Z[ii[e], jj[e], :] of the t-CUR approximation of
    Algorithm 5, from the only parts of A the algorithm reads: the picked
    lateral slices Csl = A[:, cidx, :] and horizontal slices
    Rsl = A[ridx, :, :] (both unscaled). Per Fourier slice,
    Chat_k = fft(Csl)_k D_c, Rhat_k = D_r fft(Rsl)_k, Uhat_k =
    pinv_r(D_r S^T Chat_k) and Zhat_k[i, j] = Chat_k[i, :] Uhat_k Rhat_k[:, j];
    the tube is the inverse transform of Zhat[i, j, :]."""
    Csl = np.asarray(Csl, dtype=np.float64)
    Rsl = np.asarray(Rsl, dtype=np.float64)
    n3 = Csl.shape[2]
    ridx = np.asarray(ridx, dtype=np.int64)
    cscale = np.asarray(cscale, dtype=np.float64)
    rscale = np.asarray(rscale, dtype=np.float64)
    ii = np.asarray(ii, dtype=np.int64)
    jj = np.asarray(jj, dtype=np.int64)
    K = T.half_spectrum_count(n3)
    Hc = T.half_spectrum(Csl)  # (K, n1, c)
    Hr = T.half_spectrum(Rsl)  # (K, l, n2)
    Zh = np.zeros((len(ii), n3), dtype=complex)
    for k in range(K):
        Ck = (Hc[k].real if _is_real_slice(k, n3) else Hc[k]) * cscale[None, :]
        Rk = rscale[:, None] * (Hr[k].real if _is_real_slice(k, n3) else Hr[k])
        Uk = pinv_r(rscale[:, None] * Ck[ridx, :], r)
        Zh[:, k] = np.einsum("ec,ce->e", Ck[ii, :] @ Uk, Rk[:, jj])
    for k in range(K, n3):
        Zh[:, k] = Zh[:, n3 - k].conj()
    return T._real_part_checked(np.fft.ifft(Zh, axis=1))


def tproject_tubes(C, Xcols, jcols, ii, jj):
    """Selected tubes Z[ii[e], jj[e], :] of Algorithm 3's projection
    Z = C * C^+ * X, from C (n1 x c x n3) and the lateral slices of X that
    the tubes need: Xcols[:, t, :] = X[:, jcols[t], :], jj[e] in jcols. Per
    Fourier slice, Zhat_k[i, j] = (Chat_k Chat_k^+)[i, :] Xhat_k[:, j]; the
    tube is the inverse transform of Zhat[i, j, :]."""
    C = np.asarray(C, dtype=np.float64)
    Xcols = np.asarray(Xcols, dtype=np.float64)
    n3 = C.shape[2]
    pos = {int(j): t for t, j in enumerate(np.asarray(jcols, dtype=np.int64))}
    ii = np.asarray(ii, dtype=np.int64)
    tt = np.array([pos[int(j)] for j in np.asarray(jj, dtype=np.int64)], dtype=np.int64)
    K = T.half_spectrum_count(n3)
    Hc = T.half_spectrum(C)  # (K, n1, c)
    Hx = T.half_spectrum(Xcols)  # (K, n1, t)
    Zh = np.zeros((len(ii), n3), dtype=complex)
    for k in range(K):
        Ck = Hc[k].real if _is_real_slice(k, n3) else Hc[k]
        Xk = Hx[k].real if _is_real_slice(k, n3) else Hx[k]
        Pi = Ck[ii, :] @ np.linalg.pinv(Ck)  # rows ii of the projector
        Zh[:, k] = np.einsum("en,ne->e", Pi, Xk[:, tt])
    for k in range(K, n3):
        Zh[:, k] = Zh[:, n3 - k].conj()
    return T._real_part_checked(np.fft.ifft(Zh, axis=1))


def soft_threshold(V, t):
    """Entrywise shrinkage sign(v) max(|v| - t, 0): the minimiser over E of
    t ||E||_1 + 1/2 ||E - V||_F^2 (the closed-form E-update of Algorithm 7)."""
    V = np.asarray(V, dtype=np.float64)
    return np.sign(V) * np.maximum(np.abs(V) - t, 0.0)


def rpca_lambda(shape):
    """Default weight of the l1 term of eq. tlow7, which the paper leaves
    open: 1 / sqrt(max(n1, n2) n3), the value used by the tensor robust PCA
    work that eq. tlow7 is taken from."""
    n1, n2, n3 = shape
    return 1.0 / np.sqrt(max(n1, n2) * n3)


def admm_rpca(X, lam, iters=100, rho=1.1, mu0=1e-3, mu_max=1e10, L_true=None, tol=None):
    """Algorithm 7 as stated, for robust tensor PCA (eq. tlow7): minimise
    ||L||_TNN + lam ||E||_1 subject to X = L + E. From L = E = Y = 0 and
    mu = mu0 every iteration does
        L <- tsvt(X - E - Y/mu, 1/mu)                 (L-update, TNN prox)
        E <- soft_threshold(X - L - Y/mu, lam/mu)     (E-update, l1 prox)
        Y <- Y + mu (L + E - X)
        mu <- min(rho mu, mu_max)
    followed by Algorithm 7's check when tol is given (as in admm_complete),
    for at most `iters` iterations. Returns (L, E, Y, history) with the same
    per-iteration records as admm_complete."""
    X = np.asarray(X, dtype=np.float64)
    L = np.zeros_like(X)
    E = np.zeros_like(X)
    Y = np.zeros_like(X)
    mu = float(mu0)
    hist = []
    for _ in range(int(iters)):
        Lprev, Eprev = L, E
        L, ranks = tsvt(X - E - Y / mu, 1.0 / mu)
        E = soft_threshold(X - L - Y / mu, lam / mu)
        Y = Y + mu * (L + E - X)
        rec = {
            "dL": float(np.max(np.abs(L - Lprev))),
            "dE": float(np.max(np.abs(E - Eprev))),
            "res": float(np.max(np.abs(L + E - X))),
            "ranks": ranks,
            "mu": mu,
        }
        if L_true is not None:
            rec["rse"] = T.rel_fro(L, L_true)
        hist.append(rec)
        mu = min(rho * mu, mu_max)
        if _stopped(rec, tol):
            break
    return L, E, Y, hist


def cur_tnn(X, cidx, ridx, r=None, mask=None, lam=None, iters=100, rho=1.1, mu0=1e-3, mu_max=1e10):
    """Algorithm 6 (CUR t-NN) given its picks. The picked slices are taken
    as they are, without rescaling:
        C = X[:, cidx, :],  Ct = ADMM(C)
        R = X[ridx, :, :],  Rt = ADMM(R)
        W = Ct[ridx, :, :]  (l x c x n3),  U = W^+  (per Fourier slice)
        L = Ct * U * Rt
    ADMM is admm_complete on the matching part of `mask` when a mask is
    given (eq. tlow6) and admm_rpca with weight `lam` otherwise (eq.
    tlow7). The pseudo-inverse of every Fourier slice keeps at most r
    singular values (all when r is None) and drops those at or below
    max(l, c) eps sigma_1. Returns (L, Ct, Rt)."""
    X = np.asarray(X, dtype=np.float64)
    cidx = np.asarray(cidx, dtype=np.int64)
    ridx = np.asarray(ridx, dtype=np.int64)
    n3 = X.shape[2]

    def admm(part, part_mask):
        if part_mask is None:
            return admm_rpca(part, lam, iters, rho, mu0, mu_max)[0]
        return admm_complete(part, part_mask, iters, rho, mu0, mu_max)[0]

    Ct = admm(X[:, cidx, :], None if mask is None else np.asarray(mask)[:, cidx, :])
    Rt = admm(X[ridx, :, :], None if mask is None else np.asarray(mask)[ridx, :, :])
    K = T.half_spectrum_count(n3)
    Ch, Rh = T.fft3(Ct), T.fft3(Rt)
    Lh = np.zeros((X.shape[0], X.shape[1], n3), dtype=complex)
    for k in range(K):
        Ck = Ch[:, :, k].real if _is_real_slice(k, n3) else Ch[:, :, k]
        Rk = Rh[:, :, k].real if _is_real_slice(k, n3) else Rh[:, :, k]
        Uk = pinv_r(Ck[ridx, :], r)
        Lh[:, :, k] = Ck @ Uk @ Rk
    L = T._real_part_checked(T.ifft3(_mirror(Lh, K, n3)))
    return L, Ct, Rt
