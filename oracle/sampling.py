"""Slice statistics, sampling probabilities and slice picks (oracle; test
infrastructure only).

Probabilities (Section 3):
* norm2       p_j = ||A_{:j:}||_F^2 / ||A||_F^2                eq. nonoptimal_probs
* normprod    p_j ~ ||A_{:j:}||_F ||B_{j::}||_F                eq. nearly_optimal_probs
* lateral leverage    p_j ~ ||Vhat_{j::}||_F^2, V the top-r right singular
                      slices of the t-SVD                      eq. cur-col-prob
* horizontal leverage p_i ~ ||Uhat^(C)_{i::}||_F^2, U^(C) the top-r left
                      singular slices of C (the printed formula is garbled:
                      no square and the wrong factor; this reading squares
                      the Frobenius norm and normalises by the actual sum)
                                                               eq. colprob_rows_exact
All are returned unnormalised; picks only depend on ratios.

Picks (Algorithm 2 and its copies in Algorithms 4 and 5): slice i is kept
with probability min(1, c p_i) and rescaled by 1/sqrt(min(1, c p_i)).
The paper names no generator and no arithmetic for the coin flips. The
reading used here makes every decision an exact integer comparison, so CPU
and GPU agree bit for bit given the same weights:

1. weights -> q_i = floor(w_i * 2^(B-e)), e the binary exponent of max w
   (w_max = m 2^e, m in [0.5, 1)) and B = 62 - ceil(log2 n); a power-of-two
   scaling, exact in float64. S = sum q_i < 2^62 exactly.
2. u_i = word 0 of Philox4x64-10 at key (seed, stream), counter (i,0,0,0).
3. Bernoulli (the paper's scheme): keep i iff c q_i >= S or
   floor(u_i S / 2^64) < c q_i, i.e. u_i / 2^64 < c q_i / S. Output in
   ascending slice order, as Algorithm 2 fills S and D.
4. IID (exactly c draws with replacement, the n3 = 1 scheme of Drineas,
   Kannan and Mahoney that Algorithm 2 reduces to): draw t uses counter t,
   T = floor(u_t S / 2^64), j_t = the first i whose inclusive prefix sum of
   q exceeds T. Output in draw order; scale 1/sqrt(c q_j / S).
5. Uniform without replacement (Corollaries cor:proj-main and cor:gnys-main):
   the c slices with the smallest u_i (ties to the smaller index), ascending;
   scale sqrt(n / c).
Scales use float64 conversion, division and square root, each correctly
rounded.

Pins (tests/test_oracle_sampling.py): inclusion frequencies over many seeds
against min(1, c p_i) (chi-square), expected count, IID frequencies against
q_i / S, uniform draws distinct and of size c, leverage sums and the
Fourier/original-domain leverage identity used in the proof of
Theorem thm:regress-main, quantisation invariance under power-of-two scaling.
"""

import math

import numpy as np

from . import tensor as T
from .philox import uniform_u64

MASK64 = (1 << 64) - 1


# ---------------------------------------------------------------------------
# Slice statistics and probabilities
# ---------------------------------------------------------------------------

def lateral_sq_norms(A):
    """||A_{:j:}||_F^2 for every lateral slice j."""
    A = np.asarray(A, dtype=np.float64)
    return np.einsum("ijk,ijk->j", A, A)


def horizontal_sq_norms(B):
    """||B_{i::}||_F^2 for every horizontal slice i."""
    B = np.asarray(B, dtype=np.float64)
    return np.einsum("ijk,ijk->i", B, B)


def weights_norm2(A):
    """Unnormalised eq. nonoptimal_probs (beta = 1)."""
    return lateral_sq_norms(A)


def weights_normprod(A, B):
    """Unnormalised eq. nearly_optimal_probs (beta = 1)."""
    a = lateral_sq_norms(A)
    b = horizontal_sq_norms(B)
    return np.sqrt(a * b)


def weights_lateral_leverage(A, r):
    """Unnormalised eq. cur-col-prob: ||Vhat_{j::}||_F^2 summed over all n3
    Fourier slices, V the top-r right singular slices of A."""
    _, _, V, _ = T.tsvd(A, r=r)
    Vh = T.fft3(V)
    return np.sum(np.abs(Vh) ** 2, axis=(1, 2))


def weights_horizontal_leverage(C, r):
    """Unnormalised horizontal leverage: ||Uhat^(C)_{i::}||_F^2 over all n3
    Fourier slices, U^(C) the top-r left singular slices of C."""
    U, _, _, _ = T.tsvd(C, r=r)
    Uh = T.fft3(U)
    return np.sum(np.abs(Uh) ** 2, axis=(1, 2))


def normalise(w):
    w = np.asarray(w, dtype=np.float64)
    return w / w.sum()


# ---------------------------------------------------------------------------
# Exact-integer picks
# ---------------------------------------------------------------------------

def _check_weights(w):
    w = [float(x) for x in np.asarray(w, dtype=np.float64).ravel()]
    if len(w) == 0:
        raise ValueError("empty weight vector")
    for x in w:
        if not math.isfinite(x) or x < 0.0:
            raise ValueError("weights must be finite and non-negative")
    if max(w) <= 0.0:
        raise ValueError("all weights are zero")
    return w


def quantize(w):
    """Return (q, S): q_i = floor(w_i 2^(B-e)) as Python ints and their sum."""
    w = _check_weights(w)
    n = len(w)
    _, e = math.frexp(max(w))
    B = 62 - (n - 1).bit_length()
    q = [int(math.floor(math.ldexp(x, B - e))) for x in w]
    S = sum(q)
    return q, S


def _scale_from(t, S):
    p = min(1.0, float(t) / float(S))
    return 1.0 / math.sqrt(p)


def sample_bernoulli(w, c, seed, stream=0):
    """Algorithm 2's picks: keep i with probability min(1, c p_i)."""
    q, S = quantize(w)
    n = len(q)
    if not (1 <= c <= n):
        raise ValueError("need 1 <= c <= n")
    idx, scale = [], []
    for i in range(n):
        t = c * q[i]
        if t >= S:
            keep = True
        else:
            u = uniform_u64(seed, stream, i)
            keep = ((u * S) >> 64) < t
        if keep:
            idx.append(i)
            scale.append(_scale_from(t, S))
    return np.array(idx, dtype=np.int64), np.array(scale, dtype=np.float64)


def sample_iid(w, c, seed, stream=0):
    """Exactly c draws with replacement, P(j) = q_j / S."""
    q, S = quantize(w)
    n = len(q)
    if not (1 <= c <= n):
        raise ValueError("need 1 <= c <= n")
    prefix = []
    acc = 0
    for x in q:
        acc += x
        prefix.append(acc)
    idx, scale = [], []
    for t in range(c):
        u = uniform_u64(seed, stream, t)
        target = (u * S) >> 64
        # first i with prefix[i] > target (binary search over the inclusive sums)
        lo, hi = 0, n - 1
        while lo < hi:
            mid = (lo + hi) // 2
            if prefix[mid] > target:
                hi = mid
            else:
                lo = mid + 1
        idx.append(lo)
        scale.append(1.0 / math.sqrt(float(c * q[lo]) / float(S)))
    return np.array(idx, dtype=np.int64), np.array(scale, dtype=np.float64)


def sample_uniform_norepl(n, c, seed, stream=0):
    """c distinct slices, uniformly: the c smallest Philox draws."""
    if not (1 <= c <= n):
        raise ValueError("need 1 <= c <= n")
    keys = [(uniform_u64(seed, stream, i), i) for i in range(n)]
    keys.sort()
    idx = sorted(i for _, i in keys[:c])
    sc = math.sqrt(float(n) / float(c))
    return np.array(idx, dtype=np.int64), np.full(len(idx), sc)


def sample(w, c, mode, seed, stream=0):
    """Dispatch on mode in {"bernoulli", "iid", "uniform"}; ``w`` is ignored
    (only its length) for "uniform"."""
    if mode == "bernoulli":
        return sample_bernoulli(w, c, seed, stream)
    if mode == "iid":
        return sample_iid(w, c, seed, stream)
    if mode == "uniform":
        return sample_uniform_norepl(len(np.asarray(w).ravel()), c, seed, stream)
    raise ValueError(mode)
