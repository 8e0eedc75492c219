"""Raw random arrays for the synthetic workloads.

Data seeds are 17040436 + workload id; every array is drawn in float64 and
cast by the caller. Shapes and distributions:

* exact     (id 1): A 64x48x16, B 48x32x16, i.i.d. N(0, 1).
* rtprod    (id 2): A 512x2048x64, B 2048x512x64; A_{:j:} = exp(g_j) G_{:j:},
                    B_{j::} = exp(h_j) H_{j::} with G, H, g, h i.i.d. N(0, 1)
                    (lognormal(0, 1) slice scales, independent for A and B).
* lowrank   (id 3): factors G1 n1 x r x n3, G2 r x n2 x n3 ~ N(0, 1) and a
                    noise tensor N(0, v) with v = 1e-3 read as the variance;
                    default 1024x1024x128, r = 20.
* complete  (id 4): factors 256x15x100 and 15x256x100 ~ N(0, 1), noise of
                    variance 0.01, observation mask Bernoulli(0.5) as uint8.
* learned   (id 5): tensor factors with tubal rank r in 5..40 whose
                    horizontal slices of G1 and lateral slices of G2 carry
                    exp(sigma_c xi) scales, sigma_c ~ U[0, 2] (the coherence
                    knob), xi ~ N(0, 1).
"""

import numpy as np

SEED_BASE = 17040436

__all__ = [
    "SEED_BASE", "rng", "gaussian", "exact_pair", "rtprod_pair",
    "lowrank_factors", "completion_problem", "rpca_problem", "salt_pepper_problem",
    "learned_factors",
    "lognormal_weights",
]


def rng(workload_id, salt=0):
    return np.random.default_rng([SEED_BASE + int(workload_id), int(salt)])


def gaussian(shape, seed, salt=0, dtype=np.float64):
    g = np.random.default_rng([int(seed), int(salt)])
    return g.standard_normal(shape).astype(dtype)


def exact_pair(n1=64, n2=48, n4=32, n3=16, salt=0):
    g = rng(1, salt)
    A = g.standard_normal((n1, n2, n3))
    B = g.standard_normal((n2, n4, n3))
    return A, B


def rtprod_pair(n1=512, n2=2048, n4=512, n3=64, salt=0, dtype=np.float32):
    """Gaussian tensors whose lateral slices of A and horizontal slices of B
    carry independent lognormal(0, 1) scales."""
    g = rng(2, salt)
    sa = np.exp(g.standard_normal(n2))
    sb = np.exp(g.standard_normal(n2))
    A = g.standard_normal((n1, n2, n3), dtype=np.float32 if dtype == np.float32 else np.float64)
    A *= sa[None, :, None].astype(A.dtype)
    B = g.standard_normal((n2, n4, n3), dtype=np.float32 if dtype == np.float32 else np.float64)
    B *= sb[:, None, None].astype(B.dtype)
    return A.astype(dtype, copy=False), B.astype(dtype, copy=False)


def lowrank_factors(n1=1024, n2=1024, n3=128, r=20, noise_var=1e-3, salt=0, dtype=np.float32):
    """(G1, G2, N): A = G1 * G2 + N has tubal rank r plus noise."""
    g = rng(3, salt)
    f32 = np.float32 if dtype == np.float32 else np.float64
    G1 = g.standard_normal((n1, r, n3), dtype=f32)
    G2 = g.standard_normal((r, n2, n3), dtype=f32)
    N = g.standard_normal((n1, n2, n3), dtype=f32)
    N *= f32(np.sqrt(noise_var))
    return G1.astype(dtype, copy=False), G2.astype(dtype, copy=False), N.astype(dtype, copy=False)


def completion_problem(n1=256, n2=256, n3=100, r=15, noise_var=0.01, p_obs=0.5, salt=0,
                       dtype=np.float32):
    """(G1, G2, N, mask): L* = G1 * G2, X = (L* + N) on the mask."""
    g = rng(4, salt)
    G1 = g.standard_normal((n1, r, n3)).astype(dtype)
    G2 = g.standard_normal((r, n2, n3)).astype(dtype)
    N = (g.standard_normal((n1, n2, n3)) * np.sqrt(noise_var)).astype(dtype)
    mask = (g.random((n1, n2, n3)) < p_obs).astype(np.uint8)
    return G1, G2, N, mask


def rpca_problem(n1=48, n2=40, n3=6, r=2, spike_frac=0.05, spike_mag=5.0, salt=0, dtype=np.float64):
    """(G1, G2, S): L* = G1 * G2 has tubal rank r; S holds +-spike_mag on a
    spike_frac share of the entries (positions and signs uniform) and zeros
    elsewhere, so X = L* + S is a low-rank tensor with sparse gross errors."""
    g = rng(6, salt)
    G1 = g.standard_normal((n1, r, n3))
    G2 = g.standard_normal((r, n2, n3))
    hit = g.random((n1, n2, n3)) < spike_frac
    S = np.where(hit, spike_mag * np.where(g.random((n1, n2, n3)) < 0.5, -1.0, 1.0), 0.0)
    return G1.astype(dtype), G2.astype(dtype), S.astype(dtype)


def salt_pepper_problem(n1=192, n2=1140, n3=168, r=10, frac=0.2, salt=0):
    """(G1, G2, hit, high): factors of a tubal-rank-r tensor (float32) and a
    salt-and-pepper corruption pattern: hit marks a frac share of the entries
    (uniform positions), high says whether a hit entry is set to the top
    (True) or the bottom (False) of the value range. The default shape is
    that of the Extended Yale B face tensor (192 x 1140 x 168)."""
    g = rng(7, salt)
    G1 = g.standard_normal((n1, r, n3), dtype=np.float32)
    G2 = g.standard_normal((r, n2, n3), dtype=np.float32)
    hit = g.random((n1, n2, n3), dtype=np.float32) < frac
    high = g.random((n1, n2, n3), dtype=np.float32) < 0.5
    return G1, G2, hit, high


def learned_factors(index, n1=512, n2=512, n3=64, rmin=5, rmax=40, salt=0, dtype=np.float32):
    """Factors of the index-th generated tensor of the learned-proposal set.
    Returns (G1, G2, r, sigma_c)."""
    g = rng(5, 1_000_003 * int(salt) + int(index))
    r = int(g.integers(rmin, rmax + 1))
    sigma_c = float(g.uniform(0.0, 2.0))
    G1 = g.standard_normal((n1, r, n3))
    G2 = g.standard_normal((r, n2, n3))
    G1 *= np.exp(sigma_c * g.standard_normal(n1))[:, None, None]
    G2 *= np.exp(sigma_c * g.standard_normal(n2))[None, :, None]
    return G1.astype(dtype), G2.astype(dtype), r, sigma_c


def lognormal_weights(n, seed, zeros=0, sigma=1.0):
    """Positive weights exp(sigma xi) with ``zeros`` of them set to 0."""
    g = np.random.default_rng([int(seed), 77])
    w = np.exp(sigma * g.standard_normal(n))
    if zeros:
        w[g.choice(n, size=zeros, replace=False)] = 0.0
    return w
