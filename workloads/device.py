"""Device-side random arrays for the learned-proposal workload (id 5).

The set has thousands of 512x512x64 tensors, too many to draw on the host,
so their Gaussian parts are drawn on the GPU by torch's generator (seeded
per tensor) and their scalars (tubal rank r ~ U{5..40}, coherence knob
sigma_c ~ U[0, 2]) by NumPy. Only random draws live here: the caller forms
A = G1 * G2 + noise with its own t-product.

learned_parts(index) returns float32 tensors on the device:
  G1 (n1 x r x n3) with horizontal slice i scaled by exp(sigma_c xi_i),
  G2 (r x n2 x n3) with lateral slice j scaled by exp(sigma_c zeta_j), and
     latent factor t supported on a random set of
     max(1, round(n2^(1 - sigma_c u_t / 2))) lateral slices (u_t ~ U[0, 1];
     zero elsewhere), so that as sigma_c grows some directions of the
     tensor live in a handful of lateral slices (coherent, concentrated
     leverage) while at sigma_c = 0 every slice mixes all of them;
  N  (n1 x n2 x n3) i.i.d. N(0, 1) (the caller scales it relative to A),
and the scalars r and sigma_c. xi, zeta ~ N(0, 1).
"""

import numpy as np
import torch

from .generators import SEED_BASE

LEARNED_ID = 5


def learned_scalars(index, rmin=5, rmax=40):
    g = np.random.default_rng([SEED_BASE + LEARNED_ID, 7, int(index)])
    r = int(g.integers(rmin, rmax + 1))
    sigma_c = float(g.uniform(0.0, 2.0))
    u = g.uniform(0.0, 1.0, size=r)
    return r, sigma_c, u


def learned_parts(index, device="cuda", n1=512, n2=512, n3=64, rmin=5, rmax=40, with_noise=True):
    r, sigma_c, u = learned_scalars(index, rmin, rmax)
    gen = torch.Generator(device=device)
    gen.manual_seed((SEED_BASE + LEARNED_ID) * 1_000_003 + int(index))
    G1 = torch.randn((n1, r, n3), generator=gen, device=device, dtype=torch.float32)
    G2 = torch.randn((r, n2, n3), generator=gen, device=device, dtype=torch.float32)
    xi = torch.randn(n1, generator=gen, device=device, dtype=torch.float32)
    zeta = torch.randn(n2, generator=gen, device=device, dtype=torch.float32)
    G1 *= torch.exp(sigma_c * xi)[:, None, None]
    G2 *= torch.exp(sigma_c * zeta)[None, :, None]
    for t in range(r):
        m = max(1, int(round(n2 ** (1.0 - sigma_c * u[t] / 2.0))))
        keep = torch.randperm(n2, generator=gen, device=device)[:m]
        mask = torch.zeros(n2, dtype=torch.float32, device=device)
        mask[keep] = 1.0
        G2[t] *= mask[:, None]
    N = torch.randn((n1, n2, n3), generator=gen, device=device, dtype=torch.float32) if with_noise else None
    return G1, G2, N, r, sigma_c
