"""Writes completion_rse_256x256x100.txt: the oracle's ADMM completion run on
the 256x256x100 tubal-rank-15 workload (noise variance 0.01, half of the
entries observed), 100 iterations with rho = 1.1, mu0 = 1e-3, mu_max = 1e10
(Algorithm 7 and its parameters, completion variant), recording the relative
error ||L_t - L*||_F / ||L*||_F and the largest per-slice rank after every
iteration. Calls only the oracle and the seeded generators.

    python tests/golden/make_completion_rse.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import decomp as D  # noqa: E402
from oracle import tensor as T  # noqa: E402


def main():
    G1, G2, N, mask = W.completion_problem(dtype=np.float64)
    Ls = T.tprod_fft(G1, G2)
    X = (Ls + N) * mask
    _, _, _, hist = D.admm_complete(X, mask, iters=100, L_true=Ls)
    out = os.path.join(HERE, "completion_rse_256x256x100.txt")
    with open(out, "w") as f:
        f.write("# Oracle ADMM completion (Algorithm 7, completion variant; rho=1.1, mu0=1e-3, mu_max=1e10)\n")
        f.write("# workload: L* = G1 * G2 (256x15x100, 15x256x100, N(0,1)), X = (L* + N(0, 0.01)) on a\n")
        f.write("# Bernoulli(0.5) mask, seeds of workloads.completion_problem; written by make_completion_rse.py\n")
        f.write("# iteration rse max_rank mu\n")
        for i, h in enumerate(hist):
            f.write(f"{i} {h['rse']:.10e} {int(h['ranks'].max())} {h['mu']:.10e}\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
