"""FP64 CPU oracle for the t-product hot path.

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference that the
GPU library is checked against. Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library itself never
does, and it shares no code with the HIP path (no kernels, headers, helpers,
tables or pre/post-processing).

Everything is NumPy in float64 (the paper runs MATLAB, whose default is
double precision) and follows the paper's definitions in their own order:

* ``tensor``   - circ/unfold/fold t-product, t-transpose, identity, t-SVD,
                 tensor nuclear and spectral norms (Section 2).
* ``philox``   - the counter-based generator both sides draw Bernoulli picks
                 from (the paper does not name one).
* ``sampling`` - slice norms, the sampling probabilities of Section 3 and the
                 exact-integer pick procedure.
* ``decomp``   - rt-product (Algorithm 2), t-project / t-CX (Algorithms 3-4),
                 t-CUR (Algorithm 5), CUR t-NN (Algorithm 6), t-SVT and the
                 ADMM of Algorithm 7 for robust tensor PCA (eq. tlow7) and
                 for the completion problem (eq. tlow6).
* ``mlp``      - the learned leverage proposal (not in the paper).

Parity status of every function is listed in its module header.
"""
