"""GPU parity of the dense leading-r t-SVD (tp_tsvd_full) against the FP64
oracle's t-SVD from dense per-slice SVDs (t-SVD theorem, Section 2.1).

Singular vectors are unique only up to a phase per column and Fourier slice
(and within equal singular values), so the tests compare what is unique:
the singular values, the t-orthonormality U^T * U = I, the energy the
leading r columns capture in every Fourier slice, and, where the spectrum
has a gap after r, the projector U * U^T. Tolerances: the Gram matrix in
float32 squares the condition number, so a singular value carries 1e-5
relative plus 8 eps_32 sigma_max^2 / sigma; orthonormality and energy 1e-5,
projectors 1e-4. Slices whose longer side is more than four times the
shorter go through the Gram matrix ((200, 48), (30, 150), (400, 80), and
(4100, 40) and (9000, 100), the latter's Gram product on the float32
matrix cores with its long contraction split into parts); the others through the block Jacobi on the slices themselves
(on A^H through the t-transpose when tall)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import tensor as T

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1704_04362_amd.api")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def _slices(X):
    Xh = T.fft3(X)
    return [Xh[:, :, k] for k in range(X.shape[2] // 2 + 1)]


@pytest.mark.parametrize("shape,r", [((200, 48, 6), 20), ((40, 90, 5), 12), ((64, 64, 4), 64), ((50, 30, 1), 10),
                                     ((300, 130, 8), 100), ((33, 70, 7), 33), ((60, 40, 300), 10),
                                     ((30, 150, 4), 10), ((4100, 40, 4), 12), ((9000, 100, 2), 10)])
def test_tsvd_full_matches_oracle(shape, r):
    A = np.random.default_rng(sum(shape) + r).standard_normal(shape).astype(np.float32)
    Ad = A.astype(np.float64)
    U, S_ = api.tsvd_full(dev(A), r)
    U = U.cpu().numpy().astype(np.float64)
    _, _, _, sv = T.tsvd(Ad)
    # the float32 Gram perturbs an eigenvalue by ~eps_32 lambda_max, hence
    # sigma by ~eps_32 sigma_max^2 / (2 sigma): a bound of 8 eps_32 on that
    # term (the square 64 x 64 slices have sigma_max / sigma_min ~ 200)
    s_ref = sv[:, :r]
    bound = 1e-5 * s_ref + 4.8e-7 * sv.max() ** 2 / s_ref
    assert np.all(np.abs(S_.cpu().numpy() - s_ref) <= bound)
    # t-orthonormal columns: U^T * U is the r x r identity tensor
    assert rel(T.tprod_fft(T.ttranspose(U), U), T.teye(r, shape[2])) < 1e-5
    # every Fourier slice: the r columns capture the top-r energy of A_k
    for k, (Uk, Ak) in enumerate(zip(_slices(U), _slices(Ad))):
        got = np.linalg.norm(Uk.conj().T @ Ak) ** 2
        want = float(np.sum(sv[k, :r] ** 2))
        assert abs(got - want) < 1e-5 * want, k


@pytest.mark.parametrize("shape", [(400, 80, 6), (60, 150, 5)])
def test_tsvd_full_projector_on_low_rank(shape):
    # tubal rank 8 plus small noise: a clear gap after the 8th singular
    # value, so the leading subspace (the projector U * U^T) is unique
    n1, n2, n3 = shape
    G1, G2, N = W.lowrank_factors(n1, n2, n3, 8, noise_var=1e-6, salt=n1, dtype=np.float64)
    A = T.tprod_fft(G1, G2) + N
    U, _ = api.tsvd_full(dev(A.astype(np.float32)), 8)
    U = U.cpu().numpy().astype(np.float64)
    Ur = T.tsvd(A, 8)[0]
    P = T.tprod_fft(U, T.ttranspose(U))
    Pr = T.tprod_fft(Ur, T.ttranspose(Ur))
    assert rel(P, Pr) < 1e-4


@pytest.mark.parametrize("shape", [(90, 40, 4), (40, 90, 4), (200, 40, 4), (30, 150, 4)])
def test_tsvd_full_rank_deficient_gives_zero_columns(shape):
    # tubal rank 3 and r = 5: the two extra columns belong to zero singular
    # values, which every route reports as exactly 0 with a zero column; the
    # first three are orthonormal. Shapes: tall and wide slices on the direct
    # route, tall and wide on the Gram route.
    n1, n2, n3 = shape
    G1, G2, _ = W.lowrank_factors(n1, n2, n3, 3, noise_var=0.0, salt=5, dtype=np.float64)
    A = T.tprod_fft(G1, G2).astype(np.float32)
    U, S_ = api.tsvd_full(dev(A), 5)
    s = S_.cpu().numpy()
    assert np.all(s[:, 3:] == 0.0)
    assert np.all(s[:, :3] > 0.0)
    U = U.cpu().numpy().astype(np.float64)
    assert np.all(U[:, 3:, :] == 0.0)
    assert rel(T.tprod_fft(T.ttranspose(U[:, :3]), U[:, :3]), T.teye(3, n3)) < 1e-4


@pytest.mark.parametrize("shape", [(72, 40, 6), (40, 90, 5)])
def test_tsvd_full_direct_path_resolves_a_graded_spectrum(shape):
    # singular values over four decades: the Jacobi on the slices themselves
    # keeps an absolute error of a few float32 roundings of sigma_max, which
    # the Gram route (error ~ eps_32 sigma_max^2 / sigma) could not
    n1, n2, n3 = shape
    m = min(n1, n2)
    g = np.random.default_rng(n1 + n2)
    G1 = g.standard_normal((n1, m, n3))
    G2 = g.standard_normal((m, n2, n3)) * (10.0 ** (-4.0 * np.arange(m) / m))[:, None, None]
    A = T.tprod_fft(G1, G2).astype(np.float32)
    r = m // 2
    U, S_ = api.tsvd_full(dev(A), r)
    _, _, _, sv = T.tsvd(A.astype(np.float64))
    s_ref = sv[:, :r]
    assert np.all(np.abs(S_.cpu().numpy() - s_ref) <= 1e-5 * s_ref + 2e-6 * sv.max())
    U = U.cpu().numpy().astype(np.float64)
    assert rel(T.tprod_fft(T.ttranspose(U), U), T.teye(r, n3)) < 1e-5


def test_tsvd_full_reports_unconverged_slices():
    """Both routes (near-square slices and the Gram route) report 0 slices
    whose sweeps hit the cap on ordinary inputs, and give the same U and S
    with and without the count."""
    rs = np.random.default_rng(67)
    for shape, r in [((40, 48, 6), 5), ((300, 20, 5), 4)]:
        A = rs.standard_normal(shape).astype(np.float32)
        U, S, unc = api.tsvd_full(dev(A), r, with_unconverged=True)
        U2, S2 = api.tsvd_full(dev(A), r)
        assert int(unc.item()) == 0
        np.testing.assert_array_equal(U.cpu().numpy(), U2.cpu().numpy())
        np.testing.assert_array_equal(S.cpu().numpy(), S2.cpu().numpy())

