"""Thin torch binding of the C ABI (argument marshalling only).

Every function takes and returns torch tensors on the current HIP device and
enqueues its work on torch's current stream. Outputs and the workspace are
allocated with torch; all arithmetic runs in the HIP kernels of libtprod.so.
There is no CPU path: CPU tensors are rejected.
"""
import ctypes as C

import torch

from . import _lib as L

_DT = {torch.float32: L.TP_F32, torch.float64: L.TP_F64}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need_gpu(*ts):
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("tensors must live on the GPU")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")


def _out(out, shape, dtype, device):
    """The caller's output tensor after checking it can be written by the
    kernels as a dense array of `shape` and `dtype` on `device`, or a new
    one."""
    shape = tuple(int(v) for v in shape)
    if out is None:
        return torch.empty(shape, dtype=dtype, device=device)
    _need_gpu(out)
    if out.dtype != dtype:
        raise ValueError(f"out must be {dtype}, got {out.dtype}")
    if tuple(out.shape) != shape:
        raise ValueError(f"out must have shape {shape}, got {tuple(out.shape)}")
    if out.device != torch.device(device):
        raise ValueError("out must live on the inputs' device")
    return out


def _tensor(x):
    if x.dim() != 3:
        raise ValueError("expected a 3-way tensor")
    if x.dtype not in _DT:
        raise ValueError("dtype must be float32 or float64")
    return L.Tensor(x.data_ptr(), _DT[x.dtype], x.shape[0], x.shape[1], x.shape[2])


def _spectrum(re, im):
    return L.Spectrum(re.data_ptr(), im.data_ptr(), _DT[re.dtype], re.shape[0], re.shape[1], re.shape[2])


_WS_CACHE = {}


def _ws(nbytes, device):
    """Workspace for one call. One buffer is kept per (device, stream) and
    reused: calls on the same stream run in order, so a buffer is never in use
    by two calls at once; it grows when a call needs more."""
    nbytes = max(int(nbytes), 1)
    key = (torch.device(device).index, torch.cuda.current_stream(device).cuda_stream)
    buf = _WS_CACHE.get(key)
    if buf is None or buf.numel() < nbytes:
        _WS_CACHE.pop(key, None)
        buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        _WS_CACHE[key] = buf
    return buf


def half_count(n3):
    return n3 // 2 + 1


def tfft(X, out=None):
    """Half spectrum (re, im), each K x n1 x n2, of fft(X, [], 3); out =
    (re, im) to write into existing tensors."""
    _need_gpu(X)
    shape = (half_count(X.shape[2]), X.shape[0], X.shape[1])
    re = _out(out[0] if out else None, shape, X.dtype, X.device)
    im = _out(out[1] if out else None, shape, X.dtype, X.device)
    L.check(L.load().tp_tfft(C.byref(_tensor(X)), C.byref(_spectrum(re, im)), _stream()))
    return re, im


def tifft(re, im, n3, out=None):
    """Real tensor rows x cols x n3 whose half spectrum is (re, im)."""
    _need_gpu(re, im)
    X = _out(out, (re.shape[1], re.shape[2], n3), re.dtype, re.device)
    L.check(L.load().tp_tifft(C.byref(_spectrum(re, im)), C.byref(_tensor(X)), _stream()))
    return X


def spectrum_matmul(a, b, op_a=0, op_b=0, real_last=True, prec="f32"):
    """Per-slice products C_k = op(A_k) op(B_k); a and b are (re, im) pairs."""
    are, aim = a
    bre, bim = b
    _need_gpu(are, aim, bre, bim)
    M = are.shape[2] if op_a else are.shape[1]
    N = bre.shape[1] if op_b else bre.shape[2]
    cre = torch.empty((are.shape[0], M, N), dtype=are.dtype, device=are.device)
    cim = torch.empty_like(cre)
    L.check(L.load().tp_spectrum_matmul(C.byref(_spectrum(are, aim)), int(op_a), C.byref(_spectrum(bre, bim)),
                                         int(op_b), C.byref(_spectrum(cre, cim)), int(bool(real_last)),
                                         L.PREC[prec], _stream()))
    return cre, cim


def slice_norms(A, mode="lateral"):
    """Squared Frobenius norms of lateral (mode "lateral") or horizontal
    slices, float64."""
    _need_gpu(A)
    m = 0 if mode == "lateral" else 1
    n = A.shape[1] if m == 0 else A.shape[0]
    out = torch.empty(n, dtype=torch.float64, device=A.device)
    t = _tensor(A)
    lib = L.load()
    ws = _ws(lib.tp_slice_norms_workspace(C.byref(t), m), A.device)
    L.check(lib.tp_slice_norms(C.byref(t), m, out.data_ptr(), ws.data_ptr(), ws.numel(), _stream()))
    return out


class Picks:
    """Device-resident picks: idx (int32), scale (float64), count (int64[1])."""

    def __init__(self, cap, device):
        self.idx = torch.empty(cap, dtype=torch.int32, device=device)
        self.scale = torch.empty(cap, dtype=torch.float64, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        self.cap = cap

    def struct(self):
        return L.Sample(self.idx.data_ptr(), self.scale.data_ptr(), self.cap, self.count.data_ptr())

    def host(self):
        """(idx, scale) trimmed to the live count, as CPU tensors (syncs)."""
        n = int(self.count.item())
        if n < 0:
            raise ValueError("sampling rejected the weights (non-finite, negative or all zero)")
        return self.idx[:n].cpu(), self.scale[:n].cpu()


def tsample(kind, c, mode="iid", seed=0, stream_id=0, A=None, B=None, w=None, n=None, cap=None, out=None):
    """Pick c slices (see tp_tsample). kind in {"user", "uniform", "norm2",
    "normprod"}; for "user" pass float64 device weights w."""
    _need_gpu(A, B, w)
    if n is None:
        n = A.shape[1] if A is not None else w.numel()
    device = (A if A is not None else w).device if (A is not None or w is not None) else torch.device("cuda")
    if out is None:
        out = Picks(cap if cap is not None else (n if mode == "bernoulli" else c), device)
    lib = L.load()
    ta = C.byref(_tensor(A)) if A is not None else None
    tb = C.byref(_tensor(B)) if B is not None else None
    ws_bytes = lib.tp_tsample_workspace(n)
    if A is not None:
        ws_bytes += lib.tp_slice_norms_workspace(C.byref(_tensor(A)), 0)
    ws = _ws(ws_bytes, device)
    s = out.struct()
    L.check(lib.tp_tsample(L.KIND[kind], ta, tb, w.data_ptr() if w is not None else None, int(n), int(c),
                           L.MODE[mode], int(seed), int(stream_id), C.byref(s), ws.data_ptr(), ws.numel(),
                           _stream()))
    return out


def tprod(A, B, picks=None, prec=None, out=None):
    """t-product A * B (Algorithm 1), or the rt-product of Algorithm 2 when
    picks (from tsample over A's lateral slices) are given."""
    _need_gpu(A, B)
    if prec is None:
        prec = "f64" if A.dtype == torch.float64 else "f32"
    C_ = _out(out, (A.shape[0], B.shape[1], A.shape[2]), A.dtype, A.device)
    lib = L.load()
    ta, tb, tc = _tensor(A), _tensor(B), _tensor(C_)
    ps = picks.struct() if picks is not None else None
    sp = C.byref(ps) if ps is not None else None
    ws = _ws(lib.tp_tprod_workspace(C.byref(ta), C.byref(tb), sp, L.PREC[prec]), A.device)
    L.check(lib.tp_tprod(C.byref(ta), C.byref(tb), sp, C.byref(tc), L.PREC[prec], ws.data_ptr(), ws.numel(),
                         _stream()))
    return C_


def tsvd_rand(A, r, p=10, q=1, seed=0, prec=None, picks=None):
    """Leading-r t-SVD summary by the randomized range finder: returns
    (S, lev_lateral, lev_horizontal) with S the K x r singular values of the
    Fourier slices and the unnormalised tubal leverage scores (float64).
    picks (lateral slices of A, e.g. from tsample) replace the Gaussian
    sketch by the t-CX basis."""
    S, _, _, _, lat, hor = _tsvd_rand(A, r, p, q, seed, prec, picks, scores=True)
    return S, lat, hor


def tsvd_rand_factors(A, r, p=10, q=1, seed=0, prec=None, picks=None):
    """The randomized tubal-rank-r t-SVD as tensors: returns (U, S, V, Z)
    with U (n1 x r x n3) and V (n2 x r x n3) the first r left and right
    singular slices, S their K x r singular values and Z = U * S * V^T the
    rank-r approximation (see tp_tsvd_rand)."""
    S, U, V, Z, _, _ = _tsvd_rand(A, r, p, q, seed, prec, picks, factors=True)
    return U, S, V, Z


def _tsvd_rand(A, r, p, q, seed, prec, picks, scores=False, factors=False):
    _need_gpu(A)
    if prec is None:
        prec = "f64" if A.dtype == torch.float64 else "f32"
    n1, n2, n3 = A.shape
    K = half_count(n3)
    S = torch.empty((K, r), dtype=torch.float64, device=A.device)
    lat = torch.empty(n2, dtype=torch.float64, device=A.device) if scores else None
    hor = torch.empty(n1, dtype=torch.float64, device=A.device) if scores else None
    U = torch.empty((n1, r, n3), dtype=A.dtype, device=A.device) if factors else None
    V = torch.empty((n2, r, n3), dtype=A.dtype, device=A.device) if factors else None
    Z = torch.empty_like(A) if factors else None
    lib = L.load()
    t = _tensor(A)
    ps = picks.struct() if picks is not None else None
    sp = C.byref(ps) if ps is not None else None
    ws = _ws(lib.tp_tsvd_rand_workspace(C.byref(t), r, p, sp, L.PREC[prec]), A.device)
    opt = lambda x: C.byref(_tensor(x)) if x is not None else None  # noqa: E731
    ptr = lambda x: x.data_ptr() if x is not None else None  # noqa: E731
    L.check(lib.tp_tsvd_rand(C.byref(t), int(r), int(p), int(q), sp, int(seed), L.PREC[prec], S.data_ptr(), opt(U),
                             opt(V), opt(Z), ptr(lat), ptr(hor), ws.data_ptr(), ws.numel(), _stream()))
    return S, U, V, Z, lat, hor


def tproject(X, Cs, prec=None, out=None):
    """t-project of Algorithm 3: Z = C * C^+ * X (more than 64 lateral
    slices in C: float32 data, see tp_tproject)."""
    _need_gpu(X, Cs)
    if prec is None:
        prec = "f64" if X.dtype == torch.float64 else "f32"
    Z = _out(out, X.shape, X.dtype, X.device)
    lib = L.load()
    tx, tc, tz = _tensor(X), _tensor(Cs), _tensor(Z)
    ws = _ws(lib.tp_tproject_workspace(C.byref(tx), C.byref(tc), L.PREC[prec]), X.device)
    L.check(lib.tp_tproject(C.byref(tx), C.byref(tc), C.byref(tz), L.PREC[prec], ws.data_ptr(), ws.numel(),
                            _stream()))
    return Z


def tcx(A, c, rounds=1, r=1, col_kind="norm2", col_w=None, mode="iid", seed=0, prec=None, out=None):
    """t-CX of Algorithm 4 boosted by repetition (the projection onto the
    union of `rounds` independent draws of c slices): returns (Z, picks)."""
    _need_gpu(A, col_w)
    if prec is None:
        prec = "f64" if A.dtype == torch.float64 else "f32"
    cols = Picks(c * rounds, A.device)
    Z = _out(out, A.shape, A.dtype, A.device)
    lib = L.load()
    ta, tz = _tensor(A), _tensor(Z)
    cs = cols.struct()
    ws = _ws(lib.tp_tcx_workspace(C.byref(ta), int(c), int(rounds), int(r), L.KIND[col_kind], L.PREC[prec]),
             A.device)
    L.check(lib.tp_tcx(C.byref(ta), int(c), int(rounds), int(r), L.KIND[col_kind],
                       col_w.data_ptr() if col_w is not None else None, L.MODE[mode], int(seed), C.byref(cs),
                       C.byref(tz), L.PREC[prec], ws.data_ptr(), ws.numel(), _stream()))
    return Z, cols


def tcur(A, c, l, r, col_kind="lev", row_kind="lev", col_w=None, row_w=None, mode="iid", seed=0, prec=None,
         want_z=True, out=None, row_mode=None, mlp=None, want_core=False):
    """t-CUR of Algorithm 5: returns (Z, column picks, row picks), plus the
    float64 core (re, im), each K x c x l, when want_core. Z is None when
    want_z is False. mode picks the columns, row_mode (default: mode) the
    rows; "uniform" modes take the "uniform" kind. mlp = (params, phi,
    alpha) for col_kind "learned"."""
    _need_gpu(A, col_w, row_w)
    if prec is None:
        prec = "f64" if A.dtype == torch.float64 else "f32"
    row_mode = mode if row_mode is None else row_mode
    n1, n2, n3 = A.shape
    capc = n2 if mode == "bernoulli" else c
    capl = n1 if row_mode == "bernoulli" else l
    cols = Picks(capc, A.device)
    rows = Picks(capl, A.device)
    Z = _out(out, A.shape, A.dtype, A.device) if want_z else None
    core = None
    if want_core:
        core = (torch.empty((half_count(n3), capc, capl), dtype=torch.float64, device=A.device),
                torch.empty((half_count(n3), capc, capl), dtype=torch.float64, device=A.device))
    m = None
    if mlp is not None:
        params, phi, alpha = mlp
        _need_gpu(params, phi)
        m = L.Mlp(params.data_ptr(), phi.data_ptr(), float(alpha))
    lib = L.load()
    t = _tensor(A)
    tz = _tensor(Z) if Z is not None else None
    tc = _spectrum(*core) if core is not None else None
    cs, rs_ = cols.struct(), rows.struct()
    ws = _ws(lib.tp_tcur_workspace(C.byref(t), c, l, r, L.KIND[col_kind], L.MODE[mode], L.KIND[row_kind],
                                   L.MODE[row_mode], L.PREC[prec]), A.device)
    L.check(lib.tp_tcur(C.byref(t), int(c), int(l), int(r), L.KIND[col_kind],
                        col_w.data_ptr() if col_w is not None else None, L.MODE[mode], L.KIND[row_kind],
                        row_w.data_ptr() if row_w is not None else None, L.MODE[row_mode],
                        C.byref(m) if m is not None else None, int(seed), C.byref(cs), C.byref(rs_),
                        C.byref(tc) if tc is not None else None, C.byref(tz) if tz is not None else None,
                        L.PREC[prec], ws.data_ptr(), ws.numel(), _stream()))
    if want_core:
        return Z, cols, rows, core
    return Z, cols, rows


def tsvd_full(A, r, out=None, with_unconverged=False):
    """Dense leading-r t-SVD (see tp_tsvd_full): returns (U, S) with U the
    n1 x r x n3 first left singular slices of A (float32) and S the K x r
    singular values of the Fourier slices (float64, descending); with
    with_unconverged also a device int32 count of the Fourier slices whose
    Jacobi sweeps hit their cap."""
    _need_gpu(A)
    n1, n2, n3 = A.shape
    U = _out(out, (n1, r, n3), torch.float32, A.device)
    S = torch.empty((half_count(n3), r), dtype=torch.float64, device=A.device)
    unc = torch.zeros(1, dtype=torch.int32, device=A.device) if with_unconverged else None
    lib = L.load()
    t, tu = _tensor(A), _tensor(U)
    ws = _ws(lib.tp_tsvd_full_workspace(C.byref(t), int(r)), A.device)
    L.check(lib.tp_tsvd_full(C.byref(t), int(r), C.byref(tu), S.data_ptr(),
                             unc.data_ptr() if unc is not None else None, ws.data_ptr(), ws.numel(), _stream()))
    return (U, S, unc) if with_unconverged else (U, S)


def tsvt(M, tau, out=None, with_unconverged=False):
    """Per-Fourier-slice singular value thresholding with threshold tau:
    returns (L, ranks), and with with_unconverged also a device int32 count
    of the slices whose Jacobi sweeps hit their cap."""
    _need_gpu(M)
    L_ = _out(out, M.shape, M.dtype, M.device)
    ranks = torch.empty(half_count(M.shape[2]), dtype=torch.int32, device=M.device)
    unc = torch.zeros(1, dtype=torch.int32, device=M.device) if with_unconverged else None
    lib = L.load()
    tm, tl = _tensor(M), _tensor(L_)
    ws = _ws(lib.tp_tsvt_workspace(C.byref(tm)), M.device)
    L.check(lib.tp_tsvt(C.byref(tm), float(tau), C.byref(tl), ranks.data_ptr(),
                        unc.data_ptr() if unc is not None else None, L.PREC["f32"], ws.data_ptr(), ws.numel(),
                        _stream()))
    return (L_, ranks, unc) if with_unconverged else (L_, ranks)


def _admm_status(status, info, done):
    """TP_ENOCONV (a stop tolerance not met within the cap) is a result, not
    an error: report it in info; raise for anything else."""
    if info is not None:
        info["iters"] = int(done.value)
        info["converged"] = status == 0
    if status != L.TP_ENOCONV:
        L.check(status)


def tcomplete(X, mask, iters=100, rho=1.1, mu0=1e-3, mu_max=1e10, tol=0.0, info=None):
    """ADMM tensor completion (Algorithm 7, completion variant): returns
    (L, E, Y, ranks of the last iteration). mask is a uint8 tensor of X's
    shape, nonzero where observed. tol > 0 applies Algorithm 7's stop test
    after every iteration (one host synchronisation per iteration); a dict
    passed as info receives "iters" (iterations run) and "converged"."""
    _need_gpu(X, mask)
    if mask.dtype != torch.uint8 or mask.shape != X.shape:
        raise ValueError("mask must be uint8 with X's shape")
    L_, E, Y = torch.empty_like(X), torch.empty_like(X), torch.empty_like(X)
    ranks = torch.empty(half_count(X.shape[2]), dtype=torch.int32, device=X.device)
    lib = L.load()
    tx = _tensor(X)
    ws = _ws(lib.tp_tcomplete_workspace(C.byref(tx)), X.device)
    done = C.c_int32(0)
    status = lib.tp_tcomplete(C.byref(tx), mask.data_ptr(), int(iters), float(rho), float(mu0), float(mu_max),
                              float(tol), C.byref(_tensor(L_)), C.byref(_tensor(E)), C.byref(_tensor(Y)),
                              ranks.data_ptr(), C.byref(done), L.PREC["f32"], ws.data_ptr(), ws.numel(), _stream())
    _admm_status(status, info, done)
    return L_, E, Y, ranks


def trpca(X, lam=None, iters=100, rho=1.1, mu0=1e-3, mu_max=1e10, tol=0.0, info=None):
    """Robust tensor PCA by the ADMM of Algorithm 7 (eq. tlow7): returns
    (L, E, Y, ranks of the last iteration). lam = None lets the library use
    its default 1/sqrt(max(n1, n2) n3); tol and info as for tcomplete."""
    _need_gpu(X)
    n3 = X.shape[2]
    L_, E, Y = torch.empty_like(X), torch.empty_like(X), torch.empty_like(X)
    ranks = torch.empty(half_count(n3), dtype=torch.int32, device=X.device)
    lib = L.load()
    tx = _tensor(X)
    ws = _ws(lib.tp_trpca_workspace(C.byref(tx)), X.device)
    done = C.c_int32(0)
    status = lib.tp_trpca(C.byref(tx), 0.0 if lam is None else float(lam), int(iters), float(rho), float(mu0),
                          float(mu_max), float(tol), C.byref(_tensor(L_)), C.byref(_tensor(E)), C.byref(_tensor(Y)),
                          ranks.data_ptr(), C.byref(done), L.PREC["f32"], ws.data_ptr(), ws.numel(), _stream())
    _admm_status(status, info, done)
    return L_, E, Y, ranks


def tcur_nn(X, c, l, r, mask=None, lam=None, col_kind="uniform", row_kind="uniform", col_w=None, row_w=None,
            mode="uniform", seed=0, iters=100, rho=1.1, mu0=1e-3, mu_max=1e10, out=None, row_mode=None):
    """CUR t-NN of Algorithm 6: returns (L, column picks, row picks). With a
    uint8 mask (nonzero where observed) the ADMM is the completion variant,
    otherwise robust PCA with weight lam (None: the library's default
    1/sqrt(max(n1, n2) n3))."""
    _need_gpu(X, mask, col_w, row_w)
    n1, n2, n3 = X.shape
    if mask is not None and (mask.dtype != torch.uint8 or mask.shape != X.shape):
        raise ValueError("mask must be uint8 with X's shape")
    if lam is None:
        lam = 0.0  # the library's default weight
    cols, rows = Picks(c, X.device), Picks(l, X.device)
    L_ = _out(out, X.shape, X.dtype, X.device)
    lib = L.load()
    tx = _tensor(X)
    cs, rs_ = cols.struct(), rows.struct()
    ws = _ws(lib.tp_tcur_nn_workspace(C.byref(tx), int(c), int(l), int(r), L.KIND[col_kind], L.KIND[row_kind],
                                      1 if mask is not None else 0), X.device)
    row_mode = mode if row_mode is None else row_mode
    L.check(lib.tp_tcur_nn(C.byref(tx), mask.data_ptr() if mask is not None else None, float(lam), int(c), int(l),
                           int(r), L.KIND[col_kind], col_w.data_ptr() if col_w is not None else None, L.MODE[mode],
                           L.KIND[row_kind], row_w.data_ptr() if row_w is not None else None, L.MODE[row_mode],
                           int(seed), int(iters), float(rho), float(mu0), float(mu_max), C.byref(cs), C.byref(rs_),
                           C.byref(_tensor(L_)), L.PREC["f32"], ws.data_ptr(), ws.numel(), _stream()))
    return L_, cols, rows


# ---------------------------------------------------------------------------
# launch tracing
# ---------------------------------------------------------------------------

def trace_enable(on=True):
    """Start (clearing earlier records) or stop recording stage timings:
    True / 1 every stage, 2 the per-slice product stages only, False / 0
    stop."""
    mode = (1 if on else 0) if isinstance(on, bool) else int(on)
    L.check(L.load().tp_trace_enable(mode))


def trace_read():
    """{stage name: (calls, total ms)} of the recorded stages (waits for
    their events)."""
    lib = L.load()
    n = lib.tp_trace_count()
    if n < 0:
        L.check(n)
    out = {}
    for i in range(n):
        buf = C.create_string_buffer(64)
        calls = C.c_int64()
        ms = C.c_double()
        L.check(lib.tp_trace_entry(i, buf, 64, C.byref(calls), C.byref(ms)))
        out[buf.value.decode()] = (int(calls.value), float(ms.value))
    return out


# ---------------------------------------------------------------------------
# learned leverage proposal
# ---------------------------------------------------------------------------

def mlp_param_count():
    return int(L.load().tp_mlp_param_count())


def mlp_pack(P, device="cuda"):
    """Flat float32 device parameter vector from a dict with W1 (17x128), b1,
    W2 (128x128), b2, w3 (128), b3 (1)."""
    import numpy as np
    flat = np.concatenate([np.asarray(P[k], dtype=np.float64).ravel() for k in ("W1", "b1", "W2", "b2", "w3", "b3")])
    return torch.from_numpy(flat.astype(np.float32)).to(device)


def mlp_features(A, phi):
    """n2 x 17 float32 features of A's lateral slices (phi: (n1 n3) x 16)."""
    _need_gpu(A, phi)
    feat = torch.empty((A.shape[1], 17), dtype=torch.float32, device=A.device)
    lib = L.load()
    t = _tensor(A)
    ws = _ws(lib.tp_mlp_features_workspace(C.byref(t)), A.device)
    L.check(lib.tp_mlp_features(C.byref(t), phi.data_ptr(), feat.data_ptr(), ws.data_ptr(), ws.numel(), _stream()))
    return feat


def mlp_forward(params, feat):
    _need_gpu(params, feat)
    out = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device)
    L.check(L.load().tp_mlp_forward(params.data_ptr(), feat.data_ptr(), feat.shape[0], out.data_ptr(), _stream()))
    return out


def mlp_train_step(params, m, v, step, lr, feat, target, want_grad=False):
    """One step (see tp_mlp_train_step); returns (loss tensor, grad or None)."""
    _need_gpu(params, m, v, feat, target)
    T, n = target.shape
    loss = torch.empty(1, dtype=torch.float32, device=feat.device)
    grad = torch.empty_like(params) if want_grad else None
    lib = L.load()
    ws = _ws(lib.tp_mlp_train_workspace(T, n), feat.device)
    L.check(lib.tp_mlp_train_step(params.data_ptr(), m.data_ptr(), v.data_ptr(), int(step), float(lr),
                                  feat.data_ptr(), target.data_ptr(), T, n, loss.data_ptr(),
                                  grad.data_ptr() if grad is not None else None, ws.data_ptr(), ws.numel(),
                                  _stream()))
    return loss, grad


def mlp_proposal(params, A, phi, alpha=0.4):
    """float64 sampling weights for A's lateral slices from the network."""
    _need_gpu(params, A, phi)
    w = torch.empty(A.shape[1], dtype=torch.float64, device=A.device)
    lib = L.load()
    t = _tensor(A)
    ws = _ws(lib.tp_mlp_proposal_workspace(C.byref(t)), A.device)
    L.check(lib.tp_mlp_proposal(params.data_ptr(), C.byref(t), phi.data_ptr(), float(alpha), w.data_ptr(),
                                ws.data_ptr(), ws.numel(), _stream()))
    return w
