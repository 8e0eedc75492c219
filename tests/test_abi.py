"""The C-ABI library loads and exports what include/tprod.h declares; host
argument validation rejects bad calls before touching the GPU."""
import ctypes as C
import subprocess

import pytest

from paper_1704_04362_amd import _lib as L


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = L.header_symbols()
    assert "tp_tprod" in names and "tp_tsample" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert f" T {n}" in out, n


def test_trace_modes():
    # host-side bookkeeping only: no device work
    lib = L.load()
    for mode in (-1, 3):
        assert lib.tp_trace_enable(mode) == -1  # TP_EINVAL
    for mode in (2, 1, 0):
        assert lib.tp_trace_enable(mode) == 0
    assert lib.tp_trace_count() == 0


def test_status_strings_and_version():
    lib = L.load()
    assert lib.tp_version() >= 100
    assert lib.tp_status_string(0) == b"ok"
    assert lib.tp_status_string(-2) == b"shape mismatch"


def _t(n1, n2, n3, dtype=L.TP_F32, data=0x1000):
    return L.Tensor(data, dtype, n1, n2, n3)


@pytest.mark.parametrize("case", ["null", "inner", "tube", "outC", "dtype", "prec", "ws"])
def test_tprod_validation(case):
    lib = L.load()
    A, B, Cc = _t(4, 5, 6), _t(5, 3, 6), _t(4, 3, 6)
    prec = L.PREC["f32"]
    ws, wsb = C.c_void_p(0x2000), 1 << 30
    if case == "null":
        A = _t(4, 5, 6, data=0)
        want = -1
    elif case == "inner":
        B = _t(6, 3, 6)
        want = -2
    elif case == "tube":
        B = _t(5, 3, 7)
        want = -2
    elif case == "outC":
        Cc = _t(4, 4, 6)
        want = -2
    elif case == "dtype":
        B = _t(5, 3, 6, dtype=L.TP_F64)
        want = -3
    elif case == "prec":
        prec = L.PREC["f64"]
        want = -3
    else:
        wsb = 16
        want = -4
    rc = lib.tp_tprod(C.byref(A), C.byref(B), None, C.byref(Cc), prec, ws, wsb, None)
    assert rc == want, lib.tp_last_error()
    assert lib.tp_last_error()


def test_tsample_validation():
    lib = L.load()
    s = L.Sample(0x1000, 0x2000, 10, 0x3000)
    ws = C.c_void_p(0x4000)
    # c out of range
    assert lib.tp_tsample(0, None, None, C.c_void_p(0x5000), 10, 11, 1, 0, 0, C.byref(s), ws, 1 << 20, None) == -1
    assert lib.tp_tsample(0, None, None, C.c_void_p(0x5000), 10, 0, 1, 0, 0, C.byref(s), ws, 1 << 20, None) == -1
    # Bernoulli needs capacity n
    s2 = L.Sample(0x1000, 0x2000, 5, 0x3000)
    assert lib.tp_tsample(0, None, None, C.c_void_p(0x5000), 10, 3, 0, 0, 0, C.byref(s2), ws, 1 << 20, None) == -1
    # user weights missing
    assert lib.tp_tsample(0, None, None, None, 10, 3, 1, 0, 0, C.byref(s), ws, 1 << 20, None) == -1
    # workspace too small
    assert lib.tp_tsample(0, None, None, C.c_void_p(0x5000), 10, 3, 1, 0, 0, C.byref(s), ws, 8, None) == -4
    # norm2 with mismatched n
    A = _t(4, 5, 6)
    assert lib.tp_tsample(2, C.byref(A), None, None, 7, 3, 1, 0, 0, C.byref(s), ws, 1 << 20, None) == -2


def test_spectrum_and_transform_validation():
    lib = L.load()
    X = _t(4, 5, 8)
    bad = L.Spectrum(0x1000, 0x2000, L.TP_F32, 4, 4, 5)   # K should be 5
    assert lib.tp_tfft(C.byref(X), C.byref(bad), None) == -2
    good = L.Spectrum(0x1000, 0x2000, L.TP_F32, 5, 4, 5)
    X64 = _t(4, 5, 8, dtype=L.TP_F64)
    assert lib.tp_tfft(C.byref(X64), C.byref(good), None) == -3
    A = L.Spectrum(0x1000, 0x2000, L.TP_F32, 3, 4, 5)
    B = L.Spectrum(0x1000, 0x2000, L.TP_F32, 3, 6, 2)
    Cs = L.Spectrum(0x1000, 0x2000, L.TP_F32, 3, 4, 2)
    assert lib.tp_spectrum_matmul(C.byref(A), 0, C.byref(B), 0, C.byref(Cs), 1, 1, None) == -2
    assert lib.tp_spectrum_matmul(C.byref(A), 2, C.byref(B), 0, C.byref(Cs), 1, 1, None) == -1


@pytest.mark.parametrize("case", ["lambda", "nan_lambda", "shape", "iters", "nan_tol", "ws"])
def test_trpca_validation(case):
    lib = L.load()
    X, Lt, E, Y = _t(6, 5, 4), _t(6, 5, 4), _t(6, 5, 4), _t(6, 5, 4)
    lam, iters, tol, wsb, want = 0.1, 10, 0.0, 1 << 30, -1
    if case == "lambda":
        lam = -0.5
    elif case == "nan_lambda":
        lam = float("nan")
    elif case == "shape":
        E = _t(6, 4, 4)
        want = -2
    elif case == "iters":
        iters = 0
    elif case == "nan_tol":
        tol = float("nan")
    else:
        # lambda = 0 selects the default weight and passes validation, so
        # the call reaches the workspace check
        lam, wsb, want = 0.0, 16, -4
    done = C.c_int32(-5)
    rc = lib.tp_trpca(C.byref(X), lam, iters, 1.1, 1e-3, 1e10, tol, C.byref(Lt), C.byref(E), C.byref(Y), None,
                      C.byref(done), L.PREC["f32"], C.c_void_p(0x2000), wsb, None)
    assert rc == want, lib.tp_last_error()
    assert done.value == 0


@pytest.mark.parametrize("case", ["empty", "tau", "nan_tau", "prec", "dtype", "shape", "ws"])
def test_tsvt_validation(case):
    lib = L.load()
    M, Lt = _t(6, 5, 4), _t(6, 5, 4)
    tau, prec, wsb, want = 0.5, L.PREC["f32"], 1 << 30, -1
    if case == "empty":
        M, Lt = _t(0, 5, 4), _t(0, 5, 4)
        want = -2
    elif case == "tau":
        tau = -1.0
    elif case == "nan_tau":
        tau = float("nan")
    elif case == "prec":
        prec = L.PREC["bf16x3"]
        want = -3
    elif case == "dtype":
        M = _t(6, 5, 4, dtype=L.TP_F64)
        want = -3
    elif case == "shape":
        Lt = _t(6, 5, 5)
        want = -2
    else:
        wsb = 16
        want = -4
    rc = lib.tp_tsvt(C.byref(M), tau, C.byref(Lt), None, None, prec, C.c_void_p(0x2000), wsb, None)
    assert rc == want, lib.tp_last_error()
    assert lib.tp_last_error()


@pytest.mark.parametrize("case", ["mask", "empty", "rho", "mu", "ws"])
def test_tcomplete_validation(case):
    lib = L.load()
    X, Lt, E, Y = _t(6, 5, 4), _t(6, 5, 4), _t(6, 5, 4), _t(6, 5, 4)
    mask, rho, mu0, wsb, want = C.c_void_p(0x3000), 1.1, 1e-3, 1 << 30, -1
    if case == "mask":
        mask = None
    elif case == "empty":
        X, Lt, E, Y = _t(6, 0, 4), _t(6, 0, 4), _t(6, 0, 4), _t(6, 0, 4)
        want = -2
    elif case == "rho":
        rho = 0.5
    elif case == "mu":
        mu0 = 0.0
    else:
        wsb = 16
        want = -4
    rc = lib.tp_tcomplete(C.byref(X), mask, 10, rho, mu0, 1e10, 0.0, C.byref(Lt), C.byref(E), C.byref(Y), None,
                          None, L.PREC["f32"], C.c_void_p(0x2000), wsb, None)
    assert rc == want, lib.tp_last_error()
    # the workspace query of an empty tensor is 0
    assert lib.tp_tcomplete_workspace(C.byref(_t(6, 0, 4))) == 0


@pytest.mark.parametrize("case", ["bernoulli", "rank", "dtype", "lambda"])
def test_tcur_nn_validation(case):
    lib = L.load()
    X, Lt = _t(20, 24, 4), _t(20, 24, 4)
    cols = L.Sample(0x3000, 0x4000, 24, 0x5000)
    rows = L.Sample(0x6000, 0x7000, 20, 0x8000)
    mode, r, lam, want = L.MODE["uniform"], 2, 0.1, -1
    if case == "bernoulli":
        mode = L.MODE["bernoulli"]
    elif case == "rank":
        r = 9
    elif case == "dtype":
        X = _t(20, 24, 4, dtype=L.TP_F64)
        want = -3
    else:
        lam = -1.0
    rc = lib.tp_tcur_nn(C.byref(X), None, lam, 8, 6, r, L.KIND["uniform"], None, mode, L.KIND["uniform"], None,
                        mode, 0, 10, 1.1, 1e-3, 1e10, C.byref(cols), C.byref(rows), C.byref(Lt), L.PREC["f32"],
                        C.c_void_p(0x2000), 1 << 30, None)
    assert rc == want


@pytest.mark.parametrize("case", ["too_many", "bernoulli", "rounds", "lev_rank"])
def test_tcx_validation(case):
    lib = L.load()
    A, Z = _t(20, 100, 4), _t(20, 100, 4)
    cols = L.Sample(0x3000, 0x4000, 200, 0x5000)
    c, rounds, r, kind, mode, want = 8, 2, 2, L.KIND["norm2"], L.MODE["iid"], -1
    if case == "too_many":
        c, rounds, want = 33, 2, -7
    elif case == "bernoulli":
        mode = L.MODE["bernoulli"]
    elif case == "rounds":
        rounds = 0
    else:
        kind, r = L.KIND["lev"], 60
    rc = lib.tp_tcx(C.byref(A), c, rounds, r, kind, None, mode, 0, C.byref(cols), C.byref(Z), L.PREC["f32"],
                    C.c_void_p(0x2000), 1 << 30, None)
    assert rc == want


def test_tproject_validation():
    lib = L.load()
    X, Z = _t(20, 30, 4), _t(20, 30, 4)
    for Cs, want in ((_t(20, 65, 4), -7), (_t(21, 5, 4), -2), (_t(20, 5, 4, dtype=L.TP_F64), -3)):
        rc = lib.tp_tproject(C.byref(X), C.byref(Cs), C.byref(Z), L.PREC["f32"], C.c_void_p(0x2000), 1 << 30, None)
        assert rc == want


def test_missing_library_raises(tmp_path, monkeypatch):
    # no fallback: without the built library every call fails loudly
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "libtprod.so"))
    with pytest.raises(RuntimeError, match="missing"):
        L.load()


def test_cpu_tensors_are_rejected():
    # the binding has no CPU path
    import torch
    from paper_1704_04362_amd import api
    A = torch.zeros(4, 5, 6)
    with pytest.raises(ValueError, match="GPU"):
        api.tprod(A, torch.zeros(5, 3, 6))
    with pytest.raises(ValueError, match="GPU"):
        api.tsvt(A, 0.5)
    # an out= tensor is checked like an input before its pointer is passed:
    # a host tensor, a strided view, a wrong dtype or a wrong shape is refused
    with pytest.raises(ValueError, match="GPU"):
        api._out(torch.zeros(4, 3, 6), (4, 3, 6), torch.float32, "cuda:0")
    for bad, msg in ((torch.zeros(4, 3, 6, dtype=torch.float64), "float32"), (torch.zeros(4, 4, 6), "shape"),
                     (torch.zeros(6, 3, 4).permute(2, 1, 0), "contiguous")):
        with pytest.raises(ValueError, match=msg):
            api._out(_FakeCuda(bad), (4, 3, 6), torch.float32, "cuda:0")


class _FakeCuda:
    """A CPU tensor that reports itself as a device tensor, so the checks
    after the device test can run without a GPU."""

    def __init__(self, t):
        self._t = t
        self.is_cuda = True
        self.dtype, self.shape, self.device = t.dtype, t.shape, "cuda:0"

    def is_contiguous(self):
        return self._t.is_contiguous()


@pytest.mark.parametrize("case", ["rank", "zero_rank", "ushape", "empty", "dtype", "big", "ws"])
def test_tsvd_full_validation(case):
    lib = L.load()
    A, U, r, wsb, want = _t(30, 20, 4), _t(30, 5, 4), 5, 1 << 30, -1
    if case == "rank":
        r, U = 21, _t(30, 21, 4)
    elif case == "zero_rank":
        r, U = 0, _t(30, 1, 4)
    elif case == "ushape":
        U = _t(30, 6, 4)
        want = -2
    elif case == "empty":
        A = _t(0, 20, 4)
        want = -2
    elif case == "dtype":
        A = _t(30, 20, 4, dtype=L.TP_F64)
        want = -3
    elif case == "big":
        A, U = _t(5000, 5000, 2), _t(5000, 5, 2)
        want = -7
    else:
        wsb = 16
        want = -4
    rc = lib.tp_tsvd_full(C.byref(A), r, C.byref(U), None, None, C.c_void_p(0x2000), wsb, None)
    assert rc == want, lib.tp_last_error()


def test_tsample_noalloc_rejects_sizes_beyond_its_scratch():
    # the fixed scratch holds 32 MiB; 2^24 candidate slices need more, which
    # is refused on the host before anything is enqueued
    lib = L.load()
    assert lib.tp_tsample_noalloc_max_bytes() == 32 << 20
    n = 1 << 24
    assert lib.tp_tsample_workspace(n) > lib.tp_tsample_noalloc_max_bytes()
    out = L.Sample(0x1000, 0x2000, 8, 0x3000)
    rc = lib.tp_tsample_noalloc(L.KIND["uniform"], None, None, None, n, 8, L.MODE["iid"], 0, 0, C.byref(out), None)
    assert rc == -7
    assert b"scratch" in lib.tp_last_error()
    # bad arguments get tp_tsample's own errors
    assert lib.tp_tsample_noalloc(L.KIND["uniform"], None, None, None, 10, 11, L.MODE["iid"], 0, 0, C.byref(out),
                                  None) == -1


@pytest.mark.parametrize("case", ["uniform_with_weights", "row_uniform_with_lev", "learned_rows", "learned_no_mlp",
                                  "core_shape", "core_dtype", "ok_ws"])
def test_tcur_validation(case):
    # uniform picks without replacement use no weights: any other kind is
    # refused instead of computed and ignored; the learned kind is for
    # columns and needs its network; the core output has the picks' shape
    lib = L.load()
    A, Z = _t(40, 50, 8), _t(40, 50, 8)
    cols = L.Sample(0x3000, 0x4000, 12, 0x5000)
    rows = L.Sample(0x6000, 0x7000, 10, 0x8000)
    K = 5
    ck, cm, rk, rm, mlp, want, wsb = L.KIND["uniform"], L.MODE["uniform"], L.KIND["lev"], L.MODE["iid"], None, -1, 16
    core = None
    if case == "uniform_with_weights":
        ck = L.KIND["norm2"]
    elif case == "row_uniform_with_lev":
        rm = L.MODE["uniform"]
    elif case == "learned_rows":
        rk = L.KIND["learned"]
    elif case == "learned_no_mlp":
        ck, cm = L.KIND["learned"], L.MODE["iid"]
    elif case == "core_shape":
        core = L.Spectrum(0x9000, 0xa000, L.TP_F64, K, 12, 11)
        want = -2
    elif case == "core_dtype":
        core = L.Spectrum(0x9000, 0xa000, L.TP_F32, K, 12, 10)
        want = -2
    else:
        # the remark's procedure with a core of the right shape passes
        # validation and stops at the workspace
        core = L.Spectrum(0x9000, 0xa000, L.TP_F64, K, 12, 10)
        want = -4
    rc = lib.tp_tcur(C.byref(A), 12, 10, 3, ck, None, cm, rk, None, rm, mlp, 0, C.byref(cols), C.byref(rows),
                     C.byref(core) if core is not None else None, C.byref(Z), L.PREC["f32"], C.c_void_p(0x2000), wsb,
                     None)
    assert rc == want, lib.tp_last_error()


@pytest.mark.parametrize("case", ["u_shape", "z_shape", "v_dtype", "slices_cap", "slices_big", "ok_ws"])
def test_tsvd_rand_validation(case):
    lib = L.load()
    A = _t(40, 90, 8)
    U, V, Z = _t(40, 4, 8), _t(90, 4, 8), _t(40, 90, 8)
    sl = None
    want, wsb = -2, 16
    if case == "u_shape":
        U = _t(40, 5, 8)
    elif case == "z_shape":
        Z = _t(40, 90, 7)
    elif case == "v_dtype":
        V = _t(90, 4, 8, dtype=L.TP_F64)
    elif case == "slices_cap":
        sl = L.Sample(0x3000, 0x4000, 3, 0x5000)
        want = -1
    elif case == "slices_big":
        sl = L.Sample(0x3000, 0x4000, 70, 0x5000)
        want = -7
    else:
        sl = L.Sample(0x3000, 0x4000, 12, 0x5000)
        want = -4
    rc = lib.tp_tsvd_rand(C.byref(A), 4, 10, 1, C.byref(sl) if sl is not None else None, 0, L.PREC["f32"], None,
                          C.byref(U), C.byref(V), C.byref(Z), None, None, C.c_void_p(0x2000), wsb, None)
    assert rc == want, lib.tp_last_error()
