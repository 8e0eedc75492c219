"""ctypes view of the C ABI in include/tprod.h."""
import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtprod.so")

TP_F32, TP_F64 = 0, 1
TP_ENOCONV = -6
PREC = {"f64": 0, "f32": 1, "bf16x3": 2, "bf16": 3}
KIND = {"user": 0, "uniform": 1, "norm2": 2, "normprod": 3, "lev": 4, "learned": 5}
MODE = {"bernoulli": 0, "iid": 1, "uniform": 2}


class Tensor(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("n1", C.c_int64), ("n2", C.c_int64),
                ("n3", C.c_int64)]


class Spectrum(C.Structure):
    _fields_ = [("re", C.c_void_p), ("im", C.c_void_p), ("dtype", C.c_int32), ("K", C.c_int64),
                ("rows", C.c_int64), ("cols", C.c_int64)]


class Mlp(C.Structure):
    _fields_ = [("params", C.c_void_p), ("phi", C.c_void_p), ("alpha", C.c_double)]


class Sample(C.Structure):
    _fields_ = [("idx", C.c_void_p), ("scale", C.c_void_p), ("cap", C.c_int64), ("count", C.c_void_p)]


P = C.POINTER
_SIGS = {
    "tp_status_string": (C.c_char_p, [C.c_int]),
    "tp_last_error": (C.c_char_p, []),
    "tp_version": (C.c_int, []),
    "tp_tfft": (C.c_int, [P(Tensor), P(Spectrum), C.c_void_p]),
    "tp_tifft": (C.c_int, [P(Spectrum), P(Tensor), C.c_void_p]),
    "tp_spectrum_matmul": (C.c_int, [P(Spectrum), C.c_int, P(Spectrum), C.c_int, P(Spectrum), C.c_int, C.c_int,
                                     C.c_void_p]),
    "tp_slice_norms": (C.c_int, [P(Tensor), C.c_int, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tp_slice_norms_workspace": (C.c_size_t, [P(Tensor), C.c_int]),
    "tp_tsample": (C.c_int, [C.c_int, P(Tensor), P(Tensor), C.c_void_p, C.c_int64, C.c_int64, C.c_int,
                             C.c_uint64, C.c_uint64, P(Sample), C.c_void_p, C.c_size_t, C.c_void_p]),
    "tp_tsample_workspace": (C.c_size_t, [C.c_int64]),
    "tp_tsample_noalloc": (C.c_int, [C.c_int, P(Tensor), P(Tensor), C.c_void_p, C.c_int64, C.c_int64, C.c_int,
                                     C.c_uint64, C.c_uint64, P(Sample), C.c_void_p]),
    "tp_tsample_noalloc_max_bytes": (C.c_size_t, []),
    "tp_tprod": (C.c_int, [P(Tensor), P(Tensor), P(Sample), P(Tensor), C.c_int, C.c_void_p, C.c_size_t,
                           C.c_void_p]),
    "tp_tprod_workspace": (C.c_size_t, [P(Tensor), P(Tensor), P(Sample), C.c_int]),
    "tp_tsvd_rand": (C.c_int, [P(Tensor), C.c_int64, C.c_int64, C.c_int32, P(Sample), C.c_uint64, C.c_int,
                               C.c_void_p, P(Tensor), P(Tensor), P(Tensor), C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_size_t, C.c_void_p]),
    "tp_tsvd_rand_workspace": (C.c_size_t, [P(Tensor), C.c_int64, C.c_int64, P(Sample), C.c_int]),
    "tp_tcur": (C.c_int, [P(Tensor), C.c_int64, C.c_int64, C.c_int64, C.c_int, C.c_void_p, C.c_int, C.c_int,
                          C.c_void_p, C.c_int, P(Mlp), C.c_uint64, P(Sample), P(Sample), P(Spectrum), P(Tensor),
                          C.c_int, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tp_tcur_workspace": (C.c_size_t, [P(Tensor), C.c_int64, C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_int,
                                       C.c_int, C.c_int]),
    "tp_tsvt": (C.c_int, [P(Tensor), C.c_double, P(Tensor), C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_size_t,
                          C.c_void_p]),
    "tp_tsvt_workspace": (C.c_size_t, [P(Tensor)]),
    "tp_tsvd_full": (C.c_int, [P(Tensor), C.c_int64, P(Tensor), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                 C.c_void_p]),
    "tp_tsvd_full_workspace": (C.c_size_t, [P(Tensor), C.c_int64]),
    "tp_tcomplete": (C.c_int, [P(Tensor), C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double,
                               P(Tensor), P(Tensor), P(Tensor), C.c_void_p, P(C.c_int32), C.c_int, C.c_void_p,
                               C.c_size_t, C.c_void_p]),
    "tp_tcomplete_workspace": (C.c_size_t, [P(Tensor)]),
    "tp_tproject": (C.c_int, [P(Tensor), P(Tensor), P(Tensor), C.c_int, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tp_tproject_workspace": (C.c_size_t, [P(Tensor), P(Tensor), C.c_int]),
    "tp_tcx": (C.c_int, [P(Tensor), C.c_int64, C.c_int32, C.c_int64, C.c_int, C.c_void_p, C.c_int, C.c_uint64,
                         P(Sample), P(Tensor), C.c_int, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tp_tcx_workspace": (C.c_size_t, [P(Tensor), C.c_int64, C.c_int32, C.c_int64, C.c_int, C.c_int]),
    "tp_trpca": (C.c_int, [P(Tensor), C.c_double, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double,
                           P(Tensor), P(Tensor), P(Tensor), C.c_void_p, P(C.c_int32), C.c_int, C.c_void_p, C.c_size_t,
                           C.c_void_p]),
    "tp_trpca_workspace": (C.c_size_t, [P(Tensor)]),
    "tp_tcur_nn": (C.c_int, [P(Tensor), C.c_void_p, C.c_double, C.c_int64, C.c_int64, C.c_int64, C.c_int,
                             C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_uint64, C.c_int32, C.c_double,
                             C.c_double, C.c_double, P(Sample), P(Sample), P(Tensor), C.c_int, C.c_void_p,
                             C.c_size_t, C.c_void_p]),
    "tp_tcur_nn_workspace": (C.c_size_t, [P(Tensor), C.c_int64, C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_int]),
    "tp_trace_enable": (C.c_int, [C.c_int]),
    "tp_trace_count": (C.c_int, []),
    "tp_trace_entry": (C.c_int, [C.c_int, C.c_char_p, C.c_size_t, P(C.c_int64), P(C.c_double)]),
    "tp_mlp_param_count": (C.c_int, []),
    "tp_mlp_features": (C.c_int, [P(Tensor), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tp_mlp_features_workspace": (C.c_size_t, [P(Tensor)]),
    "tp_mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "tp_mlp_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_void_p,
                                    C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_size_t, C.c_void_p]),
    "tp_mlp_train_workspace": (C.c_size_t, [C.c_int64, C.c_int64]),
    "tp_mlp_proposal": (C.c_int, [C.c_void_p, P(Tensor), C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                  C.c_size_t, C.c_void_p]),
    "tp_mlp_proposal_workspace": (C.c_size_t, [P(Tensor)]),
}

_lib = None


def header_symbols():
    """Function names declared in include/tprod.h."""
    import re
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(here, "include", "tprod.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(tp_\w+)\s*\(", text, flags=re.M)))


def load():
    """Load libtprod.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_1704_04362_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class TpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def check(status):
    if status != 0:
        lib = load()
        raise TpError(status, lib.tp_last_error().decode() or lib.tp_status_string(status).decode())
    return status
