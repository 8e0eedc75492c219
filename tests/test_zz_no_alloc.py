"""The allocation-free sampling entry point (tp_tsample_noalloc) against
tp_tsample: on the same arguments both give the same picks, bit for bit,
through the C ABI. Two calls in a row share the fixed device scratch, the
second with a smaller input, so a result that depended on what an earlier
call left in the scratch would show here."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W
from paper_1704_04362_amd import _lib as L

pytestmark = pytest.mark.gpu


def _tensor(x):
    return L.Tensor(x.data_ptr(), L.TP_F32 if x.dtype == torch.float32 else L.TP_F64, *x.shape)


class _Picks:
    def __init__(self, cap):
        self.idx = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
        self.scale = torch.full((cap,), -7.0, dtype=torch.float64, device="cuda")
        self.count = torch.full((1,), -7, dtype=torch.int64, device="cuda")
        self.s = L.Sample(self.idx.data_ptr(), self.scale.data_ptr(), cap, self.count.data_ptr())

    def live(self):
        n = int(self.count.item())
        assert n >= 0
        return self.idx[:n].cpu().numpy(), self.scale[:n].cpu().numpy()


def _run(noalloc, kind, A, w, n, c, mode, seed):
    lib = L.load()
    cap = n if mode == "bernoulli" else c
    out = _Picks(cap)
    ta = C.byref(_tensor(A)) if A is not None else None
    wp = w.data_ptr() if w is not None else None
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        rc = lib.tp_tsample_noalloc(L.KIND[kind], ta, None, wp, n, c, L.MODE[mode], seed, 3, C.byref(out.s), stream)
    else:
        nbytes = lib.tp_tsample_workspace(n) + (lib.tp_slice_norms_workspace(ta, 0) if A is not None else 0)
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
        rc = lib.tp_tsample(L.KIND[kind], ta, None, wp, n, c, L.MODE[mode], seed, 3, C.byref(out.s),
                            ws.data_ptr(), ws.numel(), stream)
    assert rc == 0, L.load().tp_last_error()
    torch.cuda.synchronize()
    return out.live()


@pytest.mark.parametrize("mode", ["bernoulli", "iid", "uniform"])
def test_noalloc_picks_equal_workspace_picks(mode):
    A1, _ = W.rtprod_pair(n1=96, n2=3000, n4=8, n3=12, salt=41)
    A2, _ = W.rtprod_pair(n1=40, n2=700, n4=8, n3=12, salt=42)
    w1 = W.lognormal_weights(5000, seed=43)
    w2 = W.lognormal_weights(900, seed=44, zeros=100)
    cases = [("norm2", torch.from_numpy(A1).cuda(), None, 3000, 300),
             ("norm2", torch.from_numpy(A2).cuda(), None, 700, 50),
             ("user", None, torch.from_numpy(w1).cuda(), 5000, 400),
             ("user", None, torch.from_numpy(w2).cuda(), 900, 64)]
    for seed, (kind, A, w, n, c) in enumerate(cases):
        got = _run(True, kind, A, w, n, c, mode, seed)
        want = _run(False, kind, A, w, n, c, mode, seed)
        assert np.array_equal(got[0], want[0]), (kind, n)
        assert np.array_equal(got[1], want[1]), (kind, n)
        assert len(got[0]) > 0

