"""Library calls captured into a HIP graph: no allocation, no host
synchronisation and no memset inside a call, so a captured t-product,
rt-product and t-CUR replay to the eager results bit for bit. Every replay
is checked, with eager work and synchronisations between the replays."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1704_04362_amd.api")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_replays_equal_eager_calls():
    A, B = W.rtprod_pair(n1=96, n2=512, n4=80, n3=16)
    Ad, Bd = dev(A), dev(B)
    G1, G2, N = W.lowrank_factors(n1=96, n2=80, n3=8, r=4, salt=3)
    X = dev(G1.astype(np.float32))
    X = api.tprod(X, dev(G2.astype(np.float32)), prec="f32") + dev(N.astype(np.float32))
    C1 = torch.empty(96, 80, 16, device="cuda")
    C2 = torch.empty(96, 80, 16, device="cuda")
    Z = torch.empty_like(X)

    def calls():
        api.tprod(Ad, Bd, prec="bf16x3", out=C1)
        picks = api.tsample("norm2", 64, mode="iid", seed=5, A=Ad)
        api.tprod(Ad, Bd, picks=picks, prec="f32", out=C2)
        api.tcur(X, 24, 24, 4, col_kind="lev", row_kind="lev", seed=2, prec="f32", out=Z)

    calls()  # eager (also sets up the transform tables before capture)
    torch.cuda.synchronize()
    ref = [C1.clone(), C2.clone(), Z.clone()]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        calls()
    torch.cuda.synchronize()
    other = dev(np.ones((8, 8, 4), np.float32))
    for rep in range(3):
        for t in (C1, C2, Z):
            t.fill_(float("nan"))
        api.tprod(other, other, prec="f32")  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for got, want in zip((C1, C2, Z), ref):
            assert torch.equal(got, want), rep


def test_svt_sweeps_on_two_streams_replay_equal_eager():
    # 33 slices of 256 x 256 give 264 pair steps per launch, enough for the
    # sweeps to split over the caller's stream and the side stream; the
    # fork and join are captured with the rest of the call
    g0 = torch.Generator().manual_seed(11)
    M = torch.randn(256, 256, 64, generator=g0).cuda()
    L1 = torch.empty_like(M)
    holder = {}

    def call():
        holder["L"], holder["ranks"] = api.tsvt(M, 30.0, out=L1)

    call()
    torch.cuda.synchronize()
    ref_L, ref_ranks = L1.clone(), holder["ranks"].clone()
    assert int(ref_ranks.min()) > 0 and int(ref_ranks.max()) < 256
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    torch.cuda.synchronize()
    for rep in range(3):
        L1.fill_(float("nan"))
        holder["ranks"].fill_(-1)
        api.tsvt(M[:64, :64, :8].contiguous(), 1.0)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(L1, ref_L), rep
        assert torch.equal(holder["ranks"], ref_ranks), rep
