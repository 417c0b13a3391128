"""Parity of the interleaved-layout ("mrhs") FP32 stencil with the FP64 oracle.

The operator is D_S of eq. 3 on several right-hand sides sharing links and clover
(Sect. 3.3 names several right-hand sides as the cache-friendly form), with the SU(3)
products on the vector units or on the matrix cores.  Bar: FP32, 1e-5 relative per
right-hand side against the oracle.  Lattices span several workgroups with ragged
tails (6x6x6x10: V/2 = 1080), right-hand-side counts cover one group (1..16, padded
to a multiple of four lanes), several groups (17..32) and uneven ones.
"""
import ctypes

import numpy as np
import pytest
import torch

from gpu_common import Case, rel, to_dev, to_host
from oracle import solvers
from paper_2407_08092_amd import api
from paper_2407_08092_amd._lib import lib

pytestmark = pytest.mark.gpu

ENGINES = [api.DDQ_ENGINE_VALU, api.DDQ_ENGINE_MFMA]
ENGINE_IDS = ["valu", "mfma"]
_cases = {}


def case(dims, link12=False, eps=0.3, c_sw=1.0, m0=-0.1, seed=101):
    key = (dims, link12, eps, c_sw, m0, seed)
    if key not in _cases:
        c = Case(dims, eps, c_sw, m0, seed)
        if link12:
            api.set_gauge(c.lat, torch.from_numpy(c.U).cuda(), link12=True)
            api.set_clover(c.lat, c_sw, m0)
        _cases[key] = c
    return _cases[key]


def to_mrhs(x):
    """oracle vectors [n, V/2, 12] -> mrhs layout [V/2, 6, n, 2] complex64 on the GPU."""
    n, vh, _ = x.shape
    a = np.transpose(x, (1, 2, 0)).reshape(vh, 6, 2, n)  # [Vh, 6, 2, n]
    a = np.ascontiguousarray(np.transpose(a, (0, 1, 3, 2)))  # [Vh, 6, n, 2]
    return torch.from_numpy(a).to(device="cuda", dtype=torch.complex64).contiguous()


def from_mrhs(t):
    """mrhs layout [V/2, 6, n, 2] -> oracle vectors [n, V/2, 12] complex128."""
    a = t.detach().cpu().numpy().astype(np.complex128)  # [Vh, 6, n, 2]
    vh, _, n, _ = a.shape
    a = np.transpose(a, (2, 0, 1, 3)).reshape(n, vh, 12)
    return np.ascontiguousarray(a)


def per_rhs(got, ref):
    return max(rel(got[r], ref[r]) for r in range(ref.shape[0]))


@pytest.mark.parametrize("n", [1, 3, 12, 20])
def test_pack_unpack_roundtrip(n):
    c = case((4, 6, 8, 10))
    x = c.vec(301, n)
    planar = to_dev(x, torch.complex64)
    packed = api.mrhs_pack(c.lat, planar)
    torch.cuda.synchronize()
    assert torch.equal(packed, to_mrhs(x))  # the layout stated in the header
    back = api.mrhs_unpack(c.lat, packed)
    torch.cuda.synchronize()
    assert torch.equal(back.reshape(planar.shape), planar)


APPLY_CASES = [((4, 4, 4, 4), 1), ((4, 4, 4, 4), 12), ((4, 6, 8, 10), 2), ((4, 6, 8, 10), 5),
               ((4, 6, 8, 10), 16), ((6, 6, 6, 10), 3), ((6, 6, 6, 10), 12), ((6, 6, 6, 10), 17),
               ((8, 8, 8, 16), 8), ((8, 8, 8, 16), 13), ((8, 8, 8, 16), 32), ((2, 2, 2, 2), 4)]


@pytest.mark.parametrize("stage", [0, 1], ids=["direct", "staged"])
@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
@pytest.mark.parametrize("dims,n", APPLY_CASES)
def test_apply_matches_oracle(dims, n, engine, stage):
    c = case(dims)
    x = c.vec(302, n)
    api.mrhs_set_launch(c.lat, 1, 0, 0, stage)
    try:
        y = api.mrhs_apply_schur(c.lat, to_mrhs(x), engine=engine)
        torch.cuda.synchronize()
    finally:
        api.mrhs_set_launch(c.lat, 1, 0)
    ref = np.stack([c.op.schur(x[r]) for r in range(n)])
    assert per_rhs(from_mrhs(y), ref) < 1e-5


@pytest.mark.parametrize("stage", [0, 1], ids=["direct", "staged"])
@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
@pytest.mark.parametrize("n", [4, 12])
def test_apply_link12(n, engine, stage):
    c = case((6, 6, 6, 10), link12=True)
    x = c.vec(303, n)
    api.mrhs_set_launch(c.lat, 1, 0, 0, stage)
    try:
        y = api.mrhs_apply_schur(c.lat, to_mrhs(x), engine=engine)
        torch.cuda.synchronize()
    finally:
        api.mrhs_set_launch(c.lat, 1, 0)
    ref = np.stack([c.op.schur(x[r]) for r in range(n)])
    assert per_rhs(from_mrhs(y), ref) < 1e-5


@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
@pytest.mark.parametrize("dims,n", [((4, 6, 8, 10), 12), ((8, 8, 8, 16), 5)])
def test_richardson_matches_oracle(dims, n, engine):
    c = case(dims)
    b = c.vec(304, n)
    x0 = c.vec(305, n)
    omega = 0.12
    x = to_mrhs(x0)
    api.mrhs_richardson_smooth(c.lat, x, to_mrhs(b), 6, omega, engine=engine)
    torch.cuda.synchronize()
    ref = np.stack([solvers.richardson(c.op.schur, b[r], x0[r], 6, omega) for r in range(n)])
    assert per_rhs(from_mrhs(x), ref) < 1e-5


LAUNCHES = [(0, 0, 0, 0), (0, 48, 0, 0), (1, 0, 0, 0), (1, 48, 0, 0), (2, 0, 1, 0), (2, 0, 2, 0), (2, 32, 3, 0),
            (2, 0, 5, 0), (1, 0, 0, 1), (0, 0, 0, 1), (2, 0, 3, 1), (2, 64, 5, 1)]


@pytest.mark.parametrize("n", [3, 12, 24])
def test_engines_agree_and_orders_are_bitwise_equal(n):
    # plain, slab and t-walk orders (walks of 1, 2, 3 and 5 = Lt / 2 slices) with and
    # without an LDS cap: every lane's arithmetic is the same, so results are bitwise equal
    c = case((6, 6, 6, 10))
    x = to_mrhs(c.vec(306, n))
    ys = {}
    for engine in ENGINES:
        for order, lds, ts, stage in LAUNCHES:
            api.mrhs_set_launch(c.lat, order, lds, ts, stage)
            ys[(engine, order, lds, ts, stage)] = api.mrhs_apply_schur(c.lat, x, engine=engine)
    api.mrhs_set_launch(c.lat, 1, 0)
    torch.cuda.synchronize()
    for engine in ENGINES:
        ref = ys[(engine, 1, 0, 0, 0)]
        for key, y in ys.items():
            if key[0] == engine:
                assert torch.equal(y, ref), key  # the arithmetic of a lane does not depend on the order
    a = from_mrhs(ys[(0, 1, 0, 0, 0)])
    b = from_mrhs(ys[(1, 1, 0, 0, 0)])
    assert per_rhs(b, a) < 2e-6  # two FP32 summation orders of the same sums


@pytest.mark.parametrize("stage", [0, 1], ids=["direct", "staged"])
@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
@pytest.mark.parametrize("dims,n,ts", [((4, 6, 8, 10), 12, 1), ((4, 6, 8, 10), 5, 3), ((8, 8, 8, 16), 12, 8),
                                       ((8, 8, 8, 16), 20, 3), ((2, 2, 2, 2), 4, 1)])
def test_twalk_matches_oracle(dims, n, ts, engine, stage):
    c = case(dims)
    api.mrhs_set_launch(c.lat, 2, 0, ts, stage)
    try:
        x = c.vec(310, n)
        y = api.mrhs_apply_schur(c.lat, to_mrhs(x), engine=engine)
        b = c.vec(311, n)
        z = to_mrhs(x)
        api.mrhs_richardson_smooth(c.lat, z, to_mrhs(b), 3, 0.12, engine=engine)
        torch.cuda.synchronize()
    finally:
        api.mrhs_set_launch(c.lat, 1, 0)
    ref = np.stack([c.op.schur(x[r]) for r in range(n)])
    assert per_rhs(from_mrhs(y), ref) < 1e-5
    ref = np.stack([solvers.richardson(c.op.schur, b[r], x[r], 3, 0.12) for r in range(n)])
    assert per_rhs(from_mrhs(z), ref) < 1e-5


def test_matches_planar_multi_rhs_kernels():
    # the same operator through ddq_apply_schur's FP32 path on [nrhs][6][V/2][2] vectors
    c = case((8, 8, 8, 16))
    x = c.vec(307, 12)
    planar = to_dev(x, torch.complex64)
    yp = api.apply_schur(c.lat, planar)
    ym = api.mrhs_apply_schur(c.lat, api.mrhs_pack(c.lat, planar), engine=api.DDQ_ENGINE_MFMA)
    torch.cuda.synchronize()
    assert per_rhs(from_mrhs(ym), to_host(yp)) < 2e-6


def test_argument_errors():
    c = case((4, 4, 4, 4))
    L = lib()
    x = to_mrhs(c.vec(308, 4))
    y = torch.empty_like(x)
    px, py = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())
    api.reserve(c.lat, 4)
    assert L.ddq_mrhs_apply_schur(c.lat.handle, 4, px, py, 2) == -1  # unknown engine
    assert L.ddq_mrhs_apply_schur(c.lat.handle, 0, px, py, 0) == -1
    assert L.ddq_mrhs_apply_schur(c.lat.handle, 4, px, px, 0) == -1  # x and y overlap
    assert L.ddq_mrhs_richardson_smooth(c.lat.handle, 4, px, px, 1, 0.1, 0) == -1
    assert L.ddq_mrhs_set_launch(c.lat.handle, 3, 0, 0, 0) == -1
    assert L.ddq_mrhs_set_launch(c.lat.handle, 1, 161, 0, 0) == -1
    assert L.ddq_mrhs_set_launch(c.lat.handle, 2, 0, 0, 0) == -1  # a t walk of no slices
    assert L.ddq_mrhs_set_launch(c.lat.handle, 2, 0, 3, 0) == -1  # more than Lt / 2 = 2
    assert L.ddq_mrhs_set_launch(c.lat.handle, 1, 0, 0, 2) == -1
    assert L.ddq_mrhs_pack(c.lat.handle, 4, px, px) == -1
    # beyond the reservation: DDQ_ERR_STATE, nothing allocated
    big = to_mrhs(c.vec(309, 200))
    out = torch.empty_like(big)
    st = L.ddq_mrhs_apply_schur(c.lat.handle, 200, ctypes.c_void_p(big.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), 1)
    assert st == -2


@pytest.mark.parametrize("engine", ENGINES, ids=ENGINE_IDS)
@pytest.mark.parametrize("order", [1, 0], ids=["slab", "plain"])
def test_chunked_launches_are_bitwise_equal(engine, order):
    # kernels A and B launched per range of t-slices (ddq_set_sweep_chunks) give the one-launch
    # apply and sweeps bit for bit
    c = case((6, 6, 6, 10))
    x = to_mrhs(c.vec(312, 12))
    b = to_mrhs(c.vec(313, 12))
    outs = {}
    for nc in (1, 2, 3, 7, 10):
        api.set_sweep_chunks(c.lat, nc)
        api.mrhs_set_launch(c.lat, order)
        y = api.mrhs_apply_schur(c.lat, x, engine=engine)
        z = x.clone()
        api.mrhs_richardson_smooth(c.lat, z, b, 3, 0.12, engine=engine)
        torch.cuda.synchronize()
        outs[nc] = (y, z)
    api.set_sweep_chunks(c.lat, 0)
    api.mrhs_set_launch(c.lat, 1)
    for nc in (2, 3, 7, 10):
        assert torch.equal(outs[nc][0], outs[1][0]), nc
        assert torch.equal(outs[nc][1], outs[1][1]), nc
