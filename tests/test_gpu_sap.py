"""SAP(n, m) of Alg. 1 (4^4 blocks, block-local odd-even Minimal Residual) through the C
ABI, against the FP64 oracle's SAP with the same blocks: 1e-12 relative with FP64 block
solves, 1e-5 with FP32 ones (FP32 links, 18- or 12-real, and clover; the residuals and
the update stay FP64).

Lattices: 4^4 (one block spanning every direction: the wrap-around hops, with the
antiperiodic sign in t, stay inside it), 8x4x4x4 (two blocks along x, one colour each),
8x8x4x8 (a checkerboard of eight blocks), 12x4x8x4 (three blocks along x: two
neighbouring blocks share a colour).
"""
import numpy as np
import pytest
import torch

from gpu_common import Case, rel
from oracle import solvers
from paper_2407_08092_amd import api, synth

pytestmark = pytest.mark.gpu

DIMS = [(4, 4, 4, 4), (8, 4, 4, 4), (8, 8, 4, 8), (12, 4, 8, 4)]
_cases = {}


def case(dims):
    if dims not in _cases:
        _cases[dims] = Case(dims, 0.4, 1.0, -0.2, 501)
    return _cases[dims]


# 8^4: FP32 blocks with 18-real links keep the block's links in LDS (no block spans y, z
# or t); the other lattices take the kernel that reads them from memory
@pytest.mark.parametrize("m", [1, 4])
@pytest.mark.parametrize("dims", DIMS + [(8, 8, 8, 8)], ids=lambda d: "x".join(map(str, d)))
def test_sap_matches_oracle(dims, m):
    c = case(dims)
    b = c.full(502)
    x0 = c.full(503) * 0.1
    n = 2
    ref = solvers.sap(c.op, b, x0, n, m)
    for prec, tol in ((api.DDQ_F64, 1e-12), (api.DDQ_F32, 1e-5)):
        x = torch.from_numpy(x0.copy()).cuda()
        api.sap_smooth(c.lat, torch.from_numpy(b).cuda(), x, n, m, prec=prec)
        torch.cuda.synchronize()
        assert rel(x.cpu().numpy(), ref) < tol, prec


# FP32 block solves with 12-real links keep the block's links in LDS and the clover
# slots in registers; 8^4 has no direction that a block spans (no wrap-around hop)
@pytest.mark.parametrize("m", [1, 4])
@pytest.mark.parametrize("dims", DIMS + [(8, 8, 8, 8)], ids=lambda d: "x".join(map(str, d)))
def test_sap_f32_with_twelve_real_links(dims, m):
    c = case(dims)
    lat = api.create_lattice(dims)
    api.set_gauge(lat, torch.from_numpy(c.U).cuda(), link12=True)
    api.set_clover(lat, 1.0, -0.2)
    b = c.full(504)
    x0 = c.full(505) * 0.1
    ref = solvers.sap(c.op, b, x0, 2, m)
    x = torch.from_numpy(x0.copy()).cuda()
    api.sap_smooth(lat, torch.from_numpy(b).cuda(), x, 2, m, prec=api.DDQ_F32)
    torch.cuda.synchronize()
    api.destroy_lattice(lat)
    assert rel(x.cpu().numpy(), ref) < 1e-5


@pytest.mark.parametrize("dims", [(12, 8, 8, 8), (8, 12, 8, 8), (4, 8, 8, 8)], ids=lambda d: "x".join(map(str, d)))
def test_sap_odd_block_count(dims):
    """Three blocks along x (a row of blocks holds two of one colour and one of the other:
    the on-chip block solves' grid covers both colours' rows) or along y (neighbouring
    blocks across the boundary share a colour), and one block along x (the x hops wrap
    inside the block, all in LDS); FP64, FP32 18-real and FP32 12-real block solves, all
    on chip, against one oracle run."""
    c = case(dims)
    b = c.full(506)
    x0 = c.full(507) * 0.1
    ref = solvers.sap(c.op, b, x0, 2, 2)
    for prec, tol in ((api.DDQ_F64, 1e-12), (api.DDQ_F32, 1e-5)):
        x = torch.from_numpy(x0.copy()).cuda()
        api.sap_smooth(c.lat, torch.from_numpy(b).cuda(), x, 2, 2, prec=prec)
        torch.cuda.synchronize()
        assert rel(x.cpu().numpy(), ref) < tol, prec
    lat = api.create_lattice(dims)
    api.set_gauge(lat, torch.from_numpy(c.U).cuda(), link12=True)
    api.set_clover(lat, 1.0, -0.2)
    x = torch.from_numpy(x0.copy()).cuda()
    api.sap_smooth(lat, torch.from_numpy(b).cuda(), x, 2, 2, prec=api.DDQ_F32)
    torch.cuda.synchronize()
    api.destroy_lattice(lat)
    assert rel(x.cpu().numpy(), ref) < 1e-5


@pytest.mark.parametrize("dims", [(8, 8, 4, 8), (8, 8, 8, 8)], ids=lambda d: "x".join(map(str, d)))
def test_sap_without_mr_steps(dims):
    """m = 0: every block solve leaves the even sites alone and solves the block's odd rows
    (e_o = A_oo^-1 r_o); 8x8x4x8 takes the block kernel that reads links from memory for
    FP64 and FP32 18-real, 8^4 the on-chip one; FP32 12-real on both."""
    c = case(dims)
    b = c.full(512)
    x0 = c.full(513) * 0.1
    ref = solvers.sap(c.op, b, x0, 2, 0)
    for prec, tol in ((api.DDQ_F64, 1e-12), (api.DDQ_F32, 1e-5)):
        x = torch.from_numpy(x0.copy()).cuda()
        api.sap_smooth(c.lat, torch.from_numpy(b).cuda(), x, 2, 0, prec=prec)
        torch.cuda.synchronize()
        assert rel(x.cpu().numpy(), ref) < tol, prec
    lat = api.create_lattice(dims)
    api.set_gauge(lat, torch.from_numpy(c.U).cuda(), link12=True)
    api.set_clover(lat, 1.0, -0.2)
    x = torch.from_numpy(x0.copy()).cuda()
    api.sap_smooth(lat, torch.from_numpy(b).cuda(), x, 2, 0, prec=api.DDQ_F32)
    torch.cuda.synchronize()
    api.destroy_lattice(lat)
    assert rel(x.cpu().numpy(), ref) < 1e-5


def test_sap_reduces_the_residual_and_zero_sweeps():
    c = case((8, 8, 4, 8))
    b = c.full(511)
    bd = torch.from_numpy(b).cuda()
    x0 = torch.from_numpy(c.full(514)).cuda()
    x = x0.clone()
    api.sap_smooth(c.lat, bd, x, 0, 4)
    torch.cuda.synchronize()
    assert torch.equal(x, x0)  # n = 0: x unchanged
    res = []
    for n in (1, 2, 4):
        x = torch.zeros_like(bd)
        api.sap_smooth(c.lat, bd, x, n, 4)
        res.append(solvers.vnorm(b - c.op.D(x.cpu().numpy())) / solvers.vnorm(b))
    assert res[0] < 0.5 and res[2] < res[1] < res[0]


def test_sap_argument_errors():
    c = case((4, 4, 4, 4))
    b = torch.from_numpy(c.full(521)).cuda()
    with pytest.raises(api.DDQError):
        api.sap_smooth(c.lat, b, b, 1, 2)  # x and b overlap
    with pytest.raises(api.DDQError):
        api.sap_smooth(c.lat, b, torch.zeros_like(b), 1, -1)
    c6 = Case((6, 6, 6, 10), 0.4, 1.0, -0.2, 522)  # extents not multiples of 4
    b6 = torch.from_numpy(c6.full(523)).cuda()
    with pytest.raises(api.DDQError):
        api.sap_smooth(c6.lat, b6, torch.zeros_like(b6), 1, 2)


@pytest.mark.parametrize("sap_n,sap_m,prec", [(1, 4, api.DDQ_F64), (2, 2, api.DDQ_F64), (1, 4, api.DDQ_F32)])
def test_fgmres_with_sap_matches_oracle(sap_n, sap_m, prec):
    c = case((8, 8, 4, 8))
    b = c.full(531)
    x, info, ok = api.fgmres_sap_solve(c.lat, torch.from_numpy(b).cuda(), m=20, max_cycles=20, tol=1e-10,
                                       sap_n=sap_n, sap_m=sap_m, inner_prec=prec)
    assert ok, info
    xh = x.cpu().numpy()
    assert solvers.vnorm(b - c.op.D(xh)) <= 1e-10 * solvers.vnorm(b)
    res = solvers.gmres(c.op.D, b, np.zeros_like(b), 20, 20, 1e-10 * solvers.vnorm(b),
                        solvers.sap_preconditioner(c.op, sap_n, sap_m))
    assert res.converged
    assert abs(info["iters"] - res.iters) <= (1 if prec == api.DDQ_F64 else 2)
    assert rel(xh, res.x) < 1e-8
    with pytest.raises(api.DDQError):
        api.fgmres_sap_solve(c.lat, torch.from_numpy(b).cuda(), m=8, sap_n=1, sap_m=-1)
