"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: FP64 path <= 1e-12 relative, FP32 path <= 1e-5 relative (norm-wise over all
sites and components, per right-hand side).  Lattices: the degenerate 2^4, the
4^4 lattice of the first workload, distinct extents 4x6x8x10 (catches axis
mix-ups; V/2 = 960 spans four 256-site workgroups with a ragged tail), 6x6x6x10
(ragged), and an 8^3x16 lattice of 16 full workgroups.
"""
import numpy as np
import pytest
import torch

from gpu_common import Case, rel, to_dev, to_host
from oracle import solvers
from paper_2407_08092_amd import api, synth

pytestmark = pytest.mark.gpu

DIMS = [(2, 2, 2, 2), (4, 4, 4, 4), (4, 6, 8, 10), (6, 6, 6, 10), (8, 8, 8, 16)]
_cases = {}


def case(dims, eps=0.3, c_sw=1.0, m0=-0.1, seed=101):
    key = (dims, eps, c_sw, m0, seed)
    if key not in _cases:
        _cases[key] = Case(dims, eps, c_sw, m0, seed)
    return _cases[key]


@pytest.mark.parametrize("dims", DIMS)
def test_clover_blocks(dims):
    c = case(dims, eps=0.5, c_sw=1.2, m0=-0.25, seed=7)
    A_ee, A_oo_inv = (t.cpu().numpy() for t in api.get_clover(c.lat))
    A = c.op.A_ee
    # oracle 12x12 -> two 6x6 chiral blocks
    ref_ee = np.stack([A[:, :6, :6], A[:, 6:, 6:]], 1)
    Ai = c.op.A_oo_inv
    ref_oo = np.stack([Ai[:, :6, :6], Ai[:, 6:, 6:]], 1)
    assert rel(A_ee, ref_ee) < 1e-14
    assert rel(A_oo_inv, ref_oo) < 1e-13
    assert np.abs(Ai[:, :6, 6:]).max() < 1e-14


@pytest.mark.parametrize("dims", DIMS)
def test_apply_schur_f64(dims):
    c = case(dims)
    x = c.vec(11)
    y = api.apply_schur(c.lat, to_dev(x))
    torch.cuda.synchronize()
    assert rel(to_host(y), c.op.schur(x)) < 1e-12


@pytest.mark.parametrize("dims", DIMS)
def test_apply_schur_f32(dims):
    c = case(dims)
    x = c.vec(12)
    y = api.apply_schur(c.lat, to_dev(x, torch.complex64))
    torch.cuda.synchronize()
    assert rel(to_host(y), c.op.schur(x)) < 1e-5


@pytest.mark.parametrize("dims", DIMS)
def test_apply_schur_dagger(dims):
    c = case(dims)
    x = c.vec(13)
    y = api.apply_schur(c.lat, to_dev(x), dagger=True)
    y32 = api.apply_schur(c.lat, to_dev(x, torch.complex64), dagger=True)
    torch.cuda.synchronize()
    ref = c.op.schur_adjoint(x)
    assert rel(to_host(y), ref) < 1e-12
    assert rel(to_host(y32), ref) < 1e-5


@pytest.mark.parametrize("dims,n", [((4, 6, 8, 10), 3), ((8, 8, 8, 16), 5), ((6, 6, 6, 10), 12), ((2, 2, 2, 2), 2)])
def test_apply_schur_multi_rhs(dims, n):
    # several right-hand sides per launch (workgroups of 64 sites x 4 right-hand sides,
    # ragged counts leave idle wavefronts)
    c = case(dims)
    x = c.vec(14, n=n)
    y = api.apply_schur(c.lat, to_dev(x))
    y32 = api.apply_schur(c.lat, to_dev(x, torch.complex64))
    yd = api.apply_schur(c.lat, to_dev(x), dagger=True)
    torch.cuda.synchronize()
    for r in range(n):
        assert rel(to_host(y)[r], c.op.schur(x[r])) < 1e-12
        assert rel(to_host(y32)[r], c.op.schur(x[r])) < 1e-5
        assert rel(to_host(yd)[r], c.op.schur_adjoint(x[r])) < 1e-12


def test_richardson_multi_rhs():
    c = case((4, 6, 8, 10))
    b = c.vec(16, n=4)
    x0 = c.vec(17, n=4)
    xd = to_dev(x0)
    api.richardson_smooth(c.lat, xd, to_dev(b), 6, 0.15)
    x32 = to_dev(x0, torch.complex64)
    api.richardson_smooth(c.lat, x32, to_dev(b, torch.complex64), 6, 0.15)
    torch.cuda.synchronize()
    for r in range(4):
        ref = solvers.richardson(c.op.schur, b[r], x0[r], 6, 0.15)
        assert rel(to_host(xd)[r], ref) < 1e-12
        assert rel(to_host(x32)[r], ref) < 1e-5


def test_periodic_t_lattice():
    c = Case((4, 6, 8, 10), 0.4, 1.0, -0.15, 55, antiperiodic=False)
    x = c.vec(15)
    y = api.apply_schur(c.lat, to_dev(x))
    torch.cuda.synchronize()
    assert rel(to_host(y), c.op.schur(x)) < 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 8, 10), (6, 6, 6, 10)])
def test_richardson_f64(dims):
    c = case(dims)
    b = c.vec(21)
    lam = solvers.power_iteration(c.op.schur, c.vec(22), 50)
    for omega in (0.8 / lam, 0.8):  # Alg. 4 weight delta/|lambda_max| with delta = 0.8, and 0.8 literally
        x0 = c.vec(23)
        ref = solvers.richardson(c.op.schur, b, x0, 10, omega)
        xd = to_dev(x0)
        api.richardson_smooth(c.lat, xd, to_dev(b), 10, omega)
        torch.cuda.synchronize()
        assert rel(to_host(xd), ref) < 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 8, 10), (8, 8, 8, 16)])
def test_richardson_f32(dims):
    c = case(dims)
    b = c.vec(24)
    lam = solvers.power_iteration(c.op.schur, c.vec(25), 50)
    omega = 0.8 / lam
    ref = solvers.richardson(c.op.schur, b, np.zeros_like(b), 20, omega)
    xd = api.parity_vector(c.lat, dtype=torch.complex64).zero_()
    api.richardson_smooth(c.lat, xd, to_dev(b, torch.complex64), 20, omega)
    torch.cuda.synchronize()
    assert rel(to_host(xd), ref) < 1e-5


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 6, 8, 10), (8, 8, 8, 16)])
def test_link12_f32(dims):
    # FP32 links stored as two rows, the third rebuilt from unitarity in the kernel
    c = Case(dims, 0.5, 1.0, -0.2, 301)
    api.set_gauge(c.lat, torch.from_numpy(c.U).cuda(), link12=True)
    api.set_clover(c.lat, 1.0, -0.2)
    x = c.vec(71)
    y = api.apply_schur(c.lat, to_dev(x, torch.complex64))
    yd = api.apply_schur(c.lat, to_dev(x, torch.complex64), dagger=True)
    y64 = api.apply_schur(c.lat, to_dev(x))  # FP64 keeps all 18 reals
    torch.cuda.synchronize()
    assert rel(to_host(y), c.op.schur(x)) < 1e-5
    assert rel(to_host(yd), c.op.schur_adjoint(x)) < 1e-5
    assert rel(to_host(y64), c.op.schur(x)) < 1e-12
    b = c.vec(72)
    ref = solvers.richardson(c.op.schur, b, np.zeros_like(b), 20, 0.17)
    xd = api.parity_vector(c.lat, dtype=torch.complex64).zero_()
    api.richardson_smooth(c.lat, xd, to_dev(b, torch.complex64), 20, 0.17)
    torch.cuda.synchronize()
    assert rel(to_host(xd), ref) < 1e-5


def test_richardson_zero_sweeps_is_identity():
    c = case((4, 4, 4, 4))
    x0 = c.vec(26)
    xd = to_dev(x0)
    api.richardson_smooth(c.lat, xd, to_dev(c.vec(27)), 0, 0.3)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(xd), x0)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 6, 8, 10), (6, 6, 6, 10)])
def test_prepare_reconstruct(dims):
    c = case(dims)
    b = c.full(31)
    bd = torch.from_numpy(b).cuda()
    bt = api.oe_prepare(c.lat, bd)
    torch.cuda.synchronize()
    assert rel(to_host(bt), c.op.prepare(b)) < 1e-12
    xe = c.vec(32)
    x = api.oe_reconstruct(c.lat, to_dev(xe), bd)
    torch.cuda.synchronize()
    assert rel(x.cpu().numpy(), c.op.reconstruct(xe, b)) < 1e-12


@pytest.mark.parametrize("dims", [(4, 6, 8, 10)])
def test_pack_unpack_roundtrip_bitwise(dims):
    c = case(dims)
    f = torch.from_numpy(c.full(41)).cuda()
    e = api.pack_parity(c.lat, f, 0)
    o = api.pack_parity(c.lat, f, 1)
    g = api.unpack_parity(c.lat, e, 0)
    api.unpack_parity(c.lat, o, 1, out=g)
    f32 = f.to(torch.complex64)
    e32 = api.pack_parity(c.lat, f32, 0)
    g32 = api.unpack_parity(c.lat, e32, 0)
    torch.cuda.synchronize()
    assert torch.equal(g, f)
    assert np.array_equal(to_host(e), c.olat.to_parity(c.full(41), 0))
    assert torch.equal(e32, api.convert_parity(c.lat, e, torch.complex64))
    assert torch.equal(e32, to_dev(to_host(e), torch.complex64))
    even = torch.from_numpy(np.broadcast_to(c.olat.parity == 0, f.shape[:4]).copy()).cuda()[..., None, None]
    assert torch.equal(g32 * even, f32 * even)
    # FP32 -> FP64 widening is exact
    assert torch.equal(api.convert_parity(c.lat, e32, torch.complex128), to_dev(to_host(e32)))


def test_power_iteration_matches_oracle():
    c = case((4, 4, 4, 4))
    v0 = c.vec(51)
    ref = solvers.power_iteration(c.op.schur, v0, 50)
    got = api.estimate_lambda_max(c.lat, 50, to_dev(v0))
    assert abs(got / ref - 1) < 1e-12


def _true_relres(c, x, b):
    return solvers.vnorm(b - c.op.D(x)) / solvers.vnorm(b)


def test_gmres_f64_first_workload():
    # 4^4, eps 0.3, c_sw 1.0, m0 -0.1, odd-even GMRES(30) to 1e-10
    c = case((4, 4, 4, 4), eps=0.3, c_sw=1.0, m0=-0.1, seed=101)
    b = synth.gaussian_spinor((4, 4, 4, 4), 102)
    x, info, ok = api.oe_gmres_solve(c.lat, torch.from_numpy(b).cuda(), m=30, max_cycles=100, tol=1e-10)
    assert ok
    xh = x.cpu().numpy()
    assert _true_relres(c, xh, b) <= 1e-10
    x_ref, res = solvers.oe_solve(c.op, b, 30, 100, 1e-10)
    assert res.converged
    assert rel(xh, x_ref) < 1e-8
    assert abs(info["iters"] - res.iters) <= 2
    assert info["true_relres"] <= 1e-10


@pytest.mark.parametrize("inner,sweeps", [(api.DDQ_F64, 10), (api.DDQ_F32, 0), (api.DDQ_F32, 10)])
def test_gmres_variants(inner, sweeps):
    dims = (6, 6, 6, 10)
    c = case(dims, eps=0.5, c_sw=1.0, m0=-0.2, seed=201)
    b = synth.gaussian_spinor(dims, 202)
    lam = solvers.power_iteration(c.op.schur, c.vec(203), 50)
    x, info, ok = api.oe_gmres_solve(c.lat, torch.from_numpy(b).cuda(), m=30, max_cycles=60, tol=1e-10,
                                     inner_prec=inner, smoother_sweeps=sweeps, omega=0.8 / lam)
    assert ok, info
    assert _true_relres(c, x.cpu().numpy(), b) <= 1e-10
    if inner == api.DDQ_F32:
        assert info["applies_lo"] > 0


def test_gmres_not_converged_status():
    c = case((4, 4, 4, 4))
    b = synth.gaussian_spinor((4, 4, 4, 4), 61)
    x, info, ok = api.oe_gmres_solve(c.lat, torch.from_numpy(b).cuda(), m=2, max_cycles=1, tol=1e-12)
    assert not ok
    assert info["cycles"] == 1 and info["iters"] == 2


def test_zero_rhs_is_converged_before_any_step():
    """b = 0 from x = 0: |b - D x| = 0 <= tol |b| holds before the first Arnoldi step (Alg. 2
    stops on the initial residual), for odd-even GMRES, FGMRES with M_nu and FGMRES with
    SAP; x stays zero."""
    c = case((4, 4, 4, 4))
    b = torch.zeros(c.lat.full_shape, dtype=torch.complex128, device="cuda")
    runs = [(api.oe_gmres_solve, {}), (api.fgmres_solve, {"omega": 0.1}), (api.fgmres_sap_solve, {})]
    for solve, kw in runs:
        x, info, ok = solve(c.lat, b, m=8, **kw)
        torch.cuda.synchronize()
        assert ok, solve.__name__
        assert info["iters"] == 0 and info["true_relres"] == 0.0, (solve.__name__, info)
        assert torch.count_nonzero(x) == 0, solve.__name__


def test_gmres_nonfinite_rhs_rejected():
    c = case((4, 4, 4, 4))
    b = synth.gaussian_spinor((4, 4, 4, 4), 62)
    b[0, 0, 0, 0, 0, 0] = np.nan
    with pytest.raises(api.DDQError) as e:
        api.oe_gmres_solve(c.lat, torch.from_numpy(b).cuda(), m=4, max_cycles=2)
    assert e.value.status == -6


def test_not_positive_definite_clover_reported():
    lat = api.create_lattice((4, 4, 4, 4))
    api.set_gauge(lat, torch.from_numpy(synth.gauge_field((4, 4, 4, 4), 0.9, 5)).cuda())
    with pytest.raises(api.DDQError) as e:
        api.set_clover(lat, 10.0, -4.0)
    assert e.value.status == -5


def test_call_order_errors():
    lat = api.create_lattice((4, 4, 4, 4))
    x = torch.zeros((12, lat.Vh), dtype=torch.complex128, device="cuda")
    with pytest.raises(api.DDQError) as e:
        api.apply_schur(lat, x)
    assert e.value.status == -2
    api.set_gauge(lat, torch.from_numpy(synth.gauge_field((4, 4, 4, 4), 0.3, 5)).cuda())
    with pytest.raises(api.DDQError):
        api.apply_schur(lat, x)
    with pytest.raises(api.DDQError):
        api.set_clover(lat, float("nan"), 0.0)


@pytest.mark.parametrize("dims", [(4, 6, 8, 10), (6, 6, 6, 10), (8, 8, 8, 16)])
@pytest.mark.parametrize("nc", [2, 3, 4, 10])
def test_chunked_sweeps_equal_plain_sweeps(dims, nc):
    # Richardson sweeps launched per range of t-slices give the plain sweep's result bit for
    # bit (every site computes the same sums from the same inputs), FP64 and FP32
    c = case(dims)
    nc = min(nc, dims[3])
    b, x0 = c.vec(131), c.vec(132)
    omega = 0.12
    outs = {}
    for dt in (torch.complex128, torch.complex64):
        for k in (1, nc):
            api.set_sweep_chunks(c.lat, k)
            x = to_dev(x0, dt)
            api.richardson_smooth(c.lat, x, to_dev(b, dt), 4, omega)
            torch.cuda.synchronize()
            outs[(dt, k)] = x
    api.set_sweep_chunks(c.lat, 0)
    for dt in (torch.complex128, torch.complex64):
        assert torch.equal(outs[(dt, 1)], outs[(dt, nc)])
    ref = solvers.richardson(c.op.schur, b, x0, 4, omega)
    assert rel(to_host(outs[(torch.complex128, nc)]), ref) < 1e-12
    assert rel(to_host(outs[(torch.complex64, nc)]), ref) < 1e-5


@pytest.mark.parametrize("dims", [(4, 6, 8, 10), (8, 8, 8, 16)])
@pytest.mark.parametrize("nc", [2, 5, 16])
@pytest.mark.parametrize("dagger", [False, True], ids=["plain", "dagger"])
def test_chunked_apply_equals_plain_apply(dims, nc, dagger):
    # the Schur apply launched per range of t-slices: bit for bit the one-launch apply
    c = case(dims)
    nc = min(nc, dims[3])
    x = c.vec(133)
    outs = {}
    for dt in (torch.complex128, torch.complex64):
        for k in (1, nc):
            api.set_sweep_chunks(c.lat, k)
            outs[(dt, k)] = api.apply_schur(c.lat, to_dev(x, dt), dagger=dagger)
            torch.cuda.synchronize()
    api.set_sweep_chunks(c.lat, 0)
    for dt in (torch.complex128, torch.complex64):
        assert torch.equal(outs[(dt, 1)], outs[(dt, nc)])
    ref = c.op.schur_adjoint(x) if dagger else c.op.schur(x)
    assert rel(to_host(outs[(torch.complex128, nc)]), ref) < 1e-12
    assert rel(to_host(outs[(torch.complex64, nc)]), ref) < 1e-5


def test_chunk_count_arguments():
    c = case((4, 4, 4, 4))
    with pytest.raises(api.DDQError):
        api.set_sweep_chunks(c.lat, -1)
    with pytest.raises(api.DDQError):
        api.set_sweep_chunks(c.lat, 5)  # more ranges than t-slices
    api.set_sweep_chunks(c.lat, 4)
    api.set_sweep_chunks(c.lat, 0)
