"""16-bit storage (FP16 and BF16 vectors, 12-real links and clover blocks; FP32
arithmetic) through the C ABI, against the FP64 oracle.

Tolerances follow from the storage rounding: with u the unit roundoff of the
format (FP16: 2^-11 = 4.9e-4, BF16: 2^-8 = 3.9e-3) every stored input of one
apply (the spinor, the links, whose third row is rebuilt from two rounded rows,
the clover slots) and the stored output carry a relative error of at most u, so a
bound of 10 u norm-wise per right-hand side for one apply, and 10 u per sweep for
the Richardson smoother, leaves room for the sums of a few such errors.  Solves
that use the 16-bit smoother only as the preconditioner of FP64-refined GMRES are
held to the same 1e-10 true residual as every other solve.
"""
import numpy as np
import pytest
import torch

from gpu_common import Case, rel, to_dev, to_dev16, to_host
from oracle import solvers
from paper_2407_08092_amd import api, synth

pytestmark = pytest.mark.gpu

U_ROUND = {torch.float16: 2.0 ** -11, torch.bfloat16: 2.0 ** -8}
PREC = {torch.float16: api.DDQ_F16, torch.bfloat16: api.DDQ_BF16}
DTYPES = [torch.float16, torch.bfloat16]
DIMS = [(4, 4, 4, 4), (4, 6, 8, 10), (6, 6, 6, 10)]
_cases = {}


def case(dims):
    if dims not in _cases:
        c = Case(dims, 0.5, 1.0, -0.2, 81)
        api.set_gauge(c.lat, torch.from_numpy(c.U).cuda(), store=(api.DDQ_F64, api.DDQ_F32, api.DDQ_F16, api.DDQ_BF16))
        api.set_clover(c.lat, 1.0, -0.2)
        lam = solvers.power_iteration(c.op.schur, c.vec(82), 50)
        _cases[dims] = (c, 0.8 / lam)
    return _cases[dims]


def per_rhs_err(got, ref):
    return max(rel(got[r], ref[r]) for r in range(ref.shape[0]))


@pytest.mark.parametrize("dtype", DTYPES, ids=["f16", "bf16"])
def test_conversion_matches_host_rounding(dtype):
    c, _ = case((4, 6, 8, 10))
    x = c.vec(83, 2)
    lib16 = api.convert_parity(c.lat, to_dev(x), dtype)
    host16 = to_dev16(x, dtype)
    assert torch.equal(lib16, host16)  # FP16: one rounding from FP64; BF16: through FP32
    back = api.convert_parity(c.lat, lib16, torch.complex128)
    assert torch.equal(back, to_dev(to_host(host16)))  # widening is exact
    f32 = api.convert_parity(c.lat, lib16, torch.complex64)
    assert torch.equal(f32, to_dev(to_host(host16), torch.complex64))


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("dtype", DTYPES, ids=["f16", "bf16"])
def test_apply_schur_16bit(dims, dtype):
    c, _ = case(dims)
    x = c.vec(84, 3)
    y = api.apply_schur(c.lat, to_dev16(x, dtype))
    ref = np.stack([c.op.schur(x[r]) for r in range(3)])
    err = per_rhs_err(to_host(y), ref)
    assert err < 10 * U_ROUND[dtype], err


@pytest.mark.parametrize("n", [1, 2, 4, 5, 6])
def test_apply_16bit_rhs_counts(n):
    # 1, 2 or 3 right-hand sides per thread (the largest dividing n), ragged 6x6x6x10
    c, _ = case((6, 6, 6, 10))
    x = c.vec(91, n)
    xd = to_dev16(x, torch.float16)
    y = api.apply_schur(c.lat, xd if n > 1 else xd[0])
    ref = np.stack([c.op.schur(x[r]) for r in range(n)])
    got = to_host(y) if n > 1 else to_host(y)[None]
    assert per_rhs_err(got, ref) < 10 * U_ROUND[torch.float16]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("dtype", DTYPES, ids=["f16", "bf16"])
def test_richardson_16bit(dims, dtype):
    c, omega = case(dims)
    x0, b = c.vec(85, 2), c.vec(86, 2)
    xs = to_dev16(x0, dtype)
    api.richardson_smooth(c.lat, xs, to_dev16(b, dtype), 3, omega)
    ref = np.stack([solvers.richardson(c.op.schur, b[r], x0[r], 3, omega) for r in range(2)])
    err = per_rhs_err(to_host(xs), ref)
    assert err < 30 * U_ROUND[dtype], err


@pytest.mark.parametrize("dtype", DTYPES, ids=["f16", "bf16"])
def test_gmres_with_16bit_smoother(dtype):
    dims = (6, 6, 6, 10)
    c, omega = case(dims)
    b = synth.gaussian_spinor(dims, 87)
    x, info, ok = api.oe_gmres_solve(c.lat, torch.from_numpy(b).cuda(), m=30, max_cycles=60, tol=1e-10,
                                     inner_prec=api.DDQ_F32, smoother_sweeps=4, omega=omega,
                                     smoother_prec=PREC[dtype])
    assert ok, info
    res = solvers.vnorm(b - c.op.D(x.cpu().numpy())) / solvers.vnorm(b)
    assert res <= 1e-10


def test_batch_with_16bit_smoother():
    c1, om1 = case((4, 4, 4, 4))
    c2, om2 = case((4, 6, 8, 10))
    bs = [np.stack([synth.gaussian_spinor(c.dims, 90 + r) for r in range(n)]) for c, n in ((c1, 2), (c2, 3))]
    batch = api.batch_create([c1.lat, c2.lat], [2, 3])
    xs, infos, ok = api.batch_solve(batch, [torch.from_numpy(b).cuda() for b in bs], m=30, tol=1e-10,
                                    smoother_sweeps=4, omega=[om1, om2], smoother_prec=api.DDQ_F16)
    assert ok, infos
    for c, b, x in ((c1, bs[0], xs[0]), (c2, bs[1], xs[1])):
        xh = x.cpu().numpy()
        for r in range(b.shape[0]):
            assert solvers.vnorm(b[r] - c.op.D(xh[r])) / solvers.vnorm(b[r]) <= 1e-10


def test_16bit_errors():
    c, omega = case((4, 4, 4, 4))
    x = to_dev16(c.vec(88), torch.float16)
    with pytest.raises(api.DDQError):
        api.apply_schur(c.lat, x, dagger=True)
    with pytest.raises(api.DDQError):  # FP32 -> 16 bit is not offered
        api.convert_parity(c.lat, to_dev(c.vec(88), torch.complex64), torch.float16)
    lat = api.create_lattice((4, 4, 4, 4))
    api.set_gauge(lat, torch.from_numpy(c.U).cuda())  # no 16-bit storage requested
    api.set_clover(lat, 1.0, -0.2)
    with pytest.raises(api.DDQError) as e:
        api.apply_schur(lat, x)
    assert e.value.status == -2
    b = torch.from_numpy(synth.gaussian_spinor((4, 4, 4, 4), 89)).cuda()
    with pytest.raises(api.DDQError):
        api.oe_gmres_solve(lat, b, m=8, inner_prec=api.DDQ_F32, smoother_sweeps=2, omega=omega,
                           smoother_prec=api.DDQ_F16)
    with pytest.raises(api.DDQError):  # a 16-bit smoother under an FP64 inner solve
        api.oe_gmres_solve(c.lat, b, m=8, inner_prec=api.DDQ_F64, smoother_sweeps=2, omega=omega,
                           smoother_prec=api.DDQ_F16)


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("dtype", DTYPES, ids=["f16", "bf16"])
def test_fp32_clover_variant(dims, dtype):
    # 16-bit links and spinors with the FP32 clover blocks: the same bars (one rounding
    # fewer per apply), and the profiler counts 36 FP32 slot pairs per site
    c, omega = case(dims)
    x, b = c.vec(92, 2), c.vec(93, 2)
    api.set_h16_clover(c.lat, True)
    try:
        api.profile_begin(c.lat)
        y = api.apply_schur(c.lat, to_dev16(x, dtype))
        stats = api.profile_end(c.lat)
        xs = to_dev16(x, dtype)
        api.richardson_smooth(c.lat, xs, to_dev16(b, dtype), 3, omega)
        torch.cuda.synchronize()
    finally:
        api.set_h16_clover(c.lat, False)
    ref = np.stack([c.op.schur(x[r]) for r in range(2)])
    assert per_rhs_err(to_host(y), ref) < 10 * U_ROUND[dtype]
    ref = np.stack([solvers.richardson(c.op.schur, b[r], x[r], 3, omega) for r in range(2)])
    assert per_rhs_err(to_host(xs), ref) < 30 * U_ROUND[dtype]
    tag = "bf16" if dtype == torch.bfloat16 else "f16"
    vh = c.olat.Vh
    per_site = {f"hop_clinv_{tag}_c32_x2": (2 * 24 + 48) * 4 + 36 * 8, f"hop_apply_{tag}_c32_x2": (2 * 36 + 48) * 4 + 36 * 8}
    for name, bps in per_site.items():
        assert name in stats, list(stats)
        assert stats[name]["bytes_per_launch"] == bps * vh


def test_fp32_clover_needs_fp32_storage():
    c, _ = case((4, 4, 4, 4))
    lat = api.create_lattice((4, 4, 4, 4))
    api.set_gauge(lat, torch.from_numpy(c.U).cuda(), store=(api.DDQ_F64, api.DDQ_F16))
    api.set_clover(lat, 1.0, -0.2)
    with pytest.raises(api.DDQError) as e:
        api.set_h16_clover(lat, True)
    assert e.value.status == -2
