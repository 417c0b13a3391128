"""The full operator D, the odd-even smoother M_nu (Sect. 2.4.5) and FGMRES on the full
D through the C ABI, against the FP64 oracle: D and M_nu with FP64 sweeps to 1e-12
relative, M_nu with FP32 sweeps to 1e-5, FGMRES to the 1e-10 true residual; the matrix
D M_3 on 4^4 (the right panel of Fig. 1), built column by column on the GPU, against
eq. 2's dense factorised form, and its spectrum on a smaller lattice against the closed
form {1 - (1 - omega lambda)^nu : lambda in spec(D_S)} plus 1 on the odd half.

Lattices: 2^4 (two-site extents: neighbours coincide), 4x6x8x10 and 6x6x6x10 (V/2 not a
multiple of 64 or 256).
"""
import numpy as np
import pytest
import torch

from gpu_common import Case, rel
from oracle import dirac, solvers
from oracle.dirac import dense_schur, sparse_D
from paper_2407_08092_amd import api, synth

pytestmark = pytest.mark.gpu

DIMS = [(2, 2, 2, 2), (4, 6, 8, 10), (6, 6, 6, 10)]
_cases = {}


def case(dims, eps=0.5, c_sw=1.0, m0=-0.2, seed=301):
    key = (tuple(dims), eps, c_sw, m0, seed)
    if key not in _cases:
        _cases[key] = Case(dims, eps, c_sw, m0, seed)
    return _cases[key]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("dims", DIMS)
def test_apply_dirac_matches_oracle(dims):
    c = case(dims)
    x = c.full(311)
    y = api.apply_dirac(c.lat, dev(x))
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), c.op.D(x)) < 1e-13
    xs = np.stack([c.full(312), c.full(313), c.full(314)])
    ys = api.apply_dirac(c.lat, dev(xs)).cpu().numpy()
    for r in range(3):
        assert rel(ys[r], c.op.D(xs[r])) < 1e-13


@pytest.mark.parametrize("nu", [0, 1, 3])
@pytest.mark.parametrize("dims", DIMS)
def test_oe_smoother_matches_oracle(dims, nu):
    c = case(dims)
    r = c.full(321)
    omega = 0.12
    ref = solvers.oe_smoother(c.op, nu, omega)(r)
    z = api.oe_smoother(c.lat, dev(r), nu, omega).cpu().numpy()
    assert rel(z, ref) < 1e-12
    z32 = api.oe_smoother(c.lat, dev(r), nu, omega, prec=api.DDQ_F32).cpu().numpy()
    assert rel(z32, ref) < 1e-5
    if nu == 0:  # p_{R,0} = 0: the even half is exactly zero
        even = c.olat.parity == 0
        assert np.all(z[even] == 0) and np.all(z32[even] == 0)


def test_oe_smoother_several_rhs_match_single():
    c = case((4, 6, 8, 10))
    rs = np.stack([c.full(331 + k) for k in range(4)])
    zs = api.oe_smoother(c.lat, dev(rs), 3, 0.12).cpu().numpy()
    for k in range(4):
        z1 = api.oe_smoother(c.lat, dev(rs[k]), 3, 0.12).cpu().numpy()
        assert rel(zs[k], z1) < 1e-14


@pytest.mark.parametrize("inner", [api.DDQ_F64, api.DDQ_F32], ids=["f64", "f32"])
def test_fgmres_full_matches_oracle(inner):
    dims = (4, 6, 8, 10)
    c = case(dims, eps=0.4, seed=341)
    b = c.full(342)
    omega = 0.8 / solvers.power_iteration(c.op.schur, c.vec(343), 50)
    x, info, ok = api.fgmres_solve(c.lat, dev(b), m=16, max_cycles=30, tol=1e-10, smoother_sweeps=3, omega=omega,
                                   inner_prec=inner)
    assert ok, info
    xh = x.cpu().numpy()
    assert solvers.vnorm(b - c.op.D(xh)) <= 1e-10 * solvers.vnorm(b)
    assert info["true_relres"] <= 1e-10
    x_ref, res = solvers.fgmres_full(c.op, b, 16, 30, 1e-10, 3, omega)
    assert res.converged
    assert rel(xh, x_ref) < 1e-8
    if inner == api.DDQ_F64:
        assert abs(info["iters"] - res.iters) <= 1
    else:
        assert info["applies_lo"] > 0 and abs(info["iters"] - res.iters) <= 3


def test_fgmres_initial_guess_status_and_errors():
    c = case((4, 4, 4, 4), eps=0.3, m0=-0.1, seed=351)
    b = synth.gaussian_spinor((4, 4, 4, 4), 352)
    x_ref = np.linalg.solve(sparse_D(c.op).toarray(), b.ravel()).reshape(b.shape)
    # an exact initial guess converges at the first residual check
    x, info, ok = api.fgmres_solve(c.lat, dev(b), x0=dev(x_ref), m=8, tol=1e-10, smoother_sweeps=2, omega=0.15)
    assert ok and info["iters"] == 0 and info["cycles"] == 0
    x, info, ok = api.fgmres_solve(c.lat, dev(b), m=2, max_cycles=1, tol=1e-12, smoother_sweeps=1, omega=0.15)
    assert not ok and info["cycles"] == 1 and info["iters"] == 2
    with pytest.raises(api.DDQError):
        api.fgmres_solve(c.lat, dev(b), m=129)
    bad = b.copy()
    bad[0, 0, 0, 0, 0, 0] = np.nan
    with pytest.raises(api.DDQError) as e:
        api.fgmres_solve(c.lat, dev(bad), m=4, smoother_sweeps=1, omega=0.15)
    assert e.value.status == -6
    with pytest.raises(api.DDQError):
        api.oe_smoother(c.lat, dev(b), 2, 0.1, prec=api.DDQ_F16)


def _gpu_DM(c, nu, omega):
    """D M_nu as a dense matrix: M_nu applied to every unit vector at once (one right-
    hand side per column), then D, both on the GPU"""
    n = 12 * c.olat.V
    eye = torch.eye(n, dtype=torch.complex128, device="cuda").reshape((n,) + c.lat.full_shape)
    DMt = api.apply_dirac(c.lat, api.oe_smoother(c.lat, eye, nu, omega))
    return DMt.reshape(n, n).T.cpu().numpy()  # row r of DMt is column r of D M


def test_D_M3_matrix_on_4444():
    # the lattice of Fig. 1; delta = 1: omega = 1 / |lambda_max(D_S)|
    c = case((4, 4, 4, 4), eps=0.3, m0=-0.1, seed=101)
    D = sparse_D(c.op).toarray()
    e, o = dirac.parity_dofs(c.olat, 0), dirac.parity_dofs(c.olat, 1)
    Dee, Deo, Doe, Doo = D[np.ix_(e, e)], D[np.ix_(e, o)], D[np.ix_(o, e)], D[np.ix_(o, o)]
    Doo_inv = np.linalg.inv(Doo)
    DS = Dee - Deo @ Doo_inv @ Doe
    omega = 1.0 / np.abs(np.linalg.eigvals(DS)).max()
    Ie = np.eye(len(e))
    pS = (Ie - np.linalg.matrix_power(Ie - omega * DS, 3)) @ np.linalg.inv(DS)
    n = D.shape[0]
    M = np.zeros((n, n), complex)  # eq. 2 with D_S^-1 -> p_{R,3}(D_S), in the natural order
    R = np.eye(n, dtype=complex)[e] - Deo @ Doo_inv @ np.eye(n)[o]  # right factor: even rows
    Xe = pS @ R
    M[e] = Xe
    M[o] = Doo_inv @ np.eye(n)[o] - Doo_inv @ Doe @ Xe
    assert rel(_gpu_DM(c, 3, omega), D @ M) < 1e-12


def test_D_M_spectrum_closed_form():
    c = case((4, 4, 2, 2), eps=0.3, m0=-0.1, seed=361)
    lS = np.linalg.eigvals(dense_schur(c.op))
    omega = 0.8 / np.abs(lS).max()
    from scipy.optimize import linear_sum_assignment
    for nu in (1, 3):
        got = np.linalg.eigvals(_gpu_DM(c, nu, omega))
        expect = np.concatenate([1 - (1 - omega * lS) ** nu, np.ones(len(lS))])
        cost = np.abs(got[:, None] - expect[None, :])
        r, k = linear_sum_assignment(cost)
        assert cost[r, k].max() < 1e-9
