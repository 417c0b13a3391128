"""The boundary's resource and multi-right-hand-side contract, through the raw C ABI
where it matters:

* apply, smooth, SAP and solve allocate nothing: past the reservation they return
  DDQ_ERR_STATE and do nothing; after ddq_reserve they run, leave the device's free
  memory unchanged and give the results of the per-right-hand-side calls (the HIP
  runtime takes device memory of its own when it first loads a source file's code
  object or instantiates graphs; in the suite's order the earlier tests have done that,
  and the SAP test does it itself);
* ddq_oe_gmres_solve with several right-hand sides: every system meets the full
  residual bar |b - D x| <= 1e-10 |b| with the oracle's D and equals its one-system
  solve;
* ddq_autotune writes the tuned tiles and a fresh lattice of the same extents picks
  them up from the file (seen in the kernel names of the library's profiler).
"""
import ctypes as C
import json

import numpy as np
import pytest
import torch

from gpu_common import Case, rel, to_dev, to_host
from oracle import solvers
from paper_2407_08092_amd import _lib, api, synth

pytestmark = pytest.mark.gpu

ERR_STATE = -2


def _p(t):
    return C.c_void_p(t.data_ptr())


def _free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_apply_and_smooth_allocate_nothing():
    L = _lib.lib()
    c = Case((8, 8, 8, 8), 0.5, 1.0, -0.2, 31)
    n = 8
    x = to_dev(c.vec(32, n))
    y = torch.empty_like(x)
    # set_gauge / set_clover reserved one right-hand side: eight are refused untouched
    y.fill_(7.0)
    assert L.ddq_apply_schur(c.lat.handle, 0, n, _p(x), _p(y), 0) == ERR_STATE
    assert b"ddq_reserve" in L.ddq_last_error()
    assert L.ddq_richardson_smooth(c.lat.handle, 0, n, _p(y), _p(x), 2, 0.1) == ERR_STATE
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
    assert L.ddq_reserve(c.lat.handle, n, 0, 0) == 0
    free0 = _free_bytes()
    for dag in (0, 1):
        assert L.ddq_apply_schur(c.lat.handle, 0, n, _p(x), _p(y), dag) == 0
        for r in range(n):
            y1 = api.apply_schur(c.lat, x[r].contiguous(), dagger=bool(dag))
            assert torch.equal(y[r], y1)
    x32 = api.convert_parity(c.lat, x, torch.complex64)
    b32 = api.convert_parity(c.lat, to_dev(c.vec(33, n)), torch.complex64)
    assert L.ddq_richardson_smooth(c.lat.handle, 1, n, _p(x32), _p(b32), 3, 0.1) == 0
    assert _free_bytes() == free0
    # a smaller count runs in the same reservation
    assert L.ddq_apply_schur(c.lat.handle, 0, 3, _p(x), _p(y), 0) == 0
    assert _free_bytes() == free0


def test_solvers_need_their_reservation():
    L = _lib.lib()
    c = Case((4, 4, 4, 4), 0.3, 1.0, -0.1, 101)
    b = torch.from_numpy(c.full(102)).cuda()
    x = torch.zeros_like(b)
    p = _lib.GmresParams(30, 100, 1e-10, 0, 0, 0.0, 0.0, 0, 2, 0)
    info = _lib.SolveInfo()
    assert L.ddq_oe_gmres_solve(c.lat.handle, 1, _p(x), _p(b), C.byref(p), C.byref(info)) == ERR_STATE
    assert L.ddq_fgmres_solve(c.lat.handle, _p(x), _p(b), C.byref(p), C.byref(info)) == ERR_STATE
    assert L.ddq_sap_smooth(c.lat.handle, 0, _p(x), _p(b), 1, 2) == ERR_STATE
    assert L.ddq_apply_dirac(c.lat.handle, 1, _p(b), _p(x)) == ERR_STATE
    g = torch.empty(c.lat.full_shape[:4] + (4, 3, 3), dtype=torch.complex128, device="cuda")
    v = to_dev(c.vec(3))
    assert L.ddq_backward_link_force(c.lat.handle, _p(v), _p(v), _p(g), None, 0) == ERR_STATE
    # a reservation for m = 20 does not cover m = 30
    assert L.ddq_reserve(c.lat.handle, 1, 20, 1) == 0
    assert L.ddq_oe_gmres_solve(c.lat.handle, 1, _p(x), _p(b), C.byref(p), C.byref(info)) == ERR_STATE
    assert L.ddq_reserve(c.lat.handle, 1, 30, 1) == 0
    free0 = _free_bytes()
    assert L.ddq_oe_gmres_solve(c.lat.handle, 1, _p(x), _p(b), C.byref(p), C.byref(info)) == 0
    assert _free_bytes() == free0
    assert solvers.vnorm(c.full(102) - c.op.D(x.cpu().numpy())) <= 1e-10 * solvers.vnorm(c.full(102))
    assert info.true_relres <= 1e-10


def test_batch_needs_its_reservation():
    L = _lib.lib()
    c = Case((4, 4, 4, 4), 0.5, 1.0, -0.2, 402)
    batch = api.batch_create([c.lat], [2])
    b = torch.from_numpy(np.stack([c.full(1402), c.full(1403)])).cuda()
    x = torch.zeros_like(b)
    xp, bp = (C.c_void_p * 1)(x.data_ptr()), (C.c_void_p * 1)(b.data_ptr())
    p = _lib.GmresParams(20, 40, 1e-10, 1, 3, 0.1, 0.0, 1, 2, 0)
    infos = (_lib.SolveInfo * 2)()
    assert L.ddq_batch_solve(batch.handle, xp, bp, C.byref(p), None, infos) == ERR_STATE
    assert L.ddq_batch_reserve(batch.handle, 20, 0) == 0
    free0 = _free_bytes()
    assert L.ddq_batch_solve(batch.handle, xp, bp, C.byref(p), None, infos) == 0
    assert _free_bytes() == free0
    p.cycle_graph = 1  # cycle mode was not reserved
    assert L.ddq_batch_solve(batch.handle, xp, bp, C.byref(p), None, infos) == ERR_STATE
    xh = x.cpu().numpy()
    for r in range(2):
        bb = c.full(1402 + r)
        assert solvers.vnorm(bb - c.op.D(xh[r])) <= 1e-10 * solvers.vnorm(bb)


@pytest.mark.parametrize("inner,sweeps", [(api.DDQ_F64, 0), (api.DDQ_F32, 6)])
def test_oe_gmres_several_right_hand_sides(inner, sweeps):
    dims = (4, 6, 8, 10)
    c = Case(dims, 0.5, 1.0, -0.2, 203)
    bs = np.stack([c.full(204 + r) for r in range(3)])
    omega = 0.8 / solvers.power_iteration(c.op.schur, c.vec(207), 50)
    x, infos, ok = api.oe_gmres_solve(c.lat, torch.from_numpy(bs).cuda(), m=20, tol=1e-10, inner_prec=inner,
                                      smoother_sweeps=sweeps, omega=omega)
    assert ok and len(infos) == 3
    xh = x.cpu().numpy()
    for r in range(3):
        assert solvers.vnorm(bs[r] - c.op.D(xh[r])) <= 1e-10 * solvers.vnorm(bs[r])
        assert infos[r]["true_relres"] <= 1e-10
        x1, info1, ok1 = api.oe_gmres_solve(c.lat, torch.from_numpy(bs[r]).cuda(), m=20, tol=1e-10,
                                            inner_prec=inner, smoother_sweeps=sweeps, omega=omega)
        assert ok1 and torch.equal(x[r], x1)


def test_autotune_cache_round_trip(tmp_path):
    path = tmp_path / "tiles.json"
    dims = (8, 8, 8, 16)
    c = Case(dims, 0.5, 1.0, -0.2, 41)
    chosen, _ = api.tune_multi_rhs(c.lat, 4, reps=2)
    api.autotune(c.lat, str(path))
    doc = json.loads(path.read_text())
    mine = [e for e in doc["tiles"] if e["nrhs"] == 4 and "8x8x8x16" in e["key"]]
    assert len(mine) == 1
    assert (mine[0]["nb"], mine[0]["waves"], mine[0]["xcd_map"]) == (chosen["nb"], chosen["waves"],
                                                                      chosen["xcd_map"])
    # a fresh lattice of the same extents takes the cached tile (here replaced by a known
    # one), and an entry of another lattice survives the rewrite
    mine[0].update(nb=2, waves=4, xcd_map=8)
    other = {"key": "other/1cu/2x2x2x2/link18", "nrhs": 2, "nb": 1, "waves": 1, "xcd_map": 0, "passes": 1,
             "lds_kb": 0, "ms": 1.0}
    entries = [e for e in doc["tiles"] if e is not mine[0]] + [mine[0], other]
    path.write_text('{"ddq_autotune": 1, "tiles": [\n' + ",\n".join(json.dumps(e) for e in entries) + "\n]}\n")
    lat2 = api.create_lattice(dims)
    api.set_gauge(lat2, torch.from_numpy(c.U).cuda())
    api.set_clover(lat2, 1.0, -0.2)
    api.autotune(lat2, str(path))
    after = json.loads(path.read_text())["tiles"]
    assert other in after
    assert [(e["nb"], e["waves"], e["xcd_map"]) for e in after if e["key"] == mine[0]["key"]] == [(2, 4, 8)]
    x = api.convert_parity(lat2, to_dev(c.vec(42, 4)), torch.complex64)
    api.profile_begin(lat2)
    y = api.apply_schur(lat2, x)
    names = list(api.profile_end(lat2))
    assert any(n.endswith("_x4_nb2g4x8") for n in names), names
    ref = np.stack([c.op.schur(v) for v in c.vec(42, 4)])
    assert rel(to_host(y), ref) < 1e-5


def test_sap_allocates_nothing_after_its_reservation():
    """DDQ_RESERVE_SAP covers the SAP-order copies of the block solves (FP64, FP32
    12-real) and of the residual (FP64 links, A_ee, A_oo): the first calls after the
    reservation build them there, so no SAP call changes the device's free memory."""
    L = _lib.lib()
    dims = (8, 8, 8, 8)
    c = Case(dims, 0.5, 1.0, -0.2, 41)
    # the HIP runtime loads sap.hip's code object on the first launch of one of its
    # kernels (device memory of its own): a SAP call on another lattice does that first
    warm = torch.from_numpy(c.full(43)).cuda()
    api.sap_smooth(c.lat, warm, torch.zeros_like(warm), 1, 1, prec=api.DDQ_F64)
    lat = api.create_lattice(dims)
    api.set_gauge(lat, torch.from_numpy(c.U).cuda(), link12=True)
    api.set_clover(lat, 1.0, -0.2)
    b = torch.from_numpy(c.full(42)).cuda()
    x = torch.zeros_like(b)
    assert L.ddq_sap_smooth(lat.handle, api.DDQ_F64, _p(x), _p(b), 1, 2) == ERR_STATE
    assert L.ddq_reserve(lat.handle, 1, 0, api.DDQ_RESERVE_SAP) == 0
    free0 = _free_bytes()
    for prec in (api.DDQ_F64, api.DDQ_F32, api.DDQ_F64):
        assert L.ddq_sap_smooth(lat.handle, prec, _p(x), _p(b), 1, 2) == 0
        assert _free_bytes() == free0
    assert torch.isfinite(torch.view_as_real(x)).all()
    api.destroy_lattice(lat)
