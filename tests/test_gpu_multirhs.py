"""FP32 multi-right-hand-side stencil tiles through the C ABI, against the FP64
oracle applied to each right-hand side on its own (FP32 bar: 1e-5 relative per
right-hand side), and against the one-right-hand-side-per-thread kernel.

Every tile is covered: nb (right-hand sides per thread) 0..4, one or four
wavefronts per site block, XCD order off, in chunks of 1, 8, 32 site blocks
(more chunks than the small lattices have blocks: the padded grid) or slab order
(t-slices cut into eight pieces of 64-site groups: on these lattices some XCDs get
none), 18- and 12-real links; and tiles that split the right-hand sides into passes or
request LDS to cap the resident workgroups.
Lattices 4x6x8x10 (V/2 = 960: 15 blocks of 64 sites, 3.75 of 256) and 6x6x6x10
(V/2 = 1080: ragged for both) with 12 right-hand sides (divisible by 1, 2, 3, 4).
"""
import itertools

import numpy as np
import pytest
import torch

from gpu_common import Case, rel, to_dev, to_host
from oracle import solvers
from paper_2407_08092_amd import api

pytestmark = pytest.mark.gpu

NRHS = 12
DIMS = [(4, 6, 8, 10), (6, 6, 6, 10)]
TILES = [(0, 4, 0), (0, 4, -1)] + list(itertools.product((1, 2, 3, 4), (1, 4), (-1, 0, 1, 8, 32)))
# right-hand sides split into passes and workgroups capped by an LDS request
PASS_TILES = [(1, 4, -1, 2, 64), (2, 1, -1, 3, 48), (3, 4, -1, 2, 96), (4, 4, -1, 3, 0), (1, 1, -1, 4, 0),
              (2, 4, 0, 2, 160)]
_cache = {}


def setup(dims):
    if dims not in _cache:
        c = Case(dims, 0.5, 1.0, -0.2, 71)
        lat12 = api.create_lattice(dims)
        api.set_gauge(lat12, torch.from_numpy(c.U).cuda(), link12=True)
        api.set_clover(lat12, 1.0, -0.2)
        x = c.vec(72, NRHS)
        b = c.vec(73, NRHS)
        lam = solvers.power_iteration(c.op.schur, c.vec(74), 50)
        omega = 0.8 / lam
        y_ref = np.stack([c.op.schur(x[r]) for r in range(NRHS)])
        x_rich = np.stack([solvers.richardson(c.op.schur, b[r], x[r], 3, omega) for r in range(NRHS)])
        _cache[dims] = (c, lat12, x, b, omega, y_ref, x_rich)
    return _cache[dims]


def per_rhs_err(got, ref):
    return max(rel(got[r], ref[r]) for r in range(ref.shape[0]))


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("link12", [False, True])
@pytest.mark.parametrize("tile", TILES + PASS_TILES, ids=lambda t: "nb{}w{}x{}".format(*t[:3]) +
                         ("p{}l{}".format(*t[3:]) if len(t) > 3 else ""))
def test_tile_apply_and_richardson(dims, link12, tile):
    c, lat12, x, b, omega, y_ref, x_rich = setup(dims)
    lat = lat12 if link12 else c.lat
    api.set_multi_rhs_tile(lat, NRHS, *tile)
    xd = to_dev(x, torch.complex64)
    y = api.apply_schur(lat, xd)
    assert per_rhs_err(to_host(y), y_ref) < 1e-5
    xs = xd.clone()
    api.richardson_smooth(lat, xs, to_dev(b, torch.complex64), 3, omega)
    assert per_rhs_err(to_host(xs), x_rich) < 1e-5
    # the same arithmetic as one right-hand side per thread
    api.set_multi_rhs_tile(lat, NRHS, 0, 4, 0)
    y0 = api.apply_schur(lat, xd)
    assert rel(to_host(y), to_host(y0)) < 1e-6


def test_tile_reaches_uneven_rhs_counts():
    # nb must divide nrhs: a tile with nb = 4 is refused for 6 right-hand sides,
    # nb = 3 is used
    c, lat12, x, b, omega, y_ref, x_rich = setup(DIMS[0])
    with pytest.raises(api.DDQError):
        api.set_multi_rhs_tile(c.lat, 6, 4, 4, 0)
    api.set_multi_rhs_tile(c.lat, 6, 3, 1, 1)
    y = api.apply_schur(c.lat, to_dev(x[:6], torch.complex64))
    assert per_rhs_err(to_host(y), y_ref[:6]) < 1e-5


def test_autotuner_picks_the_fastest_valid_tile():
    c, lat12, x, b, omega, y_ref, x_rich = setup(DIMS[1])
    best, cands = api.tune_multi_rhs(c.lat, NRHS, reps=3)
    seen = [(t["nb"], t["waves"], t["xcd_map"], t["passes"], t["lds_kb"]) for t in cands]
    assert all(tuple(t) + (1, 0) in seen for t in TILES)
    assert any(t[3] > 1 for t in seen) and any(t[4] > 0 for t in seen)
    assert all(t["ms"] > 0 for t in cands)
    assert best["ms"] == min(t["ms"] for t in cands)
    assert (best["nb"], best["waves"], best["xcd_map"], best["passes"], best["lds_kb"]) in seen
    y = api.apply_schur(c.lat, to_dev(x, torch.complex64))
    assert per_rhs_err(to_host(y), y_ref) < 1e-5
    # 7 right-hand sides: only nb = 1 tiles in one pass and the default are candidates
    best7, cands7 = api.tune_multi_rhs(c.lat, 7, reps=2)
    assert {t["nb"] for t in cands7} == {0, 1}
    assert {t["passes"] for t in cands7} == {1}
