"""The interleaved-layout ("mrhs") FP32 stencil at the batching workload's full size:
24^3 x 48, 12 right-hand sides (eps 0.5, c_sw 1.0, m0 -0.2, gauge seed 401).

The oracle's apply at this size is slow, so the check is against the library's
one-right-hand-side FP32 stencil (itself held to the oracle at 1e-5 on the parity
lattices and checked at full size by the free-field and gauge-covariance tests): both
engines, apply and Richardson sweeps, agree with it to FP32 summation-order noise,
and repeated launches are bitwise identical.
"""
import numpy as np
import pytest
import torch

from gpu_common import rel
from paper_2407_08092_amd import api, synth

pytestmark = pytest.mark.gpu

DIMS = (24, 24, 24, 48)
N = 12
_state = {}


def _setup():
    if not _state:
        lat = api.create_lattice(DIMS)
        api.set_gauge(lat, synth.gauge_field(DIMS, 0.5, 401, device="cuda"))
        api.set_clover(lat, 1.0, -0.2)
        g = torch.Generator(device="cuda").manual_seed(1401)
        x = torch.randn((N,) + tuple(api.parity_vector(lat, None, torch.complex64).shape),
                        dtype=torch.complex64, device="cuda", generator=g)
        _state.update(lat=lat, x=x)
    return _state["lat"], _state["x"]


def per_rhs(a, b):
    return max(rel(a[r].cpu().numpy(), b[r].cpu().numpy()) for r in range(b.shape[0]))


LAUNCH = [(1, 0, 0, 0), (2, 0, 6, 0), (2, 64, 24, 0), (1, 0, 0, 1), (2, 0, 2, 1)]


@pytest.mark.parametrize("launch", LAUNCH, ids=["slab", "twalk6", "twalk24_lds64", "slab_staged", "twalk2_staged"])
@pytest.mark.parametrize("engine", [api.DDQ_ENGINE_VALU, api.DDQ_ENGINE_MFMA], ids=["valu", "mfma"])
def test_fullsize_apply_matches_single_rhs_kernel(engine, launch):
    lat, x = _setup()
    api.mrhs_set_launch(lat, *launch)
    ref = torch.stack([api.apply_schur(lat, x[r].contiguous()) for r in range(N)])
    xm = api.mrhs_pack(lat, x)
    y1 = api.mrhs_apply_schur(lat, xm, engine=engine)
    y2 = api.mrhs_apply_schur(lat, xm, engine=engine)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    got = api.mrhs_unpack(lat, y1)
    api.mrhs_set_launch(lat, 1, 0)
    assert per_rhs(got, ref) < 2e-6


@pytest.mark.parametrize("launch", LAUNCH, ids=["slab", "twalk6", "twalk24_lds64", "slab_staged", "twalk2_staged"])
@pytest.mark.parametrize("engine", [api.DDQ_ENGINE_VALU, api.DDQ_ENGINE_MFMA], ids=["valu", "mfma"])
def test_fullsize_sweeps_match_single_rhs_kernel(engine, launch):
    lat, x = _setup()
    api.mrhs_set_launch(lat, *launch)
    b = x.flip(0).contiguous()
    omega = 0.15
    ref = x.clone()
    for r in range(N):
        api.richardson_smooth(lat, ref[r], b[r].contiguous(), 3, omega)
    xm = api.mrhs_pack(lat, x)
    api.mrhs_richardson_smooth(lat, xm, api.mrhs_pack(lat, b), 3, omega, engine=engine)
    torch.cuda.synchronize()
    api.mrhs_set_launch(lat, 1, 0)
    assert per_rhs(api.mrhs_unpack(lat, xm), ref) < 5e-6
