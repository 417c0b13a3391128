"""ddq_apply_schur_noalloc: the Schur apply of eq. 3 with its u_o work space in the
library's fixed device array instead of the lattice's reservation.

Checked through the C ABI against ddq_apply_schur (the same kernels, so the outputs
must agree bit for bit) and against the FP64 oracle at the parity bars (FP64 1e-12,
FP32 1e-5, 16-bit 10u); several calls in a row, each later one smaller than the one
before, so a call that read what an earlier call left in the shared array would show;
requests beyond the array's 64 MiB are refused before any launch.
"""
import ctypes

import numpy as np
import pytest
import torch

from gpu_common import Case, rel, to_dev, to_dev16, to_host
from paper_2407_08092_amd import api
from paper_2407_08092_amd._lib import lib

pytestmark = pytest.mark.gpu

LIMIT = 64 << 20


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _noalloc(c, x, dagger=False):
    y = torch.empty_like(x)
    y.view(torch.uint8).fill_(0xFF)  # NaN in every precision: the call must overwrite all of y
    api.apply_schur_noalloc(c.lat, x, y, dagger)
    torch.cuda.synchronize()
    return y


def _ref(c, x, dagger=False):
    y = api.apply_schur(c.lat, x, dagger=dagger)
    torch.cuda.synchronize()
    return y


def test_noalloc_matches_apply_schur_twice_shrinking():
    big = Case((8, 8, 8, 16), 0.5, 1.2, -0.25, 301)
    small = Case((4, 6, 8, 10), 0.3, 1.0, -0.1, 101)

    # call 1: three FP64 right-hand sides on 8^3 x 16 (u_o: 2.4 MiB of the array)
    x1 = big.vec(21, 3)
    d1 = to_dev(x1)
    y1 = _noalloc(big, d1)
    assert torch.equal(y1, _ref(big, d1))
    for r in range(3):
        assert rel(to_host(y1[r]), big.op.schur(x1[r])) < 1e-12

    # call 2: one FP32 right-hand side on the smaller 4x6x8x10 lattice
    x2 = small.vec(22)
    d2 = to_dev(x2, torch.complex64)
    y2 = _noalloc(small, d2)
    assert torch.equal(y2, _ref(small, d2))
    assert rel(to_host(y2), small.op.schur(x2)) < 1e-5

    # call 3: the daggered FP64 apply, one right-hand side of 4x6x8x10
    d3 = to_dev(x2)
    y3 = _noalloc(small, d3, dagger=True)
    assert torch.equal(y3, _ref(small, d3, dagger=True))
    assert rel(to_host(y3), small.op.schur_adjoint(x2)) < 1e-12


def test_noalloc_16bit():
    c = Case((4, 6, 8, 10), 0.3, 1.0, -0.1, 101)
    api.set_gauge(c.lat, torch.from_numpy(c.U).cuda(), store=(api.DDQ_F64, api.DDQ_F32, api.DDQ_F16, api.DDQ_BF16))
    api.set_clover(c.lat, 1.0, -0.1)
    x = c.vec(23, 2)
    for dt, u in ((torch.float16, 2.0 ** -11), (torch.bfloat16, 2.0 ** -8)):
        d = to_dev16(x, dt)
        y = _noalloc(c, d)
        assert torch.equal(y, _ref(c, d))
        for r in range(2):
            assert rel(to_host(y[r]), c.op.schur(x[r])) < 10 * u


def test_noalloc_refuses_beyond_limit():
    c = Case((8, 8, 8, 16), 0.3, 1.0, -0.1, 101)
    vh = c.olat.Vh
    n = LIMIT // (vh * 12 * 16) + 1  # FP64: one right-hand side more than fits
    x = to_dev(c.vec(24))
    y = torch.empty_like(x)
    st = lib().ddq_apply_schur_noalloc(c.lat.handle, 0, int(n), _ptr(x), _ptr(y), 0)
    assert st == -1  # DDQ_ERR_ARG, refused before any launch
    assert b"fixed work space" in lib().ddq_last_error()
    # the largest count that fits is accepted (checked without launching: nrhs - 1 of
    # them would need vectors this test does not allocate, so only the limit is probed)
    assert (n - 1) * vh * 12 * 16 <= LIMIT
