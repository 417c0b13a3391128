"""The C-ABI library loads, exports every symbol include/ddq.h declares, and
rejects bad arguments on the host before touching the GPU (CPU only)."""
import ctypes as C
import os
import re

import pytest

from paper_2407_08092_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ddq_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ddq_create_lattice", "ddq_set_gauge", "ddq_set_clover", "ddq_apply_schur",
                     "ddq_richardson_smooth", "ddq_oe_gmres_solve", "ddq_oe_prepare", "ddq_oe_reconstruct"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    assert set(declared_functions()) == set(_lib._SIGNATURES)


@pytest.mark.parametrize("dims", [(4, 5, 4, 4), (0, 4, 4, 4), (4, 4, 4, 1), (4, 4, -2, 4)])
def test_bad_extents_rejected_on_host(dims):
    L = _lib.lib()
    h = C.c_void_p()
    arr = (C.c_int * 4)(*dims)
    st = L.ddq_create_lattice(arr, 1, None, C.byref(h))
    assert st == -1
    assert h.value is None
    assert b"even" in L.ddq_last_error()


def test_null_arguments_rejected_on_host():
    L = _lib.lib()
    assert L.ddq_create_lattice(None, 1, None, None) == -1
    assert L.ddq_apply_schur(None, 0, 1, None, None, 0) == -1
    assert L.ddq_destroy_lattice(None) == 0
    assert L.ddq_set_clover(None, 1.0, 0.0) == -1


def test_too_large_volume_rejected():
    L = _lib.lib()
    h = C.c_void_p()
    arr = (C.c_int * 4)(2048, 2048, 2048, 2)
    assert L.ddq_create_lattice(arr, 1, None, C.byref(h)) == -1


def test_no_cpu_fallback_in_product_package():
    # the product package never imports the oracle
    pkg = os.path.join(ROOT, "paper_2407_08092_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f


def test_coarse_sizes_and_bad_arguments_on_host():
    L = _lib.lib()
    cd = (C.c_int * 4)(3, 4, 3, 5)
    nb = C.c_int64()
    # N_v = 24: 2N_v = 48 -> 3 row tiles x 6 pairs of k-slices x 1 KB per (site, block)
    assert L.ddq_coarse_packed_bytes(cd, 24, 1, C.byref(nb)) == 0 and nb.value == 180 * 9 * 3 * 6 * 1024
    # N_v = 20: 2N_v = 40 padded to 48 rows and 40 columns (5 pairs of 4-wide k-slices)
    assert L.ddq_coarse_packed_bytes(cd, 20, 1, C.byref(nb)) == 0 and nb.value == 180 * 9 * 3 * 5 * 1024
    assert L.ddq_coarse_packed_bytes(cd, 0, 1, C.byref(nb)) == -1
    assert L.ddq_coarse_packed_bytes(cd, 33, 1, C.byref(nb)) == -1
    assert L.ddq_coarse_packed_bytes((C.c_int * 4)(3, 0, 3, 3), 8, 1, C.byref(nb)) == -1
    assert L.ddq_coarse_packed_bytes((C.c_int * 4)(512, 512, 512, 1), 8, 1, C.byref(nb)) == -1
    # FP16 / BF16 storage: half the bytes
    assert L.ddq_coarse_packed_bytes(cd, 24, 2, C.byref(nb)) == 0 and nb.value == 180 * 9 * 3 * 6 * 512
    assert L.ddq_coarse_packed_bytes(cd, 24, 3, C.byref(nb)) == 0 and nb.value == 180 * 9 * 3 * 6 * 512
    assert L.ddq_coarse_packed_bytes(cd, 24, 0, C.byref(nb)) == -1  # no FP64 storage
    fake = C.c_void_p(1 << 20)  # never dereferenced: every call below fails its host checks
    y = C.c_void_p((1 << 20) + 4096)
    assert L.ddq_coarse_apply(cd, 8, 1, 0, fake, fake, y, 0, 0, None) == -1
    assert L.ddq_coarse_apply(cd, 8, 1, 16, fake, fake, y, 5, 0, None) == -1
    assert L.ddq_coarse_apply(cd, 8, 1, 16, fake, fake, y, 0, 3, None) == -1  # no such product form
    assert L.ddq_coarse_apply(cd, 8, 0, 16, fake, fake, y, 0, 0, None) == -1  # no such storage
    assert L.ddq_coarse_apply(cd, 8, 1, 16, fake, fake, fake, 0, 0, None) == -1  # y == v
    # y starting inside v (180 sites x 16 rows x 16 right-hand sides x 8 B = 368,640 B)
    assert L.ddq_coarse_apply(cd, 8, 1, 16, fake, fake, C.c_void_p((1 << 20) + 368640 - 8), 0, 0, None) == -1
    assert b"overlap" in L.ddq_last_error()
    assert L.ddq_coarse_apply(cd, 8, 1, 16, C.c_void_p((1 << 20) + 8), fake, y, 0, 0,
                              None) == -1  # packed not 16-byte aligned
    assert L.ddq_coarse_pack_blocks(cd, 8, 1, 2, fake, fake, None) == -1  # 16-bit input blocks are not taken
    assert L.ddq_coarse_pack_blocks(cd, 8, 1, 1, fake, C.c_void_p((1 << 20) + 1024), None) == -1  # overlap
    assert b"overlap" in L.ddq_last_error()
    assert L.ddq_coarse_apply(cd, 8, 1, 16, None, fake, fake, 0, 0, None) == -1


def test_lattice_beyond_the_descriptor_limit_refused():
    # 56^3 x 112: V/2 = 9,834,496 sites, the FP64 clover field of a parity would need
    # 5.7 GB in one 32-bit buffer descriptor
    L = _lib.lib()
    h = C.c_void_p()
    assert L.ddq_create_lattice((C.c_int * 4)(56, 56, 56, 112), 1, None, C.byref(h)) == -1
    assert h.value is None
    assert b"4 GiB" in L.ddq_last_error()


def test_reservation_and_cache_calls_reject_null_on_host():
    L = _lib.lib()
    assert L.ddq_reserve(None, 1, 0, 0) == -1
    assert L.ddq_autotune(None, b"/tmp/x.json") == -1
    assert L.ddq_batch_reserve(None, 10, 0) == -1
    assert L.ddq_oe_gmres_solve(None, 1, None, None, None, None) == -1


def test_coarse_pack_of_many_sites_is_accepted_on_host():
    # 2^22 coarse sites at N_v = 32: the pack has 2^22 * 9 * 8 * 4 * 64 > 2^32 lane elements,
    # which the grid-stride pack kernel covers; only the site bound (2^25) limits the size
    L = _lib.lib()
    nb = C.c_int64()
    assert L.ddq_coarse_packed_bytes((C.c_int * 4)(64, 64, 32, 32), 32, 1, C.byref(nb)) == 0
    assert nb.value == (1 << 22) * 9 * 8 * 4 * 64 * 16
