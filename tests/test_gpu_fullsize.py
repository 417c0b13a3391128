"""Full-size checks of the HIP path at 48^3 x 96 (the large single-GPU workload)
through closed forms that hold at any size, so no oracle run is needed:

* free field (all links 1): D_S psi_e = [(4 + m0) - H(p)^2 / (4 + m0)] psi_e on even
  plane waves, and after k Richardson sweeps from zero on an eigenvector with
  eigenvalue mu, x_k = (1 - (1 - omega mu)^k) / mu * b (Alg. 4, Sect. 2.4.5);
* pure gauge U_mu(x) = Om(x) Om(x + mu)^H: D_S (Om psi_e) = Om (closed form psi_e),
  which checks link placement, daggering and the clover vanishing at full size;
* gauge covariance with random links and a non-trivial clover: the clover blocks
  and D_S rotate with a random site field Om.
The even-site coordinates are recomputed here in torch, independently of the
library's indexing.
"""
import numpy as np
import pytest
import torch

from paper_2407_08092_amd import api, synth
from planewave import momentum, schur_of_p

pytestmark = pytest.mark.gpu

DIMS = (48, 48, 48, 96)
M0 = -0.25


def even_coords(dims, dev):
    lx, ly, lz, lt = dims
    vh = lx * ly * lz * lt // 2
    i = torch.arange(vh, device=dev, dtype=torch.int64)
    xh = i % (lx // 2)
    r = i // (lx // 2)
    y = r % ly
    r = r // ly
    z = r % lz
    t = r // lz
    x = 2 * xh + ((y + z + t) % 2)
    return x, y, z, t


def plane_even(dims, p, u, dev):
    x, y, z, t = (c.to(torch.float64) for c in even_coords(dims, dev))
    # float64 coordinates: an int64 tensor times a Python float would round to float32
    ph = torch.exp(1j * (float(p[0]) * x + float(p[1]) * y + float(p[2]) * z + float(p[3]) * t))
    uu = torch.as_tensor(np.asarray(u).reshape(12), dtype=torch.complex128, device=dev)
    return uu[:, None] * ph[None, :]  # ABI layout [12, V/2]


def relerr(a, b):
    return (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()


@pytest.fixture(scope="module")
def free_lattice():
    lat = api.create_lattice(DIMS)
    U = torch.zeros(synth.field_shape(DIMS) + (4, 3, 3), dtype=torch.complex128, device="cuda")
    U[..., 0, 0] = 1
    U[..., 1, 1] = 1
    U[..., 2, 2] = 1
    api.set_gauge(lat, U)
    del U
    api.set_clover(lat, 1.2, M0)
    return lat


@pytest.mark.parametrize("k", [(1, 0, 0, 0), (0, 3, 0, 5), (7, 11, 13, 47)])
def test_free_field_schur_fullsize(free_lattice, k):
    p = momentum(DIMS, k)
    u = synth.gaussian_complex((4, 3), 3)
    psi = plane_even(DIMS, p, u, "cuda")
    expect = plane_even(DIMS, p, np.einsum("st,ta->sa", schur_of_p(p, M0), u), "cuda")
    y = api.apply_schur(free_lattice, psi)
    assert relerr(y, expect) < 1e-12
    y32 = api.apply_schur(free_lattice, api.convert_parity(free_lattice, psi, torch.complex64))
    assert relerr(api.convert_parity(free_lattice, y32, torch.complex128), expect) < 1e-5


def test_richardson_eigenvector_fullsize(free_lattice):
    p = momentum(DIMS, (2, 5, 1, 9))
    ev, W = np.linalg.eig(schur_of_p(p, M0))
    mu = ev[0]
    u = np.outer(W[:, 0], synth.gaussian_complex((3,), 4))
    b = plane_even(DIMS, p, u, "cuda")
    omega, n = 0.8 / 4.82, 20
    expect = (1 - (1 - omega * mu) ** n) / mu * b
    x = torch.zeros_like(b)
    api.richardson_smooth(free_lattice, x, b, n, omega)
    assert relerr(x, expect) < 1e-12
    x32 = api.parity_vector(free_lattice, dtype=torch.complex64).zero_()
    api.richardson_smooth(free_lattice, x32, api.convert_parity(free_lattice, b, torch.complex64), n, omega)
    assert relerr(api.convert_parity(free_lattice, x32, torch.complex128), expect) < 1e-5


def test_pure_gauge_fullsize():
    dev = "cuda"
    Om = synth.random_su3_sites(DIMS, 77, device=dev)  # [Lt, Lz, Ly, Lx, 3, 3]
    U = torch.empty(synth.field_shape(DIMS) + (4, 3, 3), dtype=torch.complex128, device=dev)
    for mu, axis in enumerate((3, 2, 1, 0)):
        U[..., mu, :, :] = Om @ torch.roll(Om, -1, dims=axis).conj().transpose(-1, -2)
    lat = api.create_lattice(DIMS)
    api.set_gauge(lat, U)
    del U
    api.set_clover(lat, 1.2, M0)
    A_ee, _ = api.get_clover(lat)
    eye6 = torch.eye(6, dtype=torch.complex128, device=dev) * (4 + M0)
    assert (A_ee - eye6).abs().max().item() < 1e-13
    del A_ee
    lx, ly, lz, lt = DIMS
    x, y, z, t = even_coords(DIMS, dev)
    lexi = x + lx * (y + ly * (z + lz * t))
    Om_e = Om.reshape(-1, 3, 3)[lexi]  # [V/2, 3, 3]
    del Om
    p = momentum(DIMS, (3, 1, 4, 1))
    u = synth.gaussian_complex((4, 3), 5)
    psi = plane_even(DIMS, p, u, dev)
    expect = plane_even(DIMS, p, np.einsum("st,ta->sa", schur_of_p(p, M0), u), dev)

    def rot(v):  # Om(x) acting on colour of an ABI-layout vector [12, V/2]
        w = v.reshape(4, 3, -1).permute(2, 0, 1)  # [V/2, 4, 3]
        return torch.einsum("nab,nsb->nsa", Om_e, w).permute(1, 2, 0).reshape(12, -1).contiguous()

    got = api.apply_schur(lat, rot(psi))
    assert relerr(got, rot(expect)) < 1e-12


def test_gauge_covariance_random_links_fullsize():
    """Random links (eps 0.5, c_sw 1.2, m0 -0.25) at the benchmarked size: under
    U'_mu(x) = Om(x) U_mu(x) Om(x + mu)^H the clover blocks rotate, A' = Om A Om^H, and
    D_S'(Om psi) = Om (D_S psi) (eq. 3 with the 6x6 clover blocks of Sect. 2.4.5), so
    the link and clover-slot indexing of every site is exercised with a non-trivial
    clover, in FP64 (1e-12) and FP32 (1e-5)."""
    dev = "cuda"
    x, y, z, t = even_coords(DIMS, dev)
    lx, ly, lz, lt = DIMS
    lexi = x + lx * (y + ly * (z + lz * t))
    del x, y, z, t
    psi = torch.from_numpy(synth.gaussian_complex((12, lexi.numel()), 303)).to(dev)
    U = synth.gauge_field(DIMS, 0.5, 301, device=dev)
    every = 4099  # sampled sites of the clover comparison

    def applies(lat, v):
        y64 = api.apply_schur(lat, v)
        y32 = api.apply_schur(lat, api.convert_parity(lat, v, torch.complex64))
        return y64, api.convert_parity(lat, y32, torch.complex128)

    lat = api.create_lattice(DIMS)
    api.set_gauge(lat, U)
    api.set_clover(lat, 1.2, M0)
    y64, y32 = applies(lat, psi)
    A_ee, _ = api.get_clover(lat)
    A_sample = A_ee[::every].clone()
    del A_ee, lat
    torch.cuda.empty_cache()
    Om = synth.random_su3_sites(DIMS, 304, device=dev)
    for mu, axis in enumerate((3, 2, 1, 0)):
        U[..., mu, :, :] = Om @ U[..., mu, :, :] @ torch.roll(Om, -1, dims=axis).conj().transpose(-1, -2)
    Om_e = Om.reshape(-1, 3, 3)[lexi]  # [V/2, 3, 3]
    del Om

    def rot(v):  # Om(x) on the colour index of an ABI-layout vector [12, V/2]
        w = v.reshape(4, 3, -1).permute(2, 0, 1)
        return torch.einsum("nab,nsb->nsa", Om_e, w).permute(1, 2, 0).reshape(12, -1).contiguous()

    lat = api.create_lattice(DIMS)
    api.set_gauge(lat, U)
    del U
    api.set_clover(lat, 1.2, M0)
    # A' = Om A Om^H on both 6x6 blocks (Om on the colour index of each spin)
    A2, _ = api.get_clover(lat)
    Os = Om_e[::every]
    O6 = torch.zeros((Os.shape[0], 1, 6, 6), dtype=torch.complex128, device=dev)
    O6[:, 0, :3, :3] = Os
    O6[:, 0, 3:, 3:] = Os
    expect_A = O6 @ A_sample @ O6.conj().transpose(-1, -2)
    assert ((A2[::every] - expect_A).abs().max() / A_sample.abs().max()).item() < 1e-13
    del A2
    y64b, y32b = applies(lat, rot(psi))
    assert relerr(y64b, rot(y64)) < 1e-12
    assert relerr(y32b, rot(y64)) < 1e-5
    assert relerr(rot(y32), y64b) < 1e-5


def test_sap_gauge_covariance_fullsize():
    """SAP(1, 2) of Alg. 1 at the benchmarked size is gauge covariant: the 4^4 blocks do
    not depend on the links, and the block operators, the residuals and the Minimal
    Residual coefficients transform with the site field Om, so SAP on
    (U' = Om U Om(+mu)^H, Om b) returns Om x.  Checks the colour-restricted residual and
    the on-chip block solves over all 20,736 blocks of a colour: FP64 blocks (whole
    18-real links in LDS; 1e-12) and FP32 blocks with 12-real and with 18-real links
    (1e-5, and 1e-5 from FP64)."""
    dev = "cuda"
    U = synth.gauge_field(DIMS, 0.5, 311, device=dev)
    b = torch.from_numpy(synth.gaussian_spinor(DIMS, 312)).to(dev)

    def sap(U_, b_):
        out = []
        for link12 in (True, False):  # FP32 blocks with 12-real, then 18-real links
            lat = api.create_lattice(DIMS)
            api.set_gauge(lat, U_, link12=link12)
            api.set_clover(lat, 1.2, M0)
            for prec in ((api.DDQ_F64, api.DDQ_F32) if link12 else (api.DDQ_F32,)):
                x = torch.zeros_like(b_)
                api.sap_smooth(lat, b_, x, 1, 2, prec=prec)
                out.append(x)
            torch.cuda.synchronize()
            api.destroy_lattice(lat)
            torch.cuda.empty_cache()
        return out

    x64, x32, x18 = sap(U, b)
    assert relerr(x32, x64) < 1e-5
    assert relerr(x18, x64) < 1e-5
    Om = synth.random_su3_sites(DIMS, 313, device=dev)
    for mu, axis in enumerate((3, 2, 1, 0)):
        U[..., mu, :, :] = Om @ U[..., mu, :, :] @ torch.roll(Om, -1, dims=axis).conj().transpose(-1, -2)

    def rot(v):  # Om(x) on the colour index of a full vector [t][z][y][x][4][3]
        return (Om.unsqueeze(-3) @ v.unsqueeze(-1)).squeeze(-1)

    y64, y32, y18 = sap(U, rot(b))
    del U
    assert relerr(y64, rot(x64)) < 1e-12
    assert relerr(y32, rot(x32)) < 1e-5
    assert relerr(y18, rot(x18)) < 1e-5
