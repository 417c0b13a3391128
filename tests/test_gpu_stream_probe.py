"""The stencil streaming-ceiling probe (ddq_stencil_stream) through the C ABI.

It is a measurement aid with no oracle value: what is checked is that it visits
every site once in the stencil's workgroup order (each output site changes when the
first element row of its own input changes), that it is deterministic, and that it
rejects what it does not take.  Lattices: 4x6x8x10 and 6x6x6x10 (V/2 not a multiple
of the 256-site workgroup; t-slices not a multiple of 8 groups of 64 sites) and
24^3 x 48.
"""
import pytest
import torch

from paper_2407_08092_amd import api, synth

pytestmark = pytest.mark.gpu

DIMS = [(4, 6, 8, 10), (6, 6, 6, 10), (24, 24, 24, 48)]


@pytest.fixture(scope="module", params=DIMS, ids=lambda d: "x".join(map(str, d)))
def lat(request):
    dims = request.param
    lat = api.create_lattice(dims)
    api.set_gauge(lat, synth.gauge_field(dims, 0.5, 501, device="cuda"))
    api.set_clover(lat, 1.0, -0.2)
    return lat


def bits(t):
    r = torch.view_as_real(t)
    return r.view(torch.int64 if r.dtype == torch.float64 else torch.int32)


def per_site_bits(t):
    """[rows, V/2, words] integer view of a parity vector's element rows"""
    b = bits(t)
    if t.dtype == torch.complex128:  # [12, Vh, 2]
        return b
    return b.reshape(6, t.shape[1], 4)  # [6, Vh, 2, 2] -> 4 words per element


@pytest.mark.parametrize("kernel", [0, 1, 2])
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["f32", "f64"])
def test_visits_every_site_once_and_repeats(lat, kernel, dtype):
    g = torch.Generator(device="cuda").manual_seed(11 + kernel)
    shp = (12, lat.Vh) if dtype == torch.complex128 else (6, lat.Vh, 2)
    vin, x, b = (torch.randn(shp, dtype=dtype, device="cuda", generator=g) for _ in range(3))
    out1, out2, out3 = (torch.empty_like(vin) for _ in range(3))
    api.stencil_stream(lat, kernel, vin, out1, x, b)
    api.stencil_stream(lat, kernel, vin, out2, x, b)
    vin2 = vin.clone()
    vin2[0] += 1.0  # the first element row of every site's input
    api.stencil_stream(lat, kernel, vin2, out3, x, b)
    torch.cuda.synchronize()
    assert torch.equal(bits(out1), bits(out2))
    changed = (per_site_bits(out1) != per_site_bits(out3)).any(dim=-1)  # [rows, Vh]
    assert bool(changed.all()), int((~changed).sum())


def test_twelve_real_links_and_errors():
    dims = (6, 6, 6, 10)
    lat = api.create_lattice(dims)
    api.set_gauge(lat, synth.gauge_field(dims, 0.5, 502, device="cuda"), link12=True)
    api.set_clover(lat, 1.0, -0.2)
    v = torch.randn((6, lat.Vh, 2), dtype=torch.complex64, device="cuda")
    o1, o2 = torch.empty_like(v), torch.empty_like(v)
    api.stencil_stream(lat, 2, v, o1, v.clone(), v.clone())
    api.stencil_stream(lat, 2, v, o2, v.clone(), v.clone())
    torch.cuda.synchronize()
    assert torch.equal(bits(o1), bits(o2))
    with pytest.raises(api.DDQError):
        api.stencil_stream(lat, 3, v, o1, v, v)  # no such kernel
    with pytest.raises(api.DDQError):
        api.stencil_stream(lat, 1, v, o1)  # B reads x
    with pytest.raises(ValueError):
        api.stencil_stream(lat, 0, v.unsqueeze(0), o1.unsqueeze(0))  # one right-hand side
    h = torch.zeros((3, lat.Vh, 4, 2), dtype=torch.float16, device="cuda")
    with pytest.raises(api.DDQError):
        api.stencil_stream(lat, 0, h, torch.empty_like(h))  # FP32 / FP64 only
