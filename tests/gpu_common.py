"""Shared set-up for the GPU parity tests: the same seeded inputs go to the oracle
and, through the C ABI, to the HIP library.  Layout changes between the oracle's
[V/2, 12] parity vectors and the ABI's [12, V/2] are done here, in test code."""
import numpy as np
import torch

from oracle.dirac import Lattice, WilsonClover
from paper_2407_08092_amd import api, synth


def to_dev(v_np, dtype=torch.complex128):
    """oracle parity vector [V/2, 12] (or [n, V/2, 12]) -> ABI layout on the GPU:
    complex128 [.., 12, V/2]; complex64 [.., 6, V/2, 2] (rows 2k, 2k+1 paired)."""
    a = np.swapaxes(v_np, -1, -2)  # [.., 12, Vh]
    if dtype == torch.complex64:
        vh = a.shape[-1]
        a = np.swapaxes(a.reshape(a.shape[:-2] + (6, 2, vh)), -1, -2)  # [.., 6, Vh, 2]
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to(device="cuda", dtype=dtype).contiguous()


def to_dev16(v_np, dtype):
    """oracle parity vector [.., V/2, 12] -> 16-bit ABI layout [.., 3, V/2, 4, 2]
    (float16 / bfloat16), rounded on the host as the library narrows: FP16 in one
    rounding from FP64 (numpy's conversion is correctly rounded), BF16 through FP32
    (two roundings to nearest even)."""
    a = np.swapaxes(v_np, -1, -2)  # [.., 12, Vh]
    vh = a.shape[-1]
    a = np.swapaxes(a.reshape(a.shape[:-2] + (3, 4, vh)), -1, -2)  # [.., 3, Vh, 4]
    r = np.ascontiguousarray(np.stack([a.real, a.imag], axis=-1))  # [.., 3, Vh, 4, 2] float64
    if dtype == torch.float16:
        return torch.from_numpy(r.astype(np.float16)).contiguous().cuda()
    return torch.from_numpy(r).to(torch.float32).to(dtype).contiguous().cuda()


def to_host(t):
    """ABI parity vector -> oracle layout [.., V/2, 12] (complex128 numpy)."""
    if t.dtype in (torch.float16, torch.bfloat16):
        a = torch.view_as_complex(t.detach().cpu().to(torch.float64).contiguous()).numpy()  # [.., 3, Vh, 4]
        a = np.swapaxes(a, -1, -2)  # [.., 3, 4, Vh]
        a = a.reshape(a.shape[:-3] + (12, a.shape[-1]))
        return np.ascontiguousarray(np.swapaxes(a, -1, -2))
    a = t.detach().cpu().numpy().astype(np.complex128)
    if t.dtype == torch.complex64:
        a = np.swapaxes(a, -1, -2)  # [.., 6, 2, Vh]
        a = a.reshape(a.shape[:-3] + (12, a.shape[-1]))
    return np.ascontiguousarray(np.swapaxes(a, -1, -2))


class Case:
    """One lattice with its oracle operator and its GPU twin."""

    def __init__(self, dims, eps, c_sw, m0, seed, antiperiodic=True):
        self.dims = tuple(dims)
        self.olat = Lattice(dims, antiperiodic)
        self.U = synth.gauge_field(dims, eps, seed)
        self.op = WilsonClover(self.olat, self.U, c_sw, m0)
        self.lat = api.create_lattice(dims, antiperiodic)
        api.set_gauge(self.lat, torch.from_numpy(self.U).cuda())
        api.set_clover(self.lat, c_sw, m0)

    def vec(self, seed, n=None):
        shape = (self.olat.Vh, 12) if n is None else (n, self.olat.Vh, 12)
        return synth.gaussian_complex(shape, seed)

    def full(self, seed):
        return synth.gaussian_spinor(self.dims, seed)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
