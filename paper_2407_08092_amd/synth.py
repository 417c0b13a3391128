"""Seeded synthetic inputs for the odd-even Wilson-clover path.

This module draws random numbers and turns them into inputs: SU(3) gauge
links, Gaussian complex spinor fields and random SU(3) site matrices.  It holds
no part of the Dirac operator, the Schur complement or the solvers, so that the
oracle and the HIP library can both be fed from it without sharing any of the
method's arithmetic.

Canonical layouts (shared with the C ABI):
  gauge links  U[t][z][y][x][mu][a][b], complex128, mu = 0..3 = x, y, z, t
  full spinor  psi[t][z][y][x][spin][colour], complex128

Gauge links follow U = exp(i eps sum_k a_k T_k), a_k ~ N(0, 1), T_k = lambda_k/2
(Gell-Mann matrices), drawn in one numpy ``default_rng(seed)`` stream of shape
(Lt, Lz, Ly, Lx, 4, 8).  The paper's gauge configuration is not available; these
fields stand in for it at the paper's lattice shapes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gellmann_T",
    "su3_coefficients",
    "gauge_field",
    "random_su3_sites",
    "gaussian_spinor",
    "gaussian_complex",
    "field_shape",
]


def field_shape(dims):
    """Array shape (Lt, Lz, Ly, Lx) of a lattice with extents dims = (Lx, Ly, Lz, Lt)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx)


def gellmann_T() -> np.ndarray:
    """The eight su(3) generators T_k = lambda_k / 2, normalised tr(T_a T_b) = delta_ab / 2."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam / 2


def su3_coefficients(dims, seed: int) -> np.ndarray:
    """The N(0,1) coefficients a_k of every link, shape (Lt, Lz, Ly, Lx, 4, 8)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(field_shape(dims) + (4, 8))


def _expi(a: np.ndarray, eps: float, device=None, chunk: int = 1 << 22):
    """exp(i eps sum_k a_k T_k) for a[..., 8]; returns complex128 [..., 3, 3].

    Uses torch.linalg.matrix_exp so that large fields can be built on a GPU;
    for device None the result is a numpy array computed on the CPU.
    """
    import torch

    T = torch.from_numpy(gellmann_T())
    lead = a.shape[:-1]
    flat = a.reshape(-1, 8)
    dev = torch.device("cpu") if device is None else torch.device(device)
    out = torch.empty((flat.shape[0], 3, 3), dtype=torch.complex128, device=dev)
    Td = T.to(dev)
    for s in range(0, flat.shape[0], chunk):
        ak = torch.from_numpy(np.ascontiguousarray(flat[s:s + chunk])).to(dev)
        X = torch.einsum("nk,kab->nab", ak.to(torch.complex128), Td) * eps
        out[s:s + chunk] = torch.linalg.matrix_exp(1j * X)
    out = out.reshape(lead + (3, 3))
    if device is None:
        return out.numpy()
    return out


def gauge_field(dims, eps: float, seed: int, device=None):
    """Seeded SU(3) gauge field, canonical layout U[t][z][y][x][mu][a][b].

    device None: numpy complex128 on the host; otherwise a torch complex128
    tensor on that device (the random draws are identical either way; only the
    rounding of the exponential may differ).
    """
    return _expi(su3_coefficients(dims, seed), eps, device=device)


def random_su3_sites(dims, seed: int, eps: float = 3.0, device=None):
    """One random SU(3) matrix per site, shape (Lt, Lz, Ly, Lx, 3, 3) (numpy, or a
    torch tensor on `device`)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(field_shape(dims) + (8,))
    return _expi(a, eps, device=device)


def gaussian_complex(shape, seed: int) -> np.ndarray:
    """Complex128 array with Re and Im each iid N(0, 1), from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(tuple(shape) + (2,))
    return g[..., 0] + 1j * g[..., 1]


def gaussian_spinor(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Gaussian complex full spinor field [t][z][y][x][4][3] (or [nrhs][...])."""
    shape = field_shape(dims) + (4, 3)
    if nrhs is not None:
        shape = (nrhs,) + shape
    return gaussian_complex(shape, seed)
