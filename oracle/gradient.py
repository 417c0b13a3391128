"""Oracle: gradients of the Schur operator with respect to the gauge links (FP64, CPU).

Test infrastructure only: the HIP library never imports this module.

The operator of ``oracle.dirac`` is written out a second time in torch complex128 on the
CPU (same conventions: chiral basis, H with (1 - g) forward, A = (4 + m0) +
(i c_sw / 4) sum sigma F, F = (Q - Q^H) / 8, antiperiodic t) so that autograd can
differentiate it.  For a real function L of the complex links the autograd gradient is
G = dL/dRe U + i dL/dIm U, so dL = Re tr(G^H dU).  Under the left perturbation
U -> exp(i e T_a) U the derivative is F_a = dL/de = -Im tr(T_a U G^H) (``project_su3``).

Independent pin: ``fd_force`` takes central differences of L on the NumPy oracle,
L(exp(+i h T_a) U) - L(exp(-i h T_a) U), accumulated site by site.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dirac

_GAMMA = torch.from_numpy(dirac.GAMMA)
_SIGMA = torch.from_numpy(dirac.SIGMA)


def _T():
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


T_GEN = _T()  # su(3) generators lambda_a / 2


class TorchSchur:
    """D_S(U) phi_e in torch, differentiable in U and phi_e."""

    def __init__(self, lat: dirac.Lattice, c_sw: float, m0: float):
        self.lat = lat
        self.c_sw, self.m0 = float(c_sw), float(m0)
        self.even = torch.from_numpy(lat.even)
        self.odd = torch.from_numpy(lat.odd)
        lt = lat.shape[0]
        sf = torch.ones(lt, dtype=torch.float64)
        sb = torch.ones(lt, dtype=torch.float64)
        if lat.antiperiodic_t:
            sf[lt - 1] = -1
            sb[0] = -1
        self.sign_f, self.sign_b = sf, sb

    def _shift(self, f, mu, step, signed):
        g = torch.roll(f, -step, dims=3 - mu)
        if signed and mu == 3:
            s = self.sign_f if step == 1 else self.sign_b
            g = g * s.view(-1, *([1] * (f.dim() - 1)))
        return g

    def _dag(self, M):
        return M.conj().transpose(-1, -2)

    def clover(self, U):
        sh = lambda f, st: self._roll(f, st)
        A = torch.zeros(self.lat.shape + (12, 12), dtype=torch.complex128)
        for mu in range(4):
            for nu in range(mu + 1, 4):
                Um, Un = U[..., mu, :, :], U[..., nu, :, :]
                l1 = Um @ sh(Un, {mu: 1}) @ self._dag(sh(Um, {nu: 1})) @ self._dag(Un)
                l2 = Un @ self._dag(sh(Um, {mu: -1, nu: 1})) @ self._dag(sh(Un, {mu: -1})) @ sh(Um, {mu: -1})
                l3 = (self._dag(sh(Um, {mu: -1})) @ self._dag(sh(Un, {mu: -1, nu: -1}))
                      @ sh(Um, {mu: -1, nu: -1}) @ sh(Un, {nu: -1}))
                l4 = self._dag(sh(Un, {nu: -1})) @ sh(Um, {nu: -1}) @ sh(Un, {mu: 1, nu: -1}) @ self._dag(Um)
                Q = l1 + l2 + l3 + l4
                F = (Q - self._dag(Q)) / 8
                A = A + 2 * torch.einsum("st,...ab->...satb", _SIGMA[mu, nu], F).reshape(self.lat.shape + (12, 12))
        A = A * (1j * self.c_sw / 4)
        return A + (4 + self.m0) * torch.eye(12, dtype=torch.complex128)

    def _roll(self, f, steps):
        for mu, s in steps.items():
            f = torch.roll(f, -s, dims=3 - mu)
        return f

    def hop(self, U, psi):
        out = torch.zeros_like(psi)
        for mu in range(4):
            fw = torch.einsum("...ab,...sb->...sa", U[..., mu, :, :], self._shift(psi, mu, 1, True))
            out = out + fw - torch.einsum("st,...ta->...sa", _GAMMA[mu], fw)
            bw = torch.einsum("...ba,...sb->...sa", U[..., mu, :, :].conj(), psi)
            bw = self._shift(bw, mu, -1, True)
            out = out + bw + torch.einsum("st,...ta->...sa", _GAMMA[mu], bw)
        return 0.5 * out

    def _full(self, v, parity):
        V = self.lat.V
        idx = self.even if parity == 0 else self.odd
        f = torch.zeros((V, 12), dtype=torch.complex128)
        f = f.index_put((idx,), v)
        return f.reshape(self.lat.shape + (4, 3))

    def _part(self, f, parity):
        idx = self.even if parity == 0 else self.odd
        return f.reshape(self.lat.V, 12)[idx]

    def schur(self, U, x_e):
        """D_S x_e = A_ee x_e - H_eo A_oo^-1 H_oe x_e, parity vectors [V/2, 12]."""
        A = self.clover(U).reshape(self.lat.V, 12, 12)
        A_ee, A_oo = A[self.even], A[self.odd]
        h = self._part(self.hop(U, self._full(x_e, 0)), 1)
        u = torch.linalg.solve(A_oo, h.unsqueeze(-1)).squeeze(-1)
        h2 = self._part(self.hop(U, self._full(u, 1)), 0)
        return torch.einsum("nij,nj->ni", A_ee, x_e) - h2


def autograd_link_gradient(lat, U, phi_e, c_sw, m0, chi_e=None):
    """Gradient G (torch convention, dL = Re tr(G^H dU)) of
    L = |D_S phi|^2 (chi_e None) or L = Re(chi^H D_S phi); returns (G, dL/dphi) as numpy."""
    op = TorchSchur(lat, c_sw, m0)
    Ut = torch.from_numpy(np.asarray(U, dtype=np.complex128)).clone().requires_grad_(True)
    ph = torch.from_numpy(np.asarray(phi_e, dtype=np.complex128)).clone().requires_grad_(True)
    y = op.schur(Ut, ph)
    if chi_e is None:
        L = (y.conj() * y).real.sum()
    else:
        L = (torch.from_numpy(np.asarray(chi_e)).conj() * y).real.sum()
    L.backward()
    return Ut.grad.detach().numpy(), ph.grad.detach().numpy()


def project_su3(U, G):
    """F_a = -Im tr(T_a U G^H) per link: [..., 4, 8]."""
    M = np.einsum("...ab,...cb->...ac", U, np.conj(G))  # U G^H
    return -np.einsum("kba,...ab->...k", T_GEN, M).imag


def _expm_herm(X):
    w, v = np.linalg.eigh(X)
    return (v * np.exp(1j * w)[None, :]) @ v.conj().T


def fd_force(lat, U, phi_e, c_sw, m0, links, h=1e-6, chi_e=None):
    """Central finite differences of L on the NumPy oracle for the links
    [(t, z, y, x, mu), ...] and all 8 generators: array [len(links), 8]."""
    out = np.zeros((len(links), 8))
    for n, site in enumerate(links):
        for a in range(8):
            ys = []
            for sgn in (+1, -1):
                Up = np.array(U, copy=True)
                Up[site] = _expm_herm(sgn * h * T_GEN[a]) @ Up[site]
                op = dirac.WilsonClover(lat, Up, c_sw, m0)
                ys.append(op.schur(phi_e))
            if chi_e is None:
                diff = np.sum(np.abs(ys[0]) ** 2 - np.abs(ys[1]) ** 2)
            else:
                diff = np.sum((np.conj(chi_e) * (ys[0] - ys[1])).real)
            out[n, a] = diff / (2 * h)
    return out
