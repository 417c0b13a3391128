"""Oracle: Wilson-clover Dirac operator, odd-even split and Schur complement (FP64, CPU).

Test infrastructure only (see the package docstring): the HIP library never
imports this module.

The paper (Sect. 2.3) names the operator -- Wilson-Dirac with a clover term,
twelve degrees of freedom per site, nine 12x12 blocks per block row -- but
does not write it down.  This module fixes the textbook operator in the
following conventions:

* Lattice extents dims = (Lx, Ly, Lz, Lt), all even; arrays are shaped
  (Lt, Lz, Ly, Lx, ...), directions mu = 0..3 = x, y, z, t.  Periodic in x, y,
  z; antiperiodic in t (a hop across the t boundary carries a factor -1).
* Chiral gamma basis: gamma_k = [[0, -i s_k], [i s_k, 0]] for k = 1, 2, 3 and
  gamma_4 = [[0, 1], [1, 0]], so gamma_5 = diag(1, 1, -1, -1).  This is the
  basis in which D_ee and D_oo consist of 6x6 blocks (Sect. 2.4.5).
* D psi(x) = A(x) psi(x) - H psi(x), with the hopping term
      H psi(x) = 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                              + (1 + gamma_mu) U_mu(x - mu)^H psi(x - mu) ]
  and the site term
      A(x) = (4 + m0) 1 + (i c_sw / 4) sum_{mu != nu} sigma_munu (x) F_munu(x),
      sigma_munu = (i/2)[gamma_mu, gamma_nu],  F_munu = (Q_munu - Q_munu^H) / 8,
  Q_munu(x) being the sum of the four counter-clockwise plaquette leaves in the
  mu-nu plane that start at x.  The clover uses the links without the boundary
  sign (it cancels in every closed loop).
* Odd-even split (Sect. 2.4.5): a site is even when x + y + z + t is even; even
  sites come first (eq. 1).  Within a parity the sites are in increasing
  lexicographic order n = x + Lx (y + Ly (z + Lz t)).  A parity vector is an
  array [V/2, 12] with index 3 * spin + colour.
* With D_ee = A_ee, D_oo = A_oo, D_eo = -H_eo, D_oe = -H_oe the Schur
  complement of eq. 3 is D_S = A_ee - H_eo A_oo^-1 H_oe.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# ---------------------------------------------------------------------------
# Spin algebra
# ---------------------------------------------------------------------------
_S1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_S2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_S3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)
PAULI = np.array([_S1, _S2, _S3])


def _chiral_gamma(s):
    return np.block([[_Z2, -1j * s], [1j * s, _Z2]])


GAMMA = np.array([_chiral_gamma(_S1), _chiral_gamma(_S2), _chiral_gamma(_S3),
                  np.block([[_Z2, _I2], [_I2, _Z2]])])
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
SIGMA = np.array([[0.5j * (GAMMA[m] @ GAMMA[n] - GAMMA[n] @ GAMMA[m]) for n in range(4)]
                  for m in range(4)])
I4 = np.eye(4, dtype=np.complex128)

# array axis of direction mu in a field shaped (Lt, Lz, Ly, Lx, ...)
_AXIS = (3, 2, 1, 0)


def dag(M):
    """Conjugate transpose over the last two axes."""
    return np.conj(np.swapaxes(M, -1, -2))


# ---------------------------------------------------------------------------
# Lattice geometry
# ---------------------------------------------------------------------------
class Lattice:
    """Geometry of an Lx x Ly x Lz x Lt lattice with its odd-even split (Sect. 2.4.5)."""

    def __init__(self, dims, antiperiodic_t: bool = True):
        dims = tuple(int(d) for d in dims)
        if len(dims) != 4 or any(d < 2 or d % 2 for d in dims):
            raise ValueError(f"extents must be four even numbers >= 2, got {dims}")
        self.dims = dims
        self.shape = (dims[3], dims[2], dims[1], dims[0])
        self.V = int(np.prod(dims))
        self.Vh = self.V // 2
        self.antiperiodic_t = bool(antiperiodic_t)
        t, z, y, x = np.indices(self.shape)
        self.coords = (x, y, z, t)
        self.parity = (x + y + z + t) % 2
        flat = self.parity.ravel()
        # even sites first, each parity in increasing lexicographic order (eq. 1)
        self.even = np.flatnonzero(flat == 0)
        self.odd = np.flatnonzero(flat == 1)

    # f(x + mu) and f(x - mu) for a field (boundary sign applied when signed)
    def fwd(self, f, mu, signed=True):
        g = np.roll(f, -1, axis=_AXIS[mu])
        if signed and mu == 3 and self.antiperiodic_t:
            g = g.copy()
            g[self.shape[0] - 1] *= -1
        return g

    def bwd(self, f, mu, signed=True):
        g = np.roll(f, 1, axis=_AXIS[mu])
        if signed and mu == 3 and self.antiperiodic_t:
            g = g.copy()
            g[0] *= -1
        return g

    def shift(self, f, steps):
        """Periodic shift, f(x + sum_mu steps[mu] mu); used for gauge loops."""
        for mu, s in steps.items():
            if s:
                f = np.roll(f, -s, axis=_AXIS[mu])
        return f

    # parity vectors <-> full fields
    def to_parity(self, psi, parity):
        sites = self.even if parity == 0 else self.odd
        return psi.reshape(self.V, 12)[sites].copy()

    def from_parity(self, v, parity):
        full = np.zeros((self.V, 12), dtype=np.complex128)
        sites = self.even if parity == 0 else self.odd
        full[sites] = v
        return full.reshape(self.shape + (4, 3))

    def neighbour(self, n, mu, step):
        """Lexicographic index of site n shifted by step*mu (periodic) and the
        boundary sign of that hop."""
        lx, ly, lz, lt = self.dims
        c = [n % lx, (n // lx) % ly, (n // (lx * ly)) % lz, n // (lx * ly * lz)]
        c[mu] += step
        sign = 1.0
        if mu == 3 and self.antiperiodic_t and (c[3] < 0 or c[3] >= lt):
            sign = -1.0
        c[mu] %= self.dims[mu]
        return c[0] + lx * (c[1] + ly * (c[2] + lz * c[3])), sign


# ---------------------------------------------------------------------------
# Gauge loops and the clover term
# ---------------------------------------------------------------------------
def field_strength(lat: Lattice, U):
    """F_munu = (Q_munu - Q_munu^H) / 8 for mu < nu, as a dict {(mu, nu): [...,3,3]}."""
    F = {}
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Um, Un = U[..., mu, :, :], U[..., nu, :, :]
            S = lat.shift
            leaf1 = Um @ S(Un, {mu: 1}) @ dag(S(Um, {nu: 1})) @ dag(Un)
            leaf2 = Un @ dag(S(Um, {mu: -1, nu: 1})) @ dag(S(Un, {mu: -1})) @ S(Um, {mu: -1})
            leaf3 = (dag(S(Um, {mu: -1})) @ dag(S(Un, {mu: -1, nu: -1}))
                     @ S(Um, {mu: -1, nu: -1}) @ S(Un, {nu: -1}))
            leaf4 = dag(S(Un, {nu: -1})) @ S(Um, {nu: -1}) @ S(Un, {mu: 1, nu: -1}) @ dag(Um)
            Q = leaf1 + leaf2 + leaf3 + leaf4
            F[(mu, nu)] = (Q - dag(Q)) / 8.0
    return F


def clover_matrix(lat: Lattice, U, c_sw: float, m0: float):
    """A(x) = (4 + m0) 1 + (i c_sw / 4) sum_{mu != nu} sigma_munu (x) F_munu(x); [..., 12, 12].

    The sum over ordered pairs is twice the sum over mu < nu because both
    sigma_munu and F_munu are antisymmetric in (mu, nu).
    """
    F = field_strength(lat, U)
    A = np.zeros(lat.shape + (12, 12), dtype=np.complex128)
    for (mu, nu), Fmn in F.items():
        # kron(sigma, F) with index 3 * spin + colour
        A += 2.0 * np.einsum("st,...ab->...satb", SIGMA[mu, nu], Fmn).reshape(lat.shape + (12, 12))
    A *= 1j * c_sw / 4.0
    A += (4.0 + m0) * np.eye(12)
    return A


# ---------------------------------------------------------------------------
# The operator
# ---------------------------------------------------------------------------
def _colour(Um, psi):
    """U psi on every spin: out[..., s, a] = sum_b U[..., a, b] psi[..., s, b]."""
    return np.einsum("...ab,...sb->...sa", Um, psi)


def _spin(G, psi):
    """G psi on the spin index: out[..., s, a] = sum_t G[s, t] psi[..., t, a]."""
    return np.einsum("st,...ta->...sa", G, psi)


def hopping(lat: Lattice, U, psi, adjoint: bool = False):
    """H psi, or the adjoint H^H psi when adjoint is set.

    H^H is written out as its own stencil: the adjoint of the block
    (1 -+ gamma_mu) U at (x, x +- mu) is (1 -+ gamma_mu) U^H at (x +- mu, x), so
    the forward hop carries (1 + gamma_mu) U_mu(x) and the backward hop
    (1 - gamma_mu) U_mu(x - mu)^H.
    """
    sf, sb = (1.0, -1.0) if adjoint else (-1.0, 1.0)
    out = np.zeros_like(psi)
    for mu in range(4):
        fw = _colour(U[..., mu, :, :], lat.fwd(psi, mu))
        out += fw + sf * _spin(GAMMA[mu], fw)
        bw = lat.bwd(_colour(dag(U[..., mu, :, :]), psi), mu)
        out += bw + sb * _spin(GAMMA[mu], bw)
    return 0.5 * out


class WilsonClover:
    """Wilson-clover operator on a lattice, with the odd-even pieces of eqs. 1-3."""

    def __init__(self, lat: Lattice, U, c_sw: float, m0: float):
        self.lat = lat
        self.U = np.asarray(U, dtype=np.complex128)
        assert self.U.shape == lat.shape + (4, 3, 3)
        self.c_sw, self.m0 = float(c_sw), float(m0)
        self.A = clover_matrix(lat, self.U, c_sw, m0)
        Af = self.A.reshape(lat.V, 12, 12)
        self.A_ee = Af[lat.even]
        self.A_oo = Af[lat.odd]
        # D_oo^-1: a plain 12x12 inverse per odd site (Sect. 2.4.5: storing it is cheap)
        self.A_oo_inv = np.linalg.inv(self.A_oo)

    # full operator -------------------------------------------------------
    def site_term(self, psi):
        return np.einsum("...ij,...j->...i", self.A, psi.reshape(self.lat.shape + (12,))
                         ).reshape(psi.shape)

    def H(self, psi, adjoint=False):
        return hopping(self.lat, self.U, psi, adjoint)

    def D(self, psi):
        """D psi for a full field [..., 4, 3]."""
        return self.site_term(psi) - self.H(psi)

    # blocks of eq. 1 as maps between parity vectors ----------------------
    def D_eo(self, v_o):
        return -self.lat.to_parity(self.H(self.lat.from_parity(v_o, 1)), 0)

    def D_oe(self, v_e):
        return -self.lat.to_parity(self.H(self.lat.from_parity(v_e, 0)), 1)

    def D_ee(self, v_e):
        return np.einsum("nij,nj->ni", self.A_ee, v_e)

    def D_oo_inv(self, v_o):
        return np.einsum("nij,nj->ni", self.A_oo_inv, v_o)

    # Schur complement, eq. 3 ----------------------------------------------
    def schur(self, v_e):
        """D_S v_e = D_ee v_e - D_eo D_oo^-1 D_oe v_e."""
        return self.D_ee(v_e) - self.D_eo(self.D_oo_inv(self.D_oe(v_e)))

    def schur_adjoint(self, v_e):
        """D_S^H v_e, built from the adjoint stencil and conjugate-transposed
        site blocks (not from gamma_5):
        D_S^H = D_ee^H - (D^H)_eo (D_oo^-1)^H (D^H)_oe with (D^H)_eo = -(H^H)_eo."""
        lat = self.lat
        t1 = -lat.to_parity(self.H(lat.from_parity(v_e, 0), adjoint=True), 1)
        t2 = np.einsum("nij,nj->ni", dag(self.A_oo_inv), t1)
        t3 = -lat.to_parity(self.H(lat.from_parity(t2, 1), adjoint=True), 0)
        return np.einsum("nij,nj->ni", dag(self.A_ee), v_e) - t3

    # eq. 2: the factorised inverse --------------------------------------
    def prepare(self, b):
        """Right-hand side of the Schur system: b~_e = b_e - D_eo D_oo^-1 b_o."""
        b_e = self.lat.to_parity(b, 0)
        b_o = self.lat.to_parity(b, 1)
        return b_e - self.D_eo(self.D_oo_inv(b_o))

    def reconstruct(self, x_e, b):
        """Full solution from the even half: x_o = D_oo^-1 (b_o - D_oe x_e)."""
        b_o = self.lat.to_parity(b, 1)
        x_o = self.D_oo_inv(b_o - self.D_oe(x_e))
        return self.lat.from_parity(x_e, 0) + self.lat.from_parity(x_o, 1)


# ---------------------------------------------------------------------------
# Explicit matrices (brute force for small lattices)
# ---------------------------------------------------------------------------
def sparse_D(op: WilsonClover):
    """D as a sparse 12V x 12V matrix assembled site by site from its nine 12x12
    blocks per block row (Sect. 2.3): the site block A(x) and, for every mu,
    -1/2 (1 - gamma_mu) (x) U_mu(x) in block column x + mu and
    -1/2 (1 + gamma_mu) (x) U_mu(x - mu)^H in block column x - mu, each times
    the boundary sign of that hop.  Blocks that land on the same column (2-site
    extents) add."""
    lat = op.lat
    V = lat.V
    Uf = op.U.reshape(V, 4, 3, 3)
    Af = op.A.reshape(V, 12, 12)
    rows, cols, vals = [], [], []
    ii, jj = np.meshgrid(np.arange(12), np.arange(12), indexing="ij")

    def put(n, m, blk):
        rows.append(12 * n + ii.ravel())
        cols.append(12 * m + jj.ravel())
        vals.append(blk.ravel())

    for n in range(V):
        put(n, n, Af[n])
        for mu in range(4):
            m, s = lat.neighbour(n, mu, +1)
            put(n, m, -0.5 * s * np.kron(I4 - GAMMA[mu], Uf[n, mu]))
            m, s = lat.neighbour(n, mu, -1)
            put(n, m, -0.5 * s * np.kron(I4 + GAMMA[mu], dag(Uf[m, mu])))
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(12 * V, 12 * V))
    return M.tocsr()


def parity_dofs(lat: Lattice, parity):
    sites = lat.even if parity == 0 else lat.odd
    return (12 * sites[:, None] + np.arange(12)[None, :]).ravel()


def dense_schur(op: WilsonClover):
    """D_S = D_ee - D_eo D_oo^-1 D_oe from the dense blocks of D in even-first order."""
    D = sparse_D(op).toarray()
    e, o = parity_dofs(op.lat, 0), parity_dofs(op.lat, 1)
    Dee, Deo = D[np.ix_(e, e)], D[np.ix_(e, o)]
    Doe, Doo = D[np.ix_(o, e)], D[np.ix_(o, o)]
    return Dee - Deo @ np.linalg.solve(Doo, Doe)


def norm(v):
    return float(np.sqrt(np.sum(np.abs(v) ** 2)))


def rel_err(a, b):
    """|a - b|_2 / |b|_2 over all entries."""
    return norm(np.asarray(a) - np.asarray(b)) / norm(b)
