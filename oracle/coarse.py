"""Oracle: the coarse-grid operator of Sect. 2.3 (FP64, CPU).

Test infrastructure only: the HIP library never imports this module.

Aggregation-based prolongation (Sect. 2.3): the lattice is cut into aggregates of fixed
extent aligned at the origin; on every aggregate and for each chirality (spins 0, 1 and
spins 2, 3 of the chiral basis) the N_v test vectors, restricted to the aggregate's
sites and to that chirality's spin components, are orthonormalised (QR) and become the
columns of P.  R = P^H and D_c = R D P (Sect. 2.2's Galerkin coarse operator): a
nearest-neighbour operator on the coarse lattice with nine 2 N_v x 2 N_v complex blocks
per coarse site (self and the eight neighbours), coarse d.o.f. (chirality, k) ordered
chirality-major.  Readings: the test vectors are inputs (the paper obtains them in the
setup phase, which is not built); the coarse lattice is periodic in every direction
(the fine antiperiodic sign lives inside the blocks); block d = 0 is the site's own,
d = 1 + 2 mu + s its neighbour in direction mu forward (s = 0) or backward (s = 1).
"""
from __future__ import annotations

import numpy as np


def coarse_dims(lat, agg):
    assert all(L % a == 0 for L, a in zip(lat.dims, agg))
    return tuple(L // a for L, a in zip(lat.dims, agg))


def coarse_index(cd, c):
    """lexicographic index (x fastest) of coarse coordinates c = (x, y, z, t)"""
    return c[0] + cd[0] * (c[1] + cd[1] * (c[2] + cd[2] * c[3]))


def coarse_coords(cd, i):
    c = []
    for L in cd:
        c.append(i % L)
        i //= L
    return c


def coarse_neighbour(cd, i, d):
    """coarse site of block d of site i (periodic)"""
    if d == 0:
        return i
    mu, s = (d - 1) // 2, (d - 1) % 2
    c = coarse_coords(cd, i)
    c[mu] = (c[mu] + (1 if s == 0 else -1)) % cd[mu]
    return coarse_index(cd, c)


def aggregate_of_sites(lat, agg):
    """coarse site index of every fine site, in the lattice's array order"""
    cd = coarse_dims(lat, agg)
    idx = np.indices(lat.shape)  # axes: t, z, y, x
    c = [idx[3 - mu] // agg[mu] for mu in range(4)]
    return c[0] + cd[0] * (c[1] + cd[1] * (c[2] + cd[2] * c[3]))


class Prolongation:
    """P of Sect. 2.3 from test vectors (list of full fields [..., 4, 3])."""

    def __init__(self, lat, agg, test_vectors):
        self.lat, self.agg = lat, tuple(agg)
        self.cd = coarse_dims(lat, agg)
        self.Vc = int(np.prod(self.cd))
        self.nv = len(test_vectors)
        self.site_agg = aggregate_of_sites(lat, agg).ravel()
        T = np.stack([np.asarray(t).reshape(lat.V, 4, 3) for t in test_vectors], axis=-1)  # [V, 4, 3, nv]
        # Q[a][c]: (sites of a) x 2 spins x 3 colours by nv, orthonormal columns
        self.sites = [np.flatnonzero(self.site_agg == a) for a in range(self.Vc)]
        self.Q = []
        for a in range(self.Vc):
            qa = []
            for c in range(2):
                block = T[self.sites[a]][:, 2 * c:2 * c + 2, :, :].reshape(-1, self.nv)
                q, _ = np.linalg.qr(block)
                qa.append(q)
            self.Q.append(qa)

    def prolong(self, vc):
        """fine field from a coarse vector vc[Vc, 2, nv]"""
        f = np.zeros((self.lat.V, 4, 3), complex)
        for a in range(self.Vc):
            for c in range(2):
                f[self.sites[a], 2 * c:2 * c + 2, :] = (self.Q[a][c] @ vc[a, c]).reshape(-1, 2, 3)
        return f.reshape(self.lat.shape + (4, 3))

    def restrict(self, f):
        """P^H f: coarse vector [Vc, 2, nv]"""
        ff = np.asarray(f).reshape(self.lat.V, 4, 3)
        vc = np.zeros((self.Vc, 2, self.nv), complex)
        for a in range(self.Vc):
            for c in range(2):
                vc[a, c] = self.Q[a][c].conj().T @ ff[self.sites[a], 2 * c:2 * c + 2, :].reshape(-1)
        return vc


def galerkin_blocks(op, P):
    """the nine blocks A[Vc, 9, 2 nv, 2 nv] of D_c = P^H D P, column by column from
    matrix-free applies of D to prolonged coarse unit vectors (coarse extents >= 3, so
    that every neighbour direction reaches a distinct coarse site)"""
    assert all(c >= 3 for c in P.cd)
    n2 = 2 * P.nv
    A = np.zeros((P.Vc, 9, n2, n2), complex)
    for y in range(P.Vc):
        for q in range(n2):
            e = np.zeros((P.Vc, 2, P.nv), complex)
            e[y, q // P.nv, q % P.nv] = 1.0
            col = P.restrict(op.D(P.prolong(e))).reshape(P.Vc, n2)
            for x in range(P.Vc):
                if not np.any(col[x]):
                    continue
                ds = [d for d in range(9) if coarse_neighbour(P.cd, x, d) == y]
                assert len(ds) == 1, "coupling outside the nearest-neighbour pattern"
                A[x, ds[0], :, q] = col[x]
    return A


def coarse_apply(A, cd, v):
    """y[x] = sum over d of A[x, d] v[neighbour(x, d)]; v[Vc, 2 nv] or [Vc, 2 nv, nrhs]"""
    Vc = A.shape[0]
    y = np.zeros_like(v, dtype=complex)
    for x in range(Vc):
        for d in range(9):
            y[x] = y[x] + A[x, d] @ v[coarse_neighbour(cd, x, d)]
    return y
