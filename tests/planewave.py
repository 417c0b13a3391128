"""Closed forms used to pin the oracle and, at full size, the HIP path.

Free Wilson operator (all links 1, clover term zero), chiral basis
gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_4 = [[0, 1], [1, 0]]:
  on psi(x) = exp(i p.x) u:      D psi = [m0 + sum(1 - cos p) + i sum gamma_mu sin p_mu] psi
  on the even part psi_e of it:  D_S psi_e = [(4 + m0) - H(p)^2 / (4 + m0)] psi_e,
                                 H(p) = sum cos p_mu - i sum gamma_mu sin p_mu,
because the staggered partner exp(i (p + pi) x) flips the sign of H(p).
Momenta: p_i = 2 pi k_i / L_i, p_t = (2 k_t + 1) pi / L_t (t antiperiodic).
These formulas are written here from the definition of the operator, not
taken from the oracle.
"""
import numpy as np

_s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]),
      np.array([[1, 0], [0, -1]], complex)]
_z = np.zeros((2, 2), complex)
G = [np.block([[_z, -1j * s], [1j * s, _z]]) for s in _s] + [
    np.block([[_z, np.eye(2)], [np.eye(2), _z]])]
G5 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(complex)


def momentum(dims, k):
    lx, ly, lz, lt = dims
    return np.array([2 * np.pi * k[0] / lx, 2 * np.pi * k[1] / ly,
                     2 * np.pi * k[2] / lz, (2 * k[3] + 1) * np.pi / lt])


def plane_wave(dims, p, u):
    """exp(i p.x) u on the full lattice, shape (Lt, Lz, Ly, Lx, 4, 3)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.indices((lt, lz, ly, lx))
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return ph[..., None, None] * np.asarray(u).reshape(4, 3)


def even_mask(dims):
    lx, ly, lz, lt = dims
    t, z, y, x = np.indices((lt, lz, ly, lx))
    return ((x + y + z + t) % 2) == 0


def H_of_p(p):
    return sum(np.cos(p[m]) * np.eye(4) - 1j * np.sin(p[m]) * G[m] for m in range(4))


def D_of_p(p, m0):
    return (4 + m0) * np.eye(4) - H_of_p(p)


def schur_of_p(p, m0):
    Hp = H_of_p(p)
    return (4 + m0) * np.eye(4) - Hp @ Hp / (4 + m0)


def schur_free_eigs(dims, m0):
    """All eigenvalues of the free D_S (each with multiplicity 3 in colour x
    2 in spin x 1/2 for the p, p+pi pairing = 3), by enumeration of momenta."""
    lx, ly, lz, lt = dims
    out = []
    for kx in range(lx):
        for ky in range(ly):
            for kz in range(lz):
                for kt in range(lt):
                    p = momentum(dims, (kx, ky, kz, kt))
                    c = np.cos(p).sum()
                    s = np.sqrt((np.sin(p) ** 2).sum())
                    out.append((4 + m0) - (c - 1j * s) ** 2 / (4 + m0))
                    out.append((4 + m0) - (c + 1j * s) ** 2 / (4 + m0))
    return np.array(out)


def schur_free_extremes(dims, m0):
    """min and max |eigenvalue| of the free D_S, by enumeration over the
    distinct |cos| / |sin| combinations per axis (fast at any size)."""
    lx, ly, lz, lt = dims
    per_axis = []
    for L, anti in ((lx, 0), (ly, 0), (lz, 0), (lt, 1)):
        k = np.arange(L)
        p = (2 * k + anti) * np.pi / L
        per_axis.append(np.unique(np.round(np.stack([np.cos(p), np.sin(p) ** 2], 1), 14), axis=0))
    mn, mx = np.inf, 0.0
    for a in per_axis[0]:
        for b in per_axis[1]:
            for c_ in per_axis[2]:
                for d in per_axis[3]:
                    c = a[0] + b[0] + c_[0] + d[0]
                    s = np.sqrt(a[1] + b[1] + c_[1] + d[1])
                    for sg in (1, -1):
                        mu = abs((4 + m0) - (c - sg * 1j * s) ** 2 / (4 + m0))
                        mn, mx = min(mn, mu), max(mx, mu)
    return mn, mx
