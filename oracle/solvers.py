"""Oracle: the iterative methods of Sect. 2.4 on the Schur complement (FP64, CPU).

Test infrastructure only: the HIP library never imports this module.

Each solver takes ``apply``, a callable for the matrix (normally
``WilsonClover.schur``), and plain numpy vectors, and follows the paper's
algorithm in its order and notation.  Readings of points the paper leaves open:

* Richardson (Alg. 4): omega is an input.  The algorithm's
  omega = delta / |lambda_max| is formed by the caller from
  ``power_iteration``; the returned value is the final iterate x^(n), which the
  listing leaves unnamed.
* Power iteration (Sect. 2.4.4 says a few steps suffice): gamma_5-hermiticity
  pairs the eigenvalues of D_S as (lambda, conj(lambda)), so the iteration
  cannot settle on one eigenvector; the estimate is the geometric mean growth
  (|A^N v0| / |v0|)^(1/N), which tends to |lambda_max|.
* GMRES (Alg. 2): standard Arnoldi, v_1 = r/beta and v_{k+1} = w / h_{k+1,k}
  (the listing's v_k = r / h_{k,k-1} is read this way), h_{jk} = v_j^H w with
  modified Gram-Schmidt in the listing's order, least squares by a dense
  ``lstsq`` at every step.  A cycle ends early when the least-squares residual
  falls to the absolute target or on breakdown h_{k+1,k} <= 1e-14 beta;
  convergence is declared only on the recomputed residual at the restart (the
  listing's line "check convergence via beta").
* Flexible GMRES: the same with a right preconditioner z_k = M v_k and the
  update x += Z_k y_k.
* Odd-even smoother M_nu (Sect. 2.4.5, the right panel of Fig. 1): eq. 2's
  factorised D^-1 with D_S^-1 replaced by the Richardson polynomial
  p_{R,nu}(D_S) = (I - (I - omega D_S)^nu) D_S^-1 of Sect. 2.4.4, i.e. prepare,
  nu Richardson sweeps on D_S from zero, reconstruct.  nu = 0 is p = 0: the
  even half of M_0 r is zero and its odd half is D_oo^-1 r_o.
* FGMRES on the full D (Sect. 2.3: the fine level runs FGMRES; here M_nu alone
  is its right preconditioner, the smoother of a two-level method without the
  coarse-grid correction); the tolerance is relative to |b|.
* SAP(n, m) (Sect. 2.4.1, Alg. 1): the lattice is cut into blocks of fixed extent
  aligned at the origin; a block's colour is the parity of the sum of its block
  coordinates.  The block system D_kk e = r_k is D restricted to the block's rows
  and columns (couplings that leave the block dropped, those that wrap around the
  lattice inside one block kept), solved approximately by odd-even preconditioning
  on the block (eq. 2 with the block's hopping terms) and m Minimal Residual steps
  on the block's Schur complement from zero.  Red (colour 0) blocks first, all from
  one residual, then black from a recomputed one; the listing's convergence exit is
  left out (a fixed n, as a smoother).
* Minimal Residual (the block solver of Alg. 1, the textbook method Sect. 2.4.1
  cites): from x = 0, r = b; each step q = A r, alpha = (q^H r) / (q^H q),
  x += alpha r, r -= alpha q.
"""
from __future__ import annotations

import numpy as np


def vnorm(v):
    return float(np.sqrt(np.sum(np.abs(v) ** 2)))


def vdot(a, b):
    """a^H b over all entries."""
    return complex(np.vdot(a.ravel(), b.ravel()))


def richardson(apply, b, x0, n: int, omega: float):
    """Alg. 4: n sweeps of x <- x + omega (b - A x) from x0."""
    x = np.array(x0, dtype=np.complex128, copy=True)
    for _ in range(n):
        r = b - apply(x)
        x = x + omega * r
    return x


def power_iteration(apply, v0, n: int):
    """|lambda_max| estimate (|A^n v0| / |v0|)^(1/n), normalising every step."""
    v = np.array(v0, dtype=np.complex128, copy=True)
    nv = vnorm(v)
    v = v / nv
    log_growth = 0.0
    for _ in range(n):
        w = apply(v)
        g = vnorm(w)
        log_growth += np.log(g)
        v = w / g
    return float(np.exp(log_growth / n))


class GmresResult:
    def __init__(self, x, converged, cycles, iters, history):
        self.x = x
        self.converged = converged
        self.cycles = cycles
        self.iters = iters
        self.history = history  # residual estimate after every Arnoldi step


def gmres(apply, b, x0, m: int, max_cycles: int, tol_abs: float, precond=None,
          breakdown: float = 1e-14):
    """Restarted GMRES(n = max_cycles, m) of Alg. 2 (flexible if precond is given).

    Stops when the true residual |b - A x| at a restart is <= tol_abs.
    """
    x = np.array(x0, dtype=np.complex128, copy=True)
    history = []
    iters = 0
    for cycle in range(max_cycles + 1):
        r = b - apply(x)
        beta = vnorm(r)
        if beta <= tol_abs:
            return GmresResult(x, True, cycle, iters, history)
        if cycle == max_cycles:
            break
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        k_used = 0
        y = None
        for k in range(m):
            z = V[k] if precond is None else precond(V[k])
            Z.append(z)
            w = apply(z)
            for j in range(k + 1):
                H[j, k] = vdot(V[j], w)
                w = w - H[j, k] * V[j]
            H[k + 1, k] = vnorm(w)
            iters += 1
            k_used = k + 1
            y, *_ = np.linalg.lstsq(H[:k + 2, :k + 1], g[:k + 2], rcond=None)
            est = vnorm(g[:k + 2] - H[:k + 2, :k + 1] @ y)
            history.append(est)
            if est <= tol_abs or H[k + 1, k].real <= breakdown * beta:
                break
            V.append(w / H[k + 1, k])
        basis = Z if precond is not None else V
        for j in range(k_used):
            x = x + y[j] * basis[j]
    return GmresResult(x, False, max_cycles, iters, history)


def oe_solve(op, b, m: int, max_cycles: int, tol: float, precond=None):
    """Odd-even solve of D x = b: eq. 2's prepare, GMRES on the Schur complement
    to |b~_e - D_S x_e| <= tol |b|, reconstruct.  Returns (x, GmresResult)."""
    bt = op.prepare(b)
    res = gmres(op.schur, bt, np.zeros_like(bt), m, max_cycles, tol * vnorm(b), precond)
    return op.reconstruct(res.x, b), res


def richardson_preconditioner(apply, nsweeps: int, omega: float):
    """M v = nsweeps Richardson sweeps on A z = v from z = 0 (Alg. 4)."""
    def M(v):
        return richardson(apply, v, np.zeros_like(v), nsweeps, omega)
    return M


def oe_smoother(op, nsweeps: int, omega: float):
    """M_nu r: prepare (eq. 2), nu Richardson sweeps on D_S from zero (Alg. 4),
    reconstruct (eq. 2) -- eq. 2 with D_S^-1 replaced by p_{R,nu}(D_S)."""
    def M(r):
        bt = op.prepare(r)
        xe = richardson(op.schur, bt, np.zeros_like(bt), nsweeps, omega)
        return op.reconstruct(xe, r)
    return M


def fgmres_full(op, b, m: int, max_cycles: int, tol: float, nsweeps: int, omega: float, x0=None):
    """FGMRES(m) of Alg. 2 on the full D x = b with M_nu as right preconditioner,
    to |b - D x| <= tol |b|.  Returns (x, GmresResult)."""
    x0 = np.zeros_like(b) if x0 is None else x0
    res = gmres(op.D, b, x0, m, max_cycles, tol * vnorm(b), oe_smoother(op, nsweeps, omega))
    return res.x, res


def minimal_residual(apply, b, m: int):
    """m Minimal Residual steps on A x = b from x = 0."""
    x = np.zeros_like(b)
    r = np.array(b, dtype=np.complex128, copy=True)
    for _ in range(m):
        q = apply(r)
        qq = vdot(q, q)
        if qq == 0:
            break
        alpha = vdot(q, r) / qq
        x = x + alpha * r
        r = r - alpha * q
    return x


def sap_blocks(lat, block):
    """(block index of every site, colour of every block, number of blocks) for
    blocks of extent `block` (per direction, dividing the lattice)."""
    assert all(L % b == 0 for L, b in zip(lat.dims, block))
    nb = [L // b for L, b in zip(lat.dims, block)]
    coords = np.indices(lat.shape)  # lattice axes in the order of lat.shape
    # lat.shape lists the directions from t down to x; block extents are given x first
    bc = [coords[3 - mu] // block[mu] for mu in range(4)]
    idx = bc[0] + nb[0] * (bc[1] + nb[1] * (bc[2] + nb[2] * bc[3]))
    colour_of_site = (bc[0] + bc[1] + bc[2] + bc[3]) % 2
    nblk = nb[0] * nb[1] * nb[2] * nb[3]
    colour = np.zeros(nblk, dtype=int)
    colour[idx.ravel()] = colour_of_site.ravel()
    return idx, colour, nblk


def block_solve(op, in_block, r, m: int):
    """Approximate solution of D_kk e = r_k on one block (in_block: boolean per site):
    eq. 2 with the block's hopping terms, m Minimal Residual steps on the block Schur
    complement from zero; returns e as a full field, zero outside the block."""
    lat = op.lat
    me = lat.to_parity(in_block.astype(float)[..., None, None] * np.ones(lat.shape + (4, 3)), 0)
    mo = lat.to_parity(in_block.astype(float)[..., None, None] * np.ones(lat.shape + (4, 3)), 1)

    def D_eo_k(v_o):
        return me * op.D_eo(mo * v_o)

    def D_oe_k(v_e):
        return mo * op.D_oe(me * v_e)

    def S_k(v_e):
        return me * op.D_ee(v_e) - D_eo_k(op.D_oo_inv(D_oe_k(v_e)))

    r_e = me * lat.to_parity(r, 0)
    r_o = mo * lat.to_parity(r, 1)
    bt = r_e - D_eo_k(op.D_oo_inv(r_o))
    x_e = minimal_residual(S_k, bt, m)
    x_o = mo * op.D_oo_inv(r_o - D_oe_k(x_e))
    return lat.from_parity(x_e, 0) + lat.from_parity(x_o, 1)


def sap(op, b, x0, n: int, m: int, block=(4, 4, 4, 4)):
    """SAP(n, m) of Alg. 1 on D x = b from x0."""
    idx, colour, nblk = sap_blocks(op.lat, block)
    x = np.array(x0, dtype=np.complex128, copy=True)
    for _ in range(n):
        for c in (0, 1):
            r = b - op.D(x)
            for k in range(nblk):
                if colour[k] == c:
                    x = x + block_solve(op, idx == k, r, m)
    return x


def sap_preconditioner(op, n: int, m: int, block=(4, 4, 4, 4)):
    """M v = SAP(n, m) on D z = v from z = 0 (Alg. 1)."""
    def M(v):
        return sap(op, v, np.zeros_like(v), n, m, block)
    return M
