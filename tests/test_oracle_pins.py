"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

P1  gamma_5-hermiticity of D and D_S; explicit D_S^H stencil
P2  free-field plane waves: closed-form D and D_S on distinct extents
P3  pure gauge fields
P4  gauge covariance of D, the clover blocks and D_S
P5  constant abelian field: closed-form clover blocks
P6  the factorised inverse of eq. 2 and the Schur complement of eq. 3 vs brute force
P7  Richardson (Alg. 4) and its polynomial (Sect. 2.4.5)
P8  GMRES (Alg. 2): finite termination, residual minimisation, monotone estimates
P9  power iteration vs dense eigenvalues
P11 the qualitative claims of Fig. 1 on a 4^4 lattice
Structure: nine 12x12 blocks per block row (Sect. 2.3), 6x6 site blocks (Sect. 2.4.5).
"""
import json
import os

import numpy as np
import pytest

from oracle import dirac, solvers
from oracle.dirac import Lattice, WilsonClover, dense_schur, rel_err, sparse_D
from paper_2407_08092_amd import synth
from planewave import (G, G5, D_of_p, even_mask, momentum, plane_wave, schur_free_eigs,
                       schur_free_extremes, schur_of_p)

HERE = os.path.dirname(os.path.abspath(__file__))
DISTINCT = (4, 6, 8, 10)


def free_links(dims):
    lat = Lattice(dims)
    U = np.zeros(lat.shape + (4, 3, 3), complex)
    U[...] = np.eye(3)
    return lat, U


def rand_vec(n, seed):
    return synth.gaussian_complex((n, 12), seed)


def apply_spin_colour(M4, psi):
    """(M4 (x) 1_colour) psi for psi[..., 4, 3]."""
    return np.einsum("st,...ta->...sa", M4, psi)


def omega_transform(U, Om, lat):
    """U'_mu(x) = Om(x) U_mu(x) Om(x + mu)^H (periodic shift of Om)."""
    Up = np.empty_like(U)
    for mu in range(4):
        Om_fwd = lat.shift(Om, {mu: 1})
        Up[..., mu, :, :] = Om @ U[..., mu, :, :] @ dirac.dag(Om_fwd)
    return Up


def colour_rotate(Om, psi):
    return np.einsum("...ab,...sb->...sa", Om, psi)


# --------------------------------------------------------------------------
# basis and layout
# --------------------------------------------------------------------------
def test_gamma_basis():
    # Clifford algebra, hermiticity, gamma_5 = gamma1 gamma2 gamma3 gamma4 = diag(1,1,-1,-1)
    for m in range(4):
        assert np.allclose(dirac.GAMMA[m], G[m])
        for n in range(4):
            ac = dirac.GAMMA[m] @ dirac.GAMMA[n] + dirac.GAMMA[n] @ dirac.GAMMA[m]
            assert np.allclose(ac, 2 * np.eye(4) * (m == n))
    assert np.allclose(dirac.GAMMA5, G5)
    # sigma_munu commutes with gamma_5: A(x) splits into two 6x6 blocks (Sect. 2.4.5)
    for m in range(4):
        for n in range(4):
            assert np.allclose(dirac.SIGMA[m, n] @ G5, G5 @ dirac.SIGMA[m, n])


def test_parity_order_is_halved_lexicographic_index():
    lat = Lattice(DISTINCT)
    assert np.array_equal(lat.even >> 1, np.arange(lat.Vh))
    assert np.array_equal(lat.odd >> 1, np.arange(lat.Vh))


def test_odd_extent_rejected():
    with pytest.raises(ValueError):
        Lattice((4, 5, 4, 4))


# --------------------------------------------------------------------------
# P2 free field
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k", [(1, 0, 0, 0), (0, 2, 0, 1), (0, 0, 3, 2), (1, 5, 7, 4), (3, 1, 2, 9)])
def test_free_field_full_operator(k):
    m0 = -0.17
    lat, U = free_links(DISTINCT)
    op = WilsonClover(lat, U, c_sw=1.3, m0=m0)  # clover vanishes for unit links
    p = momentum(DISTINCT, k)
    u = synth.gaussian_complex((4, 3), 11)
    psi = plane_wave(DISTINCT, p, u)
    expect = apply_spin_colour(D_of_p(p, m0), psi)
    assert rel_err(op.D(psi), expect) < 1e-13


@pytest.mark.parametrize("k", [(1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1), (2, 5, 3, 7)])
def test_free_field_schur(k):
    m0 = -0.1
    lat, U = free_links(DISTINCT)
    op = WilsonClover(lat, U, c_sw=1.0, m0=m0)
    p = momentum(DISTINCT, k)
    u = synth.gaussian_complex((4, 3), 12)
    psi = plane_wave(DISTINCT, p, u) * even_mask(DISTINCT)[..., None, None]
    xe = lat.to_parity(psi, 0)
    expect = lat.to_parity(apply_spin_colour(schur_of_p(p, m0), psi), 0)
    assert rel_err(op.schur(xe), expect) < 1e-13


def test_free_field_schur_spectrum_4444():
    dims, m0 = (4, 4, 4, 4), -0.1
    lat, U = free_links(dims)
    op = WilsonClover(lat, U, 1.0, m0)
    ev = np.linalg.eigvals(dense_schur(op))
    ref = np.repeat(schur_free_eigs(dims, m0), 3)
    key = lambda z: np.lexsort((np.round(z.imag, 8), np.round(z.real, 8)))
    assert np.allclose(ev[key(ev)], ref[key(ref)], atol=1e-10)
    with open(os.path.join(HERE, "golden", "free_field_extremes.json")) as f:
        gold = json.load(f)["cases"]
    for case in gold:
        mn, mx = schur_free_extremes(tuple(case["dims"]), case["m0"])
        assert abs(mn - case["min_abs"]) < 6e-4 and abs(mx - case["max_abs"]) < 6e-4
        if tuple(case["dims"]) == dims:
            assert abs(np.abs(ev).min() - case["min_abs"]) < 6e-4
            assert abs(np.abs(ev).max() - case["max_abs"]) < 6e-4


def test_antiperiodic_sign_matters():
    # with periodic t the momentum set differs; the closed form must then fail
    m0 = -0.1
    lat = Lattice(DISTINCT, antiperiodic_t=False)
    U = np.zeros(lat.shape + (4, 3, 3), complex)
    U[...] = np.eye(3)
    op = WilsonClover(lat, U, 1.0, m0)
    p = momentum(DISTINCT, (0, 0, 0, 1))
    psi = plane_wave(DISTINCT, p, synth.gaussian_complex((4, 3), 3))
    assert rel_err(op.D(psi), apply_spin_colour(D_of_p(p, m0), psi)) > 1e-2


# --------------------------------------------------------------------------
# P3 pure gauge, P4 gauge covariance
# --------------------------------------------------------------------------
def test_pure_gauge():
    m0 = -0.2
    lat = Lattice(DISTINCT)
    Om = synth.random_su3_sites(DISTINCT, 21)
    U1 = np.zeros(lat.shape + (4, 3, 3), complex)
    U1[...] = np.eye(3)
    U = omega_transform(U1, Om, lat)
    op = WilsonClover(lat, U, 1.7, m0)
    assert np.allclose(op.A, (4 + m0) * np.eye(12), atol=1e-13)
    p = momentum(DISTINCT, (1, 2, 3, 4))
    psi = plane_wave(DISTINCT, p, synth.gaussian_complex((4, 3), 22)) * even_mask(DISTINCT)[..., None, None]
    got = op.schur(lat.to_parity(colour_rotate(Om, psi), 0))
    expect = lat.to_parity(colour_rotate(Om, apply_spin_colour(schur_of_p(p, m0), psi)), 0)
    assert rel_err(got, expect) < 1e-12


def test_gauge_covariance():
    lat = Lattice(DISTINCT)
    U = synth.gauge_field(DISTINCT, 0.5, 31)
    Om = synth.random_su3_sites(DISTINCT, 32)
    op = WilsonClover(lat, U, 1.0, -0.2)
    opp = WilsonClover(lat, omega_transform(U, Om, lat), 1.0, -0.2)
    # A'(x) = Om(x) A(x) Om(x)^H acting on colour
    OmS = np.einsum("st,...ab->...satb", np.eye(4), Om).reshape(lat.shape + (12, 12))
    assert np.allclose(opp.A, OmS @ op.A @ dirac.dag(OmS), atol=1e-13)
    psi = synth.gaussian_spinor(DISTINCT, 33)
    assert rel_err(opp.D(colour_rotate(Om, psi)), colour_rotate(Om, op.D(psi))) < 1e-13
    xe = lat.to_parity(psi, 0)
    got = opp.schur(lat.to_parity(colour_rotate(Om, lat.from_parity(xe, 0)), 0))
    expect = lat.to_parity(colour_rotate(Om, lat.from_parity(op.schur(xe), 0)), 0)
    assert rel_err(got, expect) < 1e-13


# --------------------------------------------------------------------------
# P5 constant abelian field
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k", [1, 2])
def test_constant_abelian_clover(k):
    dims = (8, 4, 6, 4)
    c_sw, m0 = 1.3, -0.25
    lat = Lattice(dims)
    b = 4 * np.pi * k / dims[0]
    T = np.diag([0.5, -0.5, 0.0])
    x = lat.coords[0]
    U = np.zeros(lat.shape + (4, 3, 3), complex)
    U[...] = np.eye(3)
    for a in range(3):
        U[..., 1, a, a] = np.exp(1j * b * x * T[a, a])
    op = WilsonClover(lat, U, c_sw, m0)
    sinbT = np.sin(b * np.diag(T))
    spin_sign = np.array([1, -1, 1, -1])  # diag(s3, s3) in the chiral basis
    diag = (4 + m0) + 0.5 * c_sw * np.kron(spin_sign, sinbT)
    assert np.allclose(op.A, np.diag(diag), atol=1e-13)


def test_abelian_field_clover_leaf_average():
    # U_y(x) = exp(i phi(x_1) T) with arbitrary phi: the xy plaquette based at x
    # is exp(i Delta(x_1) T), Delta(x_1) = phi(x_1 + 1) - phi(x_1); two of the four
    # clover leaves sit at x_1 and two at x_1 - 1, so
    # F_xy(x) = (i/2) [sin(Delta(x_1) T) + sin(Delta(x_1 - 1) T)] and
    # A(x) = (4 + m0) + (c_sw / 4) diag(s3, s3) (x) [sin(Delta(x_1) T) + sin(Delta(x_1 - 1) T)].
    dims = (6, 4, 2, 4)
    c_sw, m0 = 0.9, -0.3
    lat = Lattice(dims)
    phi = np.random.default_rng(5).uniform(-2, 2, dims[0])
    Tdiag = np.array([0.5, -0.5, 0.0])
    x = lat.coords[0]
    U = np.zeros(lat.shape + (4, 3, 3), complex)
    U[...] = np.eye(3)
    for a in range(3):
        U[..., 1, a, a] = np.exp(1j * phi[x] * Tdiag[a])
    op = WilsonClover(lat, U, c_sw, m0)
    delta = np.roll(phi, -1) - phi
    spin_sign = np.array([1, -1, 1, -1])
    for xi in range(dims[0]):
        s = np.sin(delta[xi] * Tdiag) + np.sin(delta[xi - 1] * Tdiag)
        diag = (4 + m0) + 0.25 * c_sw * np.kron(spin_sign, s)
        sites = op.A[:, :, :, xi]
        assert np.allclose(sites, np.diag(diag), atol=1e-13)


# --------------------------------------------------------------------------
# P1 gamma_5-hermiticity, explicit adjoint
# --------------------------------------------------------------------------
def test_gamma5_hermiticity():
    lat = Lattice(DISTINCT)
    op = WilsonClover(lat, synth.gauge_field(DISTINCT, 0.5, 41), 1.0, -0.2)
    g5 = lambda v: apply_spin_colour(G5, v.reshape(-1, 4, 3)).reshape(v.shape)
    xi, eta = rand_vec(lat.Vh, 42), rand_vec(lat.Vh, 43)
    lhs = np.vdot(xi, g5(op.schur(g5(eta))))
    rhs = np.vdot(op.schur(xi), eta)
    assert abs(lhs - rhs) / abs(rhs) < 1e-13
    # explicit adjoint stencil == gamma5 D_S gamma5 == <D_S xi, eta> = <xi, D_S^H eta>
    assert rel_err(op.schur_adjoint(eta), g5(op.schur(g5(eta)))) < 1e-13
    lhs2 = np.vdot(xi, op.schur_adjoint(eta))
    assert abs(lhs2 - rhs) / abs(rhs) < 1e-13
    # full operator too
    psi, chi = synth.gaussian_spinor(DISTINCT, 44), synth.gaussian_spinor(DISTINCT, 45)
    g5f = lambda v: apply_spin_colour(G5, v)
    assert abs(np.vdot(psi, g5f(op.D(g5f(chi)))) - np.vdot(op.D(psi), chi)) < 1e-12 * abs(np.vdot(op.D(psi), chi))


def test_adjoint_matches_dense_conjugate_transpose():
    lat = Lattice((4, 4, 4, 4))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 51), 1.0, -0.1)
    DS = dense_schur(op)
    v = rand_vec(lat.Vh, 52)
    assert rel_err(op.schur_adjoint(v).ravel(), DS.conj().T @ v.ravel()) < 1e-13


# --------------------------------------------------------------------------
# structure and brute force (P6)
# --------------------------------------------------------------------------
def test_nine_blocks_per_block_row():
    lat = Lattice((4, 4, 4, 4))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 61), 1.0, -0.1)
    D = sparse_D(op).tocsr()
    for n in (0, 17, 200):
        cols = D[12 * n:12 * n + 12].nonzero()[1]
        assert len(np.unique(cols // 12)) == 9
    # 2^4: +mu and -mu neighbours coincide -> 5 distinct block columns
    lat2 = Lattice((2, 2, 2, 2))
    op2 = WilsonClover(lat2, synth.gauge_field(lat2.dims, 0.3, 62), 1.0, -0.1)
    cols = sparse_D(op2).tocsr()[0:12].nonzero()[1]
    assert len(np.unique(cols // 12)) == 5


def test_site_blocks_are_6x6_hermitian():
    lat = Lattice((4, 4, 4, 4))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.5, 63), 1.0, -0.1)
    A = op.A.reshape(-1, 12, 12)
    assert np.abs(A[:, :6, 6:]).max() == 0.0 and np.abs(A[:, 6:, :6]).max() == 0.0
    assert np.allclose(A, dirac.dag(A), atol=1e-15)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), DISTINCT])
def test_matrix_free_vs_assembled(dims):
    lat = Lattice(dims)
    op = WilsonClover(lat, synth.gauge_field(dims, 0.5, 71), 1.0, -0.2)
    psi = synth.gaussian_spinor(dims, 72)
    assert rel_err(op.D(psi).ravel(), sparse_D(op) @ psi.ravel()) < 1e-14


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4)])
def test_schur_matrix_free_vs_dense(dims):
    lat = Lattice(dims)
    op = WilsonClover(lat, synth.gauge_field(dims, 0.3, 81), 1.0, -0.1)
    DS = dense_schur(op)
    v = rand_vec(lat.Vh, 82)
    assert rel_err(op.schur(v).ravel(), DS @ v.ravel()) < 1e-14


SMALL_DISTINCT = (4, 2, 6, 8)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), SMALL_DISTINCT])
def test_factorised_inverse_eq2(dims):
    lat = Lattice(dims)
    op = WilsonClover(lat, synth.gauge_field(dims, 0.4, 91), 1.0, -0.1)
    b = synth.gaussian_spinor(dims, 92)
    x_ref = np.linalg.solve(sparse_D(op).toarray(), b.ravel()).reshape(b.shape)
    # exact Schur solve (dense on the even half)
    bt = op.prepare(b)
    xe = np.linalg.solve(dense_schur(op), bt.ravel()).reshape(bt.shape)
    x = op.reconstruct(xe, b)
    assert rel_err(x, x_ref) < 1e-11


def test_prepare_reconstruct_plain_definition():
    # b~_e = b_e + H_eo A_oo^-1 b_o and x_o = A_oo^-1 (b_o + H_oe x_e), in terms of H
    lat = Lattice(DISTINCT)
    op = WilsonClover(lat, synth.gauge_field(DISTINCT, 0.4, 93), 1.0, -0.1)
    b = synth.gaussian_spinor(DISTINCT, 94)
    b_o = lat.to_parity(b, 1)
    Hu = op.H(lat.from_parity(np.einsum("nij,nj->ni", op.A_oo_inv, b_o), 1))
    assert rel_err(op.prepare(b), lat.to_parity(b, 0) + lat.to_parity(Hu, 0)) < 1e-14
    xe = rand_vec(lat.Vh, 95)
    x = op.reconstruct(xe, b)
    xo = np.einsum("nij,nj->ni", op.A_oo_inv, b_o + lat.to_parity(op.H(lat.from_parity(xe, 0)), 1))
    assert rel_err(lat.to_parity(x, 1), xo) < 1e-14
    # full residual of the odd rows vanishes after reconstruct
    r = b - op.D(x)
    assert solvers.vnorm(lat.to_parity(r, 1)) < 1e-12 * solvers.vnorm(b)


# --------------------------------------------------------------------------
# P7 Richardson
# --------------------------------------------------------------------------
def test_richardson_on_free_eigenvector():
    dims, m0, omega, n = DISTINCT, -0.1, 0.17, 10
    lat, U = free_links(dims)
    op = WilsonClover(lat, U, 1.0, m0)
    p = momentum(dims, (1, 2, 3, 0))
    M = schur_of_p(p, m0)
    ev, W = np.linalg.eig(M)
    u = np.outer(W[:, 0], synth.gaussian_complex((3,), 101))
    psi = plane_wave(dims, p, u) * even_mask(dims)[..., None, None]
    b = lat.to_parity(psi, 0)
    x = solvers.richardson(op.schur, b, np.zeros_like(b), n, omega)
    mu = ev[0]
    assert rel_err(x, (1 - (1 - omega * mu) ** n) / mu * b) < 1e-13


def test_richardson_polynomial_dense():
    lat = Lattice((2, 2, 2, 2))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 111), 1.0, -0.1)
    DS = dense_schur(op)
    b = rand_vec(lat.Vh, 112)
    omega, k = 0.8 / 4.7, 7
    x = solvers.richardson(op.schur, b, np.zeros_like(b), k, omega)
    Id = np.eye(DS.shape[0])
    r_expect = np.linalg.matrix_power(Id - omega * DS, k) @ b.ravel()
    assert rel_err((b - op.schur(x)).ravel(), r_expect) < 1e-12
    # p_{R,k}(D) = (I - (I - w D)^k) D^-1
    pR = (Id - np.linalg.matrix_power(Id - omega * DS, k)) @ np.linalg.inv(DS)
    assert rel_err(x.ravel(), pR @ b.ravel()) < 1e-12
    # nonzero initial guess: x_k = x0 + p(D) r0
    x0 = rand_vec(lat.Vh, 113)
    xk = solvers.richardson(op.schur, b, x0, k, omega)
    assert rel_err(xk.ravel(), x0.ravel() + pR @ (b - op.schur(x0)).ravel()) < 1e-12


# --------------------------------------------------------------------------
# P8 GMRES
# --------------------------------------------------------------------------
def test_gmres_finite_termination():
    dims, m0 = (4, 4, 4, 4), -0.1
    lat, U = free_links(dims)
    op = WilsonClover(lat, U, 1.0, m0)
    b = np.zeros((lat.Vh, 12), complex)
    mus = []
    for i, k in enumerate([(1, 0, 0, 0), (1, 1, 0, 0), (1, 1, 1, 1), (0, 0, 0, 0)]):
        p = momentum(dims, k)
        ev, W = np.linalg.eig(schur_of_p(p, m0))
        j = int(np.argmax(ev.imag))
        mus.append(ev[j])
        u = np.outer(W[:, j], synth.gaussian_complex((3,), 120 + i))
        b += lat.to_parity(plane_wave(dims, p, u) * even_mask(dims)[..., None, None], 0)
    assert len(np.unique(np.round(mus, 8))) == 4
    res = solvers.gmres(op.schur, b, np.zeros_like(b), 10, 1, 1e-12 * solvers.vnorm(b))
    assert res.iters == 4
    assert res.converged
    assert solvers.vnorm(b - op.schur(res.x)) < 1e-12 * solvers.vnorm(b)


def test_gmres_minimises_over_krylov_space():
    lat = Lattice((2, 2, 2, 2))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.5, 131), 1.0, -0.1)
    DS = dense_schur(op)
    b = rand_vec(lat.Vh, 132).ravel()
    for k in (1, 3, 6, 9):
        res = solvers.gmres(lambda v: (DS @ v.ravel()).reshape(v.shape), b, np.zeros_like(b), k, 1, 0.0)
        # brute force: orthonormal Krylov basis by QR, dense least squares
        K = np.stack([np.linalg.matrix_power(DS, j) @ b for j in range(k)], 1)
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(DS @ Q, b, rcond=None)
        best = np.linalg.norm(b - DS @ Q @ y)
        assert abs(np.linalg.norm(b - DS @ res.x) - best) < 1e-10 * np.linalg.norm(b)
        assert abs(res.history[-1] - best) < 1e-10 * np.linalg.norm(b)


def test_gmres_restarted_converges_monotone():
    lat = Lattice((4, 4, 4, 4))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 101), 1.0, -0.1)
    b = rand_vec(lat.Vh, 102)
    res = solvers.gmres(op.schur, b, np.zeros_like(b), 30, 50, 1e-10 * solvers.vnorm(b))
    assert res.converged
    assert solvers.vnorm(b - op.schur(res.x)) <= 1e-10 * solvers.vnorm(b)
    h = np.array(res.history)
    # within every cycle the least-squares residual never grows
    assert np.all(np.diff(h[:min(len(h), 30)]) <= 1e-12 * h[0])


def test_flexible_gmres_with_richardson_preconditioner():
    lat = Lattice((4, 4, 4, 4))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 101), 1.0, -0.1)
    b = rand_vec(lat.Vh, 102)
    M = solvers.richardson_preconditioner(op.schur, 10, 0.8 / 4.9)
    res = solvers.gmres(op.schur, b, np.zeros_like(b), 30, 20, 1e-10 * solvers.vnorm(b), precond=M)
    plain = solvers.gmres(op.schur, b, np.zeros_like(b), 30, 20, 1e-10 * solvers.vnorm(b))
    assert res.converged and res.iters < plain.iters
    assert solvers.vnorm(b - op.schur(res.x)) <= 1e-10 * solvers.vnorm(b)


def test_oe_solve_matches_full_solve():
    dims = SMALL_DISTINCT
    lat = Lattice(dims)
    op = WilsonClover(lat, synth.gauge_field(dims, 0.5, 141), 1.0, -0.2)
    b = synth.gaussian_spinor(dims, 142)
    x, res = solvers.oe_solve(op, b, 30, 100, 1e-10)
    assert res.converged
    assert solvers.vnorm(b - op.D(x)) <= 1e-10 * solvers.vnorm(b)
    x_ref = np.linalg.solve(sparse_D(op).toarray(), b.ravel()).reshape(b.shape)
    assert rel_err(x, x_ref) < 1e-8


# --------------------------------------------------------------------------
# P9 power iteration
# --------------------------------------------------------------------------
def test_power_iteration():
    lat = Lattice((4, 4, 4, 4))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 101), 1.0, -0.1)
    lam = np.abs(np.linalg.eigvals(dense_schur(op))).max()
    v0 = rand_vec(lat.Vh, 103)
    est50 = solvers.power_iteration(op.schur, v0, 50)
    est400 = solvers.power_iteration(op.schur, v0, 400)
    assert abs(est50 / lam - 1) < 0.06
    assert abs(est400 / lam - 1) < abs(est50 / lam - 1) + 1e-3
    assert abs(est400 / lam - 1) < 0.01
    # free field: closed form
    latf, Uf = free_links((4, 4, 4, 4))
    opf = WilsonClover(latf, Uf, 1.0, -0.1)
    estf = solvers.power_iteration(opf.schur, rand_vec(latf.Vh, 104), 400)
    assert abs(estf / schur_free_extremes((4, 4, 4, 4), -0.1)[1] - 1) < 0.01


# --------------------------------------------------------------------------
# P11 Fig. 1, qualitative (the paper's 4^4 gauge field is unknown)
# --------------------------------------------------------------------------
def test_fig1_qualitative_4444():
    lat = Lattice((4, 4, 4, 4))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 101), 1.0, -0.1)
    D = sparse_D(op).toarray()
    DS = dense_schur(op)
    lD, lS = np.linalg.eigvals(D), np.linalg.eigvals(DS)
    assert np.abs(lD).max() > 6.0                       # spec(D) extends beyond 6
    assert np.abs(lS).max() < np.abs(lD).max()          # top end moves towards 0
    assert np.abs(lS).min() > np.abs(lD).min()          # low end moves away from 0
    assert (np.abs(lS).max() / np.abs(lS).min()) < (np.abs(lD).max() / np.abs(lD).min())
    # centre and right panels: Richardson polynomial of degree 3 on D and on D_S
    delta = 1.0
    wD, wS = delta / np.abs(lD).max(), delta / np.abs(lS).max()
    lDp = 1 - (1 - wD * lD) ** 3                       # spec(D p_{R,3}(D))
    e, o = dirac.parity_dofs(lat, 0), dirac.parity_dofs(lat, 1)
    Id_e = np.eye(len(e))
    pS = (Id_e - np.linalg.matrix_power(Id_e - wS * DS, 3)) @ np.linalg.inv(DS)
    Doo_inv = np.linalg.inv(D[np.ix_(o, o)])
    Deo, Doe = D[np.ix_(e, o)], D[np.ix_(o, e)]
    n = D.shape[0]
    L = np.eye(n); Dg = np.zeros((n, n), complex); Uu = np.eye(n, dtype=complex)
    perm = np.concatenate([e, o]); ne = len(e)
    L = L.astype(complex)
    L[ne:, :ne] = -Doo_inv @ Doe
    Dg[:ne, :ne] = pS
    Dg[ne:, ne:] = Doo_inv
    Uu[:ne, ne:] = -Deo @ Doo_inv
    M3 = L @ Dg @ Uu                                     # eq. 2 with D_S^-1 -> p_{R,3}(D_S)
    lDM = np.linalg.eigvals(D[np.ix_(perm, perm)] @ M3)
    assert np.mean(np.abs(1 - lDM)) < np.mean(np.abs(1 - lDp))
    assert np.abs(lDM).min() > np.abs(lDp).min()        # spectrum kept away from zero


# --------------------------------------------------------------------------
# P12 the odd-even smoother M_nu and FGMRES on the full D (Sect. 2.4.5, Fig. 1 right)
# --------------------------------------------------------------------------
def _full_vec(lat, seed):
    return synth.gaussian_complex(lat.shape + (4, 3), seed)


def _match_multisets(a, b):
    """largest distance after the best one-to-one pairing of two eigenvalue lists"""
    from scipy.optimize import linear_sum_assignment
    cost = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(cost)
    return float(cost[r, c].max())


def test_oe_smoother_nu0_closed_form():
    # p_{R,0} = 0: M_0 r = (0, D_oo^-1 r_o)
    lat = Lattice((4, 4, 2, 2))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 121), 1.0, -0.1)
    r = _full_vec(lat, 122)
    z = solvers.oe_smoother(op, 0, 0.2)(r)
    assert np.all(lat.to_parity(z, 0) == 0)
    z_o = np.linalg.solve(op.A_oo, lat.to_parity(r, 1)[..., None])[..., 0]
    assert rel_err(lat.to_parity(z, 1), z_o) < 1e-13


@pytest.mark.parametrize("nu", [1, 3, 6])
def test_oe_smoother_spectrum_closed_form(nu):
    # D M_nu is similar to diag(D_S p_{R,nu}(D_S), 1): its spectrum is
    # {1 - (1 - omega lambda)^nu : lambda in spec(D_S)} and 1 with multiplicity 12 V / 2
    lat = Lattice((4, 4, 2, 2))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 123), 1.0, -0.1)
    D = sparse_D(op).toarray()
    lS = np.linalg.eigvals(dense_schur(op))
    omega = 0.8 / np.abs(lS).max()
    M = solvers.oe_smoother(op, nu, omega)
    n = D.shape[0]
    cols = np.empty((n, n), complex)
    for j in range(n):  # the matrix of M_nu, column by column, through the oracle function
        e = np.zeros(n, complex)
        e[j] = 1.0
        cols[:, j] = M(e.reshape(lat.shape + (4, 3))).ravel()
    got = np.linalg.eigvals(D @ cols)
    expect = np.concatenate([1 - (1 - omega * lS) ** nu, np.ones(n // 2)])
    assert _match_multisets(got, expect) < 1e-10


def test_oe_smoother_matches_dense_factorisation():
    # eq. 2 with D_S^-1 -> p_{R,nu}(D_S), from the dense blocks of the assembled D
    lat = Lattice((4, 4, 2, 2))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 131), 1.0, -0.1)
    D = sparse_D(op).toarray()
    e, o = dirac.parity_dofs(lat, 0), dirac.parity_dofs(lat, 1)
    Dee, Deo, Doe, Doo = D[np.ix_(e, e)], D[np.ix_(e, o)], D[np.ix_(o, e)], D[np.ix_(o, o)]
    Doo_inv = np.linalg.inv(Doo)
    DS = Dee - Deo @ Doo_inv @ Doe
    nu, omega = 4, 0.8 / np.abs(np.linalg.eigvals(DS)).max()
    Ie = np.eye(len(e))
    p = (Ie - np.linalg.matrix_power(Ie - omega * DS, nu)) @ np.linalg.inv(DS)
    r = _full_vec(lat, 132).ravel()
    t_e = r[e] - Deo @ (Doo_inv @ r[o])          # right factor
    x_e = p @ t_e                                # middle factor
    x_o = Doo_inv @ r[o] - Doo_inv @ (Doe @ x_e)  # left factor
    z = solvers.oe_smoother(op, nu, omega)(r.reshape(lat.shape + (4, 3))).ravel()
    assert rel_err(z[e], x_e) < 1e-12 and rel_err(z[o], x_o) < 1e-12


def test_oe_smoother_tends_to_inverse():
    # omega |lambda_max| < 1 makes (I - omega D_S)^nu -> 0: M_nu r -> D^-1 r
    lat = Lattice((4, 4, 2, 2))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 124), 1.0, -0.1)
    lS = np.linalg.eigvals(dense_schur(op))
    omega = 0.8 / np.abs(lS).max()
    rate = np.abs(1 - omega * lS).max()
    r = _full_vec(lat, 125)
    x = np.linalg.solve(sparse_D(op).toarray(), r.ravel())
    errs = [rel_err(solvers.oe_smoother(op, nu, omega)(r).ravel(), x) for nu in (10, 20, 40)]
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 3 * rate ** 40 * np.linalg.cond(dense_schur(op))


def test_fgmres_full_with_oe_smoother():
    lat = Lattice(DISTINCT)
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.4, 126), 1.0, -0.2)
    b = _full_vec(lat, 127)
    omega = 0.8 / solvers.power_iteration(op.schur, rand_vec(lat.Vh, 128), 50)
    x, res = solvers.fgmres_full(op, b, 16, 30, 1e-10, 3, omega)
    assert res.converged
    assert solvers.vnorm(b - op.D(x)) <= 1e-10 * solvers.vnorm(b)
    # fewer outer steps than with the identity preconditioner on the full D
    res0 = solvers.gmres(op.D, b, np.zeros_like(b), 16, 60, 1e-10 * solvers.vnorm(b))
    assert res0.converged and res.iters < res0.iters
    # against the dense solve on a smaller lattice
    lat2 = Lattice((4, 4, 2, 2))
    op2 = WilsonClover(lat2, synth.gauge_field(lat2.dims, 0.3, 129), 1.0, -0.1)
    b2 = _full_vec(lat2, 130)
    x2, res2 = solvers.fgmres_full(op2, b2, 12, 40, 1e-12, 2, 0.2)
    assert res2.converged
    assert rel_err(x2.ravel(), np.linalg.solve(sparse_D(op2).toarray(), b2.ravel())) < 1e-10


# --------------------------------------------------------------------------
# P13 SAP(n, m) with block-local odd-even Minimal Residual (Sect. 2.4.1, Alg. 1)
# --------------------------------------------------------------------------
def _block_dofs(lat, in_block):
    sites = np.flatnonzero(in_block.ravel())
    return (12 * sites[:, None] + np.arange(12)[None, :]).ravel()


def test_minimal_residual_closed_form_and_orthogonality():
    # diagonal A, b along one axis: one step solves it exactly
    a = np.array([2.0 + 1.0j, 3.0, 0.5 - 0.25j])
    b = np.array([0.0, 0.0, 1.0 + 2.0j])
    x = solvers.minimal_residual(lambda v: a * v, b, 1)
    assert np.allclose(x, b / a, atol=1e-15)
    # a general step: the new residual is orthogonal to A r
    rng = np.random.default_rng(141)
    A = rng.normal(size=(20, 20)) + 1j * rng.normal(size=(20, 20)) + 8 * np.eye(20)
    b = rng.normal(size=20) + 1j * rng.normal(size=20)
    x1 = solvers.minimal_residual(lambda v: A @ v, b, 1)
    r1 = b - A @ x1
    assert abs(np.vdot(A @ b, r1)) < 1e-12 * np.linalg.norm(A @ b) * np.linalg.norm(b)
    norms = [np.linalg.norm(b - A @ solvers.minimal_residual(lambda v: A @ v, b, k)) for k in range(6)]
    assert all(norms[k + 1] <= norms[k] * (1 + 1e-14) for k in range(5))


def test_sap_blocks_and_colours():
    lat = Lattice((8, 4, 4, 8))
    idx, colour, nblk = solvers.sap_blocks(lat, (4, 4, 4, 4))
    assert nblk == 4 and sorted(np.bincount(idx.ravel())) == [256] * 4
    # the block of site (x, y, z, t) = (5, 1, 2, 6): block coordinates (1, 0, 0, 1), colour 0
    assert colour[idx[6, 2, 1, 5]] == 0 and idx[6, 2, 1, 5] == 1 + 2 * (0 + 1 * (0 + 1 * 1))
    # neighbouring blocks along x have different colours
    assert colour[idx[0, 0, 0, 0]] != colour[idx[0, 0, 0, 4]]


@pytest.mark.parametrize("block", [(2, 2, 2, 2), (4, 4, 2, 2)])
def test_block_solve_converges_to_dense_block_inverse(block):
    lat = Lattice((4, 4, 2, 2))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 142), 1.0, -0.1)
    D = sparse_D(op).toarray()
    idx, colour, nblk = solvers.sap_blocks(lat, block)
    r = _full_vec(lat, 143)
    for k in range(nblk):
        in_block = idx == k
        e = solvers.block_solve(op, in_block, r, 400)
        d = _block_dofs(lat, in_block)
        ek = np.linalg.solve(D[np.ix_(d, d)], r.ravel()[d])
        assert rel_err(e.ravel()[d], ek) < 1e-10
        assert np.all(e[~in_block] == 0)


def test_single_block_is_the_whole_operator():
    # one block covering the lattice keeps the couplings that wrap around it: D_kk = D
    lat = Lattice((4, 4, 2, 2))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 144), 1.0, -0.1)
    r = _full_vec(lat, 145)
    e = solvers.block_solve(op, np.ones(lat.shape, bool), r, 400)
    assert rel_err(e.ravel(), np.linalg.solve(sparse_D(op).toarray(), r.ravel())) < 1e-10


def test_sap_is_multiplicative_schwarz():
    # with converged block solves one SAP sweep is x1 = x0 + B_black (b - D x_h),
    # x_h = x0 + B_red (b - D x0), B_c = sum over blocks of colour c of P D_kk^-1 P^T
    lat = Lattice((4, 4, 2, 2))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 146), 1.0, -0.1)
    D = sparse_D(op).toarray()
    idx, colour, nblk = solvers.sap_blocks(lat, (2, 2, 2, 2))
    n = D.shape[0]
    B = [np.zeros((n, n), complex), np.zeros((n, n), complex)]
    for k in range(nblk):
        d = _block_dofs(lat, idx == k)
        B[colour[k]][np.ix_(d, d)] = np.linalg.inv(D[np.ix_(d, d)])
    b, x0 = _full_vec(lat, 147).ravel(), _full_vec(lat, 148).ravel()
    xh = x0 + B[0] @ (b - D @ x0)
    x1 = xh + B[1] @ (b - D @ xh)
    got = solvers.sap(op, b.reshape(lat.shape + (4, 3)), x0.reshape(lat.shape + (4, 3)), 1, 400, (2, 2, 2, 2))
    assert rel_err(got.ravel(), x1) < 1e-10


def _block_parity_dofs(lat, in_block):
    """dofs of the block's even and odd sites (a site is even when x + y + z + t is)"""
    par = np.indices(lat.shape).sum(axis=0) % 2
    return _block_dofs(lat, in_block & (par == 0)), _block_dofs(lat, in_block & (par == 1))


@pytest.mark.parametrize("block", [(2, 2, 2, 2), (4, 4, 2, 2)])
def test_block_solve_without_mr_steps_solves_only_the_odd_rows(block):
    """m = 0, the degenerate block solve of Alg. 1 with odd-even inside the blocks (Sect.
    2.4.5): no Minimal Residual step leaves e_e = 0, and the reconstruction of eq. 2 gives
    e_o = (D_oo^k)^-1 r_o, from the dense D of the lattice; zero outside the block."""
    lat = Lattice((4, 4, 2, 2))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 151), 1.0, -0.1)
    D = sparse_D(op).toarray()
    idx, colour, nblk = solvers.sap_blocks(lat, block)
    r = _full_vec(lat, 152)
    rv = r.ravel()
    for k in range(nblk):
        e_d, o_d = _block_parity_dofs(lat, idx == k)
        e = solvers.block_solve(op, idx == k, r, 0)
        assert np.all(e.ravel()[e_d] == 0) and np.all(e[~(idx == k)] == 0)
        assert rel_err(e.ravel()[o_d], np.linalg.solve(D[np.ix_(o_d, o_d)], rv[o_d])) < 1e-12


@pytest.mark.parametrize("block,m", [((2, 2, 2, 2), 1), ((2, 2, 2, 2), 2), ((4, 4, 2, 2), 1),
                                     ((4, 4, 2, 2), 2), ((4, 4, 2, 2), 3)])
def test_block_solve_at_few_mr_steps_is_block_odd_even_mr(block, m):
    """The block solve of SAP at the step counts a smoother uses (Sect. 2.4.5 on combining
    odd-even with SAP: MR on the Schur complement of each block).  From the dense D of the
    lattice: the block's four sub-blocks D_ee^k, D_eo^k, D_oe^k, D_oo^k (rows and columns of
    the block's even and odd sites), the block Schur complement S = D_ee^k - D_eo^k
    (D_oo^k)^-1 D_oe^k, m dense MR steps on S e_e = b~ from zero with b~ = r_e - D_eo^k
    (D_oo^k)^-1 r_o, and e_o = (D_oo^k)^-1 (r_o - D_oe^k e_e).  Also what holds for any m:
    the block's odd rows are solved exactly, and after one step the block's even residual
    is orthogonal to S b~ (the MR step's minimisation)."""
    lat = Lattice((4, 4, 2, 2))
    op = WilsonClover(lat, synth.gauge_field(lat.dims, 0.3, 149), 1.0, -0.1)
    D = sparse_D(op).toarray()
    idx, colour, nblk = solvers.sap_blocks(lat, block)
    r = _full_vec(lat, 150)
    rv = r.ravel()
    for k in range(nblk):
        e_d, o_d = _block_parity_dofs(lat, idx == k)
        Dee, Deo = D[np.ix_(e_d, e_d)], D[np.ix_(e_d, o_d)]
        Doe, Doo = D[np.ix_(o_d, e_d)], D[np.ix_(o_d, o_d)]
        Doo_inv = np.linalg.inv(Doo)
        S = Dee - Deo @ Doo_inv @ Doe
        bt = rv[e_d] - Deo @ (Doo_inv @ rv[o_d])
        xe, res = np.zeros_like(bt), bt.copy()
        for _ in range(m):
            q = S @ res
            alpha = np.vdot(q, res) / np.vdot(q, q)
            xe, res = xe + alpha * res, res - alpha * q
        xo = Doo_inv @ (rv[o_d] - Doe @ xe)
        e = solvers.block_solve(op, idx == k, r, m).ravel()
        assert rel_err(e[e_d], xe) < 1e-12 and rel_err(e[o_d], xo) < 1e-12
        # odd rows of the block system hold exactly, for any m
        assert rel_err(Doe @ e[e_d] + Doo @ e[o_d], rv[o_d]) < 1e-12
        if m == 1:
            # one step: e_e = alpha b~ with alpha = (S b~)^H b~ / |S b~|^2, whose residual is
            # orthogonal to S b~
            sb = S @ bt
            assert rel_err(e[e_d], (np.vdot(sb, bt) / np.vdot(sb, sb)) * bt) < 1e-12
            ree = rv[e_d] - Dee @ e[e_d] - Deo @ e[o_d]
            assert abs(np.vdot(sb, ree)) < 1e-12 * np.linalg.norm(sb) * np.linalg.norm(bt)
