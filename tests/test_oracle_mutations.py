"""The pins have teeth: plausible mistakes planted in the oracle (on the CPU) must
make at least one pin fail.  Each mutant is patched in with monkeypatch and the
pin is expected to raise AssertionError."""
import numpy as np
import pytest

import test_oracle_pins as pins
from oracle import dirac


def _hop_swapped_projectors(lat, U, psi, adjoint=False):
    # mistake: (1 + gamma) on the forward hop, (1 - gamma) on the backward hop
    return _orig_hop(lat, U, psi, adjoint=not adjoint)


def _hop_undaggered_backward(lat, U, psi, adjoint=False):
    # mistake: U_mu(x - mu) instead of U_mu(x - mu)^H on the backward hop
    out = np.zeros_like(psi)
    for mu in range(4):
        fw = dirac._colour(U[..., mu, :, :], lat.fwd(psi, mu))
        out += fw - dirac._spin(dirac.GAMMA[mu], fw)
        bw = lat.bwd(dirac._colour(np.swapaxes(U[..., mu, :, :], -1, -2), psi), mu)
        out += bw + dirac._spin(dirac.GAMMA[mu], bw)
    return 0.5 * out


def _hop_no_half(lat, U, psi, adjoint=False):
    return 2.0 * _orig_hop(lat, U, psi, adjoint)


def _hop_axes_swapped(lat, U, psi, adjoint=False):
    # mistake: the link of direction mu paired with the shift along the next axis
    Us = U[..., [1, 0, 2, 3], :, :]
    return _orig_hop(lat, Us, psi, adjoint)


def _field_strength_quarter(lat, U):
    return {k: 2.0 * v for k, v in _orig_fs(lat, U).items()}


def _field_strength_reversed(lat, U):
    return {k: -v for k, v in _orig_fs(lat, U).items()}


def _field_strength_one_leaf(lat, U):
    out = {}
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Um, Un = U[..., mu, :, :], U[..., nu, :, :]
            S = lat.shift
            Q = 4 * Um @ S(Un, {mu: 1}) @ dirac.dag(S(Um, {nu: 1})) @ dirac.dag(Un)
            out[(mu, nu)] = (Q - dirac.dag(Q)) / 8.0
    return out


_orig_hop = dirac.hopping
_orig_fs = dirac.field_strength


@pytest.mark.parametrize("mutant,pin", [
    (_hop_swapped_projectors, lambda: pins.test_free_field_full_operator((1, 5, 7, 4))),
    (_hop_undaggered_backward, pins.test_pure_gauge),
    (_hop_undaggered_backward, pins.test_gamma5_hermiticity),
    (_hop_no_half, lambda: pins.test_free_field_schur((2, 5, 3, 7))),
    (_hop_axes_swapped, pins.test_gauge_covariance),
    (_hop_axes_swapped, pins.test_pure_gauge),
])
def test_hopping_mutants_caught(monkeypatch, mutant, pin):
    monkeypatch.setattr(dirac, "hopping", mutant)
    with pytest.raises(AssertionError):
        pin()


@pytest.mark.parametrize("mutant", [_field_strength_quarter, _field_strength_reversed])
def test_clover_normalisation_mutants_caught(monkeypatch, mutant):
    monkeypatch.setattr(dirac, "field_strength", mutant)
    with pytest.raises(AssertionError):
        pins.test_constant_abelian_clover(1)


def test_single_leaf_clover_caught(monkeypatch):
    # four times one leaf still agrees on a constant field; the leaf average
    # over a varying abelian field tells them apart
    monkeypatch.setattr(dirac, "field_strength", _field_strength_one_leaf)
    pins.test_constant_abelian_clover(1)
    with pytest.raises(AssertionError):
        pins.test_abelian_field_clover_leaf_average()


# odd-even smoother M_nu: a skipped prepare step, one sweep too few, a reconstruct
# that drops the D_oe x_e term
from oracle import solvers  # noqa: E402

_orig_richardson = solvers.richardson


def _smoother_no_prepare(op, nsweeps, omega):
    def M(r):
        be = op.lat.to_parity(r, 0)  # mistake: b_e instead of b~_e
        xe = solvers.richardson(op.schur, be, np.zeros_like(be), nsweeps, omega)
        return op.reconstruct(xe, r)
    return M


def _smoother_short(op, nsweeps, omega):
    return _orig_smoother(op, max(nsweeps - 1, 0), omega)


def _smoother_bad_reconstruct(op, nsweeps, omega):
    def M(r):
        bt = op.prepare(r)
        xe = solvers.richardson(op.schur, bt, np.zeros_like(bt), nsweeps, omega)
        x_o = op.D_oo_inv(op.lat.to_parity(r, 1))  # mistake: D_oe x_e dropped
        return op.lat.from_parity(xe, 0) + op.lat.from_parity(x_o, 1)
    return M


_orig_smoother = solvers.oe_smoother


@pytest.mark.parametrize("mutant,pin", [
    # a wrong outer factor (prepare or reconstruct) leaves D M similar to a block-
    # triangular matrix with the same diagonal blocks: the spectrum is unchanged, but
    # M_nu is no longer eq. 2's product and no longer tends to D^-1
    (_smoother_no_prepare, pins.test_oe_smoother_tends_to_inverse),
    (_smoother_no_prepare, pins.test_oe_smoother_matches_dense_factorisation),
    (_smoother_short, lambda: pins.test_oe_smoother_spectrum_closed_form(3)),
    (_smoother_short, pins.test_oe_smoother_matches_dense_factorisation),
    (_smoother_bad_reconstruct, pins.test_oe_smoother_tends_to_inverse),
    (_smoother_bad_reconstruct, pins.test_oe_smoother_matches_dense_factorisation),
])
def test_oe_smoother_mutants_caught(monkeypatch, mutant, pin):
    monkeypatch.setattr(solvers, "oe_smoother", mutant)
    with pytest.raises(AssertionError):
        pin()


# SAP: a block solve that keeps the hops leaving the block, a Minimal Residual step with
# the conjugated step length, a black pass that reuses the red pass's residual
_orig_block_solve = solvers.block_solve
_orig_mr = solvers.minimal_residual
_orig_sap = solvers.sap


def _block_solve_leaky(op, in_block, r, m):
    lat = op.lat
    me = lat.to_parity(in_block.astype(float)[..., None, None] * np.ones(lat.shape + (4, 3)), 0)
    mo = lat.to_parity(in_block.astype(float)[..., None, None] * np.ones(lat.shape + (4, 3)), 1)

    def S(v_e):  # mistake: the full lattice's hopping terms inside the block solve
        return me * op.schur(me * v_e)

    r_e, r_o = me * lat.to_parity(r, 0), mo * lat.to_parity(r, 1)
    bt = r_e - me * op.D_eo(op.D_oo_inv(r_o))
    x_e = solvers.minimal_residual(S, bt, m)
    x_o = mo * op.D_oo_inv(r_o - op.D_oe(x_e))
    return lat.from_parity(x_e, 0) + lat.from_parity(x_o, 1)


def _mr_conj(apply, b, m):
    x = np.zeros_like(b)
    r = np.array(b, dtype=np.complex128, copy=True)
    for _ in range(m):
        q = apply(r)
        alpha = solvers.vdot(r, q) / solvers.vdot(q, q)  # mistake: r^H q
        x = x + alpha * r
        r = r - alpha * q
    return x


def _sap_stale_residual(op, b, x0, n, m, block=(4, 4, 4, 4)):
    idx, colour, nblk = solvers.sap_blocks(op.lat, block)
    x = np.array(x0, dtype=np.complex128, copy=True)
    for _ in range(n):
        r = b - op.D(x)  # mistake: one residual for both colours
        for c in (0, 1):
            for k in range(nblk):
                if colour[k] == c:
                    x = x + solvers.block_solve(op, idx == k, r, m)
    return x


def _block_solve_unreduced(op, in_block, r, m):
    # mistake: Minimal Residual on the whole block system D_kk e = r_k, without the
    # odd-even reduction to the block's Schur complement (the converged limit is the same)
    lat = op.lat
    mask = in_block.astype(float)[..., None, None] * np.ones(lat.shape + (4, 3))

    def D_kk(v):
        return mask * op.D(mask * v)

    return solvers.minimal_residual(D_kk, mask * r, m)


@pytest.mark.parametrize("name,mutant,pin", [
    ("block_solve", _block_solve_leaky, lambda: pins.test_block_solve_converges_to_dense_block_inverse((2, 2, 2, 2))),
    ("block_solve", _block_solve_unreduced,
     lambda: pins.test_block_solve_at_few_mr_steps_is_block_odd_even_mr((4, 4, 2, 2), 1)),
    ("block_solve", _block_solve_unreduced,
     lambda: pins.test_block_solve_at_few_mr_steps_is_block_odd_even_mr((2, 2, 2, 2), 2)),
    ("minimal_residual", _mr_conj, pins.test_minimal_residual_closed_form_and_orthogonality),
    ("sap", _sap_stale_residual, pins.test_sap_is_multiplicative_schwarz),
])
def test_sap_mutants_caught(monkeypatch, name, mutant, pin):
    monkeypatch.setattr(solvers, name, mutant)
    with pytest.raises(AssertionError):
        pin()


# coarse operator: forward and backward neighbours swapped
from oracle import coarse  # noqa: E402
import test_oracle_coarse as cpins  # noqa: E402

_orig_cnb = coarse.coarse_neighbour


def _cnb_swapped(cd, i, d):
    if d == 0:
        return i
    return _orig_cnb(cd, i, d + 1 if (d - 1) % 2 == 0 else d - 1)


def test_coarse_direction_mutant_caught(monkeypatch):
    monkeypatch.setattr(coarse, "coarse_neighbour", _cnb_swapped)
    with pytest.raises(AssertionError):
        cpins.test_free_field_blocks_closed_form()


# coarse operator: restriction with the transpose instead of the conjugate transpose
def _restrict_transposed(self, f):
    ff = np.asarray(f).reshape(self.lat.V, 4, 3)
    vc = np.zeros((self.Vc, 2, self.nv), complex)
    for a in range(self.Vc):
        for c in range(2):
            vc[a, c] = self.Q[a][c].T @ ff[self.sites[a], 2 * c:2 * c + 2, :].reshape(-1)
    return vc


def test_coarse_restriction_transpose_mutant_caught(monkeypatch):
    monkeypatch.setattr(coarse.Prolongation, "restrict", _restrict_transposed)
    with pytest.raises(AssertionError):
        cpins.test_prolongation_orthonormal_and_spans_the_test_vectors()


# coarse operator: test vectors orthonormalised over all four spins at once (no chirality split)
_orig_pinit = coarse.Prolongation.__init__


def _init_no_chirality_split(self, lat, agg, test_vectors):
    _orig_pinit(self, lat, agg, test_vectors)
    T = np.stack([np.asarray(t).reshape(lat.V, 4, 3) for t in test_vectors], axis=-1)
    for a in range(self.Vc):
        q, _ = np.linalg.qr(T[self.sites[a]].reshape(-1, self.nv))
        q = q.reshape(len(self.sites[a]), 4, 3, self.nv)
        self.Q[a] = [q[:, 0:2].reshape(-1, self.nv), q[:, 2:4].reshape(-1, self.nv)]


def test_coarse_no_chirality_split_mutant_caught(monkeypatch):
    monkeypatch.setattr(coarse.Prolongation, "__init__", _init_no_chirality_split)
    with pytest.raises(AssertionError):
        cpins.test_prolongation_orthonormal_and_spans_the_test_vectors()


# coarse operator: Galerkin columns stored as rows
_orig_gal = coarse.galerkin_blocks


def _galerkin_transposed(op, P):
    return np.swapaxes(_orig_gal(op, P), 2, 3)


def test_coarse_galerkin_transposed_mutant_caught(monkeypatch):
    monkeypatch.setattr(coarse, "galerkin_blocks", _galerkin_transposed)
    with pytest.raises(AssertionError):
        cpins.test_galerkin_identity_and_gamma5_hermiticity()


# coarse operator: the apply leaves out the site's own block
def _apply_no_self(A, cd, v):
    y = np.zeros_like(v, dtype=complex)
    for x in range(A.shape[0]):
        for d in range(1, 9):
            y[x] = y[x] + A[x, d] @ v[coarse.coarse_neighbour(cd, x, d)]
    return y


@pytest.mark.parametrize("pin", ["test_galerkin_identity_and_gamma5_hermiticity", "test_coarse_apply_plain_definition"])
def test_coarse_apply_without_self_block_caught(monkeypatch, pin):
    monkeypatch.setattr(coarse, "coarse_apply", _apply_no_self)
    with pytest.raises(AssertionError):
        if pin == "test_coarse_apply_plain_definition":
            cpins.test_coarse_apply_plain_definition(3)
        else:
            cpins.test_galerkin_identity_and_gamma5_hermiticity()
