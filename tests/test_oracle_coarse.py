"""Pins of the coarse-grid oracle (Sect. 2.3): P orthonormal and reproducing the test
vectors, the Galerkin identity D_c v = P^H D P v, gamma_5-hermiticity of D_c, and the
free-field closed form of its nine blocks (direction, normalisation, boundary sign)."""
import numpy as np
import pytest

from oracle import coarse
from oracle.dirac import GAMMA, Lattice, WilsonClover
from paper_2407_08092_amd import synth


def _setup(dims=(6, 6, 6, 6), agg=(2, 2, 2, 2), nv=4, eps=0.3, seed=601):
    lat = Lattice(dims)
    op = WilsonClover(lat, synth.gauge_field(dims, eps, seed), 1.0, -0.1)
    tv = [synth.gaussian_spinor(dims, seed + 1 + k) for k in range(nv)]
    return lat, op, coarse.Prolongation(lat, agg, tv), tv


def test_prolongation_orthonormal_and_spans_the_test_vectors():
    lat, op, P, tv = _setup()
    vc = synth.gaussian_complex((P.Vc, 2, P.nv), 611)
    assert np.allclose(P.restrict(P.prolong(vc)), vc, atol=1e-13)
    for t in tv:  # each test vector lies in range(P) (aggregate by aggregate, chirality by chirality)
        assert np.allclose(P.prolong(P.restrict(t)), t, atol=1e-12)


def test_galerkin_identity_and_gamma5_hermiticity():
    lat, op, P, tv = _setup()
    A = coarse.galerkin_blocks(op, P)
    vc = synth.gaussian_complex((P.Vc, 2, P.nv), 612)
    got = coarse.coarse_apply(A, P.cd, vc.reshape(P.Vc, -1)).reshape(vc.shape)
    assert np.allclose(got, P.restrict(op.D(P.prolong(vc))), atol=1e-12)
    # Gamma_5 = diag(+1 on chirality 0, -1 on chirality 1) per coarse site: Gamma_5 D_c hermitian
    n2 = 2 * P.nv
    Dc = np.zeros((P.Vc * n2, P.Vc * n2), complex)
    for x in range(P.Vc):
        for d in range(9):
            y = coarse.coarse_neighbour(P.cd, x, d)
            Dc[x * n2:(x + 1) * n2, y * n2:(y + 1) * n2] += A[x, d]
    g5 = np.tile(np.concatenate([np.ones(P.nv), -np.ones(P.nv)]), P.Vc)
    G = g5[:, None] * Dc
    assert np.allclose(G, G.conj().T, atol=1e-12)


def test_free_field_blocks_closed_form():
    # U = 1, constant test vectors t_k = e(s = k // 3, a = k % 3) + e(s = 2 + k // 3, a = k % 3):
    # on a 2^4 aggregate P maps (chirality c, k) to 1/4 e(s = 2c + k // 3, a = k % 3) on all 16
    # sites; 8 fine links cross each face, so the forward block is -1/4 (1 - gamma_mu), the
    # backward one -1/4 (1 + gamma_mu) (times -1 across the antiperiodic t boundary), and the
    # self block (4 + m0) - 4 x 1/2 = 2 + m0
    dims, m0 = (6, 6, 6, 6), -0.1
    lat = Lattice(dims)
    U = np.zeros(lat.shape + (4, 3, 3), complex)
    U[...] = np.eye(3)
    op = WilsonClover(lat, U, 1.0, m0)
    tv = []
    for k in range(6):
        t = np.zeros(lat.shape + (4, 3), complex)
        t[..., k // 3, k % 3] = 1.0
        t[..., 2 + k // 3, k % 3] = 1.0
        tv.append(t)
    P = coarse.Prolongation(lat, (2, 2, 2, 2), tv)
    for a in range(P.Vc):  # fix the QR signs to the constant vectors' own
        for c in range(2):
            P.Q[a][c] = P.Q[a][c] * np.sign(P.Q[a][c].sum(axis=0).real)
    A = coarse.galerkin_blocks(op, P)
    # coarse d.o.f. q = 6 c + k is spin 2c + k // 3, colour k % 3
    spin = np.array([2 * (q // 6) + (q % 6) // 3 for q in range(12)])
    col = np.array([(q % 6) % 3 for q in range(12)])
    same_colour = (col[:, None] == col[None, :])

    def spin_block(M4):
        return M4[np.ix_(spin, spin)] * same_colour

    I4 = np.eye(4)
    for x in range(P.Vc):
        assert np.allclose(A[x, 0], (2 + m0) * np.eye(12), atol=1e-12)
        ct = coarse.coarse_coords(P.cd, x)[3]
        for mu in range(4):
            sf = -1.0 if (mu == 3 and ct == P.cd[3] - 1) else 1.0
            sb = -1.0 if (mu == 3 and ct == 0) else 1.0
            assert np.allclose(A[x, 1 + 2 * mu], sf * spin_block(-0.25 * (I4 - GAMMA[mu])), atol=1e-12)
            assert np.allclose(A[x, 2 + 2 * mu], sb * spin_block(-0.25 * (I4 + GAMMA[mu])), atol=1e-12)


@pytest.mark.parametrize("nrhs", [1, 3])
def test_coarse_apply_plain_definition(nrhs):
    cd = (3, 4, 3, 5)
    Vc, n2 = int(np.prod(cd)), 8
    A = synth.gaussian_complex((Vc, 9, n2, n2), 621)
    v = synth.gaussian_complex((Vc, n2, nrhs), 622)
    y = coarse.coarse_apply(A, cd, v)
    # one site by hand: x = (1, 2, 0, 4)
    x = coarse.coarse_index(cd, [1, 2, 0, 4])
    nb = [coarse.coarse_index(cd, c) for c in ([1, 2, 0, 4], [2, 2, 0, 4], [0, 2, 0, 4], [1, 3, 0, 4],
                                                [1, 1, 0, 4], [1, 2, 1, 4], [1, 2, 2, 4], [1, 2, 0, 0],
                                                [1, 2, 0, 3])]
    assert np.allclose(y[x], sum(A[x, d] @ v[nb[d]] for d in range(9)), atol=1e-12)
