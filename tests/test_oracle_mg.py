"""Pins of the multigrid oracle (oracle/mg.py) against what the construction
fixes:

- the prolongator's columns are orthonormal, each lies in one aggregate and
  one chirality (P commutes with gamma_5), and per aggregate and chirality
  they are the modified Gram-Schmidt basis of the vectors in order: the
  vectors' coefficients in it form an upper-triangular matrix with a
  positive real diagonal;
- the Galerkin operator inherits gamma_5-hermiticity: with Gamma_5 = +1 on
  chirality-0 and -1 on chirality-1 coarse degrees of freedom,
  Gamma_5 D_c Gamma_5 = D_c^dag (D is gamma_5-hermitian, P commutes with
  gamma_5);
- the matrix-free block columns equal the dense P^dag D P (dense D entry by
  entry from eq. (1), oracle/dense.py);
- twisted mass: P^dag (D + i tau gamma_5) P = P^dag D P + i tau Gamma_5
  (P^dag P = 1 and gamma_5 P = P Gamma_5), the twisted coarse operator
  satisfies Gamma_5 D_c(tau) Gamma_5 = D_c(-tau)^dag, and its matrix-free
  columns (oracle Operator with the twist) equal the dense ones;
- free field (unit links, periodic), block-constant vectors e_{s,c}: the
  coarse operator in closed form -- on the aggregate itself
  1 - 2 kappa sum_mu (1 - 1/b_mu), to the aggregate at -mu (it couples
  through the +mu hops of its face) -(kappa / b_mu)(1 - gamma_mu), to the one
  at +mu -(kappa / b_mu)(1 + gamma_mu), nothing to the others.
"""
import numpy as np

import oracle
from lattice_inputs import gauge_exp, gauge_unit, gaussian_spinor
from oracle import mg
from oracle.dense import dense_dirac

BC = (1.0, np.exp(0.3j), 1.0, -1.0)


def _gamma5_fine(n_sites):
    g5 = np.diag([1.0, 1.0, -1.0, -1.0])
    return np.kron(np.eye(n_sites), np.kron(g5, np.eye(3)))


def test_prolongator_orthonormal_chiral_and_gram_schmidt():
    dims, block, nv = (4, 4, 4, 4), (2, 2, 2, 2), 3
    V = gaussian_spinor(dims, 9101, nv)
    W = mg.block_orthonormalize(dims, block, V)
    P = mg.prolongator(dims, block, W)
    assert np.allclose(P.conj().T @ P, np.eye(P.shape[1]), atol=1e-13)
    # gamma_5 P = P Gamma_5
    nagg = P.shape[1] // (2 * nv)
    G5c = np.kron(np.eye(nagg), np.diag([1.0] * nv + [-1.0] * nv))
    assert np.allclose(_gamma5_fine(256) @ P, P @ G5c, atol=1e-14)
    # Gram-Schmidt order: per aggregate / chirality, V's parts = W's parts R
    # with R upper triangular, positive real diagonal
    agg = mg.aggregate_map(dims, block)
    for A in (0, 7, 15):
        for chi in range(2):
            sl = slice(2 * chi, 2 * chi + 2)
            Q = np.stack([W[k][agg == A][:, sl, :].reshape(-1) for k in range(nv)], axis=1)
            X = np.stack([V[k][agg == A][:, sl, :].reshape(-1) for k in range(nv)], axis=1)
            R = Q.conj().T @ X
            assert np.allclose(np.tril(R, -1), 0, atol=1e-12)
            assert np.all(np.abs(np.diag(R).imag) < 1e-12) and np.all(np.diag(R).real > 0)
            assert np.allclose(Q @ R, X, atol=1e-12)


def test_galerkin_operator_is_gamma5_hermitian_and_matches_columns():
    dims, block, nv = (4, 4, 4, 4), (2, 2, 2, 2), 2
    kappa, csw = 0.12, 1.3
    U = gauge_exp(dims, 0.5, 9201)
    W = mg.block_orthonormalize(dims, block, gaussian_spinor(dims, 9202, nv))
    P = mg.prolongator(dims, block, W)
    D = dense_dirac(dims, U, kappa, csw, BC)
    Dc = mg.galerkin(D, P)
    nagg = P.shape[1] // (2 * nv)
    G5c = np.kron(np.eye(nagg), np.diag([1.0] * nv + [-1.0] * nv))
    assert np.allclose(G5c @ Dc @ G5c, Dc.conj().T, atol=1e-12)
    assert not np.allclose(Dc, Dc.conj().T, atol=1e-3)  # not Hermitian itself
    # matrix-free block column of aggregate 5 = the dense one
    ref = oracle.Operator(dims, U, kappa, csw, BC)
    cols = mg.coarse_columns(ref.D, dims, block, W, 5)
    n2 = 2 * nv
    for B in range(nagg):
        assert np.allclose(cols[B], Dc[B * n2:(B + 1) * n2, 5 * n2:6 * n2], atol=1e-12)


def test_free_field_coarse_operator_closed_form():
    dims, block = (8, 4, 4, 4), (2, 2, 2, 2)
    kappa = 0.11
    nv = 6
    # v_k = e_{spin k//3, colour k%3} + e_{spin 2 + k//3, colour k%3} on every site
    shape = tuple(dims[::-1]) + (4, 3)
    V = np.zeros((nv,) + shape, dtype=np.complex128)
    for k in range(nv):
        V[k][..., k // 3, k % 3] = 1.0
        V[k][..., 2 + k // 3, k % 3] = 1.0
    W = mg.block_orthonormalize(dims, block, V)
    ref = oracle.Operator(dims, gauge_unit(dims), kappa, 0.0, (1, 1, 1, 1))
    cdims = mg.coarse_dims(dims, block)
    A0 = 1 + cdims[0] * (1 + cdims[1] * (0 + cdims[2] * 1))  # aggregate (1, 1, 0, 1)
    cols = mg.coarse_columns(ref.D, dims, block, W, A0)

    def spin_block(M4):
        # coarse dof r = chi * 6 + k  <->  spin 2 chi + k // 3, colour k % 3
        out = np.zeros((12, 12), dtype=np.complex128)
        for r in range(12):
            for c in range(12):
                (rc, rk), (cc, ck) = divmod(r, 6), divmod(c, 6)
                if rk % 3 == ck % 3:
                    out[r, c] = M4[2 * rc + rk // 3, 2 * cc + ck // 3]
        return out

    I4 = np.eye(4)
    expect = {A0: spin_block((1 - 2 * kappa * sum(1 - 1 / b for b in block)) * I4)}
    for mu in range(4):
        g = oracle.gamma(mu)
        minus = mg.neighbour(cdims, A0, 2 + 2 * mu)  # the aggregate at -mu
        plus = mg.neighbour(cdims, A0, 1 + 2 * mu)
        blk_m = spin_block(-(kappa / block[mu]) * (I4 - g))
        blk_p = spin_block(-(kappa / block[mu]) * (I4 + g))
        expect[minus] = expect.get(minus, 0) + blk_m
        expect[plus] = expect.get(plus, 0) + blk_p
    nagg = cols.shape[0]
    for B in range(nagg):
        want = expect.get(B, np.zeros((12, 12)))
        assert np.allclose(cols[B], want, atol=1e-13), B
    # the x direction (coarse extent 4) separates the two sides
    assert mg.neighbour(cdims, A0, 1) != mg.neighbour(cdims, A0, 2)


def test_twisted_galerkin_adds_i_tau_gamma5():
    dims, block, nv = (4, 4, 4, 4), (2, 2, 2, 2), 2
    kappa, tau = 0.125, 0.3
    U = gauge_exp(dims, 0.5, 9251)
    W = mg.block_orthonormalize(dims, block, gaussian_spinor(dims, 9252, nv))
    P = mg.prolongator(dims, block, W)
    Dc0 = mg.galerkin(dense_dirac(dims, U, kappa, 0.0, BC), P)
    Dcp = mg.galerkin(dense_dirac(dims, U, kappa, 0.0, BC, twist=tau), P)
    Dcm = mg.galerkin(dense_dirac(dims, U, kappa, 0.0, BC, twist=-tau), P)
    nagg = P.shape[1] // (2 * nv)
    G5c = np.kron(np.eye(nagg), np.diag([1.0] * nv + [-1.0] * nv))
    assert np.allclose(Dcp, Dc0 + 1j * tau * G5c, atol=1e-12)
    assert np.allclose(G5c @ Dcp @ G5c, Dcm.conj().T, atol=1e-12)
    assert not np.allclose(G5c @ Dcp @ G5c, Dcp.conj().T, atol=1e-3)
    ref = oracle.Operator(dims, U, kappa, 0.0, BC, twist=tau)
    cols = mg.coarse_columns(ref.D, dims, block, W, 3)
    n2 = 2 * nv
    for B in range(nagg):
        assert np.allclose(cols[B], Dcp[B * n2:(B + 1) * n2, 3 * n2:4 * n2], atol=1e-12)
