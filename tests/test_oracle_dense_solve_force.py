"""Brute-force pins of the oracle on tiny lattices.

- the matrix-free C oracle equals the dense N x N matrix assembled entry by
  entry from eq. (1) (Sec. 3) in numpy (an independent writing, with its own
  gamma matrices and clover term from path products and sigma_{mu nu});
- even-odd Schur decomposition: det D = det A_oo det M and the reconstructed
  even-odd solution equals the dense LU solution;
- the textbook solvers (CG on the normal equations, BiCGStab) reach the
  dense solution x = D^-1 b, the quantity a propagator solve computes (the
  paper's Fig. 1 loop over the 12 spin-colour sources);
- pseudofermion force: the exact S from the dense matrix, central finite
  differences along random su(3) directions, and gauge covariance.
"""
import numpy as np
import pytest

import oracle
from oracle.dense import clover_site, dense_dirac, parity_index
from lattice_inputs import (gauge_exp, gauge_haar, gauge_transform, gaussian_parity_spinor, gaussian_spinor,
                            random_su3_algebra, WORKLOADS, workload_gauge, workload_source, ANTIPERIODIC_T)

BC = (1.0, np.exp(0.9j), 1.0, -1.0)


@pytest.mark.parametrize("dims,csw", [((2, 2, 2, 2), 0.0), ((2, 2, 2, 2), 1.4), ((4, 2, 2, 4), 1.1),
                                      ((4, 4, 4, 4), 1.0)])
def test_matrix_free_equals_dense(dims, csw):
    U = gauge_haar(dims, 71)
    kappa = 0.13
    D = dense_dirac(dims, U, kappa, csw, BC)
    op = oracle.Operator(dims, U, kappa, csw, BC)
    psi = gaussian_spinor(dims, 72)
    assert np.allclose(op.D(psi).reshape(-1), D @ psi.reshape(-1), atol=1e-12)
    assert np.allclose(op.Ddag(psi).reshape(-1), D.conj().T @ psi.reshape(-1), atol=1e-12)


def test_clover_dense_writing_matches():
    dims = (4, 2, 4, 2)
    U = gauge_exp(dims, 0.7, 81)
    F = oracle.clover(dims, U, 1.7, 0.135)
    for lex in (0, 9, 31, 63):
        x = lex % 4
        y = (lex // 4) % 2
        z = (lex // 8) % 4
        t = lex // 32
        assert np.allclose(F[lex], clover_site(U, dims, (x, y, z, t), 1.7, 0.135), atol=1e-15)


def test_even_odd_determinant_and_reconstruction():
    dims = (2, 2, 2, 4)
    U = gauge_haar(dims, 91)
    kappa, csw = 0.14, 1.5
    D = dense_dirac(dims, U, kappa, csw, BC)
    ie = parity_index(dims, 0)
    io = parity_index(dims, 1)
    Aee = D[np.ix_(ie, ie)]
    Aoo = D[np.ix_(io, io)]
    Deo = D[np.ix_(ie, io)]
    Doe = D[np.ix_(io, ie)]
    Mhat = Aee - Deo @ np.linalg.solve(Aoo, Doe)
    s1, l1 = np.linalg.slogdet(D)
    s2, l2 = np.linalg.slogdet(Aoo)
    s3, l3 = np.linalg.slogdet(Mhat)
    assert abs(l1 - (l2 + l3)) < 1e-10 and abs(s1 - s2 * s3) < 1e-10
    op = oracle.Operator(dims, U, kappa, csw, BC)
    xe = gaussian_parity_spinor(dims, 92)
    assert np.allclose(op.schur(xe).reshape(-1), Mhat @ xe.reshape(-1), atol=1e-12)
    assert np.allclose(op.schur_dag(xe).reshape(-1), Mhat.conj().T @ xe.reshape(-1), atol=1e-12)
    b = gaussian_spinor(dims, 93)
    x_dense = np.linalg.solve(D, b.reshape(-1))
    x, _ = oracle.solve_eo(op, b, tol=1e-13)
    assert np.linalg.norm(x.reshape(-1) - x_dense) < 1e-11 * np.linalg.norm(x_dense)


def test_solvers_on_random_hpd_system():
    rng = np.random.default_rng(5)
    n = 60
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = a @ a.conj().T + n * np.eye(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it = oracle.cg(lambda v: A @ v, b, 1e-13)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-11 * np.linalg.norm(x)
    B = A + 5j * np.diag(rng.standard_normal(n))
    x, it = oracle.bicgstab(lambda v: B @ v, b, 1e-13)
    assert np.linalg.norm(x - np.linalg.solve(B, b)) < 1e-11 * np.linalg.norm(x)
    x, it = oracle.bicgstab(lambda v: B @ v, np.zeros(n, complex), 1e-13)
    assert it == 0 and not np.any(x)


@pytest.mark.parametrize("method", ["bicgstab", "cg"])
def test_workload_4x4x4x4_solve_matches_dense(method):
    """The 4^4 Haar-random Wilson workload: kappa = 0.12, antiperiodic in time."""
    w = WORKLOADS["wilson_4x4x4x4"]
    dims = w["dims"]
    U = workload_gauge("wilson_4x4x4x4")
    b = workload_source("wilson_4x4x4x4")
    D = dense_dirac(dims, U, w["kappa"], 0.0, ANTIPERIODIC_T)
    x_dense = np.linalg.solve(D, b.reshape(-1))
    op = oracle.Operator(dims, U, w["kappa"], 0.0, ANTIPERIODIC_T)
    x, _ = oracle.solve_eo(op, b, tol=1e-12, method=method)
    assert oracle.true_residual(op, x, b) < 1e-12
    assert np.linalg.norm(x.reshape(-1) - x_dense) < 1e-11 * np.linalg.norm(x_dense)
    # full-lattice CG on D^dag D
    xf, _ = oracle.cg(op.DdagD, op.Ddag(b), 1e-13)
    assert oracle.true_residual(op, xf, b) < 1e-12


def _expm_su3(X):
    w, v = np.linalg.eig(X)
    return (v * np.exp(w)[..., None, :]) @ np.linalg.inv(v)


def test_force_exact_action_dense():
    dims = (2, 2, 2, 4)
    U = gauge_exp(dims, 0.4, 101)
    kappa = 0.125
    op = oracle.Operator(dims, U, kappa, 0.0, BC)
    phi = gaussian_parity_spinor(dims, 102)
    D = dense_dirac(dims, U, kappa, 0.0, BC)
    ie, io = parity_index(dims, 0), parity_index(dims, 1)
    M = D[np.ix_(ie, ie)] - D[np.ix_(ie, io)] @ np.linalg.solve(D[np.ix_(io, io)], D[np.ix_(io, ie)])
    S_dense = np.vdot(phi.reshape(-1), np.linalg.solve(M.conj().T @ M, phi.reshape(-1))).real
    S, _ = oracle.pf_action_eo(op, phi)
    assert abs(S - S_dense) < 1e-11 * abs(S_dense)


@pytest.mark.parametrize("variant", ["eo", "full"])
def test_force_finite_difference(variant):
    dims = (4, 2, 2, 4)
    U = gauge_exp(dims, 0.3, 111)
    kappa = 0.125
    op = oracle.Operator(dims, U, kappa, 0.0, BC)
    if variant == "eo":
        phi = gaussian_parity_spinor(dims, 112)
        S0, Mraw, G = oracle.pf_force_eo(op, phi, tol=1e-14)

        def action(Uv):
            return oracle.pf_action_eo(oracle.Operator(dims, Uv, kappa, 0.0, BC), phi, tol=1e-14)[0]
    else:
        phi = gaussian_spinor(dims, 112)
        S0, Mraw, G = oracle.pf_force_full(op, phi, tol=1e-14)

        def action(Uv):
            o = oracle.Operator(dims, Uv, kappa, 0.0, BC)
            X, _ = oracle.cg(o.DdagD, phi, 1e-14)
            return np.vdot(phi, X).real
    for seed in (113, 114):
        X = random_su3_algebra(dims, seed)
        h = 1e-5
        Sp = action(_expm_su3(h * X) @ U)
        Sm = action(_expm_su3(-h * X) @ U)
        fd = (Sp - Sm) / (2 * h)
        pred = np.sum(np.einsum("...ab,...ab->...", np.conj(G), X).real)
        assert abs(fd - pred) < 1e-7 * max(1.0, abs(pred)), (fd, pred)
        # raw derivative: dS = sum Re tr(M dU) with dU = X U
        pred_raw = np.sum(np.einsum("...ab,...bc,...ca->...", Mraw, X, U).real)
        assert abs(pred_raw - pred) < 1e-9 * max(1.0, abs(pred))


def test_force_gauge_covariance():
    dims = (4, 2, 2, 4)
    U = gauge_exp(dims, 0.3, 121)
    Om = gauge_transform(dims, 122)
    Ut = np.empty_like(U)
    for mu in range(4):
        Om_fwd = np.roll(Om, -1, axis=3 - mu)
        Ut[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(Om_fwd, -1, -2))
    kappa = 0.125
    phi = gaussian_parity_spinor(dims, 123)
    op = oracle.Operator(dims, U, kappa, 0.0, BC)
    opt = oracle.Operator(dims, Ut, kappa, 0.0, BC)
    phi_full = oracle.from_parity(dims, phi, 0)
    phit = oracle.to_parity(dims, np.einsum("...ab,...sb->...sa", Om, phi_full), 0)
    S, _, G = oracle.pf_force_eo(op, phi, tol=1e-14)
    St, _, Gt = oracle.pf_force_eo(opt, phit, tol=1e-14)
    assert abs(S - St) < 1e-11 * abs(S)
    expect = Om[..., None, :, :] @ G @ np.conj(np.swapaxes(Om, -1, -2))[..., None, :, :]
    assert np.allclose(Gt, expect, atol=1e-10)
    # G is traceless anti-Hermitian
    assert np.allclose(G, -np.conj(np.swapaxes(G, -1, -2)), atol=1e-15)
    assert np.allclose(np.trace(G, axis1=-2, axis2=-1), 0, atol=1e-14)
