"""Pins of the oracle's twisted-mass Wilson operator D = 1 - kappa H +
i tau gamma_5 (another discretisation of the Wilson family; Sec. 4 lists
further fermion types among the framework's operators).

- U = 1: with a = 1 - 2 kappa sum cos p_mu and b_mu = 2 kappa sin p_mu,
  D - a = i (sum b_mu gamma_mu + tau gamma_5) on a plane wave, and since
  gamma_5 anticommutes with every gamma_mu, (D - a)^2 = -(|b|^2 + tau^2):
  the eigenvalues are a +- i sqrt(|b|^2 + tau^2), each six times; checked
  against the dense matrix's eigenvalues on 4^4 and 2^4 x 4^2 lattices.
- gamma_5 D(tau) gamma_5 = D(-tau)^dag on a random gauge field (the
  relation the dagger of the twisted operator satisfies in place of
  gamma_5-hermiticity), with D^dag coded separately in the oracle.
- the matrix-free oracle equals the dense entrywise writing of eq. (1) plus
  the twist, and the even-odd solve through the Schur operator equals the
  dense solve.
"""
import numpy as np
import pytest

import oracle
from oracle.dense import dense_dirac, parity_index
from lattice_inputs import gauge_exp, gauge_haar, gauge_unit, gaussian_spinor


@pytest.mark.parametrize("dims,tau,kappa", [((4, 4, 4, 4), 0.3, 0.12), ((2, 4, 2, 4), -0.7, 0.2)])
def test_free_field_twisted_spectrum_closed_form(dims, tau, kappa):
    bc = (1, 1, 1, -1)
    U = gauge_unit(dims)
    D = dense_dirac(dims, U, kappa, 0.0, bc, twist=tau)
    def canon(z):  # sorted by rounded (re, im): degenerate eigenvalues differ only by rounding
        z = np.asarray(z)
        return z[np.lexsort((np.round(z.imag, 8), np.round(z.real, 8)))]
    ev = canon(np.linalg.eigvals(D))
    want = []
    for n in np.ndindex(*dims):
        p = [(2 * np.pi * n[mu] + (np.pi if mu == 3 else 0.0)) / dims[mu] for mu in range(4)]
        a = 1 - 2 * kappa * sum(np.cos(p))
        r = np.sqrt(sum((2 * kappa * np.sin(q)) ** 2 for q in p) + tau ** 2)
        want += [a + 1j * r] * 6 + [a - 1j * r] * 6
    want = canon(want)
    assert np.abs(ev - want).max() < 1e-10


def test_gamma5_relation_of_the_dagger():
    dims, kappa, tau = (4, 4, 2, 4), 0.13, 0.4
    U = gauge_haar(dims, 1501)
    psi = gaussian_spinor(dims, 2501)
    g5 = lambda v: v * np.asarray([1, 1, -1, -1])[:, None]  # noqa: E731
    plus = oracle.Operator(dims, U, kappa, bc=(1, 1, 1, -1), twist=tau)
    minus = oracle.Operator(dims, U, kappa, bc=(1, 1, 1, -1), twist=-tau)
    lhs = g5(plus.D(g5(psi)))
    rhs = minus.Ddag(psi)
    assert np.linalg.norm(lhs - rhs) < 1e-13 * np.linalg.norm(rhs)
    # and the twist really enters: D(tau) differs from D(-tau)
    assert np.linalg.norm(plus.D(psi) - minus.D(psi)) > 0.1 * np.linalg.norm(psi)


@pytest.mark.parametrize("csw", [0.0])
def test_matrix_free_equals_dense_and_even_odd_solve(csw):
    dims, kappa, tau = (2, 2, 4, 2), 0.15, 0.25
    bc = (1, 1, 1, -1)
    U = gauge_exp(dims, 0.5, 1502)
    ref = oracle.Operator(dims, U, kappa, csw, bc, twist=tau)
    D = dense_dirac(dims, U, kappa, csw, bc, twist=tau)
    psi = gaussian_spinor(dims, 2502)
    assert np.linalg.norm(ref.D(psi).reshape(-1) - D @ psi.reshape(-1)) < 1e-13 * np.linalg.norm(psi)
    assert np.linalg.norm(ref.Ddag(psi).reshape(-1) - D.conj().T @ psi.reshape(-1)) < 1e-13 * np.linalg.norm(psi)
    # M = A_ee - kappa^2 H_eo A_oo^-1 H_oe and its dagger against the dense blocks
    e, o = parity_index(dims, 0), parity_index(dims, 1)
    M = D[np.ix_(e, e)] - D[np.ix_(e, o)] @ np.linalg.solve(D[np.ix_(o, o)], D[np.ix_(o, e)])
    xe = oracle.to_parity(dims, psi, 0)
    assert np.linalg.norm(ref.schur(xe).reshape(-1) - M @ xe.reshape(-1)) < 1e-12 * np.linalg.norm(xe)
    assert np.linalg.norm(ref.schur_dag(xe).reshape(-1) - M.conj().T @ xe.reshape(-1)) < 1e-12 * np.linalg.norm(xe)
    # the even-odd solve reconstructs the dense solution
    b = gaussian_spinor(dims, 2503)
    x, _ = oracle.solve_eo(ref, b, tol=1e-13)
    xd = np.linalg.solve(D, b.reshape(-1))
    assert np.linalg.norm(x.reshape(-1) - xd) < 1e-11 * np.linalg.norm(xd)
