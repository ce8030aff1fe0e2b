"""Pins of the oracle against the algebra and the free-field closed form.

- gamma matrices: Clifford algebra, hermiticity, gamma_5 diagonal in the
  chiral basis, rank-2 projectors (1 -/+ gamma_mu)/2.
- U = 1: plane waves are eigenvectors of eq. (1) (Sec. 3) with
  D e^{ipx} u = e^{ipx} [1 - 2 kappa sum cos p_mu + 2 i kappa sum gamma_mu sin p_mu] u,
  p_mu = (2 pi n_mu + theta_mu) / L_mu for a boundary phase e^{i theta_mu};
  the even-odd Schur operator of the Wilson matrix has the eigenvalue
  1 - kappa^2 h^2 on the even-site restriction of the same wave, where h is
  an eigenvalue of 2 sum cos p - 2 i sum gamma sin p.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import gauge_unit


def test_clifford_and_hermiticity():
    g = [oracle.gamma(mu) for mu in range(4)]
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2.0 * (mu == nu) * np.eye(4), atol=0)


def test_gamma5_chiral_diagonal():
    g5 = oracle.gamma(4)
    assert np.array_equal(g5, np.diag([1, 1, -1, -1]).astype(complex))
    for mu in range(4):
        assert np.allclose(g5 @ oracle.gamma(mu) + oracle.gamma(mu) @ g5, 0, atol=0)


def test_projectors_rank_two():
    for mu in range(4):
        g = oracle.gamma(mu)
        for s in (+1, -1):
            P = 0.5 * (np.eye(4) + s * g)
            assert np.allclose(P @ P, P, atol=1e-15)
            assert np.linalg.matrix_rank(P) == 2


def test_oracle_gammas_match_independent_dense_writing():
    from oracle.dense import chiral_gammas
    g, g5 = chiral_gammas()
    for mu in range(4):
        assert np.array_equal(oracle.gamma(mu), g[mu])
    assert np.array_equal(oracle.gamma(4), g5)


def _plane_wave(dims, n, theta, u):
    lx, ly, lz, lt = dims
    p = [(2 * np.pi * n[mu] + theta[mu]) / dims[mu] for mu in range(4)]
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return phase[..., None, None] * u.reshape(4, 3)[None, None, None, None], p


@pytest.mark.parametrize("dims,theta", [
    ((4, 4, 4, 4), (0.0, 0.0, 0.0, np.pi)),
    ((4, 2, 6, 8), (0.3, -1.1, 2.0, np.pi)),
    ((2, 2, 2, 2), (0.0, 0.7, 0.0, np.pi)),
])
def test_free_field_plane_waves(dims, theta):
    rng = np.random.default_rng(7)
    kappa = 0.137
    bc = [np.exp(1j * th) for th in theta]
    U = gauge_unit(dims)
    g = [oracle.gamma(mu) for mu in range(4)]
    for trial in range(6):
        n = [int(rng.integers(0, d)) for d in dims]
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi, p = _plane_wave(dims, n, theta, u)
        spin = (1 - 2 * kappa * sum(np.cos(p))) * np.eye(4) + 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))
        expect = np.einsum("st,...tc->...sc", spin, psi)
        got = oracle.dirac(dims, U, bc, kappa, psi)
        assert np.allclose(got, expect, atol=1e-13, rtol=0)
        spin_d = (1 - 2 * kappa * sum(np.cos(p))) * np.eye(4) - 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))
        got_d = oracle.dirac(dims, U, bc, kappa, psi, dagger=True)
        assert np.allclose(got_d, np.einsum("st,...tc->...sc", spin_d, psi), atol=1e-13, rtol=0)


def test_free_field_spectrum_dense_eigenvalues():
    """All 12 V eigenvalues of the dense free operator on 2^2 x 4 x 4
    (antiperiodic in t) are the closed-form ones, each 6-fold."""
    from oracle.dense import dense_dirac
    dims = (2, 2, 4, 4)
    kappa = 0.11
    bc = (1, 1, 1, -1)
    D = dense_dirac(dims, gauge_unit(dims), kappa, 0.0, bc)
    ev = np.sort_complex(np.round(np.linalg.eigvals(D), 12))
    expect = []
    theta = (0, 0, 0, np.pi)
    for n0 in range(dims[0]):
        for n1 in range(dims[1]):
            for n2 in range(dims[2]):
                for n3 in range(dims[3]):
                    n = (n0, n1, n2, n3)
                    p = [(2 * np.pi * n[m] + theta[m]) / dims[m] for m in range(4)]
                    re = 1 - 2 * kappa * sum(np.cos(p))
                    im = 2 * kappa * np.sqrt(sum(np.sin(q) ** 2 for q in p))
                    expect += [re + 1j * im] * 6 + [re - 1j * im] * 6
    expect = np.sort_complex(np.round(np.asarray(expect), 12))
    assert np.allclose(ev, expect, atol=1e-10)


def test_free_field_even_odd_schur_eigenvalue():
    dims = (4, 4, 4, 8)
    theta = (0.0, 0.0, 0.0, np.pi)
    bc = [np.exp(1j * th) for th in theta]
    kappa = 0.124
    op = oracle.Operator(dims, gauge_unit(dims), kappa, 0.0, bc)
    g = [oracle.gamma(mu) for mu in range(4)]
    rng = np.random.default_rng(3)
    for trial in range(4):
        n = [int(rng.integers(0, d)) for d in dims]
        p = [(2 * np.pi * n[mu] + theta[mu]) / dims[mu] for mu in range(4)]
        Hp = 2 * sum(np.cos(p)) * np.eye(4) - 2j * sum(g[m] * np.sin(p[m]) for m in range(4))
        w, vecs = np.linalg.eig(Hp)
        for k in range(4):
            u = np.outer(vecs[:, k], rng.standard_normal(3) + 1j * rng.standard_normal(3))
            psi, _ = _plane_wave(dims, n, theta, u)
            xe = oracle.to_parity(dims, psi, 0)
            got = op.schur(xe)
            assert np.allclose(got, (1 - kappa ** 2 * w[k] ** 2) * xe, atol=1e-12)
