"""Pins of the oracle against symmetries and closed forms of eq. (1) (Sec. 3).

- gamma_5-hermiticity: D^dag = gamma_5 D gamma_5 (D^dag is coded separately,
  not as gamma_5 D gamma_5) and <chi, D psi> = <D^dag chi, psi>;
- gauge covariance: D[U^Omega](Omega psi) = Omega D[U] psi with
  U^Omega_mu(x) = Omega(x) U_mu(x) Omega(x+mu)^dag, and F -> Omega F Omega^dag;
- clover term (the paper: a 12x12 Hermitian matrix made of the links):
  Hermitian, zero at U = 1, block diagonal in the chiral basis, and equal to
  the closed form for abelian fields: for a constant field phi in the x-y
  plane, F = c_sw kappa sin(phi) sigma_12 (x) diag(-1, 1, 0); for diagonal
  U(1)^2 links, colour component c of Fhat_{mu nu}(x) is (i/4) times the sum
  of the sines of the four plaquette angles.
- clover inverse: A A^-1 = 1, and singular blocks are reported.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import (gauge_abelian_twist, gauge_exp, gauge_haar, gauge_transform, gauge_u1_diag,
                            gauge_unit, gaussian_spinor)

BC = (1.0, np.exp(0.4j), 1.0, -1.0)


def _gamma5_full(psi):
    g5 = oracle.gamma(4)
    return np.einsum("st,...tc->...sc", g5, psi)


@pytest.mark.parametrize("csw", [0.0, 1.3])
def test_gamma5_hermiticity(csw):
    dims = (4, 2, 4, 6)
    U = gauge_haar(dims, 11)
    op = oracle.Operator(dims, U, 0.13, csw, BC)
    psi = gaussian_spinor(dims, 12)
    chi = gaussian_spinor(dims, 13)
    assert np.allclose(op.Ddag(psi), _gamma5_full(op.D(_gamma5_full(psi))), atol=1e-13)
    lhs = np.vdot(chi, op.D(psi))
    rhs = np.vdot(op.Ddag(chi), psi)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def _transform_links(U, Om):
    Ut = np.empty_like(U)
    for mu in range(4):
        axis = 3 - mu
        Om_fwd = np.roll(Om, -1, axis=axis)
        Ut[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(Om_fwd, -1, -2))
    return Ut


@pytest.mark.parametrize("csw", [0.0, 1.7])
def test_gauge_covariance(csw):
    dims = (4, 4, 2, 6)
    U = gauge_exp(dims, 0.6, 21)
    Om = gauge_transform(dims, 22)
    Ut = _transform_links(U, Om)
    psi = gaussian_spinor(dims, 23)
    # periodic phases: a gauge transformation commutes with constant phases too
    op = oracle.Operator(dims, U, 0.12, csw, BC)
    opt = oracle.Operator(dims, Ut, 0.12, csw, BC)
    Om_psi = np.einsum("...ab,...sb->...sa", Om, psi)
    lhs = opt.D(Om_psi)
    rhs = np.einsum("...ab,...sb->...sa", Om, op.D(psi))
    assert np.allclose(lhs, rhs, atol=1e-12)
    if csw:
        F = op.F.reshape(-1, 4, 3, 4, 3)
        Ft = opt.F.reshape(-1, 4, 3, 4, 3)
        O = Om.reshape(-1, 3, 3)
        expect = np.einsum("xab,xsbtc,xdc->xsatd", O, F, np.conj(O))
        assert np.allclose(Ft, expect, atol=1e-13)


def test_clover_hermitian_blockdiag_and_unit():
    dims = (4, 4, 4, 4)
    F = oracle.clover(dims, gauge_haar(dims, 31), 1.9, 0.14)
    assert np.allclose(F, np.conj(np.swapaxes(F, -1, -2)), atol=1e-15)
    F4 = F.reshape(-1, 4, 3, 4, 3)
    assert np.allclose(F4[:, :2, :, 2:, :], 0, atol=0)
    assert np.allclose(F4[:, 2:, :, :2, :], 0, atol=0)
    # colour-traceless for every spin pair
    assert np.allclose(np.einsum("xsata->xst", F4), 0, atol=1e-15)
    assert np.max(np.abs(F)) > 0.05
    F1 = oracle.clover(dims, gauge_unit(dims), 1.9, 0.14)
    assert np.max(np.abs(F1)) == 0.0


@pytest.mark.parametrize("n_flux", [1, 2, 3])
def test_clover_abelian_constant_field(n_flux):
    dims = (8, 4, 2, 2)
    csw, kappa = 1.7, 0.13
    phi = 2 * np.pi * n_flux / dims[0]
    F = oracle.clover(dims, gauge_abelian_twist(dims, n_flux), csw, kappa, traceless=True)
    g = [oracle.gamma(mu) for mu in range(4)]
    sigma12 = 0.5j * (g[0] @ g[1] - g[1] @ g[0])
    expect = csw * kappa * np.sin(phi) * np.kron(sigma12, np.diag([-1.0, 1.0, 0.0]))
    assert np.allclose(F, expect[None], atol=1e-15)


def test_clover_abelian_plaquette_angles():
    """Diagonal links: every leaf is a product of phases; check Fhat colour
    by colour against the plaquette-angle sum (no trace removal)."""
    dims = (4, 2, 4, 2)
    U = gauge_u1_diag(dims, 41, amp=0.8)
    csw, kappa = 1.0, 0.125
    F = oracle.clover(dims, U, csw, kappa, traceless=False).reshape(dims[::-1] + (4, 3, 4, 3))
    ang = np.angle(np.stack([U[..., :, c, c] for c in range(3)], axis=-1))  # [t,z,y,x,mu,c]
    g = [oracle.gamma(mu) for mu in range(4)]

    def sh(a, mu, d):
        return np.roll(a, -d, axis=3 - mu)

    expect = np.zeros_like(F)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a_mu = ang[..., mu, :]
            a_nu = ang[..., nu, :]

            def plaq(base_mu, base_nu):
                # plaquette angle of the square with lower-left corner x + base
                am = sh(sh(a_mu, mu, base_mu), nu, base_nu)
                an = sh(sh(a_nu, mu, base_mu), nu, base_nu)
                return am + sh(an, mu, 1) - sh(am, nu, 1) - an

            s = sum(np.sin(plaq(bm, bn)) for bm, bn in ((0, 0), (-1, 0), (-1, -1), (0, -1)))
            Fh = 0.25j * s  # [t,z,y,x,c], diagonal in colour
            gg = g[mu] @ g[nu]
            for c in range(3):
                expect[..., :, c, :, c] += -csw * kappa * gg[None, None, None, None] * Fh[..., c, None, None]
    assert np.allclose(F, expect, atol=1e-14)


def test_clover_inverse_and_singular():
    dims = (4, 4, 2, 2)
    op = oracle.Operator(dims, gauge_haar(dims, 51), 0.13, 1.5, BC)
    prod = np.einsum("xij,xjk->xik", op.A, op.Ainv)
    assert np.allclose(prod, np.eye(12)[None], atol=1e-13)
    M = np.tile(np.eye(12, dtype=complex), (3, 1, 1))
    M[1, 5, :] = M[1, 4, :]  # two equal rows
    inv, nsing = oracle.site_invert(M)
    assert nsing == 1
    assert np.array_equal(inv[1], np.zeros((12, 12)))
    assert np.allclose(inv[0], np.eye(12)) and np.allclose(inv[2], np.eye(12))


def test_sites_variants_match_full():
    dims = (4, 4, 4, 2)
    U = gauge_haar(dims, 61)
    op = oracle.Operator(dims, U, 0.12, 1.1, BC)
    psi = gaussian_spinor(dims, 62)
    full = op.D(psi).reshape(-1, 4, 3)
    sites = np.array([0, 5, 17, 100, 127])
    got = oracle.dirac_sites(dims, U, BC, 0.12, psi, sites, op.F)
    assert np.array_equal(got, full[sites])
    Fs = oracle.clover_sites(dims, U, 1.1, 0.12, sites)
    assert np.array_equal(Fs, op.F[sites])
    # the per-site hopping sum, both signs, against the full-lattice one
    for dag in (False, True):
        hfull = op.H(psi, dagger=dag).reshape(-1, 4, 3)
        hs = oracle.hop_sites(dims, U, BC, psi, sites, dagger=dag)
        assert np.array_equal(hs, hfull[sites])
    # and on a lattice with extent-2 directions (coincident neighbours summed),
    # every site, against D = A - kappa H rearranged: H = (A psi - D psi) / kappa
    dims2 = (2, 4, 2, 4)
    U2 = gauge_haar(dims2, 63)
    psi2 = gaussian_spinor(dims2, 64)
    op2 = oracle.Operator(dims2, U2, 0.2, 0.0, BC)
    all_sites = np.arange(oracle.volume(dims2))
    for dag in (False, True):
        d = (op2.Ddag if dag else op2.D)(psi2).reshape(-1, 4, 3)
        hs = oracle.hop_sites(dims2, U2, BC, psi2, all_sites, dagger=dag)
        assert np.allclose(hs, (psi2.reshape(-1, 4, 3) - d) / 0.2, rtol=0, atol=1e-13)
