"""Pins of the clover pseudofermion-force oracle (oracle/force_clover.py),
which takes the force as the autograd gradient of a dense action:

- its dense D equals the matrix-free C oracle's D (itself pinned by the free
  field, gamma-5 hermiticity, covariance and the abelian closed form) on a
  lattice with an extent-2 direction and a complex boundary phase;
- at c_sw = 0 the even-odd and full-lattice forces equal the Wilson forces of
  oracle/__init__.py, which are written out from the hopping-term derivative
  (an independent formula);
- central finite differences of the action along a random su(3) direction
  (both variants, traceless and not);
- gauge covariance: G[U^Omega, Omega phi](x) = Omega(x) G[U, phi](x) Omega(x)^dag;
- the matrix-free variant (C-oracle solve, autograd of the bilinear only)
  equals the dense one, and at c_sw = 0 the hand-written Wilson forces.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import (gauge_exp, gauge_transform, gaussian_parity_spinor, gaussian_spinor,
                            random_su3_algebra)

torch = pytest.importorskip("torch")
from oracle import force_clover as fc  # noqa: E402

BC = (1.0, 1.0, 1.0, -1.0)


def _expm_ah(X):
    """exp(X) for anti-Hermitian 3x3 X (eigendecomposition of the Hermitian iX)."""
    w, v = np.linalg.eigh(1j * X)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(-1j * w), v.conj())


def _transform_links(U, Om):
    out = np.empty_like(U)
    for mu in range(4):
        ax = 3 - mu
        out[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(np.roll(Om, -1, axis=ax), -1, -2))
    return out


def test_dense_torch_operator_equals_c_oracle():
    dims = (4, 4, 2, 4)
    bc = (1.0, np.exp(0.3j), 1.0, -1.0)
    U = gauge_exp(dims, 0.5, 71)
    psi = gaussian_spinor(dims, 72)
    for csw, traceless in ((1.3, True), (0.8, False), (0.0, True)):
        D = fc.dense_dirac_torch(torch.from_numpy(U), dims, 0.13, csw, bc, traceless).numpy()
        ref = oracle.Operator(dims, U, 0.13, csw, bc, traceless)
        got = (D @ psi.reshape(-1)).reshape(psi.shape)
        want = ref.D(psi)
        assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-14


def test_reduces_to_wilson_force_at_csw_zero():
    dims = (4, 4, 4, 4)
    U = gauge_exp(dims, 0.4, 81)
    ref = oracle.Operator(dims, U, 0.125, 0.0, BC)
    phi = gaussian_parity_spinor(dims, 82)
    S, M, G = fc.pf_force_clover(dims, U, 0.125, 0.0, BC, phi, "eo")
    Sw, Mw, Gw = oracle.pf_force_eo(ref, phi, tol=1e-14)
    assert abs(S - Sw) < 1e-11 * abs(Sw)
    assert np.linalg.norm(M - Mw) / np.linalg.norm(Mw) < 1e-10
    phif = gaussian_spinor(dims, 83)
    S, M, G = fc.pf_force_clover(dims, U, 0.125, 0.0, BC, phif, "full")
    Sw, Mw, Gw = oracle.pf_force_full(ref, phif, tol=1e-14)
    assert abs(S - Sw) < 1e-11 * abs(Sw)
    assert np.linalg.norm(M - Mw) / np.linalg.norm(Mw) < 1e-10


@pytest.mark.parametrize("variant,traceless", [("eo", True), ("full", True), ("eo", False)])
def test_force_matches_finite_differences(variant, traceless):
    dims = (4, 4, 4, 4)
    kappa, csw = 0.12, 1.7
    U = gauge_exp(dims, 0.4, 91)
    phi = gaussian_parity_spinor(dims, 92) if variant == "eo" else gaussian_spinor(dims, 92)
    S, M, G = fc.pf_force_clover(dims, U, kappa, csw, BC, phi, variant, traceless)
    X = random_su3_algebra(dims, 93)
    eps = 1e-5
    Sp = fc.pf_action_clover(dims, _expm_ah(eps * X) @ U, kappa, csw, BC, phi, variant, traceless)
    Sm = fc.pf_action_clover(dims, _expm_ah(-eps * X) @ U, kappa, csw, BC, phi, variant, traceless)
    fd = (Sp - Sm) / (2 * eps)
    pred = float(np.sum(np.real(np.conj(G) * X)))
    assert abs(fd - pred) < 1e-7 * max(1.0, abs(pred))
    # the raw matrix gives the same derivative: dS = sum Re tr(M dU), dU = X U
    pred_m = float(np.sum(np.real(np.trace(M @ (X @ U), axis1=-2, axis2=-1))))
    assert abs(pred_m - pred) < 1e-9 * max(1.0, abs(pred))


def test_force_gauge_covariant():
    dims = (4, 4, 4, 4)
    kappa, csw = 0.12, 1.7
    U = gauge_exp(dims, 0.4, 101)
    Om = gauge_transform(dims, 102)
    phi = gaussian_spinor(dims, 103)
    S, M, G = fc.pf_force_clover(dims, U, kappa, csw, BC, phi, "full")
    St, Mt, Gt = fc.pf_force_clover(dims, _transform_links(U, Om), kappa, csw, BC,
                                    np.einsum("...ab,...sb->...sa", Om, phi), "full")
    expect = Om[..., None, :, :] @ G @ np.conj(np.swapaxes(Om, -1, -2))[..., None, :, :]
    assert abs(S - St) < 1e-11 * abs(S)
    assert np.linalg.norm(Gt - expect) / np.linalg.norm(expect) < 1e-10


@pytest.mark.parametrize("dims,variant,traceless", [((4, 4, 4, 4), "eo", True), ((4, 4, 2, 6), "full", False)])
def test_matrix_free_equals_dense(dims, variant, traceless):
    bc = (1.0, np.exp(0.3j), 1.0, -1.0)
    U = gauge_exp(dims, 0.4, 111)
    phi = gaussian_parity_spinor(dims, 112) if variant == "eo" else gaussian_spinor(dims, 112)
    S, M, G = fc.pf_force_clover(dims, U, 0.12, 1.7, bc, phi, variant, traceless)
    S2, M2, G2 = fc.pf_force_clover_mf(dims, U, 0.12, 1.7, bc, phi, variant, traceless)
    assert abs(S - S2) < 1e-12 * abs(S)
    assert np.linalg.norm(M - M2) / np.linalg.norm(M) < 1e-11
    assert np.linalg.norm(G - G2) / np.linalg.norm(G) < 1e-11


def test_matrix_free_reduces_to_wilson():
    dims = (4, 4, 4, 6)
    bc = (1.0, np.exp(0.3j), 1.0, -1.0)
    U = gauge_exp(dims, 0.4, 121)
    ref = oracle.Operator(dims, U, 0.125, 0.0, bc)
    phi = gaussian_parity_spinor(dims, 122)
    S, M, G = fc.pf_force_clover_mf(dims, U, 0.125, 0.0, bc, phi, "eo")
    Sw, Mw, Gw = oracle.pf_force_eo(ref, phi, tol=1e-13)
    assert abs(S - Sw) < 1e-11 * abs(Sw)
    assert np.linalg.norm(M - Mw) / np.linalg.norm(Mw) < 1e-10


@pytest.mark.parametrize("variant", ["eo", "full"])
def test_twisted_mass_force_matches_finite_differences(variant):
    """Twisted mass (A = 1 + i tau gamma_5, no clover): the autograd force
    of the dense action against central finite differences, and the
    matrix-free force against the dense one; the twist term does not depend
    on the links, so the force changes with tau only through X and Y."""
    dims = (4, 4, 4, 4)
    kappa, tau = 0.125, 0.3
    U = gauge_exp(dims, 0.4, 191)
    phi = gaussian_parity_spinor(dims, 192) if variant == "eo" else gaussian_spinor(dims, 192)
    S, M, G = fc.pf_force_clover(dims, U, kappa, 0.0, BC, phi, variant, twist=tau)
    X = random_su3_algebra(dims, 193)
    eps = 1e-5
    Sp = fc.pf_action_clover(dims, _expm_ah(eps * X) @ U, kappa, 0.0, BC, phi, variant, twist=tau)
    Sm = fc.pf_action_clover(dims, _expm_ah(-eps * X) @ U, kappa, 0.0, BC, phi, variant, twist=tau)
    fd = (Sp - Sm) / (2 * eps)
    pred = float(np.sum(np.real(np.conj(G) * X)))
    assert abs(fd - pred) < 1e-7 * max(1.0, abs(pred))
    S2, M2, G2 = fc.pf_force_clover_mf(dims, U, kappa, 0.0, BC, phi, variant, twist=tau)
    assert abs(S - S2) < 1e-12 * abs(S)
    assert np.linalg.norm(G - G2) / np.linalg.norm(G) < 1e-11
    # the twist changes the action and the force
    S0, _, G0 = fc.pf_force_clover(dims, U, kappa, 0.0, BC, phi, variant)
    assert abs(S0 - S) > 1e-3 * abs(S) and np.linalg.norm(G - G0) > 1e-3 * np.linalg.norm(G)
