"""Pins of the molecular-dynamics oracle (oracle/hmc.py):

- the gauge action vanishes at U = 1 and takes its closed form on an abelian
  constant field (only the (x, y) plaquettes carry the angle phi);
- the gauge force matches central finite differences of the action along a
  random su(3) direction, is gauge covariant, and vanishes at U = 1;
- the exponential of an anti-Hermitian matrix equals scipy's expm (Pade),
  is unitary, and has unit determinant when traceless;
- the integrators are reversible (flip P, integrate back) and their energy
  violation falls as the step squared (both second order), Omelyan's below
  leapfrog's at the same step;
- with the even-odd Wilson pseudofermion: reversibility and the step-squared
  fall of the energy violation.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import gauge_exp, gauge_transform, gauge_unit, gaussian_parity_spinor, random_su3_algebra

pytest.importorskip("torch")
from oracle import hmc  # noqa: E402

BC = (1.0, 1.0, 1.0, -1.0)


def test_gauge_action_unit_and_abelian_closed_form():
    dims = (4, 6, 4, 4)
    assert abs(hmc.gauge_action(gauge_unit(dims), 5.5)) < 1e-12
    lx = dims[0]
    phi = 2 * np.pi * 1 / lx
    U = gauge_unit(dims).copy()
    x = np.arange(lx)
    # U_y(x) = diag(e^{i phi x}, e^{-i phi x}, 1): P_xy = diag(e^{i phi}, e^{-i phi}, 1) everywhere
    U[..., 1, 0, 0] = np.exp(1j * phi * x)
    U[..., 1, 1, 1] = np.exp(-1j * phi * x)
    V = int(np.prod(dims))
    beta = 5.5
    want = beta * V * (2.0 / 3.0) * (1.0 - np.cos(phi))
    assert abs(hmc.gauge_action(U, beta) - want) < 1e-10 * want


def test_gauge_force_finite_differences_and_covariance():
    dims = (4, 4, 4, 4)
    beta = 5.5
    U = gauge_exp(dims, 0.4, 401)
    S, M, G = hmc.gauge_force(U, beta)
    assert abs(S - hmc.gauge_action(U, beta)) < 1e-10 * abs(S)
    X = random_su3_algebra(dims, 402)
    eps = 1e-5
    fd = (hmc.gauge_action(hmc.expm_ah(eps * X) @ U, beta) - hmc.gauge_action(hmc.expm_ah(-eps * X) @ U, beta)) / (2 * eps)
    pred = float(np.sum(np.real(np.conj(G) * X)))
    assert abs(fd - pred) < 1e-7 * max(1.0, abs(pred))
    Om = gauge_transform(dims, 403)
    Ut = np.empty_like(U)
    for mu in range(4):
        Ut[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(np.roll(Om, -1, axis=3 - mu), -1, -2))
    St, _, Gt = hmc.gauge_force(Ut, beta)
    expect = Om[..., None, :, :] @ G @ np.conj(np.swapaxes(Om, -1, -2))[..., None, :, :]
    assert abs(S - St) < 1e-11 * abs(S)
    assert np.linalg.norm(Gt - expect) / np.linalg.norm(expect) < 1e-11
    _, _, G1 = hmc.gauge_force(gauge_unit(dims), beta)
    assert np.abs(G1).max() < 1e-13


def test_expm_matches_pade_and_is_special_unitary():
    scipy_linalg = pytest.importorskip("scipy.linalg")
    X = random_su3_algebra((2, 2, 2, 2), 411) * 1.7
    E = hmc.expm_ah(X)
    ref = np.stack([scipy_linalg.expm(x) for x in X.reshape(-1, 3, 3)]).reshape(E.shape)
    assert np.abs(E - ref).max() < 1e-13
    eye = np.eye(3)
    assert np.abs(E @ np.conj(np.swapaxes(E, -1, -2)) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(E) - 1).max() < 1e-13


@pytest.mark.parametrize("integrator", ["leapfrog", "omelyan"])
def test_pure_gauge_reversible_and_second_order(integrator):
    dims = (4, 4, 4, 4)
    U0 = gauge_exp(dims, 0.3, 421)
    P0 = random_su3_algebra(dims, 422)
    act = hmc.Action(dims, 5.5)
    U1, P1, H0, H1 = hmc.trajectory(act, U0, P0, 0.2, 8, integrator)
    U2, P2, _, _ = hmc.trajectory(act, U1, -P1, 0.2, 8, integrator)
    assert np.abs(U2 - U0).max() < 1e-12 and np.abs(P2 + P0).max() < 1e-12
    dH = [sum(hmc.trajectory(act, U0, P0, 0.2, n, integrator)[3]) - sum(H0) for n in (8, 16)]
    ratio = abs(dH[0] / dH[1])
    assert 3.7 < ratio < 4.3, (dH, ratio)
    if integrator == "omelyan":
        dH_lf = sum(hmc.trajectory(act, U0, P0, 0.2, 8, "leapfrog")[3]) - sum(H0)
        assert abs(dH[0]) < abs(dH_lf)


def test_with_wilson_pseudofermion_reversible_and_second_order():
    dims = (4, 4, 4, 4)
    U0 = gauge_exp(dims, 0.3, 431)
    P0 = random_su3_algebra(dims, 432)
    phi = gaussian_parity_spinor(dims, 433)
    act = hmc.Action(dims, 5.5, fermion=(0.12, 0.0, BC, True), phi=phi, tol=1e-14)
    U1, P1, H0, H1 = hmc.trajectory(act, U0, P0, 0.3, 4, "leapfrog")
    U2, P2, _, _ = hmc.trajectory(act, U1, -P1, 0.3, 4, "leapfrog")
    assert np.abs(U2 - U0).max() < 1e-11 and np.abs(P2 + P0).max() < 1e-11
    dH = [sum(hmc.trajectory(act, U0, P0, 0.3, n, "leapfrog")[3]) - sum(H0) for n in (4, 8)]
    ratio = abs(dH[0] / dH[1])
    assert 3.3 < ratio < 4.7, (dH, ratio)
