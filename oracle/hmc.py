"""Hybrid Monte Carlo molecular dynamics for the gauge-field generation of
Sec. 2 (the Monte Carlo that produces the ensembles on which the solves of
eq. (1) run): the Wilson plaquette gauge action, its force, the
pseudofermion action of the even-odd fermion matrix, and the leapfrog and
Omelyan (second-order minimum-norm) integrators of the equations of motion
dU/dt = P U, dP/dt = -G with G the su(3) force.

TEST INFRASTRUCTURE ONLY.  Plain numpy / torch CPU in FP64, written from the
definitions:

  gauge action   S_g = beta sum_x sum_{mu<nu} (1 - Re tr P_{mu nu}(x) / 3),
                 P_{mu nu}(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag;
  its force      G = -TA(U M) with M the torch autograd gradient of S_g
                 (dS = sum Re tr(M dU)), as for the fermion forces;
  kinetic term   T = 1/2 sum_{x,mu} tr(P^dag P);
  link update    U <- exp(e P) U, with exp of an anti-Hermitian matrix from
                 the eigendecomposition of the Hermitian matrix i X.

The integrators are written step by step as their definitions read (no
merging of consecutive momentum updates).  Random numbers (momenta,
pseudofermion sources) are inputs.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Operator, cg, pf_force_eo, traceless_antihermitian
from . import force_clover as _fc

_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}  # direction mu -> axis of [t, z, y, x]


def _h(a):
    return np.conj(np.swapaxes(a, -1, -2))


def plaquette_sum(U) -> float:
    """sum_x sum_{mu<nu} Re tr P_{mu nu}(x)."""
    tot = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a, b = U[..., mu, :, :], U[..., nu, :, :]
            p = a @ np.roll(b, -1, axis=_AXIS[mu]) @ _h(np.roll(a, -1, axis=_AXIS[nu])) @ _h(b)
            tot += float(np.trace(p, axis1=-2, axis2=-1).real.sum())
    return tot


def gauge_action(U, beta) -> float:
    V = int(np.prod(U.shape[:4]))
    return float(beta) * (6.0 * V - plaquette_sum(U) / 3.0)


def _gauge_action_torch(Ut, beta):
    tot = torch.zeros((), dtype=torch.float64)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a, b = Ut[..., mu, :, :], Ut[..., nu, :, :]
            p = a @ torch.roll(b, -1, dims=_AXIS[mu]) @ torch.roll(a, -1, dims=_AXIS[nu]).conj().transpose(-1, -2) \
                @ b.conj().transpose(-1, -2)
            tot = tot + torch.diagonal(p, dim1=-2, dim2=-1).sum().real
    V = int(np.prod(Ut.shape[:4]))
    return float(beta) * (6.0 * V - tot / 3.0)


def gauge_force(U, beta):
    """(S_g, Mraw, G) of the Wilson gauge action: dS_g = sum Re tr(Mraw dU),
    G = -TA(U Mraw)."""
    Ut = torch.from_numpy(np.ascontiguousarray(U, dtype=np.complex128)).clone().requires_grad_(True)
    S = _gauge_action_torch(Ut, beta)
    S.backward()
    g = Ut.grad.detach().numpy()
    Mraw = _h(g)
    return float(S.detach()), Mraw, -traceless_antihermitian(np.asarray(U) @ Mraw)


def expm_ah(X):
    """exp(X) for anti-Hermitian X (last two axes): iX = V diag(w) V^dag,
    exp(X) = V diag(exp(-i w)) V^dag."""
    w, v = np.linalg.eigh(1j * X)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(-1j * w), v.conj())


def kinetic(P) -> float:
    return 0.5 * float(np.sum(np.abs(P) ** 2))


class Action:
    """S(U) = S_g(U) + S_f(U) and its force, for a fixed pseudofermion phi on
    the even sites (fermion=None: pure gauge).  fermion = (kappa, csw, bc,
    traceless); S_f = phi^dag (M^dag M)^-1 phi with the even-odd M."""

    def __init__(self, dims, beta, fermion=None, phi=None, tol=1e-13):
        self.dims = tuple(int(v) for v in dims)
        self.beta = float(beta)
        self.fermion = fermion
        self.phi = phi
        self.tol = tol
        self.n_force = 0

    def value(self, U):
        S = gauge_action(U, self.beta)
        Sf = 0.0
        if self.fermion is not None:
            kappa, csw, bc, traceless = self.fermion
            op = Operator(self.dims, U, kappa, csw, bc, traceless)
            X, _ = cg(op.schur_normal, self.phi, self.tol)
            Sf = float(np.vdot(self.phi.reshape(-1), X.reshape(-1)).real)
        return S, Sf

    def force(self, U):
        """(S_g, S_f, G) at U."""
        self.n_force += 1
        Sg, _, G = gauge_force(U, self.beta)
        Sf = 0.0
        if self.fermion is not None:
            kappa, csw, bc, traceless = self.fermion
            if csw == 0.0:
                Sf, _, Gf = pf_force_eo(Operator(self.dims, U, kappa, 0.0, bc), self.phi, self.tol)
            else:
                Sf, _, Gf = _fc.pf_force_clover_mf(self.dims, U, kappa, csw, bc, self.phi, "eo", traceless, self.tol)
            G = G + Gf
        return Sg, Sf, G


def leapfrog(action, U, P, tau, nsteps):
    """Each step: P half step, U full step, P half step."""
    e = tau / nsteps
    for _ in range(nsteps):
        P = P - 0.5 * e * action.force(U)[2]
        U = expm_ah(e * P) @ U
        P = P - 0.5 * e * action.force(U)[2]
    return U, P


OMELYAN_LAMBDA = 0.1931833275037836


def omelyan(action, U, P, tau, nsteps, lam=OMELYAN_LAMBDA):
    """Each step: P by lam e, U by e/2, P by (1 - 2 lam) e, U by e/2, P by lam e."""
    e = tau / nsteps
    for _ in range(nsteps):
        P = P - lam * e * action.force(U)[2]
        U = expm_ah(0.5 * e * P) @ U
        P = P - (1.0 - 2.0 * lam) * e * action.force(U)[2]
        U = expm_ah(0.5 * e * P) @ U
        P = P - lam * e * action.force(U)[2]
    return U, P


def trajectory(action, U, P, tau, nsteps, integrator="leapfrog"):
    """Molecular-dynamics trajectory; returns (U, P, H0 parts, H1 parts) with
    parts = (T, S_g, S_f)."""
    Sg0, Sf0 = action.value(U)
    T0 = kinetic(P)
    if integrator == "leapfrog":
        U1, P1 = leapfrog(action, U, P, tau, nsteps)
    else:
        U1, P1 = omelyan(action, U, P, tau, nsteps)
    Sg1, Sf1 = action.value(U1)
    return U1, P1, (T0, Sg0, Sf0), (kinetic(P1), Sg1, Sf1)
