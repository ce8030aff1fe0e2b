"""Pseudofermion force of the HIP library (lq_pf_force) against the oracle
gradient, central finite differences of the GPU action along random su(3)
directions, gauge covariance, and the autograd.Function wrapper.

Tolerances: FP64 force with an FP64 solve to 1e-12 matches the oracle to
1e-9 relative (the solution error bound cond * 1e-12 with cond < 20, plus
rounding); the FP32 force kernel after a mixed solve to 1e-12 matches to
1e-5; finite differences with step 1e-5 agree to 1e-6 relative
(O(h^2) truncation plus solve error / h).
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import (ANTIPERIODIC_T, WORKLOADS, gauge_exp, gauge_transform, gaussian_parity_spinor,
                            gaussian_spinor, random_su3_algebra, workload_gauge)
from tests.gpu_common import announce, have_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lq():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


BC = (1.0, np.exp(0.3j), 1.0, -1.0)
DIMS = (4, 4, 4, 8)
KAPPA = 0.125


def _expm(X):
    w, v = np.linalg.eig(X)
    return (v * np.exp(w)[..., None, :]) @ np.linalg.inv(v)


@pytest.fixture(scope="module")
def case():
    U = gauge_exp(DIMS, 0.3, 1301)
    phi_e = gaussian_parity_spinor(DIMS, 2301)
    phi = gaussian_spinor(DIMS, 2302)
    ref = oracle.Operator(DIMS, U, KAPPA, 0.0, BC)
    return U, phi_e, phi, ref


@pytest.mark.parametrize("variant", ["eo", "full"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_force_matches_oracle(lq, case, variant, prec):
    U, phi_e, phi, ref = case
    announce("force: variant=%s prec=%s" % (variant, prec))
    if variant == "eo":
        S_ref, M_ref, G_ref = oracle.pf_force_eo(ref, phi_e, tol=1e-14)
        src = phi_e
    else:
        S_ref, M_ref, G_ref = oracle.pf_force_full(ref, phi, tol=1e-14)
        src = phi
    op = lq.Operator(DIMS, KAPPA, 0.0, BC)
    op.set_gauge(to_dev(U))
    prm = lq.SolverParams(solver="cgne", tol=1e-12, inner="f64" if prec == "f64" else "f32")
    S, grad, G, X, st = lq.pf_force(op, to_dev(src), prm, variant, prec, want_x=True)
    tol = 1e-9 if prec == "f64" else 1e-5
    grad = to_host(grad)
    G = to_host(G)
    announce("  S %.12e (oracle %.12e) iters %d diff %.1e | grad err %.2e G err %.2e" %
             (S, S_ref, st.nconv, st.diff, rel_err(grad, np.conj(np.swapaxes(M_ref, -1, -2))), rel_err(G, G_ref)))
    assert st.converged and st.diff <= 1e-12
    assert abs(S - S_ref) < 1e-10 * abs(S_ref)
    assert rel_err(grad, np.conj(np.swapaxes(M_ref, -1, -2))) < tol
    assert rel_err(G, G_ref) < tol
    op.close()


def test_force_finite_differences_of_gpu_action(lq, case):
    U, phi_e, _, _ = case
    op = lq.Operator(DIMS, KAPPA, 0.0, BC)
    prm = lq.SolverParams(solver="cgne", tol=1e-13, inner="f64")

    def action(Uv):
        op.set_gauge(to_dev(Uv))
        return lq.pf_force(op, to_dev(phi_e), prm)[0]

    op.set_gauge(to_dev(U))
    _, _, G, _, _ = lq.pf_force(op, to_dev(phi_e), prm)
    G = to_host(G)
    for seed in (1401, 1402):
        X = random_su3_algebra(DIMS, seed)
        h = 1e-5
        fd = (action(_expm(h * X) @ U) - action(_expm(-h * X) @ U)) / (2 * h)
        pred = float(np.sum(np.einsum("...ab,...ab->...", np.conj(G), X).real))
        announce("  FD %.10e  predicted %.10e" % (fd, pred))
        assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred))
    op.close()


def test_force_gauge_covariance(lq, case):
    U, phi_e, _, _ = case
    Om = gauge_transform(DIMS, 1501)
    Ut = np.empty_like(U)
    for mu in range(4):
        Ut[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(np.roll(Om, -1, axis=3 - mu), -1, -2))
    phit = oracle.to_parity(DIMS, np.einsum("...ab,...sb->...sa", Om, oracle.from_parity(DIMS, phi_e, 0)), 0)
    op = lq.Operator(DIMS, KAPPA, 0.0, BC)
    prm = lq.SolverParams(solver="cgne", tol=1e-13, inner="f64")
    op.set_gauge(to_dev(U))
    S, _, G, _, _ = lq.pf_force(op, to_dev(phi_e), prm)
    op.set_gauge(to_dev(Ut))
    St, _, Gt, _, _ = lq.pf_force(op, to_dev(phit), prm)
    G, Gt = to_host(G), to_host(Gt)
    expect = Om[..., None, :, :] @ G @ np.conj(np.swapaxes(Om, -1, -2))[..., None, :, :]
    assert abs(S - St) < 1e-10 * abs(S)
    assert rel_err(Gt, expect) < 1e-9
    op.close()


def test_autograd_function(lq, case):
    """PseudofermionAction backward against finite differences of its own
    forward along random complex directions in U and phi."""
    torch = pytest.importorskip("torch")
    U, phi_e, _, _ = case
    op = lq.Operator(DIMS, KAPPA, 0.0, BC)
    prm = lq.SolverParams(solver="cgne", tol=1e-13, inner="f64")
    Ud = to_dev(U).requires_grad_(True)
    pd = to_dev(phi_e).requires_grad_(True)
    S = lq.PseudofermionAction.apply(Ud, pd, op, prm)
    S.backward()
    gU, gp = to_host(Ud.grad), to_host(pd.grad)
    rng = np.random.default_rng(7)
    dU = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
    dp = rng.standard_normal(phi_e.shape) + 1j * rng.standard_normal(phi_e.shape)
    h = 1e-6
    with torch.no_grad():
        Sp = lq.PseudofermionAction.apply(to_dev(U + h * dU), to_dev(phi_e + h * dp), op, prm).item()
        Sm = lq.PseudofermionAction.apply(to_dev(U - h * dU), to_dev(phi_e - h * dp), op, prm).item()
    fd = (Sp - Sm) / (2 * h)
    pred = float(np.sum((np.conj(gU) * dU).real) + np.sum((np.conj(gp) * dp).real))
    announce("  autograd FD %.10e predicted %.10e" % (fd, pred))
    assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred))
    op.close()


def test_force_wilson_16x16x16x16_workload(lq):
    """The 16^4 even-odd Wilson workload (kappa 0.125, links exp(i 0.3 H)):
    FP64 and FP32 force against the oracle gradient."""
    w = WORKLOADS["wilson_16x16x16x16"]
    dims = w["dims"]
    U = workload_gauge("wilson_16x16x16x16")
    phi_e = gaussian_parity_spinor(dims, 2004)
    ref = oracle.Operator(dims, U, w["kappa"], 0.0, ANTIPERIODIC_T)
    announce("force: 16^4 oracle reference")
    S_ref, M_ref, G_ref = oracle.pf_force_eo(ref, phi_e, tol=1e-13)
    op = lq.Operator(dims, w["kappa"], 0.0, ANTIPERIODIC_T)
    op.set_gauge(to_dev(U))
    for prec, inner, tol in (("f64", "f64", 1e-9), ("f32", "f32", 1e-5)):
        S, grad, G, _, st = lq.pf_force(op, to_dev(phi_e), lq.SolverParams(solver="cgne", tol=1e-12, inner=inner),
                                        "eo", prec)
        e = rel_err(to_host(G), G_ref)
        announce("  16^4 %s: S %.10e (oracle %.10e) iters %d G err %.2e" % (prec, S, S_ref, st.nconv, e))
        assert abs(S - S_ref) < 1e-10 * abs(S_ref) and e < tol
    op.close()
