"""Clover pseudofermion force of the HIP library (lq_pf_force with c_sw != 0)
against the oracle's autograd gradient of the dense clover action, central
finite differences of the GPU action, gauge covariance and the
autograd.Function wrapper.

Tolerances as for the Wilson force: FP64 force after an FP64 solve to 1e-12
matches the oracle to 1e-9 relative; with the hopping part in FP32 (the
clover part stays FP64) to 1e-5; finite differences with step 1e-5 to 1e-6.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import (ANTIPERIODIC_T, WORKLOADS, gauge_exp, gauge_transform, gaussian_parity_spinor,
                            gaussian_spinor, random_su3_algebra, workload_gauge)
from tests.gpu_common import announce, have_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

BC = (1.0, np.exp(0.3j), 1.0, -1.0)
KAPPA, CSW = 0.12, 1.7


@pytest.fixture(scope="module")
def lq():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


def _fc():
    pytest.importorskip("torch")
    from oracle import force_clover
    return force_clover


def _expm(X):
    w, v = np.linalg.eig(X)
    return (v * np.exp(w)[..., None, :]) @ np.linalg.inv(v)


_REF = {}


def _reference(dims, variant, traceless, seed):
    """Oracle (S, Mraw, G) and the inputs, cached per case."""
    key = (dims, variant, traceless, seed)
    if key not in _REF:
        U = gauge_exp(dims, 0.4, seed)
        phi = gaussian_parity_spinor(dims, seed + 1) if variant == "eo" else gaussian_spinor(dims, seed + 1)
        S, M, G = _fc().pf_force_clover(dims, U, KAPPA, CSW, BC, phi, variant, traceless)
        _REF[key] = (U, phi, S, M, G)
    return _REF[key]


@pytest.mark.parametrize("dims,variant,traceless,prec", [
    ((4, 4, 4, 4), "eo", True, "f64"),
    ((4, 4, 4, 4), "eo", True, "f32"),
    ((4, 4, 4, 4), "full", True, "f64"),
    ((4, 4, 4, 4), "full", True, "f32"),
    ((4, 4, 4, 4), "eo", False, "f64"),
    ((4, 4, 2, 6), "eo", True, "f64"),   # an extent-2 direction: both neighbours are one site
    ((4, 4, 2, 6), "full", False, "f64"),
])
def test_clover_force_matches_oracle(lq, dims, variant, traceless, prec):
    announce("clover force: dims=%s variant=%s traceless=%s prec=%s" % (dims, variant, traceless, prec))
    U, phi, S_ref, M_ref, G_ref = _reference(dims, variant, traceless, 3101)
    op = lq.Operator(dims, KAPPA, CSW, BC, traceless=traceless)
    op.set_gauge(to_dev(U))
    prm = lq.SolverParams(solver="cgne", tol=1e-12, inner="f64" if prec == "f64" else "f32")
    S, grad, G, _, st = lq.pf_force(op, to_dev(phi), prm, variant, prec)
    grad, G = to_host(grad), to_host(G)
    want_grad = np.conj(np.swapaxes(M_ref, -1, -2))
    tol = 1e-9 if prec == "f64" else 1e-5
    announce("  S %.12e (oracle %.12e) iters %d | grad err %.2e G err %.2e" %
             (S, S_ref, st.nconv, rel_err(grad, want_grad), rel_err(G, G_ref)))
    assert st.converged and st.diff <= 1e-12
    assert abs(S - S_ref) < 1e-10 * abs(S_ref)
    assert rel_err(grad, want_grad) < tol
    assert rel_err(G, G_ref) < tol
    op.close()


def test_clover_force_finite_differences_of_gpu_action(lq):
    dims = (4, 4, 4, 4)
    U = gauge_exp(dims, 0.4, 3201)
    phi_e = gaussian_parity_spinor(dims, 3202)
    op = lq.Operator(dims, KAPPA, CSW, BC)
    prm = lq.SolverParams(solver="cgne", tol=1e-13, inner="f64")

    def action(Uv):
        op.set_gauge(to_dev(Uv))
        return lq.pf_force(op, to_dev(phi_e), prm)[0]

    op.set_gauge(to_dev(U))
    _, _, G, _, _ = lq.pf_force(op, to_dev(phi_e), prm)
    G = to_host(G)
    for seed in (3203, 3204):
        X = random_su3_algebra(dims, seed)
        h = 1e-5
        fd = (action(_expm(h * X) @ U) - action(_expm(-h * X) @ U)) / (2 * h)
        pred = float(np.sum(np.einsum("...ab,...ab->...", np.conj(G), X).real))
        announce("  clover FD %.10e  predicted %.10e" % (fd, pred))
        assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred))
    op.close()


def test_clover_force_gauge_covariance(lq):
    dims = (4, 4, 4, 4)
    U = gauge_exp(dims, 0.4, 3301)
    phi_e = gaussian_parity_spinor(dims, 3302)
    Om = gauge_transform(dims, 3303)
    Ut = np.empty_like(U)
    for mu in range(4):
        Ut[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(np.roll(Om, -1, axis=3 - mu), -1, -2))
    phit = oracle.to_parity(dims, np.einsum("...ab,...sb->...sa", Om, oracle.from_parity(dims, phi_e, 0)), 0)
    op = lq.Operator(dims, KAPPA, CSW, BC)
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


def test_clover_autograd_function(lq):
    """PseudofermionAction on a clover operator: backward against finite
    differences of its own forward along random complex directions."""
    torch = pytest.importorskip("torch")
    dims = (4, 4, 4, 4)
    U = gauge_exp(dims, 0.4, 3401)
    phi_e = gaussian_parity_spinor(dims, 3402)
    op = lq.Operator(dims, KAPPA, CSW, BC)
    prm = lq.SolverParams(solver="cgne", tol=1e-13, inner="f64")
    Ud = to_dev(U).requires_grad_(True)
    pd = to_dev(phi_e).requires_grad_(True)
    S = lq.PseudofermionAction.apply(Ud, pd, op, prm)
    S.backward()
    gU, gp = to_host(Ud.grad), to_host(pd.grad)
    rng = np.random.default_rng(8)
    dU = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
    dp = rng.standard_normal(phi_e.shape) + 1j * rng.standard_normal(phi_e.shape)
    h = 1e-6
    with torch.no_grad():
        Sp = lq.PseudofermionAction.apply(to_dev(U + h * dU), to_dev(phi_e + h * dp), op, prm).item()
        Sm = lq.PseudofermionAction.apply(to_dev(U - h * dU), to_dev(phi_e - h * dp), op, prm).item()
    fd = (Sp - Sm) / (2 * h)
    pred = float(np.sum((np.conj(gU) * dU).real) + np.sum((np.conj(gp) * dp).real))
    announce("  clover autograd FD %.10e predicted %.10e" % (fd, pred))
    assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred))
    op.close()


@pytest.mark.parametrize("dims,variant,prec", [
    ((8, 8, 8, 8), "eo", "f64"),
    ((8, 8, 8, 8), "eo", "f32"),
    ((6, 4, 4, 10), "full", "f64"),  # 480 sites per parity: a ragged last workgroup
])
def test_clover_force_matrix_free_oracle(lq, dims, variant, prec):
    """Larger lattices against the matrix-free oracle (C-oracle CG solve,
    autograd of the bilinear), at the 16^3x32 clover workload's kappa, c_sw
    and link spread."""
    fc = _fc()
    w = WORKLOADS["clover_16x16x16x32"]
    announce("clover force (matrix-free oracle): dims=%s variant=%s prec=%s" % (dims, variant, prec))
    key = ("mf", dims, variant)
    if key not in _REF:
        U = workload_gauge("clover_16x16x16x32", dims)
        phi = gaussian_parity_spinor(dims, 3501) if variant == "eo" else gaussian_spinor(dims, 3501)
        _REF[key] = (U, phi) + fc.pf_force_clover_mf(dims, U, w["kappa"], w["csw"], ANTIPERIODIC_T, phi, variant)
    U, phi, S_ref, M_ref, G_ref = _REF[key]
    op = lq.Operator(dims, w["kappa"], w["csw"], ANTIPERIODIC_T)
    op.set_gauge(to_dev(U))
    prm = lq.SolverParams(solver="cgne", tol=1e-12, inner="f64" if prec == "f64" else "f32")
    S, grad, G, _, st = lq.pf_force(op, to_dev(phi), prm, variant, prec)
    grad, G = to_host(grad), to_host(G)
    tol = 1e-9 if prec == "f64" else 1e-5
    e_grad = rel_err(grad, np.conj(np.swapaxes(M_ref, -1, -2)))
    announce("  S %.12e (oracle %.12e) iters %d | grad err %.2e G err %.2e" % (S, S_ref, st.nconv, e_grad,
                                                                             rel_err(G, G_ref)))
    assert st.converged
    assert abs(S - S_ref) < 1e-10 * abs(S_ref)
    assert e_grad < tol and rel_err(G, G_ref) < tol
    op.close()


def test_clover_force_16x16x16x32_covariance(lq):
    """The 16^3x32 clover workload: the force of a gauge-rotated field and
    source is the rotated force (a property that holds at any size)."""
    name = "clover_16x16x16x32"
    w = WORKLOADS[name]
    dims = w["dims"]
    announce("clover force: %s gauge covariance" % name)
    U = workload_gauge(name)
    phi_e = gaussian_parity_spinor(dims, 3601)
    Om = gauge_transform(dims, 3602)
    Ut = np.empty_like(U)
    for mu in range(4):
        Ut[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(np.roll(Om, -1, axis=3 - mu), -1, -2))
    phit = oracle.to_parity(dims, np.einsum("...ab,...sb->...sa", Om, oracle.from_parity(dims, phi_e, 0)), 0)
    op = lq.Operator(dims, w["kappa"], w["csw"], ANTIPERIODIC_T)
    prm = lq.SolverParams(solver="cgne", tol=1e-13, inner="f32")
    op.set_gauge(to_dev(U))
    S, _, G, _, st = lq.pf_force(op, to_dev(phi_e), prm)
    op.set_gauge(to_dev(Ut))
    St, _, Gt, _, st2 = lq.pf_force(op, to_dev(phit), prm)
    G, Gt = to_host(G), to_host(Gt)
    expect = Om[..., None, :, :] @ G @ np.conj(np.swapaxes(Om, -1, -2))[..., None, :, :]
    e = rel_err(Gt, expect)
    announce("  S %.12e / %.12e iters %d/%d  covariance err %.2e" % (S, St, st.nconv, st2.nconv, e))
    assert st.converged and st2.converged
    assert abs(S - St) < 1e-10 * abs(S)
    assert e < 1e-8
    op.close()
