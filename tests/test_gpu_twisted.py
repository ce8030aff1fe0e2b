"""The twisted-mass Wilson operator D = 1 - kappa H + i tau gamma_5 of the
HIP library against the oracle: every operator kind element by element in
FP64 / FP32 / FP16 storage (tolerances as for the Wilson and clover
operators: 1e-12, 1e-5, 5e-3), and mixed-precision solves of D x = b
(BiCGStab on M and on the A_ee^-1-preconditioned system, CG on M^dag M)
reaching the oracle's true residual and the oracle's solution; the dagger
modes (D^dag = gamma_5 D(-tau) gamma_5) against the oracle's D^dag and
D^dag D; a ragged batch of twisted operators equals the separate solves bit
for bit; the pseudofermion action and force against the oracle's gradient of
the dense action; a twisted molecular-dynamics trajectory that is reversible
and second order in the step.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import gauge_exp, gauge_haar, gaussian_parity_spinor, gaussian_spinor, random_su3_algebra
from tests.gpu_common import announce, have_gpu, rel_err, to_dev, to_host
from tests.test_gpu_apply import KINDS, TOL, _reference

pytestmark = pytest.mark.gpu

BC = (1.0, np.exp(0.7j), 1.0, -1.0)
DIMS, KAPPA, TAU = (6, 4, 6, 10), 0.13, 0.35


@pytest.fixture(scope="module")
def lq():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


@pytest.fixture(scope="module")
def case():
    U = gauge_haar(DIMS, 1601)
    return U, oracle.Operator(DIMS, U, KAPPA, 0.0, BC, twist=TAU)


@pytest.mark.parametrize("prec,recon", [("f64", 18), ("f64", 12), ("f32", 12), ("f16", 12), ("f16", 18)])
def test_twisted_apply_all_kinds(lq, case, prec, recon):
    U, ref = case
    op = lq.Operator(DIMS, KAPPA, 0.0, BC, link_recon=recon, twist=TAU)
    op.set_gauge(to_dev(U))
    full = gaussian_spinor(DIMS, 2601, 2)
    par = gaussian_parity_spinor(DIMS, 2602, 2)
    worst = {}
    for kind in KINDS:
        src = full if kind in ("D", "Ddag", "DdagD") else par
        got = to_host(op.apply(kind, to_dev(src), prec))
        for r in range(2):
            e = rel_err(got[r], _reference(ref, kind, src[r]))
            worst[kind] = max(worst.get(kind, 0.0), e)
            assert e < TOL[prec], (kind, prec, e)
    announce("twisted %s recon %d worst %.2e (%s)" % (prec, recon, max(worst.values()), max(worst, key=worst.get)))
    op.close()


@pytest.mark.parametrize("solver,inner,left", [("bicgstab", "f64", False), ("bicgstab", "f32", True),
                                               ("bicgstab", "f16", True), ("cgne", "f32", False)])
def test_twisted_solves_against_oracle(lq, case, solver, inner, left):
    U, ref = case
    b = gaussian_spinor(DIMS, 2603, 2)
    op = lq.Operator(DIMS, KAPPA, 0.0, BC, link_recon=12, twist=TAU)
    op.set_gauge(to_dev(U))
    prm = lq.SolverParams(solver=solver, tol=1e-10, inner=inner, inner_tol=5e-3 if inner == "f16" else 1e-5,
                          left_precond=left)
    x, st = op.solve(to_dev(b), "D", prm)
    x = to_host(x)
    for r in range(2):
        res = oracle.true_residual(ref, x[r], b[r])
        xr, _ = oracle.solve_eo(ref, b[r], tol=1e-13)
        announce("  twisted %s inner %s left %s: iters %d residual %.2e err %.2e"
                 % (solver, inner, left, st[r].nconv, res, rel_err(x[r], xr)))
        assert st[r].converged and res <= 1.01e-10
        assert rel_err(x[r], xr) < 50 * 1e-10
    op.close()


@pytest.mark.parametrize("mode", ["Ddag", "DdagD"])
def test_twisted_dagger_modes_against_oracle(lq, case, mode):
    """D^dag = gamma_5 D(-tau) gamma_5: the dagger modes solve with the sign
    of the twist flipped for the call; the operator keeps +tau afterwards
    (an LQ_D solve after them equals one before, bit for bit)."""
    U, ref = case
    announce("twisted mode %s" % mode)
    b = gaussian_spinor(DIMS, 2621, 2)
    op = lq.Operator(DIMS, KAPPA, 0.0, BC, link_recon=12, twist=TAU)
    op.set_gauge(to_dev(U))
    prm = lq.SolverParams(tol=1e-10, inner="f16", inner_tol=5e-3)
    xd0, _ = op.solve(to_dev(b), "D", prm)
    x, st = op.solve(to_dev(b), mode, prm)
    x = to_host(x)
    apply = ref.Ddag if mode == "Ddag" else ref.DdagD
    for r in range(2):
        res = np.linalg.norm(apply(x[r]) - b[r]) / np.linalg.norm(b[r])
        announce("  rhs %d: iters %d outer %d oracle residual %.2e" % (r, st[r].nconv, st[r].nouter, res))
        assert st[r].converged and res <= 1.01e-10
    # the Hermitian-conjugate solve is not the plain one
    assert rel_err(x[0], to_host(xd0)[0]) > 1e-3
    xd1, _ = op.solve(to_dev(b), "D", prm)
    assert np.array_equal(to_host(xd0), to_host(xd1))
    # deflation belongs to +tau: refused in the dagger modes
    with pytest.raises(lq.LQError, match="twisted"):
        op.solve(to_dev(b), mode, lq.SolverParams(tol=1e-10, deflate=True))
    op.close()


_FREF = {}


def _force_reference(dims, variant, seed):
    pytest.importorskip("torch")
    from oracle import force_clover as fc
    key = (dims, variant, seed)
    if key not in _FREF:
        U = gauge_exp(dims, 0.4, seed)
        phi = gaussian_parity_spinor(dims, seed + 1) if variant == "eo" else gaussian_spinor(dims, seed + 1)
        S, M, G = fc.pf_force_clover(dims, U, KAPPA, 0.0, BC, phi, variant, twist=TAU)
        _FREF[key] = (U, phi, S, M, G)
    return _FREF[key]


@pytest.mark.parametrize("dims,variant,prec", [
    ((4, 4, 4, 4), "eo", "f64"), ((4, 4, 4, 4), "eo", "f32"),
    ((4, 4, 4, 4), "full", "f64"), ((4, 4, 2, 6), "eo", "f64"),
])
def test_twisted_force_matches_oracle(lq, dims, variant, prec):
    """Pseudofermion action and force of the twisted operator against the
    oracle's autograd gradient of the dense action (the twist term does not
    depend on the links; it enters through the inverses).  Tolerances as
    for the Wilson force: 1e-9 (FP64) and 1e-5 (FP32 force kernel)."""
    announce("twisted force: dims=%s variant=%s prec=%s" % (dims, variant, prec))
    U, phi, S_ref, M_ref, G_ref = _force_reference(dims, variant, 3601)
    op = lq.Operator(dims, KAPPA, 0.0, BC, twist=TAU)
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


def test_twisted_trajectory_reversible_and_second_order(lq):
    """A molecular-dynamics trajectory with the twisted pseudofermion (its
    force pinned above): flipping P and integrating back recovers the start,
    and halving the leapfrog step quarters the energy violation."""
    dims, beta = (8, 8, 8, 8), 5.5
    announce("twisted trajectory %s" % (dims,))
    U0 = gauge_exp(dims, 0.3, 3701)
    P0 = random_su3_algebra(dims, 3702)
    phi = gaussian_parity_spinor(dims, 3703)
    prm = lq.SolverParams(solver="cgne", tol=1e-12, inner="f64")

    def run(U, P, n):
        op = lq.Operator(dims, KAPPA, 0.0, BC, twist=TAU)
        Ud, Pd = to_dev(U).clone(), to_dev(P).clone()
        md = lq.MDParams(beta=beta, tau=0.2, nsteps=n, integrator="leapfrog", fermion=True)
        st = lq.md_trajectory(op, Ud, Pd, to_dev(phi), md, prm)
        op.close()
        return to_host(Ud), to_host(Pd), st

    U1, P1, st = run(U0, P0, 8)
    U2, P2, _ = run(U1, -P1, 8)
    announce("  back: U err %.2e P err %.2e; Sf0 %.6e" % (rel_err(U2, U0), rel_err(P2, -P0), st.Sf0))
    assert st.converged
    assert rel_err(U2, U0) < 1e-10 and rel_err(P2, -P0) < 1e-10
    dh8, dh16 = st.dH, run(U0, P0, 16)[2].dH
    announce("  dH %.4e (8 steps) %.4e (16 steps)" % (dh8, dh16))
    assert 3.5 < abs(dh8 / dh16) < 4.5


def test_twisted_multi_rhs_shapes_bitwise(lq, case):
    """Several right-hand sides of a twisted operator: two per thread and
    four per workgroup (links in LDS) give the bits of one per thread, in
    every kind and precision, and so does a multi-RHS solve."""
    U, ref = case
    op = lq.Operator(DIMS, KAPPA, 0.0, BC, link_recon=12, twist=TAU)
    op.set_gauge(to_dev(U))
    nrhs = 5
    xe = to_dev(np.stack([gaussian_parity_spinor(DIMS, 2640 + i) for i in range(nrhs)]))
    for p in ("f16", "f32", "f64"):
        for kind in ("schur", "schur_dag", "schur_left", "schur_normal", "clover_inv_o"):
            outs = {}
            for nr in (1, 2, 4):
                op.set_option("rhs_per_thread_" + p, nr)
                outs[nr] = to_host(op.apply(kind, xe, p))
            assert np.array_equal(outs[1], outs[2]) and np.array_equal(outs[1], outs[4]), (p, kind)
    b = to_dev(gaussian_spinor(DIMS, 2650, nrhs))
    prm = lq.SolverParams(tol=1e-10, inner="f16", inner_tol=5e-3, check_every=4, left_precond=True)
    res = {}
    for nr in (1, 4):
        op.set_option("rhs_per_thread", nr)
        x, st = op.solve(b, "D", prm)
        res[nr] = (to_host(x), [s.nconv for s in st])
    assert np.array_equal(res[1][0], res[4][0]) and res[1][1] == res[4][1]
    x = res[4][0]
    bh = to_host(b)
    for r in range(nrhs):
        assert oracle.true_residual(ref, x[r], bh[r]) <= 1.01e-10
    announce("twisted multi-RHS: iterations %s" % res[4][1])
    op.close()


def test_twisted_batch_and_argument_checks(lq):
    dims_list = [(4, 4, 4, 4), (6, 6, 4, 4), (8, 4, 4, 8)]
    prm = lq.SolverParams(tol=1e-10, inner="f16", inner_tol=5e-3, left_precond=True)
    ops, bs = [], []
    for i, d in enumerate(dims_list):
        op = lq.Operator(d, KAPPA, 0.0, BC, link_recon=12, twist=TAU)
        op.set_gauge(to_dev(gauge_exp(d, 0.5, 1611 + i)))
        ops.append(op)
        bs.append(gaussian_spinor(d, 2611 + i, 2))
    batch = lq.Batch(ops, [2] * len(ops))
    xs, _ = batch.solve([to_dev(b) for b in bs], prm)
    for op, b, x in zip(ops, bs, xs):
        x1, _ = op.solve(to_dev(b), "D", prm)
        assert np.array_equal(to_host(x), to_host(x1))
    batch.close()
    for op in ops:
        op.close()
    with pytest.raises(lq.LQError, match="clover"):
        lq.Operator(DIMS, KAPPA, 1.0, BC, twist=TAU)
    with pytest.raises(lq.LQError, match="finite"):
        lq.Operator(DIMS, KAPPA, 0.0, BC, twist=float("nan"))
