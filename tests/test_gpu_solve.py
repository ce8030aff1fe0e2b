"""Solves of the HIP library against the oracle.

Every solve must reach its stated true FP64 residual |b - D x| / |b|,
recomputed here by the ORACLE's D on the returned x; the solution is also
compared with the oracle's (x = D^-1 b is unique), within the bound
|x - x*| / |x*| <= cond(D) * residual (cond <= 20 for these lattices,
so 50 * tol is asserted).
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import (ANTIPERIODIC_T, WORKLOADS, gauge_abelian_twist, gauge_exp, gaussian_spinor,
                            point_sources, workload_gauge, workload_source)
from tests.gpu_common import announce, have_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lq():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


def test_wilson_4x4x4x4_cg_full_lattice(lq):
    """Plain FP64 Wilson operator on 4^4 (Haar links, kappa 0.12,
    antiperiodic in time): one D apply, then CG on D^dag D to 1e-12."""
    announce("solve: wilson 4^4 full-lattice CGNE fp64")
    w = WORKLOADS["wilson_4x4x4x4"]
    dims = w["dims"]
    U = workload_gauge("wilson_4x4x4x4")
    b = workload_source("wilson_4x4x4x4")
    ref = oracle.Operator(dims, U, w["kappa"], 0.0, ANTIPERIODIC_T)
    op = lq.Operator(dims, w["kappa"], 0.0, ANTIPERIODIC_T)
    op.set_gauge(to_dev(U))
    assert rel_err(to_host(op.apply("D", to_dev(b))), ref.D(b)) < 1e-12
    prm = lq.SolverParams(solver="cgne", tol=1e-12, inner="f64", even_odd=False)
    x, st = op.solve(to_dev(b), "D", prm)
    x = to_host(x)
    res = oracle.true_residual(ref, x, b)
    announce("  iters %d diff %.2e oracle residual %.2e" % (st[0].nconv, st[0].diff, res))
    assert st[0].converged and res <= 1e-12
    xr, _ = oracle.solve_eo(ref, b, tol=1e-13)
    assert rel_err(x, xr) < 50 * 1e-12
    op.close()


CLOVER = dict(dims=(8, 8, 4, 8), kappa=0.13, csw=1.0, eps=0.3)


@pytest.fixture(scope="module")
def clover_case():
    d = CLOVER["dims"]
    U = gauge_exp(d, CLOVER["eps"], 1101)
    b = gaussian_spinor(d, 2101, 2)
    ref = oracle.Operator(d, U, CLOVER["kappa"], CLOVER["csw"], ANTIPERIODIC_T)
    xr = np.stack([oracle.solve_eo(ref, b[i], tol=1e-13)[0] for i in range(2)])
    return U, b, ref, xr


@pytest.mark.parametrize("solver,inner,recon", [
    ("bicgstab", "f64", 18), ("bicgstab", "f64", 12), ("bicgstab", "f32", 18), ("bicgstab", "f16", 18),
    ("bicgstab", "f16", 12),
    ("cgne", "f64", 18), ("cgne", "f32", 12), ("cgne", "f16", 18),
])
def test_clover_even_odd_solves(lq, clover_case, solver, inner, recon):
    U, b, ref, xr = clover_case
    announce("solve: clover %s %s inner=%s recon=%d" % (CLOVER["dims"], solver, inner, recon))
    op = lq.Operator(CLOVER["dims"], CLOVER["kappa"], CLOVER["csw"], ANTIPERIODIC_T, link_recon=recon)
    op.set_gauge(to_dev(U))
    tol = 1e-10
    prm = lq.SolverParams(solver=solver, tol=tol, inner=inner, inner_tol=1e-5 if inner != "f16" else 1e-2)
    x, st = op.solve(to_dev(b), "D", prm)
    x = to_host(x)
    for i in range(2):
        res = oracle.true_residual(ref, x[i], b[i])
        announce("  rhs %d: iters %d outer %d diff %.2e oracle residual %.2e err %.2e" %
                 (i, st[i].nconv, st[i].nouter, st[i].diff, res, rel_err(x[i], xr[i])))
        assert st[i].converged and res <= tol * 1.01
        assert abs(res - st[i].diff) <= 1e-2 * tol + 0.05 * res
        assert rel_err(x[i], xr[i]) < 50 * tol
    op.close()


@pytest.mark.parametrize("mode", ["Ddag", "DdagD"])
def test_other_modes(lq, clover_case, mode):
    U, b, ref, _ = clover_case
    announce("solve: mode %s" % mode)
    op = lq.Operator(CLOVER["dims"], CLOVER["kappa"], CLOVER["csw"], ANTIPERIODIC_T)
    op.set_gauge(to_dev(U))
    x, st = op.solve(to_dev(b[0]), mode, lq.SolverParams(tol=1e-10, inner="f32"))
    x = to_host(x)[0] if x.dim() == 7 else to_host(x)
    got = ref.Ddag(x) if mode == "Ddag" else ref.DdagD(x)
    res = np.linalg.norm(got - b[0]) / np.linalg.norm(b[0])
    announce("  iters %d diff %.2e oracle residual %.2e" % (st[0].nconv, st[0].diff, res))
    assert st[0].converged and res <= 1.01e-10
    op.close()


@pytest.mark.parametrize("inner", ["f32", "f16"])
def test_ddagd_near_critical(lq, inner):
    """Mode D^dag D on a near-critical Wilson lattice (8^3 x 32, kappa
    0.1245, smooth links; about 250 inner iterations): the second solve's
    tolerance is scaled by |b| / (|D| |y|), y = (D^dag)^-1 b, so that the
    normal residual |b - D^dag D x| / |b| recomputed by the oracle meets
    tol, and the residual the library reports is that one."""
    dims, kappa = (8, 8, 8, 32), 0.1245
    U = gauge_exp(dims, 0.1, 1471)
    b = gaussian_spinor(dims, 2471)
    ref = oracle.Operator(dims, U, kappa, 0.0, ANTIPERIODIC_T)
    op = lq.Operator(dims, kappa, 0.0, ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(to_dev(U))
    tol = 1e-10
    x, st = op.solve(to_dev(b), "DdagD", lq.SolverParams(tol=tol, inner=inner,
                                                        inner_tol=5e-3 if inner == "f16" else 1e-4))
    x = to_host(x).reshape(b.shape)
    res = np.linalg.norm(ref.DdagD(x) - b) / np.linalg.norm(b)
    y = ref.D(x)
    announce("  DdagD near-critical inner %s: iters %d outer %d diff %.2e oracle residual %.2e |Dx|/|b| %.1f" %
             (inner, st[0].nconv, st[0].nouter, st[0].diff, res, np.linalg.norm(y) / np.linalg.norm(b)))
    assert st[0].converged and res <= tol * 1.01
    assert abs(res - st[0].diff) <= 0.05 * res + 1e-3 * tol
    op.close()


def test_point_source_propagator_matches_single_solves(lq):
    """The 12 spin-colour point sources of Fig. 1 solved as one batch give
    the same columns as separate solves and as the oracle."""
    d = (4, 4, 4, 8)
    U = gauge_exp(d, 0.5, 1201)
    kappa, csw = 0.12, 1.7
    ref = oracle.Operator(d, U, kappa, csw, ANTIPERIODIC_T)
    src = point_sources(d)
    op = lq.Operator(d, kappa, csw, ANTIPERIODIC_T)
    op.set_gauge(to_dev(U))
    prm = lq.SolverParams(tol=1e-10, inner="f32")
    X, st = op.solve(to_dev(src), "D", prm)
    X = to_host(X)
    for k in (0, 5, 11):
        res = oracle.true_residual(ref, X[k], src[k])
        assert res <= 1.01e-10 and st[k].converged
        x1, _ = op.solve(to_dev(src[k]), "D", prm)
        assert rel_err(to_host(x1), X[k]) < 1e-8
    op.close()


def test_edge_cases(lq, clover_case):
    U, b, ref, xr = clover_case
    d = CLOVER["dims"]
    op = lq.Operator(d, CLOVER["kappa"], CLOVER["csw"], ANTIPERIODIC_T)
    op.set_gauge(to_dev(U))
    # b = 0: x = 0, nothing to do
    x, st = op.solve(to_dev(np.zeros_like(b[0])), "D", lq.SolverParams(tol=1e-10))
    assert not to_host(x).any() and st[0].diff == 0.0 and st[0].nconv == 0 and st[0].converged
    # iteration cap: result and stats still filled
    x, st = op.solve(to_dev(b[0]), "D", lq.SolverParams(tol=1e-10, max_iter=1, max_outer=1, check_every=1))
    assert not st[0].converged and st[0].nconv >= 1 and 0 < st[0].diff < 1
    # warm start from the solution: no inner iteration needed
    x, st = op.solve(to_dev(b[0]), "D", lq.SolverParams(tol=1e-10), x0=to_dev(xr[0]))
    assert st[0].converged and st[0].nconv == 0
    # non-finite right-hand side
    bad = b[0].copy()
    bad[0, 0, 0, 1, 2, 1] = np.nan
    with pytest.raises(lq.LQError) as e:
        op.solve(to_dev(bad), "D", lq.SolverParams(tol=1e-10))
    assert e.value.status == -6
    op.close()


def test_singular_clover_block_reported(lq):
    """Constant abelian field with c_sw kappa sin(phi) = 1: the block
    1 + F has the eigenvalue 0, which set_gauge reports."""
    d = (8, 4, 4, 4)
    U = gauge_abelian_twist(d, 1)
    kappa = 0.125
    csw = 1.0 / (kappa * np.sin(2 * np.pi / d[0]))
    op = lq.Operator(d, kappa, csw)
    with pytest.raises(lq.LQError) as e:
        op.set_gauge(to_dev(U))
    assert e.value.status == -5
    op.close()


@pytest.mark.parametrize("inner,recon", [("f64", 18), ("f32", 12), ("f16", 12)])
def test_left_preconditioned_inner_solves(lq, clover_case, inner, recon):
    """Inner BiCGStab on A_ee^-1 M with the source A_ee^-1 r: the outer
    FP64 loop keeps the residual of M x = b, so the solve reaches the same
    true residual and solution; the iteration counts are reported."""
    U, b, ref, xr = clover_case
    announce("solve: left-preconditioned inner=%s recon=%d" % (inner, recon))
    op = lq.Operator(CLOVER["dims"], CLOVER["kappa"], CLOVER["csw"], ANTIPERIODIC_T, link_recon=recon)
    op.set_gauge(to_dev(U))
    tol = 1e-10
    iters = {}
    for left in (False, True):
        prm = lq.SolverParams(solver="bicgstab", tol=tol, inner=inner, inner_tol=1e-5 if inner != "f16" else 1e-2,
                              left_precond=left)
        x, st = op.solve(to_dev(b), "D", prm)
        x = to_host(x)
        iters[left] = [s.nconv for s in st]
        for i in range(2):
            res = oracle.true_residual(ref, x[i], b[i])
            assert st[i].converged and res <= tol * 1.01, (left, i, res)
            assert rel_err(x[i], xr[i]) < 50 * tol
    announce("  iterations: plain %s, A_ee^-1-preconditioned %s" % (iters[False], iters[True]))
    op.close()


def test_forced_breakdown_restarts_and_converges(lq, clover_case, capfd):
    """A BiCGStab breakdown forced from the host (rho = 0 at the first inner
    solve's 3rd iteration): the system freezes, the FP64 outer loop counts a
    restart and starts a new inner solve from its iterate, and the solve
    still reaches the oracle's true residual and the oracle's solution.  The
    option is one-shot, and log level 2 prints the outer steps."""
    U, b, ref, xr = clover_case
    op = lq.Operator(CLOVER["dims"], CLOVER["kappa"], CLOVER["csw"], ANTIPERIODIC_T)
    op.set_gauge(to_dev(U))
    prm = lq.SolverParams(tol=1e-10, inner="f32", inner_tol=1e-5)
    _, st0 = op.solve(to_dev(b[0]), "D", prm)
    assert st0[0].restarts == 0
    op.set_option("break_at", 3)
    op.set_option("log_level", 2)
    x, st = op.solve(to_dev(b[0]), "D", prm)
    err = capfd.readouterr().err
    assert "lq: outer step 0" in err and "restarts" in err
    assert op.get_option("break_at") == 0
    assert st[0].restarts >= 1 and st[0].converged
    res = oracle.true_residual(ref, to_host(x), b[0])
    announce("  forced breakdown: %d restarts, %d iters (%d without), oracle residual %.2e"
             % (st[0].restarts, st[0].nconv, st0[0].nconv, res))
    assert res <= 1.01e-10 and rel_err(to_host(x), xr[0]) < 50 * 1e-10
    op.set_option("log_level", 0)
    _, st2 = op.solve(to_dev(b[0]), "D", prm)
    assert st2[0].restarts == 0
    op.close()
