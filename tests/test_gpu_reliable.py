"""Reliable updates: the mixed-precision solves with the inner Krylov space
kept across the FP64 residual replacements (lq_solver_params.reliable).

Every solve must reach its true FP64 residual |b - D x| / |b| recomputed by
the oracle's D, and the solution the oracle's within cond(D) times the
residual.  On a lattice close to the critical hopping parameter, where each
restart of CG on the normal equations discards its search direction, the
reliable FP32 solve needs no more inner iterations than the restarted one.  A
ragged batch with reliable updates equals its separate solves bit for bit,
and a forced breakdown (the system's Krylov space is discarded and restarted
afresh) still converges.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import ANTIPERIODIC_T, gauge_exp, gaussian_spinor
from tests.gpu_common import announce, have_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

CLOVER = dict(dims=(8, 8, 4, 8), kappa=0.13, csw=1.0, eps=0.3)
# near-critical Wilson lattice: ~145 iterations of FP64 CG on M^dag M
LIGHT = dict(dims=(8, 8, 8, 32), kappa=0.1245, csw=0.0, eps=0.1)


@pytest.fixture(scope="module")
def lq():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


@pytest.fixture(scope="module")
def clover_case():
    d = CLOVER["dims"]
    U = gauge_exp(d, CLOVER["eps"], 1101)
    b = gaussian_spinor(d, 2101, 2)
    ref = oracle.Operator(d, U, CLOVER["kappa"], CLOVER["csw"], ANTIPERIODIC_T)
    return U, b, ref


@pytest.fixture(scope="module")
def light_case():
    d = LIGHT["dims"]
    U = gauge_exp(d, LIGHT["eps"], 1401)
    b = gaussian_spinor(d, 2401)
    ref = oracle.Operator(d, U, LIGHT["kappa"], LIGHT["csw"], ANTIPERIODIC_T)
    return U, b, ref


def _check(ref, x, b, st, tol, tag):
    x = x.reshape((-1,) + b.shape[-6:])
    bb = b.reshape(x.shape)
    for i in range(x.shape[0]):
        res = oracle.true_residual(ref, x[i], bb[i])
        assert st[i].converged and res <= tol * 1.01, (tag, i, res)
    return x


@pytest.mark.parametrize("solver,inner,left", [
    ("bicgstab", "f32", False), ("bicgstab", "f16", False), ("bicgstab", "f16", True),
    ("cgne", "f32", False), ("cgne", "f16", False),
])
def test_reliable_solves_reach_the_oracle_residual(lq, clover_case, solver, inner, left):
    U, b, ref = clover_case
    announce("reliable: clover %s %s inner=%s left=%s" % (CLOVER["dims"], solver, inner, left))
    op = lq.Operator(CLOVER["dims"], CLOVER["kappa"], CLOVER["csw"], ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(to_dev(U))
    tol = 1e-10
    itol = 1e-2 if inner == "f16" else 1e-3
    iters = {}
    for rel in (False, True):
        prm = lq.SolverParams(solver=solver, tol=tol, inner=inner, inner_tol=itol, left_precond=left, reliable=rel)
        x, st = op.solve(to_dev(b), "D", prm)
        x = _check(ref, to_host(x), b, st, tol, (solver, inner, rel))
        iters[rel] = [(s.nconv, s.nouter) for s in st]
        if rel:
            xr = oracle.solve_eo(ref, b[0], tol=1e-13)[0]
            assert rel_err(x[0], xr) < 50 * tol
    announce("  (iterations, outer steps): restarted %s, reliable %s" % (iters[False], iters[True]))
    op.close()


@pytest.mark.parametrize("inner,itol,fewer", [("f32", 1e-1, True), ("f32", 1e-3, True), ("f16", 1e-2, False)])
def test_reliable_cgne_near_critical(lq, light_case, inner, itol, fewer):
    """FP32 storage: CG keeps its search directions across the residual
    replacements and needs no more iterations than when restarted each
    time.  Binary16 storage: both converge (its search directions carry the
    storage rounding, and which way needs fewer iterations is reported)."""
    U, b, ref = light_case
    announce("reliable: near-critical wilson %s cgne inner=%s" % (LIGHT["dims"], inner))
    op = lq.Operator(LIGHT["dims"], LIGHT["kappa"], LIGHT["csw"], ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(to_dev(U))
    tol = 1e-10
    it = {}
    for rel in (False, True):
        prm = lq.SolverParams(solver="cgne", tol=tol, inner=inner, inner_tol=itol, reliable=rel)
        x, st = op.solve(to_dev(b), "D", prm)
        _check(ref, to_host(x), b, st, tol, (inner, rel))
        it[rel] = (st[0].nconv, st[0].nouter)
    announce("  (iterations, outer steps): restarted %s, reliable %s" % (it[False], it[True]))
    if fewer:
        assert it[True][0] <= it[False][0]
    op.close()


def test_reliable_normal_equations_mode(lq, clover_case):
    """Mode D^dag D (CG on M^dag M with its own right-hand side, the
    pseudofermion force's solve) with reliable updates."""
    U, b, ref = clover_case
    op = lq.Operator(CLOVER["dims"], CLOVER["kappa"], CLOVER["csw"], ANTIPERIODIC_T)
    op.set_gauge(to_dev(U))
    x, st = op.solve(to_dev(b[0]), "DdagD", lq.SolverParams(tol=1e-10, inner="f16", inner_tol=1e-2, reliable=True))
    x = to_host(x).reshape(b[0].shape)
    res = np.linalg.norm(ref.DdagD(x) - b[0]) / np.linalg.norm(b[0])
    announce("  DdagD reliable: iters %d outer %d oracle residual %.2e" % (st[0].nconv, st[0].nouter, res))
    assert st[0].converged and res <= 1.01e-10
    op.close()


def test_reliable_batch_equals_separate_solves(lq):
    dims_list = [(4, 4, 4, 4), (6, 6, 4, 4), (8, 8, 8, 8)]
    kappa, csw = 0.135, 1.7
    prm = lq.SolverParams(tol=1e-10, inner="f16", inner_tol=1e-2, check_every=4, reliable=True)
    ops, bs, Us = [], [], []
    for i, d in enumerate(dims_list):
        U = gauge_exp(d, 0.5, 1951 + i)
        op = lq.Operator(d, kappa, csw, ANTIPERIODIC_T, link_recon=12)
        op.set_gauge(to_dev(U))
        ops.append(op)
        Us.append(U)
        bs.append(gaussian_spinor(d, 2951 + i, 2))
    batch = lq.Batch(ops, [2] * len(ops))
    xs, st = batch.solve([to_dev(b) for b in bs], prm)
    for i, (op, d) in enumerate(zip(ops, dims_list)):
        x1, s1 = op.solve(to_dev(bs[i]), "D", prm)
        assert np.array_equal(to_host(xs[i]), to_host(x1)), d
        assert [s.nconv for s in s1] == [s.nconv for s in st[2 * i:2 * i + 2]]
        ref = oracle.Operator(d, Us[i], kappa, csw, ANTIPERIODIC_T)
        _check(ref, to_host(xs[i]), bs[i], st[2 * i:2 * i + 2], 1e-10, d)
    announce("reliable batch iters %s" % [s.nconv for s in st])
    batch.close()
    for op in ops:
        op.close()


def test_reliable_forced_breakdown_starts_afresh(lq, clover_case):
    U, b, ref = clover_case
    op = lq.Operator(CLOVER["dims"], CLOVER["kappa"], CLOVER["csw"], ANTIPERIODIC_T)
    op.set_gauge(to_dev(U))
    prm = lq.SolverParams(tol=1e-10, inner="f32", inner_tol=1e-3, reliable=True)
    op.set_option("break_at", 3)
    x, st = op.solve(to_dev(b[0]), "D", prm)
    assert st[0].restarts >= 1
    _check(ref, to_host(x), b[0][None], st, 1e-10, "break")
    announce("  reliable with a forced breakdown: %d restarts, %d iters" % (st[0].restarts, st[0].nconv))
    op.close()
