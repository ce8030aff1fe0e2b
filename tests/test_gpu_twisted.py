"""The twisted-mass Wilson operator D = 1 - kappa H + i tau gamma_5 of the
HIP library against the oracle: every operator kind element by element in
FP64 / FP32 / FP16 storage (tolerances as for the Wilson and clover
operators: 1e-12, 1e-5, 5e-3), and mixed-precision solves of D x = b
(BiCGStab on M and on the A_ee^-1-preconditioned system, CG on M^dag M)
reaching the oracle's true residual and the oracle's solution; a ragged
batch of twisted operators equals the separate solves bit for bit.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import gauge_exp, gauge_haar, gaussian_parity_spinor, gaussian_spinor
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
    # the other modes are refused for a twisted operator
    with pytest.raises(lq.LQError, match="twisted"):
        op.solve(to_dev(b[0]), "Ddag", prm)
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
