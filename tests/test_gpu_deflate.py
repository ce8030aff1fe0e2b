"""Deflation inside the solve (lq_op_set_deflation + SolverParams(deflate)):
the outer FP64 loop projects each residual with eigenpairs of M^dag M
before the inner solve.

- With the complete eigenbasis of the dense M^dag M (oracle/dense.py, a
  lattice of 32 even sites: 384 pairs) the first projection is the exact
  solution M^-1 b_hat = (M^dag M)^-1 M^dag b_hat: the solve needs no inner
  iteration, and the pseudofermion force's X = (M^dag M)^-1 phi none either,
  with the oracle's residual and the undeflated force.
- On a near-critical Wilson lattice the 16 lowest pairs from lq_eigs cut the
  inner iterations of CG on the normal equations; every solve reaches the
  oracle's true residual.
- Vectors that are not eigenvectors at all (random orthonormal ones with
  made-up eigenvalues) leave the solve exact: the residual update is an
  FP64 apply.
- The deflation space belongs to the operator's current gauge field and
  parameters, needs device memory of its own, and is a solve of one operator.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import ANTIPERIODIC_T, gauge_exp, gaussian_parity_spinor, gaussian_spinor
from tests.gpu_common import announce, have_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

LIGHT = dict(dims=(8, 8, 8, 32), kappa=0.1245, csw=0.0, eps=0.1)


@pytest.fixture(scope="module")
def lq():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


def _dense_normal_eigenbasis(dims, U, kappa, csw, bc):
    from oracle.dense import dense_dirac, parity_index
    D = dense_dirac(dims, U, kappa, csw, bc)
    ie, io = parity_index(dims, 0), parity_index(dims, 1)
    M = D[np.ix_(ie, ie)] - D[np.ix_(ie, io)] @ np.linalg.solve(D[np.ix_(io, io)], D[np.ix_(io, ie)])
    w, Z = np.linalg.eigh(M.conj().T @ M)
    n = len(w)
    return w, np.ascontiguousarray(Z.T).reshape((n, n // 12, 4, 3))


def test_complete_eigenbasis_solves_by_projection(lq):
    dims = (4, 2, 2, 4)
    kappa, csw = 0.13, 1.3
    U = gauge_exp(dims, 0.5, 8101)
    w, Vh = _dense_normal_eigenbasis(dims, U, kappa, csw, ANTIPERIODIC_T)
    ref = oracle.Operator(dims, U, kappa, csw, ANTIPERIODIC_T)
    for k in (0, len(w) // 2, len(w) - 1):  # the dense ordering is the parity fields' ordering
        assert np.linalg.norm(ref.schur_normal(Vh[k]) - w[k] * Vh[k]) < 1e-10 * w[k]
    op = lq.Operator(dims, kappa, csw, ANTIPERIODIC_T)
    op.set_gauge(to_dev(U))
    op.set_deflation(list(w), to_dev(Vh))
    b = gaussian_spinor(dims, 8102, 2)
    for solver in ("bicgstab", "cgne"):
        x, st = op.solve(to_dev(b), "D", lq.SolverParams(solver=solver, tol=1e-10, inner="f32", deflate=True))
        x = to_host(x)
        for i in range(2):
            res = oracle.true_residual(ref, x[i], b[i])
            announce("  %s rhs %d: inner iterations %d, oracle residual %.2e" % (solver, i, st[i].nconv, res))
            assert st[i].converged and st[i].nconv == 0 and res <= 1e-12
    # the force's normal-equation solve: X = (M^dag M)^-1 phi from the projection
    phi = gaussian_parity_spinor(dims, 8103)
    prm = lq.SolverParams(tol=1e-12, inner="f64", solver="cgne")
    S0, g0, G0, X0, _ = lq.pf_force(op, to_dev(phi), prm, want_x=True)
    prm.deflate = True
    S1, g1, G1, X1, st = lq.pf_force(op, to_dev(phi), prm, want_x=True)
    announce("  force: S %.12e vs %.12e, inner iterations %d" % (S1, S0, st.nconv))
    assert st.nconv == 0
    assert abs(S1 - S0) <= 1e-10 * abs(S0)
    assert rel_err(to_host(G1), to_host(G0)) < 1e-9
    assert rel_err(to_host(X1), to_host(X0)) < 1e-10
    op.close()


@pytest.fixture(scope="module")
def light(lq):
    d = LIGHT["dims"]
    U = gauge_exp(d, LIGHT["eps"], 1401)
    ref = oracle.Operator(d, U, LIGHT["kappa"], LIGHT["csw"], ANTIPERIODIC_T)
    op = lq.Operator(d, LIGHT["kappa"], LIGHT["csw"], ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(to_dev(U))
    ev, res, X, st = op.eigs(16, 64, v0=to_dev(gaussian_parity_spinor(d, 8201)), tol=1e-8, vectors=True)
    assert st["nconv"] == 16
    announce("  near-critical lattice: 16 lowest eigenvalues of M^dag M %.3e .. %.3e" % (ev[0], ev[-1]))
    yield U, ref, op, ev, X
    op.close()


@pytest.mark.parametrize("solver,inner,reliable", [("cgne", "f32", False), ("cgne", "f16", True),
                                                    ("bicgstab", "f16", False), ("bicgstab", "f32", True)])
def test_deflated_solves_near_critical(lq, light, solver, inner, reliable):
    U, ref, op, ev, X = light
    b = gaussian_spinor(LIGHT["dims"], 2401)
    tol = 1e-10
    itol = 1e-2 if inner == "f16" else 1e-3
    it = {}
    for defl in (False, True):
        op.set_deflation(ev if defl else [], X if defl else None)
        prm = lq.SolverParams(solver=solver, tol=tol, inner=inner, inner_tol=itol, reliable=reliable, deflate=defl)
        x, st = op.solve(to_dev(b), "D", prm)
        res = oracle.true_residual(ref, to_host(x), b)
        assert st[0].converged and res <= tol * 1.01, (defl, res)
        it[defl] = (st[0].nconv, st[0].nouter)
    announce("  %s %s reliable=%s (iterations, outer steps): plain %s, deflated %s" %
             (solver, inner, reliable, it[False], it[True]))
    if solver == "cgne":
        assert it[True][0] < it[False][0]
    op.set_deflation([], None)


def test_poor_vectors_leave_the_solve_exact(lq):
    dims = (8, 8, 4, 8)
    kappa, csw = 0.13, 1.0
    U = gauge_exp(dims, 0.3, 8301)
    ref = oracle.Operator(dims, U, kappa, csw, ANTIPERIODIC_T)
    op = lq.Operator(dims, kappa, csw, ANTIPERIODIC_T)
    op.set_gauge(to_dev(U))
    rng = np.random.default_rng(8302)
    n = dims[0] * dims[1] * dims[2] * dims[3] // 2 * 12
    Q, _ = np.linalg.qr(rng.standard_normal((n, 8)) + 1j * rng.standard_normal((n, 8)))
    V = np.ascontiguousarray(Q.T).reshape((8, n // 12, 4, 3))
    op.set_deflation([1e-3] * 4 + [10.0] * 4, to_dev(V))
    b = gaussian_spinor(dims, 8303)
    x, st = op.solve(to_dev(b), "D", lq.SolverParams(tol=1e-10, inner="f32", deflate=True))
    res = oracle.true_residual(ref, to_host(x), b)
    announce("  random vectors: iterations %d outer %d oracle residual %.2e" % (st[0].nconv, st[0].nouter, res))
    assert st[0].converged and res <= 1.01e-10
    op.close()


def test_deflation_state_and_argument_errors(lq):
    import ctypes
    from paper_2111_04457_amd import _lib
    lib = _lib.load()
    dims = (4, 4, 4, 4)
    U = gauge_exp(dims, 0.3, 8401)
    op = lq.Operator(dims, 0.12, 1.0, ANTIPERIODIC_T)
    ev = (ctypes.c_double * 2)(0.5, 0.7)
    dummy = ctypes.c_void_p(16)  # never dereferenced: the checks fail first
    assert lib.lq_op_set_deflation(op.handle, 2, ev, dummy, None) == -2  # no gauge field
    op.set_gauge(to_dev(U))
    assert lib.lq_op_set_deflation(op.handle, -1, ev, dummy, None) == -1
    assert lib.lq_op_set_deflation(op.handle, 1025, ev, dummy, None) == -1
    assert lib.lq_op_set_deflation(op.handle, 2, None, dummy, None) == -1
    bad = (ctypes.c_double * 2)(0.5, -1.0)
    assert lib.lq_op_set_deflation(op.handle, 2, bad, dummy, None) == -1
    b = to_dev(gaussian_spinor(dims, 8402))
    with pytest.raises(lq.LQError) as e:  # no deflation space
        op.solve(b, "D", lq.SolverParams(tol=1e-10, deflate=True))
    assert e.value.status == -2
    V = to_dev(gaussian_parity_spinor(dims, 8403, 2))
    op.set_deflation([0.5, 0.7], V)
    with pytest.raises(lq.LQError) as e:  # the full-lattice solve does not deflate
        op.solve(b, "D", lq.SolverParams(tol=1e-10, solver="cgne", even_odd=False, deflate=True))
    assert e.value.status == -1
    with pytest.raises(lq.LQError) as e:  # a batch does not deflate
        op2 = lq.Operator(dims, 0.12, 1.0, ANTIPERIODIC_T)
        op2.set_gauge(to_dev(U))
        bt = lq.Batch([op, op2], [1, 1])
        try:
            bt.solve([b, b], lq.SolverParams(tol=1e-10, deflate=True))
        finally:
            bt.close()
            op2.close()
    assert e.value.status == -1
    op.set_gauge(to_dev(U))  # a new gauge field removes the space
    with pytest.raises(lq.LQError) as e:
        op.solve(b, "D", lq.SolverParams(tol=1e-10, deflate=True))
    assert e.value.status == -2
    op.set_deflation([0.5, 0.7], V)
    op.set_params(0.121, 1.0)  # so do new parameters
    with pytest.raises(lq.LQError) as e:
        op.solve(b, "D", lq.SolverParams(tol=1e-10, deflate=True))
    assert e.value.status == -2
    op.close()
    # a bound operator has no room for the space
    bop = lq.Operator(dims, 0.12, 1.0, ANTIPERIODIC_T)
    bop.bind(1)
    bop.set_gauge(to_dev(U))
    with pytest.raises(lq.LQError) as e:
        bop.set_deflation([0.5, 0.7], V)
    assert e.value.status == -2
    bop.close()
