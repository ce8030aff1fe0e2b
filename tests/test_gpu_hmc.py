"""Molecular dynamics of the HIP library (lq_gauge_force, lq_md_trajectory)
against the oracle (oracle/hmc.py): the Wilson gauge action and force, whole
leapfrog and Omelyan trajectories (pure gauge, with the even-odd Wilson and
clover pseudofermion), and, at larger sizes, properties that hold at any
size: reversibility and the step-squared fall of the energy violation.

Tolerances: the gauge force is a few FP64 roundings per staple sum
(1e-12 relative).  A trajectory compounds the link exponential (Taylor
polynomial with squaring on the GPU, eigendecomposition in the oracle; both
within a few ulps of exp) and, with fermions, forces from solves to 1e-12
(their error cond * 1e-12 with cond < 20 enters P with the step size), so
final U and P agree to 1e-9 relative and dH to 1e-7 absolute.
"""
import numpy as np
import pytest

from lattice_inputs import gauge_exp, gaussian_parity_spinor, random_su3_algebra
from tests.gpu_common import announce, have_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

BC = (1.0, 1.0, 1.0, -1.0)
BETA = 5.5


@pytest.fixture(scope="module")
def lq():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


def _hmc():
    pytest.importorskip("torch")
    from oracle import hmc
    return hmc


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 4, 10), (8, 8, 8, 8)])
def test_gauge_force_matches_oracle(lq, dims):
    hmc = _hmc()
    announce("gauge force %s" % (dims,))
    U = gauge_exp(dims, 0.4, 5101)
    S_ref, _, G_ref = hmc.gauge_force(U, BETA)
    op = lq.Operator(dims, 0.12, 0.0, BC)
    op.set_gauge(to_dev(U))
    S, G = lq.gauge_force(op, BETA)
    G = to_host(G)
    announce("  S %.15e (oracle %.15e) G err %.2e" % (S, S_ref, rel_err(G, G_ref)))
    assert abs(S - S_ref) < 1e-13 * abs(S_ref)
    assert rel_err(G, G_ref) < 1e-12
    S2, G2 = lq.gauge_force(op, 0.0)
    assert S2 == 0.0 and float(to_host(G2).__abs__().max()) == 0.0
    op.close()


def _run(lq, dims, U0, P0, phi, md, fermion=None, tol=1e-12):
    op = lq.Operator(dims, fermion[0] if fermion else 0.12, fermion[1] if fermion else 0.0, BC)
    U = to_dev(U0).clone()
    P = to_dev(P0).clone()
    st = lq.md_trajectory(op, U, P, to_dev(phi) if phi is not None else None, md,
                          lq.SolverParams(solver="cgne", tol=tol, inner="f64"))
    out = to_host(U), to_host(P), st
    op.close()
    return out


@pytest.mark.parametrize("dims,integrator,nsteps", [((4, 4, 4, 4), "leapfrog", 4), ((4, 4, 4, 4), "omelyan", 3),
                                                    ((6, 4, 4, 10), "leapfrog", 3)])
def test_pure_gauge_trajectory_matches_oracle(lq, dims, integrator, nsteps):
    hmc = _hmc()
    announce("pure gauge trajectory %s %s n=%d" % (dims, integrator, nsteps))
    U0 = gauge_exp(dims, 0.3, 5201)
    P0 = random_su3_algebra(dims, 5202)
    act = hmc.Action(dims, BETA)
    U_ref, P_ref, H0, H1 = hmc.trajectory(act, U0, P0, 0.2, nsteps, integrator)
    md = lq.MDParams(beta=BETA, tau=0.2, nsteps=nsteps, integrator=integrator, fermion=False)
    U, P, st = _run(lq, dims, U0, P0, None, md)
    dH_ref = sum(H1) - sum(H0)
    announce("  U err %.2e P err %.2e dH %.10e (oracle %.10e) forces %d" %
             (rel_err(U, U_ref), rel_err(P, P_ref), st.dH, dH_ref, st.n_force))
    assert rel_err(U, U_ref) < 1e-11 and rel_err(P, P_ref) < 1e-11
    assert abs(st.T0 - H0[0]) < 1e-11 * H0[0] and abs(st.Sg0 - H0[1]) < 1e-12 * H0[1]
    assert abs(st.dH - dH_ref) < 1e-8
    assert st.n_force == (nsteps + 1 if integrator == "leapfrog" else 2 * nsteps + 1)


@pytest.mark.parametrize("csw,integrator", [(0.0, "leapfrog"), (0.0, "omelyan"), (1.7, "leapfrog")])
def test_fermion_trajectory_matches_oracle(lq, csw, integrator):
    hmc = _hmc()
    dims = (4, 4, 4, 4)
    kappa = 0.12
    announce("fermion trajectory csw=%g %s" % (csw, integrator))
    U0 = gauge_exp(dims, 0.3, 5301)
    P0 = random_su3_algebra(dims, 5302)
    phi = gaussian_parity_spinor(dims, 5303)
    act = hmc.Action(dims, BETA, fermion=(kappa, csw, BC, True), phi=phi, tol=1e-14)
    nsteps = 3 if integrator == "leapfrog" else 2
    U_ref, P_ref, H0, H1 = hmc.trajectory(act, U0, P0, 0.15, nsteps, integrator)
    md = lq.MDParams(beta=BETA, tau=0.15, nsteps=nsteps, integrator=integrator, fermion=True)
    U, P, st = _run(lq, dims, U0, P0, phi, md, fermion=(kappa, csw))
    dH_ref = sum(H1) - sum(H0)
    announce("  U err %.2e P err %.2e dH %.10e (oracle %.10e) Sf0 %.10e (oracle %.10e) iters %d" %
             (rel_err(U, U_ref), rel_err(P, P_ref), st.dH, dH_ref, st.Sf0, H0[2], st.iters))
    assert st.converged
    assert rel_err(U, U_ref) < 1e-9 and rel_err(P, P_ref) < 1e-9
    assert abs(st.Sf0 - H0[2]) < 1e-10 * H0[2] and abs(st.Sf1 - H1[2]) < 1e-10 * H1[2]
    assert abs(st.dH - dH_ref) < 1e-7


def test_reversibility_and_second_order_8x8x8x8(lq):
    """Flip P and integrate back: the start is recovered; halving the step
    quarters dH (leapfrog and Omelyan), Omelyan's dH below leapfrog's."""
    dims = (8, 8, 8, 8)
    announce("reversibility and dH scaling 8^4 with the Wilson pseudofermion")
    U0 = gauge_exp(dims, 0.3, 5401)
    P0 = random_su3_algebra(dims, 5402)
    phi = gaussian_parity_spinor(dims, 5403)
    md = lq.MDParams(beta=BETA, tau=0.2, nsteps=8, integrator="leapfrog", fermion=True)
    U1, P1, st = _run(lq, dims, U0, P0, phi, md, fermion=(0.12, 0.0))
    U2, P2, _ = _run(lq, dims, U1, -P1, phi, md, fermion=(0.12, 0.0))
    announce("  back: U err %.2e P err %.2e" % (rel_err(U2, U0), rel_err(P2, -P0)))
    assert rel_err(U2, U0) < 1e-10 and rel_err(P2, -P0) < 1e-10
    dh = {}
    for integ in ("leapfrog", "omelyan"):
        for n in (8, 16):
            m = lq.MDParams(beta=BETA, tau=0.2, nsteps=n, integrator=integ, fermion=True)
            dh[(integ, n)] = _run(lq, dims, U0, P0, phi, m, fermion=(0.12, 0.0))[2].dH
    announce("  dH %s" % dh)
    for integ in ("leapfrog", "omelyan"):
        assert 3.5 < abs(dh[(integ, 8)] / dh[(integ, 16)]) < 4.5
    assert abs(dh[("omelyan", 8)]) < abs(dh[("leapfrog", 8)])


def test_hmc_step_accept_and_reject(lq):
    """r = 0 accepts (the operator holds the new field); r close to 1 with a
    trajectory whose dH is large rejects (U returned, operator restored)."""
    torch = pytest.importorskip("torch")
    dims = (4, 4, 4, 4)
    U0 = to_dev(gauge_exp(dims, 0.3, 5501))
    P0 = to_dev(random_su3_algebra(dims, 5502))
    eta = to_dev(gaussian_parity_spinor(dims, 5503) / np.sqrt(2.0))
    op = lq.Operator(dims, 0.12, 0.0, BC)
    sp = lq.SolverParams(solver="cgne", tol=1e-12, inner="f64")
    md = lq.MDParams(beta=BETA, tau=0.1, nsteps=5, fermion=True)
    U1, acc, st = lq.hmc_step(op, U0, P0, eta, 0.0, md, sp)
    assert acc and not torch.equal(U1, U0)
    # the pseudofermion heat bath: S_f at the start equals eta^dag eta
    assert abs(st.Sf0 - float(torch.vdot(eta.reshape(-1), eta.reshape(-1)).real)) < 1e-9 * st.Sf0
    x = to_dev(gaussian_parity_spinor(dims, 5504))
    y_new = op.apply("schur", x, "f64")
    big = lq.MDParams(beta=BETA, tau=2.0, nsteps=1, fermion=True)  # one huge step: dH >> 1
    U2, acc2, st2 = lq.hmc_step(op, U1, P0, eta, 1.0 - 1e-12, big, sp)
    announce("  accepted dH %.3e; rejected dH %.3e" % (st.dH, st2.dH))
    assert st2.dH > 1.0 and not acc2 and U2.data_ptr() == U1.data_ptr()
    assert torch.equal(op.apply("schur", x, "f64"), y_new)
    op.close()


def test_md_operator_level_argument_checks(lq):
    import ctypes
    from paper_2111_04457_amd import _lib
    lib = _lib.load()
    op = lq.Operator((4, 4, 4, 4), 0.12, 0.0, BC)
    sp = lq.SolverParams().to_c()
    st = _lib.MDStats()
    dummy = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    for field, value in (("nsteps", 0), ("integrator", 7), ("beta", float("inf")), ("fermion", 2), ("chrono", 3)):
        bad = lq.MDParams().to_c()
        setattr(bad, field, value)
        assert lib.lq_md_trajectory(op.handle, ctypes.byref(bad), ctypes.byref(sp), dummy, dummy, dummy,
                                    ctypes.byref(st), None) == -1, field
    mp = lq.MDParams().to_c()
    assert lib.lq_md_trajectory(op.handle, ctypes.byref(mp), ctypes.byref(sp), dummy, dummy, None,
                                ctypes.byref(st), None) == -1
    assert lib.lq_gauge_force(op.handle, float("nan"), dummy, None, None) == -1
    assert lib.lq_gauge_force(op.handle, 5.5, dummy, None, None) == -2  # gauge field not set
    op.close()


def test_chronological_guesses_same_trajectory_fewer_iterations(lq):
    """Starting each force solve from the previous solution (chrono 1) or
    the linear extrapolation of the last two (chrono 2) changes only the
    solver's starting point: the trajectory agrees with zero starts to the
    solver tolerance, with fewer iterations."""
    dims = (8, 8, 8, 8)
    U0 = gauge_exp(dims, 0.3, 5601)
    P0 = random_su3_algebra(dims, 5602)
    phi = gaussian_parity_spinor(dims, 5603)
    res = {}
    for chrono in (0, 1, 2):
        md = lq.MDParams(beta=BETA, tau=0.3, nsteps=6, integrator="leapfrog", fermion=True, chrono=chrono)
        res[chrono] = _run(lq, dims, U0, P0, phi, md, fermion=(0.12, 0.0))
    announce("  iterations %s, dH %s" % ({c: r[2].iters for c, r in res.items()},
                                         {c: r[2].dH for c, r in res.items()}))
    for c in (1, 2):
        assert rel_err(res[c][0], res[0][0]) < 1e-10 and rel_err(res[c][1], res[0][1]) < 1e-10
        assert abs(res[c][2].dH - res[0][2].dH) < 1e-7
    assert res[2][2].iters < res[1][2].iters < res[0][2].iters
