"""Two-level multigrid (lq_mg_*) against the multigrid oracle (oracle/mg.py).

- With no inverse iterations the near-null vectors are the start vectors,
  orthonormalised per aggregate and chirality: equal to the oracle's
  modified Gram-Schmidt of the same vectors (FP32 storage: 2e-6 relative).
- Restriction P^dag f and prolongation P c equal the oracle's with its P.
- The coarse operator equals the oracle's dense P^dag D P (D entry by entry
  from eq. (1)), as a whole on 4^4 (coarse extent 2: the two sides of a
  direction reach the same aggregate) and block by block on 8 x 4^3 (coarse
  extent 4 in x separates them); its apply equals the dense coarse matrix
  times the vector.  The build applies D in FP64 and stores FP32:
  tolerance 1e-5 of the largest entry.
- The multigrid-preconditioned solve reaches the oracle's true residual and
  solution on a near-critical Wilson lattice, a clover lattice and a
  near-critical twisted-mass lattice, with fewer fine iterations than
  BiCGStab.  The twisted coarse operator is checked against the dense
  Galerkin product of the twisted D like the clover one.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import ANTIPERIODIC_T, gauge_exp, gaussian_spinor
from oracle import mg as omg
from oracle.dense import dense_dirac
from tests.gpu_common import announce, have_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lq():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


def _hierarchy(lq, dims, kappa, csw, bc, block, nv, seed, twist=0.0):
    U = gauge_exp(dims, 0.4, seed)
    op = lq.Operator(dims, kappa, csw, bc, twist=twist)
    op.set_gauge(to_dev(U))
    v0 = gaussian_spinor(dims, seed + 1, nv)
    h = lq.Multigrid(op, to_dev(v0), lq.MGParams(block=block, nvec=nv, setup_iters=0))
    return U, op, v0, h


def test_vectors_restriction_prolongation_match_oracle(lq):
    dims, block, nv = (4, 4, 4, 8), (2, 2, 2, 2), 4
    U, op, v0, h = _hierarchy(lq, dims, 0.12, 1.0, ANTIPERIODIC_T, block, nv, 9301)
    announce("mg: vectors, restriction, prolongation on %s blocks %s nvec %d" % (dims, block, nv))
    W = omg.block_orthonormalize(dims, block, v0)
    got = to_host(h.vectors())
    assert rel_err(got, W) < 2e-6
    P = omg.prolongator(dims, block, W)
    f = gaussian_spinor(dims, 9311)
    c = to_host(h.restrict(to_dev(f)))
    assert rel_err(c.reshape(-1), omg.restrict(P, f)) < 2e-6
    rng = np.random.default_rng(9312)
    cv = rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)
    fine = to_host(h.prolong(to_dev(cv)))
    assert rel_err(fine.reshape(-1), omg.prolong(P, cv)) < 2e-6
    h.close()
    op.close()


@pytest.mark.parametrize("csw,twist", [(1.3, 0.0), (0.0, 0.3)])
def test_coarse_operator_matches_dense_galerkin(lq, csw, twist):
    dims, block, nv = (4, 4, 4, 4), (2, 2, 2, 2), 4
    bc = (1.0, np.exp(0.3j), 1.0, -1.0)
    U, op, v0, h = _hierarchy(lq, dims, 0.12, csw, bc, block, nv, 9401, twist)
    announce("mg: coarse operator against dense P^dag D P on %s (csw %g, twist %g)" % (dims, csw, twist))
    W = omg.block_orthonormalize(dims, block, v0)
    P = omg.prolongator(dims, block, W)
    Dc_ref = omg.galerkin(dense_dirac(dims, U, 0.12, csw, bc, twist=twist), P)
    cdims = omg.coarse_dims(dims, block)
    Dc = h.coarse_op()
    got = omg.stencil_to_dense(cdims, Dc)
    scale = np.abs(Dc_ref).max()
    announce("  max |entry| %.3f, max deviation %.2e" % (scale, np.abs(got - Dc_ref).max()))
    assert np.abs(got - Dc_ref).max() < 1e-5 * scale
    # its apply
    rng = np.random.default_rng(9402)
    x = rng.standard_normal((h.ncoarse, h.n2)) + 1j * rng.standard_normal((h.ncoarse, h.n2))
    y = to_host(h.coarse_apply(to_dev(x)))
    assert rel_err(y.reshape(-1), Dc_ref @ x.reshape(-1)) < 1e-5
    h.close()
    op.close()


def test_coarse_blocks_by_direction(lq):
    dims, block, nv = (8, 4, 4, 4), (2, 2, 2, 2), 3
    U, op, v0, h = _hierarchy(lq, dims, 0.125, 1.0, ANTIPERIODIC_T, block, nv, 9501)
    ref = oracle.Operator(dims, U, 0.125, 1.0, ANTIPERIODIC_T)
    W = omg.block_orthonormalize(dims, block, v0)
    cdims = omg.coarse_dims(dims, block)
    A0 = 2 + cdims[0] * (1 + cdims[1] * (1 + cdims[2] * 0))  # aggregate (2, 1, 1, 0): on the t boundary
    cols = omg.coarse_columns(ref.D, dims, block, W, A0)
    Dc = h.coarse_op()
    scale = np.abs(cols).max()
    # the aggregate itself, and x (coarse extent 4): each side on its own
    assert np.abs(Dc[A0, 0] - cols[A0]).max() < 1e-5 * scale
    bm = omg.neighbour(cdims, A0, 2)  # at -x: couples to A0 through its +x face
    bp = omg.neighbour(cdims, A0, 1)
    assert np.abs(Dc[bm, 1] - cols[bm]).max() < 1e-5 * scale
    assert np.abs(Dc[bp, 2] - cols[bp]).max() < 1e-5 * scale
    # y, z, t (coarse extent 2): both sides reach the same aggregate
    for mu in (1, 2, 3):
        B = omg.neighbour(cdims, A0, 1 + 2 * mu)
        assert np.abs(Dc[B, 1 + 2 * mu] + Dc[B, 2 + 2 * mu] - cols[B]).max() < 1e-5 * scale
    h.close()
    op.close()


@pytest.mark.parametrize("case", ["wilson_near_critical", "clover", "twisted_near_critical"])
def test_multigrid_solve_reaches_oracle_residual(lq, case):
    twist = 0.0
    if case == "wilson_near_critical":
        dims, kappa, csw, eps, block = (8, 8, 8, 32), 0.1245, 0.0, 0.1, (4, 4, 4, 4)
    elif case == "clover":
        dims, kappa, csw, eps, block = (8, 8, 8, 16), 0.1355, 1.7, 0.5, (4, 4, 4, 4)
    else:
        dims, kappa, csw, eps, block = (8, 8, 8, 32), 0.1245, 0.0, 0.1, (4, 4, 4, 4)
        twist = 0.01
    U = gauge_exp(dims, eps, 9601)
    ref = oracle.Operator(dims, U, kappa, csw, ANTIPERIODIC_T, twist=twist)
    op = lq.Operator(dims, kappa, csw, ANTIPERIODIC_T, link_recon=12, twist=twist)
    op.set_gauge(to_dev(U))
    nv = 8
    h = lq.Multigrid(op, to_dev(gaussian_spinor(dims, 9602, nv)),
                     lq.MGParams(block=block, nvec=nv, setup_iters=2, smooth_steps=4, coarse_tol=0.05))
    b = gaussian_spinor(dims, 9603)
    tol = 1e-10
    x, st = h.solve(to_dev(b), lq.SolverParams(tol=tol, inner_tol=1e-5))
    x = to_host(x)
    res = oracle.true_residual(ref, x, b)
    _, sb = op.solve(to_dev(b), "D", lq.SolverParams(tol=tol, inner="f32", inner_tol=1e-5))
    announce("mg %s %s: GCR iterations %d (outer %d), %.1f ms; oracle residual %.2e; "
             "BiCGStab (even-odd, FP32 inner) %d iterations %.1f ms" %
             (case, dims, st.nconv, st.nouter, st.t_solve_ms, res, sb[0].nconv, sb[0].t_solve_ms))
    assert st.converged and res <= tol * 1.01
    xr, _ = oracle.solve_eo(ref, b, tol=1e-13)
    assert rel_err(x, xr) < 1e-6
    assert st.nconv < sb[0].nconv
    h.close()
    op.close()


def test_multigrid_setup_groups_and_bound_operator(lq):
    """The near-null vectors' inverse iterations run as multi-RHS solves: on
    an operator bound to a workspace of 2 right-hand sides they run in
    groups of 2.  The vectors are the same whichever grouping (each system
    of a multi-RHS solve is solved as on its own only up to the outer
    loop's choices, so they are compared to the solver's tolerance), and the
    hierarchy solves to the oracle's residual."""
    dims, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 4
    U = gauge_exp(dims, 0.4, 9801)
    ref = oracle.Operator(dims, U, 0.125, 0.0, ANTIPERIODIC_T)
    v0 = to_dev(gaussian_spinor(dims, 9802, nv))
    prm = lq.MGParams(block=block, nvec=nv, setup_iters=1)
    vecs = {}
    for bound in (False, True):
        op = lq.Operator(dims, 0.125, 0.0, ANTIPERIODIC_T)
        if bound:
            op.bind(nrhs=2)
        op.set_gauge(to_dev(U))
        h = lq.Multigrid(op, v0, prm)
        vecs[bound] = to_host(h.vectors())
        b = gaussian_spinor(dims, 9803)
        x, st = h.solve(to_dev(b), lq.SolverParams(tol=1e-10, inner_tol=1e-5))
        assert st.converged and oracle.true_residual(ref, to_host(x), b) <= 1.01e-10
        if bound:
            assert op.get_option("owned_kib") == 0
        h.close()
        op.close()
    assert rel_err(vecs[True], vecs[False]) < 1e-2
    announce("mg set-up on a bound operator: vectors within %.1e of the unbound set-up" %
             rel_err(vecs[True], vecs[False]))


def test_multigrid_argument_errors(lq):
    import ctypes
    from paper_2111_04457_amd import _lib
    lib = _lib.load()
    dims = (8, 8, 8, 8)
    op = lq.Operator(dims, 0.12, 0.0, ANTIPERIODIC_T)
    v0 = to_dev(gaussian_spinor(dims, 9701, 2))
    with pytest.raises(lq.LQError) as e:  # no gauge field
        lq.Multigrid(op, v0, lq.MGParams(block=(2, 2, 2, 2), nvec=2))
    assert e.value.status == -2
    op.set_gauge(to_dev(gauge_exp(dims, 0.3, 9702)))
    for bad in (dict(block=(3, 2, 2, 2)), dict(block=(8, 2, 2, 2)), dict(block=(1, 2, 2, 2)),
                dict(block=(4, 4, 4, 4), nvec=0), dict(nvec=33), dict(gcr_restart=0), dict(coarse_tol=1.0),
                dict(setup_tol=0.0)):
        prm = dict(block=(2, 2, 2, 2), nvec=2)
        prm.update(bad)
        p = lq.MGParams(**prm).to_c()
        h = ctypes.c_void_p()
        assert lib.lq_mg_create(op.handle, ctypes.byref(p), ctypes.c_void_p(v0.data_ptr()), ctypes.byref(h),
                                None) == -1, bad
    op.close()
