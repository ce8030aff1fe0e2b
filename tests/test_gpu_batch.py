"""Multi-RHS and ragged-batch solves.

- The 12 spin-colour point sources of one propagator (Fig. 1) on a
  Wilson-clover lattice solved as one 12-RHS solve (each loaded link used
  for several right-hand sides) match the oracle's true residual.
- A ragged batch of lattices of different volumes, 4 Gaussian sources each,
  solved with lq_batch_solve (each stage of an inner iteration one launch
  over all lattices' systems, every chunk of inner iterations captured in
  one hipGraph) equals the per-lattice solves bit for bit, and every system
  reaches its true FP64 residual (oracle's D).  Batches of more lattices
  than one launch takes (8) run in groups of 8 with the same result; with
  four or more right-hand sides per lattice the batched kernels take four
  per workgroup (links in LDS) with the same bits.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import ANTIPERIODIC_T, gauge_exp, gaussian_spinor, point_sources
from tests.gpu_common import announce, have_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

KAPPA, CSW, EPS = 0.135, 1.7, 0.5


@pytest.fixture(scope="module")
def lq():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


@pytest.mark.parametrize("nr", [1, 2])
def test_twelve_point_sources_multi_rhs(lq, nr):
    dims = (8, 8, 8, 12)
    U = gauge_exp(dims, EPS, 1701)
    ref = oracle.Operator(dims, U, KAPPA, CSW, ANTIPERIODIC_T)
    src = point_sources(dims)
    op = lq.Operator(dims, KAPPA, CSW, ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(to_dev(U))
    op.set_option("rhs_per_thread", nr)
    X, st = op.solve(to_dev(src), "D", lq.SolverParams(tol=1e-10, inner="f16", inner_tol=1e-2))
    X = to_host(X)
    worst = 0.0
    for k in range(12):
        res = oracle.true_residual(ref, X[k], src[k])
        worst = max(worst, res)
        assert st[k].converged and res <= 1.01e-10, (k, res)
    announce("12 point sources nr=%d: iters %s worst oracle residual %.2e" % (nr, [s.nconv for s in st], worst))
    op.close()


def test_ragged_batch_equals_single_solves(lq):
    dims_list = [(4, 4, 4, 4), (6, 6, 6, 6), (8, 8, 8, 16), (10, 10, 10, 20)]
    Us = [gauge_exp(d, EPS, 1801 + i) for i, d in enumerate(dims_list)]
    bs = [gaussian_spinor(d, 2801 + i, 4) for i, d in enumerate(dims_list)]
    prm = lq.SolverParams(tol=1e-10, inner="f32", check_every=4)
    ops = []
    for d, U in zip(dims_list, Us):
        op = lq.Operator(d, KAPPA, CSW, ANTIPERIODIC_T)
        op.set_gauge(to_dev(U))
        ops.append(op)
    batch = lq.Batch(ops, [4] * len(ops))
    xs, st = batch.solve([to_dev(b) for b in bs], prm)
    xs2, st2 = batch.solve([to_dev(b) for b in bs], prm)  # replays the cached graphs
    for i, (op, d, U, b) in enumerate(zip(ops, dims_list, Us, bs)):
        x1, s1 = op.solve(to_dev(b), "D", prm)
        xb = to_host(xs[i])
        assert np.array_equal(xb, to_host(x1)) and np.array_equal(xb, to_host(xs2[i])), d
        ref = oracle.Operator(d, U, KAPPA, CSW, ANTIPERIODIC_T)
        for k in range(4):
            res = oracle.true_residual(ref, xb[k], b[k])
            assert res <= 1.01e-10, (d, k, res)
        assert [s.nconv for s in s1] == [s.nconv for s in st[4 * i:4 * i + 4]]
    announce("ragged batch iters %s" % [s.nconv for s in st])
    batch.close()
    for op in ops:
        op.close()


def test_batch_rejects_duplicate_operator(lq):
    d = (4, 4, 4, 4)
    op = lq.Operator(d, KAPPA, 0.0)
    with pytest.raises(lq.LQError):
        lq.Batch([op, op], [1, 1])
    op.close()


def test_ragged_batch_of_nine_lattices_left_preconditioned(lq):
    """Nine lattices (two launches of the batched hopping kernel per stage),
    1 to 3 right-hand sides each, FP16 inner BiCGStab on the
    A_ee^-1-preconditioned system: bit for bit the separate solves."""
    dims_list = [(4, 4, 4, 4), (4, 4, 2, 6), (6, 4, 4, 4), (2, 4, 4, 8), (4, 6, 4, 6), (8, 4, 4, 4),
                 (4, 4, 4, 8), (6, 6, 4, 4), (4, 8, 4, 4)]
    nr = [1 + (i % 3) for i in range(len(dims_list))]
    prm = lq.SolverParams(tol=1e-10, inner="f16", inner_tol=5e-3, check_every=3, left_precond=True)
    ops, bs, Us = [], [], []
    for i, d in enumerate(dims_list):
        U = gauge_exp(d, EPS, 1901 + i)
        op = lq.Operator(d, KAPPA, CSW, ANTIPERIODIC_T, link_recon=12)
        op.set_gauge(to_dev(U))
        ops.append(op)
        Us.append(U)
        bs.append(gaussian_spinor(d, 2901 + i, nr[i]))
    batch = lq.Batch(ops, nr)
    xs, st = batch.solve([to_dev(b) for b in bs], prm)
    k = 0
    for i, (op, d) in enumerate(zip(ops, dims_list)):
        x1, s1 = op.solve(to_dev(bs[i]), "D", prm)
        assert np.array_equal(to_host(xs[i]), to_host(x1)), d
        assert [s.nconv for s in s1] == [s.nconv for s in st[k:k + nr[i]]]
        ref = oracle.Operator(d, Us[i], KAPPA, CSW, ANTIPERIODIC_T)
        xb = to_host(xs[i]).reshape((nr[i],) + bs[i].shape[-6:])
        bb = bs[i].reshape(xb.shape)
        for r in range(nr[i]):
            assert oracle.true_residual(ref, xb[r], bb[r]) <= 1.01e-10, (d, r)
        k += nr[i]
    announce("nine-lattice batch iters %s" % [s.nconv for s in st])
    batch.close()
    for op in ops:
        op.close()


def test_ragged_batch_lds_groups_bitwise(lq):
    """With at least four right-hand sides per lattice the batched hopping
    kernels take four per workgroup with the links in LDS (groups that do
    not fill the workgroup included): the same bits as the separate solves,
    and as the batch with one right-hand side per thread."""
    dims_list = [(4, 4, 4, 4), (6, 4, 4, 8), (8, 8, 8, 8)]
    nr = [4, 5, 6]
    prm = lq.SolverParams(tol=1e-10, inner="f16", inner_tol=5e-3, check_every=4, left_precond=True)
    ops, bs, Us = [], [], []
    for i, d in enumerate(dims_list):
        U = gauge_exp(d, EPS, 1961 + i)
        op = lq.Operator(d, KAPPA, CSW, ANTIPERIODIC_T, link_recon=12)
        op.set_gauge(to_dev(U))
        ops.append(op)
        Us.append(U)
        bs.append(gaussian_spinor(d, 2961 + i, nr[i]))
    batch = lq.Batch(ops, nr)
    xs, st = batch.solve([to_dev(b) for b in bs], prm)
    k = 0
    for i, (op, d) in enumerate(zip(ops, dims_list)):
        x1, s1 = op.solve(to_dev(bs[i]), "D", prm)
        assert np.array_equal(to_host(xs[i]), to_host(x1)), d
        assert [s.nconv for s in s1] == [s.nconv for s in st[k:k + nr[i]]]
        ref = oracle.Operator(d, Us[i], KAPPA, CSW, ANTIPERIODIC_T)
        xb = to_host(xs[i])
        for r in range(nr[i]):
            assert oracle.true_residual(ref, xb[r], bs[i][r]) <= 1.01e-10, (d, r)
        k += nr[i]
    ops[0].set_option("rhs_per_thread", 1)  # the batch then runs one per thread
    xs1, _ = batch.solve([to_dev(b) for b in bs], prm)
    for i in range(len(ops)):
        assert np.array_equal(to_host(xs1[i]), to_host(xs[i]))
    announce("LDS-group batch iters %s" % [s.nconv for s in st])
    batch.close()
    for op in ops:
        op.close()


def test_batch_rejects_mixed_operators(lq):
    """A batch needs one link format and one kind of operator (all clover or
    all Wilson), and solves the even-odd system."""
    d = (4, 4, 4, 4)
    a = lq.Operator(d, KAPPA, CSW, ANTIPERIODIC_T, link_recon=12)
    b = lq.Operator(d, KAPPA, CSW, ANTIPERIODIC_T, link_recon=18)
    with pytest.raises(lq.LQError, match="link format"):
        lq.Batch([a, b], [1, 1])
    c = lq.Operator(d, KAPPA, 0.0, ANTIPERIODIC_T, link_recon=12)
    U = gauge_exp(d, EPS, 1950)
    for o in (a, c):
        o.set_gauge(to_dev(U))
    batch = lq.Batch([a, c], [1, 1])
    src = [to_dev(gaussian_spinor(d, 2950)), to_dev(gaussian_spinor(d, 2951))]
    with pytest.raises(lq.LQError, match="clover"):
        batch.solve(src, lq.SolverParams(tol=1e-10))
    batch.close()
    batch = lq.Batch([a], [1])
    with pytest.raises(lq.LQError, match="even-odd"):
        batch.solve(src[:1], lq.SolverParams(tol=1e-10, solver="cgne", even_odd=False))
    batch.close()
    for o in (a, b, c):
        o.close()
