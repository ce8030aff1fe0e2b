"""The operator on a caller-owned workspace (lq_op_workspace_bytes +
lq_op_bind: the device memory is one torch tensor, the library allocates
none) and the host-memory variants of set_gauge / apply / solve.

Each result is compared bit for bit with the same call on an operator that
allocates its own memory (the same kernels run), and against the oracle:
the Schur apply to 1e-12 (FP64), every solve to its true FP64 residual
recomputed by the oracle's D.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import ANTIPERIODIC_T, gauge_exp, gaussian_parity_spinor, gaussian_spinor
from tests.gpu_common import announce, have_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

DIMS, KAPPA, CSW = (8, 8, 4, 8), 0.13, 1.0


@pytest.fixture(scope="module")
def lq():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


@pytest.fixture(scope="module")
def case():
    U = gauge_exp(DIMS, 0.3, 1301)
    ref = oracle.Operator(DIMS, U, KAPPA, CSW, ANTIPERIODIC_T)
    return U, ref


KINDS = ("D", "Ddag", "DdagD", "schur", "schur_dag", "schur_normal", "schur_left", "hop_eo", "hop_oe",
         "clover_e", "clover_o", "clover_inv_o")


def test_bound_workspace_same_bits_and_no_allocation(lq, case):
    U, ref = case
    announce("workspace: bound 8x8x4x8 clover operator, every kind, f64/f32/f16, and a 2-rhs solve")
    torch = pytest.importorskip("torch")
    own = lq.Operator(DIMS, KAPPA, CSW, ANTIPERIODIC_T, link_recon=12)
    own.set_gauge(to_dev(U))
    op = lq.Operator(DIMS, KAPPA, CSW, ANTIPERIODIC_T, link_recon=12)
    assert op.get_option("owned_kib") == 0  # creation allocates no device memory
    ws = op.bind(nrhs=2)
    assert ws.numel() == op.workspace_bytes(2) == lq.workspace_bytes(DIMS, CSW, 12, 2)
    assert op.get_option("bound_nrhs") == 2
    op.set_gauge(to_dev(U))
    full = gaussian_spinor(DIMS, 2301, 2)
    par = gaussian_parity_spinor(DIMS, 2302, 2)
    for kind in KINDS:
        src = full if kind in ("D", "Ddag", "DdagD") else par
        for prec in ("f64", "f32", "f16"):
            a = to_host(op.apply(kind, to_dev(src), prec))
            b = to_host(own.apply(kind, to_dev(src), prec))
            assert np.array_equal(a, b), (kind, prec)
    assert rel_err(to_host(op.apply("schur", to_dev(par[0]), "f64")), ref.schur(par[0])) < 1e-12
    prm = lq.SolverParams(tol=1e-10, inner="f16", inner_tol=5e-3, left_precond=True)
    x, st = op.solve(to_dev(full), "D", prm)
    x2, _ = own.solve(to_dev(full), "D", prm)
    assert torch.equal(x, x2)
    for i in range(2):
        res = oracle.true_residual(ref, to_host(x[i]), full[i])
        announce("  rhs %d iters %d oracle residual %.2e" % (i, st[i].nconv, res))
        assert res <= 1e-10
    assert op.get_option("owned_kib") == 0, "the bound operator allocated device memory"
    # more right-hand sides than the workspace holds: an argument error
    three = gaussian_spinor(DIMS, 2303, 3)
    with pytest.raises(lq.LQError, match="bound workspace"):
        op.solve(to_dev(three), "D", prm)
    with pytest.raises(lq.LQError, match="bound workspace"):
        op.apply("D", to_dev(three), "f64")
    # unbinding gives the memory back; the operator allocates on demand again
    op.unbind()
    op.set_gauge(to_dev(U))
    assert np.array_equal(to_host(op.apply("schur", to_dev(par), "f32")), to_host(own.apply("schur", to_dev(par), "f32")))
    assert op.get_option("owned_kib") > 0
    op.close()
    own.close()


def test_bound_wilson_operator_has_no_room_for_clover(lq):
    """A Wilson operator (csw = 0) bound without clover blocks: switching the
    clover term on is refused (no room), not allocated behind the caller."""
    U = gauge_exp(DIMS, 0.3, 1302)
    op = lq.Operator(DIMS, KAPPA, 0.0, ANTIPERIODIC_T)
    op.bind(1)
    op.set_gauge(to_dev(U))
    with pytest.raises(lq.LQError) as e:
        op.set_params(KAPPA, 1.0)
    assert e.value.status == -4
    assert op.get_option("owned_kib") == 0
    op.close()


def test_host_memory_variants_equal_device_calls(lq, case):
    U, ref = case
    announce("workspace: set_gauge / apply / solve from host memory")
    dev = lq.Operator(DIMS, KAPPA, CSW, ANTIPERIODIC_T)
    dev.set_gauge(to_dev(U))
    host = lq.Operator(DIMS, KAPPA, CSW, ANTIPERIODIC_T)
    host.bind(1)
    torch = pytest.importorskip("torch")
    host.set_gauge(torch.from_numpy(U))  # host tensor: lq_op_set_gauge_host
    b = gaussian_spinor(DIMS, 2304)
    pe = gaussian_parity_spinor(DIMS, 2305)
    for kind, src in (("D", b), ("schur", pe), ("schur_left", pe)):
        h = host.apply(kind, torch.from_numpy(src), "f32")
        assert h.device.type == "cpu"
        assert np.array_equal(h.numpy(), to_host(dev.apply(kind, to_dev(src), "f32"))), kind
    prm = lq.SolverParams(tol=1e-10, inner="f32")
    xh, st = host.solve(torch.from_numpy(b), "D", prm)
    xd, _ = dev.solve(to_dev(b), "D", prm)
    assert xh.device.type == "cpu"
    assert np.array_equal(xh.numpy(), to_host(xd))
    res = oracle.true_residual(ref, xh.numpy(), b)
    announce("  host solve iters %d oracle residual %.2e" % (st[0].nconv, res))
    assert res <= 1e-10
    assert host.get_option("owned_kib") == 0
    host.close()
    dev.close()


def test_bandwidth_probe_is_below_the_hbm_peak(lq):
    """The copy and read-only probes of the library over 1 GiB report a rate
    between 1 TB/s and the 8 TB/s HBM3E peak."""
    for mode in ("copy", "read"):
        gbs = lq.bandwidth_probe(1 << 30, mode, reps=5)
        announce("  %s probe %.0f GB/s" % (mode, gbs))
        assert 1000.0 < gbs < 8000.0, (mode, gbs)
