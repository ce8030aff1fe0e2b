"""lq_op_apply_noalloc: the operator apply that allocates no device memory
(its packed fields live in a fixed per-GPU array of the library), for
callers that cannot allocate.

Checked through the C ABI against lq_op_apply on the same seeded inputs:
the two run the same kernels, so their outputs must be the same bits.  Two
calls in a row, the second with a smaller input (fewer right-hand sides,
then a smaller lattice), so that a stale tail of the shared array left by
the first call cannot go unnoticed; a call too large for the array is
rejected before any device work; and an operator that only ever used this
entry point has allocated no work buffer.
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import ANTIPERIODIC_T, gauge_exp, gaussian_parity_spinor, gaussian_spinor
from tests.gpu_common import announce, have_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

KINDS_PARITY = ("schur", "schur_dag", "schur_normal", "schur_left", "hop_oe", "clover_inv_o")
KINDS_FULL = ("D", "DdagD")


@pytest.fixture(scope="module")
def lq():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


def _op(lq, dims, seed, recon=12):
    U = gauge_exp(dims, 0.3, seed)
    op = lq.Operator(dims, 0.13, 1.0, ANTIPERIODIC_T, link_recon=recon)
    op.set_gauge(to_dev(U))
    return op, U


def _both(lq, op, kind, psi, prec):
    out = lq_out = None
    import torch
    out = torch.empty_like(psi)
    op.apply_noalloc(kind, psi, out, prec)
    lq_out = op.apply(kind, psi, prec)
    return to_host(out), to_host(lq_out)


def test_noalloc_equals_apply_two_calls_shrinking(lq):
    op_big, _ = _op(lq, (8, 8, 4, 8), 3101)
    op_small, U_small = _op(lq, (4, 4, 4, 4), 3102)
    for prec in ("f64", "f32", "f16"):
        for kind in KINDS_PARITY + KINDS_FULL:
            announce("noalloc %s %s: 8x8x4x8 nrhs 3, then nrhs 1, then 4^4 nrhs 1" % (kind, prec))
            full = kind in KINDS_FULL
            gen = gaussian_spinor if full else gaussian_parity_spinor
            calls = ((op_big, (8, 8, 4, 8), 3), (op_big, (8, 8, 4, 8), 1), (op_small, (4, 4, 4, 4), 1))
            for k, (op, dims, nrhs) in enumerate(calls):
                psi = to_dev(gen(dims, 3200 + k, nrhs if nrhs > 1 else None))
                got, want = _both(lq, op, kind, psi, prec)
                assert np.array_equal(got, want), (kind, prec, dims, nrhs)
    # the small lattice against the oracle (FP64 Schur operator)
    ref = oracle.Operator((4, 4, 4, 4), U_small, 0.13, 1.0, ANTIPERIODIC_T)
    xe = gaussian_parity_spinor((4, 4, 4, 4), 3301)
    import torch
    out = torch.empty(xe.shape, dtype=torch.complex128, device="cuda")
    op_small.apply_noalloc("schur", to_dev(xe), out, "f64")
    assert rel_err(to_host(out), ref.schur(xe)) < 1e-12
    op_big.close()
    op_small.close()


def test_noalloc_allocates_nothing_and_rejects_oversize(lq):
    import torch
    dims = (16, 16, 16, 32)
    op, _ = _op(lq, dims, 3401)
    assert op.get_option("work_kib") == 0
    xe = to_dev(gaussian_parity_spinor(dims, 3402))
    out = torch.empty_like(xe)
    # FP64 Schur operator at 16^3 x 32: three packed parity fields, 37.7 MB
    announce("noalloc schur f64 16x16x16x32")
    op.apply_noalloc("schur", xe, out, "f64")
    torch.cuda.synchronize()
    assert op.get_option("work_kib") == 0
    want = op.apply("schur", xe, "f64")
    assert np.array_equal(to_host(out), to_host(want))
    assert op.get_option("work_kib") > 0  # lq_op_apply keeps its temporaries
    # D^dag D in FP64 needs three full packed fields (75.5 MB > 64 MiB)
    b = to_dev(gaussian_spinor(dims, 3403))
    with pytest.raises(lq.LQError) as e:
        op.apply_noalloc("DdagD", b, torch.empty_like(b), "f64")
    assert e.value.status == -1 and "scratch" in str(e.value)
    op.close()
