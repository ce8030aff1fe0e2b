"""Parity of every operator apply of the HIP library against the oracle.

Element-by-element comparison on the same seeded inputs, lattices that span
several 256-site workgroups with a ragged tail, complex boundary phases,
two right-hand sides.  Tolerances (relative 2-norm of the difference):
FP64 1e-12, FP32 1e-5 (per apply), FP16 storage with FP32 arithmetic 5e-3
(binary16 rounding of links, spinors and clover, 2^-11 relative each).
"""
import numpy as np
import pytest

import oracle
from lattice_inputs import gauge_exp, gauge_haar, gaussian_parity_spinor, gaussian_spinor
from tests.gpu_common import announce, have_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 5e-3}
BC = (1.0, np.exp(0.7j), 1.0, -1.0)


@pytest.fixture(scope="module")
def lib():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


CASES = {
    # name: dims, kappa, csw, link generator
    "wilson_6x4x6x10": ((6, 4, 6, 10), 0.13, 0.0, "haar"),
    "clover_6x4x6x10": ((6, 4, 6, 10), 0.13, 1.7, "exp"),
    "clover_8x8x4x12": ((8, 8, 4, 12), 0.1355, 1.0, "exp"),
    # extent 2 in x and z: x+mu and x-mu are the same site, both terms summed
    "clover_2x4x2x6": ((2, 4, 2, 6), 0.12, 1.3, "exp"),
}


def _setup(name):
    dims, kappa, csw, gen = CASES[name]
    U = gauge_haar(dims, 501) if gen == "haar" else gauge_exp(dims, 0.5, 501)
    return dims, kappa, csw, U


_ORACLES = {}


def _oracle(name):
    if name not in _ORACLES:
        dims, kappa, csw, U = _setup(name)
        _ORACLES[name] = (oracle.Operator(dims, U, kappa, csw, BC), U)
    return _ORACLES[name]


def _reference(op, kind, psi):
    """oracle result for a kind on one right-hand side"""
    if kind == "D":
        return op.D(psi)
    if kind == "Ddag":
        return op.Ddag(psi)
    if kind == "DdagD":
        return op.DdagD(psi)
    if kind == "schur":
        return op.schur(psi)
    if kind == "schur_dag":
        return op.schur_dag(psi)
    if kind == "schur_normal":
        return op.schur_normal(psi)
    if kind == "hop_eo":
        return op.hop_to(0, psi)
    if kind == "hop_oe":
        return op.hop_to(1, psi)
    if kind == "hop_eo_dag":
        return op.hop_to(0, psi, dagger=True)
    if kind == "hop_oe_dag":
        return op.hop_to(1, psi, dagger=True)
    if kind == "clover_e":
        return op.clover_apply(0, psi)
    if kind == "clover_o":
        return op.clover_apply(1, psi)
    if kind == "clover_inv_o":
        return op.clover_apply(1, psi, inverse=True)
    if kind == "schur_left":
        # A_ee^-1 M (A = 1 for Wilson)
        return op.clover_apply(0, op.schur(psi), inverse=True)
    raise ValueError(kind)


KINDS = ["D", "Ddag", "DdagD", "schur", "schur_dag", "schur_normal", "hop_eo", "hop_oe", "hop_eo_dag",
         "hop_oe_dag", "clover_e", "clover_o", "clover_inv_o", "schur_left"]


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec,recon", [("f64", 18), ("f64", 12), ("f32", 18), ("f32", 12), ("f16", 18), ("f16", 12)])
def test_apply_all_kinds(lib, case, prec, recon):
    announce("apply parity: case=%s prec=%s recon=%d" % (case, prec, recon))
    op_ref, U = _oracle(case)
    dims, kappa, csw, _ = _setup(case)
    op = lib.Operator(dims, kappa, csw, BC, link_recon=recon)
    op.set_gauge(to_dev(U))
    nrhs = 2
    full = gaussian_spinor(dims, 601, nrhs)
    half = gaussian_parity_spinor(dims, 602, nrhs)
    for kind in KINDS:
        if csw == 0.0 and kind.startswith("clover"):
            continue
        is_full = kind in ("D", "Ddag", "DdagD")
        src = full if is_full else half
        got = to_host(op.apply(kind, to_dev(src), prec))
        for r in range(nrhs):
            ref = _reference(op_ref, kind, src[r])
            err = rel_err(got[r], ref)
            assert err < TOL[prec], (kind, r, err)
    op.close()


def test_f64_hop_bitwise_across_workgroup_sizes(lib):
    """The per-site accumulation order does not depend on the launch shape."""
    import ctypes
    case = "clover_6x4x6x10"
    dims, kappa, csw, U = _setup(case)
    op = lib.Operator(dims, kappa, csw, BC)
    op.set_gauge(to_dev(U))
    src = to_dev(gaussian_parity_spinor(dims, 603))
    outs = []
    for block in (64, 128, 256):
        lib.load().lq_op_set_block(op.handle, 0, block)
        outs.append(to_host(op.apply("schur", src, "f64")))
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    op.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_bitwise_across_workgroup_orders_and_sizes(lib, prec):
    """Every workgroup order (plain, XCD-aware, time slices interleaved) and
    size gives the same bits; 8x8x4x20 has 128 sites of a parity per time
    slice, so the interleaved order is active for 64 and 128 threads (groups
    of 2 slices) and falls back to the XCD order for 256."""
    dims, kappa, csw = (8, 8, 4, 20), 0.13, 1.5
    U = gauge_exp(dims, 0.5, 611)
    op = lib.Operator(dims, kappa, csw, BC, link_recon=12)
    op.set_gauge(to_dev(U))
    src = to_dev(gaussian_parity_spinor(dims, 612, 3))
    ref = oracle.Operator(dims, U, kappa, csw, BC)
    outs = []
    for order in (0, 1, 2):
        op.set_option("xcd_remap_" + prec, order)
        for block in (64, 128, 256):
            op.set_block(prec, block)
            outs.append(to_host(op.apply("schur", src, prec)))
            outs.append(to_host(op.apply("hop_oe_dag", src, prec)))
    for k in range(2, len(outs)):
        assert np.array_equal(outs[k % 2], outs[k]), k
    for r in range(3):
        assert rel_err(outs[0][r], ref.schur(to_host(src)[r])) < TOL[prec]
    op.close()
