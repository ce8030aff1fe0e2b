"""hipGraph capture of the solvers' inner iterations and the autotuner.

A captured chunk of inner iterations is replayed many times per solve, with
the host's eager work (scalar read-back, outer FP64 steps) between replays;
the solution must equal, bit for bit, the solution of the same solve run
eagerly.  The autotuner must give bitwise-identical operator output for the
shape it picks, write and re-read its JSON cache, and leave the solver's
results unchanged.
"""
import json
import os

import numpy as np
import pytest

import oracle
from lattice_inputs import ANTIPERIODIC_T, gauge_exp, gaussian_spinor, gaussian_parity_spinor
from tests.gpu_common import announce, have_gpu, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

DIMS = (8, 4, 8, 8)
KAPPA, CSW = 0.13, 1.2


@pytest.fixture(scope="module")
def lq():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2111_04457_amd as lq
    return lq


@pytest.fixture(scope="module")
def inputs():
    return gauge_exp(DIMS, 0.4, 1601), gaussian_spinor(DIMS, 2601, 2)


@pytest.mark.parametrize("solver,inner", [("bicgstab", "f32"), ("bicgstab", "f16"), ("cgne", "f64")])
def test_graph_replays_equal_eager(lq, inputs, solver, inner):
    U, b = inputs
    announce("graph vs eager: %s %s" % (solver, inner))
    prm = lq.SolverParams(solver=solver, tol=1e-10, inner=inner, inner_tol=1e-2 if inner == "f16" else 1e-5,
                          check_every=4)
    res = {}
    for graphs in (0, 1):
        op = lq.Operator(DIMS, KAPPA, CSW, ANTIPERIODIC_T)
        op.set_gauge(to_dev(U))
        op.set_option("graphs", graphs)
        x1, st1 = op.solve(to_dev(b), "D", prm)
        x2, st2 = op.solve(to_dev(b), "D", prm)  # second solve replays cached graphs
        res[graphs] = (to_host(x1), to_host(x2), st1, st2)
        op.close()
    e, g = res[0], res[1]
    assert np.array_equal(e[0], g[0]) and np.array_equal(e[1], g[1]) and np.array_equal(g[0], g[1])
    assert [s.nconv for s in e[2]] == [s.nconv for s in g[2]]
    assert all(s.converged for s in g[2])


def test_tuner_bitwise_cache_and_solve(lq, inputs, tmp_path):
    U, b = inputs
    ref = oracle.Operator(DIMS, U, KAPPA, CSW, ANTIPERIODIC_T)
    op = lq.Operator(DIMS, KAPPA, CSW, ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(to_dev(U))
    xe = gaussian_parity_spinor(DIMS, 2602)
    before = {p: to_host(op.apply("schur", to_dev(xe), p)) for p in ("f64", "f32", "f16")}
    cache = str(tmp_path / "tune.json")
    rep = op.tune(1, cache)
    announce("tune report %s" % json.dumps(rep))
    assert len(rep) == 3 and all(not v["cached"] for v in rep.values())
    for p in ("f64", "f32", "f16"):
        assert op.get_option("hop_block_" + p) in (64, 128, 256)
        assert np.array_equal(to_host(op.apply("schur", to_dev(xe), p)), before[p])
    data = json.load(open(cache))
    assert set(data) == set(rep)
    rep2 = op.tune(1, cache)
    assert all(v["cached"] for v in rep2.values())
    x, st = op.solve(to_dev(b[0]), "D", lq.SolverParams(tol=1e-10, inner="f16", inner_tol=1e-2))
    assert st[0].converged and oracle.true_residual(ref, to_host(x), b[0]) <= 1.01e-10
    op.close()


def test_tuner_times_the_solver_form(lq, inputs, tmp_path):
    """Tuned on the A_ee^-1-preconditioned form with the fused dot products
    (what the inner BiCGStab of left_precond runs): the cache key names that
    form, the operator keeps the reported shapes, and a left-preconditioned
    solve on those shapes gives the bits it gave on the default shapes."""
    U, b = inputs
    ref = oracle.Operator(DIMS, U, KAPPA, CSW, ANTIPERIODIC_T)
    op = lq.Operator(DIMS, KAPPA, CSW, ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(to_dev(U))
    prm = lq.SolverParams(tol=1e-10, inner="f16", inner_tol=5e-3, left_precond=True)
    x0, st0 = op.solve(to_dev(b[0]), "D", prm)
    rep = op.tune(1, str(tmp_path / "tune_left.json"), left=True)
    announce("tune(left) report %s" % json.dumps(rep))
    assert len(rep) == 3 and all(k.startswith("schur_left_red_") for k in rep)
    for k, v in rep.items():
        p = k.split("_")[3]
        assert op.get_option("hop_block_" + p) == v["block"] and op.get_option("xcd_remap_" + p) == v["xcd_remap"]
    x1, st1 = op.solve(to_dev(b[0]), "D", prm)
    assert np.array_equal(to_host(x0), to_host(x1)) and st0[0].nconv == st1[0].nconv
    assert oracle.true_residual(ref, to_host(x1), b[0]) <= 1.01e-10
    op.close()


def test_tuner_multi_rhs_shapes_bitwise(lq, inputs):
    """With several right-hand sides the tuner also sweeps the number of
    right-hand sides per thread (two per thread in binary16, four per
    workgroup in binary16 and FP32); every shape must give the same bits
    (the tuner rejects the sweep otherwise), so the output is unchanged."""
    U, _ = inputs
    op = lq.Operator(DIMS, KAPPA, CSW, ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(to_dev(U))
    xe = np.stack([gaussian_parity_spinor(DIMS, 2610 + i) for i in range(5)])
    before = {p: to_host(op.apply("schur", to_dev(xe), p)) for p in ("f64", "f32", "f16")}
    rep = op.tune(5)
    announce("tune(5) report %s" % json.dumps(rep))
    for p in ("f64", "f32", "f16"):
        assert op.get_option("rhs_per_thread_" + p) in {"f64": (1, 4), "f32": (1, 4), "f16": (1, 2, 4)}[p]
        assert np.array_equal(to_host(op.apply("schur", to_dev(xe), p)), before[p])
    for p, nr in (("f32", 1), ("f32", 2), ("f32", 4), ("f16", 1), ("f16", 2), ("f16", 4), ("f64", 2), ("f64", 4)):
        op.set_option("rhs_per_thread_" + p, nr)
        assert np.array_equal(to_host(op.apply("schur", to_dev(xe), p)), before[p]), (p, nr)
    op.close()


@pytest.mark.parametrize("dims,nrhs", [((8, 4, 8, 8), 4), ((8, 4, 8, 8), 6), ((6, 4, 4, 10), 12), ((4, 4, 2, 6), 5)])
def test_lds_shared_rhs_bitwise(lq, dims, nrhs):
    """Four right-hand sides per workgroup with the links (and, in FP16 and
    FP32, the clover blocks) staged in LDS give the bits of one right-hand
    side per thread: every kind of the hopping kernel (plain, clover on the
    result, clover on y with the axpy, the Schur operator and its dagger),
    FP16, FP32 and FP64, with
    groups of right-hand sides that do not fill the workgroup and site
    blocks that are cut by the lattice's end (480 and 96 sites per parity)."""
    U = gauge_exp(dims, 0.4, 1611)
    op = lq.Operator(dims, KAPPA, CSW, ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(to_dev(U))
    xe = to_dev(np.stack([gaussian_parity_spinor(dims, 2620 + i) for i in range(nrhs)]))
    for p in ("f16", "f32", "f64"):
        for kind in ("hop_eo", "hop_oe_dag", "clover_inv_o", "schur", "schur_dag", "schur_normal", "schur_left"):
            op.set_option("rhs_per_thread_" + p, 1)
            ref = to_host(op.apply(kind, xe, p))
            op.set_option("rhs_per_thread_" + p, 4)
            got = to_host(op.apply(kind, xe, p))
            assert np.array_equal(got, ref), (p, kind, float(np.abs(got - ref).max()))
    # a multi-RHS solve with the fused dot products in the shared kernel
    b = to_dev(gaussian_spinor(dims, 2630, nrhs))
    prm = lq.SolverParams(solver="bicgstab", tol=1e-10, inner="f16", inner_tol=1e-2, check_every=4)
    res = {}
    for nr in (1, 4):
        op.set_option("rhs_per_thread", nr)
        x, st = op.solve(b, "D", prm)
        res[nr] = (to_host(x), [s.nconv for s in st])
        assert all(s.converged for s in st)
    assert np.array_equal(res[1][0], res[4][0]) and res[1][1] == res[4][1]
    op.close()


@pytest.mark.parametrize("dims", [(16, 8, 4, 8), (32, 4, 4, 4), (16, 16, 4, 6)])
def test_lds_staged_neighbours_bitwise(lq, dims):
    """The hopping kernel with each tile's neighbour spinors staged in LDS
    (binary16, one right-hand side) gives the bits of the ordinary kernel in
    every operator kind, and a left-preconditioned solve with the fused dot
    products gives the same solution and iteration count."""
    U = gauge_exp(dims, 0.4, 1631)
    op = lq.Operator(dims, KAPPA, CSW, ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(to_dev(U))
    xe = to_dev(gaussian_parity_spinor(dims, 2640))
    xf = to_dev(gaussian_spinor(dims, 2641))
    for kind in ("hop_eo", "hop_oe", "hop_eo_dag", "hop_oe_dag", "schur", "schur_dag", "schur_normal",
                 "schur_left", "D", "Ddag", "DdagD"):
        src = xf if kind in ("D", "Ddag", "DdagD") else xe
        op.set_option("halo_f16", 0)
        ref = to_host(op.apply(kind, src, "f16"))
        op.set_option("halo_f16", 1)
        got = to_host(op.apply(kind, src, "f16"))
        assert np.array_equal(got, ref), kind
    prm = lq.SolverParams(tol=1e-10, inner="f16", inner_tol=5e-3, left_precond=True)
    res = {}
    for h in (0, 1):
        op.set_option("halo_f16", h)
        x, st = op.solve(xf, "D", prm)
        res[h] = (to_host(x), st[0].nconv)
        assert st[0].converged
    assert np.array_equal(res[0][0], res[1][0]) and res[0][1] == res[1][1]
    op.close()
