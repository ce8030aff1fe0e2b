"""Benchmark of the mixed-precision even-odd clover propagator solve.

One step = one complete solve D x = b to a true FP64 residual of 1e-10 on
the 32^3 x 64 Wilson-clover lattice (links exp(i 0.5 H), kappa 0.1355,
c_sw 1.7, antiperiodic in time): FP16-stored links and spinors with FP32
arithmetic in the inner BiCGStab (on the A_ee^-1-preconditioned Schur
operator by default), FP64 defect correction of M x = b outside, even-odd
prepare / reconstruct and the final residual included.

Printed: one JSON line.  `value` is the whole-step dslash throughput: the
algorithmic bytes of every hopping-term apply the solve performed (links,
spinor in/out, clover block, per apply) divided by the step time.  The
`roofline` entry times the solver's dominant kernels alone: the FP16
Schur operator (two fused hopping kernels, 12-real links) replayed from a
captured graph between HIP events on the stream it runs on; `cpu_baseline`
times the FP64 oracle's hopping term on the host cores.  Inputs are generated on the host and
copied to HBM before timing.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# the GPU solutions of the 16^3 x 32 ladder, compared with the oracle's in
# the cpu_baseline leg
C1_SOLUTIONS = {}


def _kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lq_common.h", "stencil.h", "dslash_impl.h", "dslash.h"):
        with open(os.path.join(ROOT, "paper_2111_04457_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic_from_profile(kernel_tag: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "schur_f16_32x32x32x64.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    # the tag names the kernels without the workgroup size the tuner picked
    if vals.get("kernel_source_hash") != _kernel_source_hash() or vals.get("kernel") != kernel_tag.split(" (")[0]:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _timed(torch, fn):
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, 1e3 * (time.perf_counter() - t)


def _graph_time_us(torch, fn, reps, replays=5):
    """Average duration of fn's launches: reps calls captured in one graph,
    each replay timed between two HIP events on the stream the kernels run
    on; the median of `replays` timed replays (after one untimed)."""
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(replays):
        e0.record(stream)
        g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    del g
    times.sort()
    return 1e3 * times[len(times) // 2] / reps


def _kernels(lq, torch, op, b_d, V, recon, reps, left):
    """Per-kernel figures on resident packed fields (no host work inside the
    timed region): the Schur operator of the solver (two fused hop kernels;
    its A_ee^-1-preconditioned form when left) in FP16 / FP32 / FP64 at the
    tuned launch shape, and the plain hopping term (even -> odd) at each
    workgroup size."""
    kind = "schur_left" if left else "schur"
    kern = {}
    roof = None
    bps_schur = {}
    for prec in ("f16", "f32", "f64"):
        fin = lq.Field(op, prec)
        fout = lq.Field(op, prec)
        fin.load(b_d.reshape(-1, 4, 3)[: V // 2].contiguous())
        us = _graph_time_us(torch, lambda: lq.apply_field(op, kind, fout, fin), reps)
        b1, f1 = op.traffic(prec, 1, clover=False)
        b2, f2 = op.traffic(prec, 1, clover=True)
        # kernel 1: clover-inverse epilogue (+ clover block); kernel 2: clover on y (or, preconditioned,
        # A_ee^-1 on the hopping term) and the axpy (+ clover block, + y)
        spinor = {"f16": 52.0, "f32": 96.0, "f64": 192.0}[prec]
        bps = (b2) + (b2 + spinor)
        bps_schur[prec] = bps
        kern["schur_%s_us" % prec] = us
        kern["schur_%s_GBs" % prec] = bps * (V // 2) / (us * 1e-6) / 1e9
        kern["schur_%s_block" % prec] = op.get_option("hop_block_" + prec)
        if prec == "f16":
            blk = op.get_option("hop_block_f16")
            gbs = kern["schur_f16_GBs"]
            roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                    "traffic": None,
                    "kernel": ("A_ee^-1-preconditioned Schur operator, FP16 storage, %d-real links: "
                               "hop_kernel<f16,%d,clov=inv> + hop_kernel<f16,%d,clov=inv on H,xpay> (%d threads)"
                               if left else
                               "Schur operator, FP16 storage, %d-real links: hop_kernel<f16,%d,clov=inv> + "
                               "hop_kernel<f16,%d,clov=y,xpay> (%d threads)") % (recon, recon, recon, blk),
                    "bytes_per_launch": bps * (V // 2), "avg_launch_us": us}
        tuned_blk = op.get_option("hop_block_" + prec)
        best = None
        for blk in (256, 128, 64):
            op.set_block(prec, blk)
            t = _graph_time_us(torch, lambda: lq.apply_field(op, "hop_oe", fout, fin), reps)
            kern["dslash_%s_b%d_us" % (prec, blk)] = t
            if best is None or t < best[1]:
                best = (blk, t)
        op.set_block(prec, tuned_blk)
        kern["dslash_%s_us" % prec] = best[1]
        kern["dslash_%s_block" % prec] = best[0]
        kern["dslash_%s_GBs" % prec] = b1 * (V // 2) / (best[1] * 1e-6) / 1e9
        # the count without spinor reuse (8 links + 8 neighbour spinors + 1
        # output = 360 reals per site, plus the binary16 spinors' 9 scales)
        rs = {"f64": 8, "f32": 4, "f16": 2}[prec]
        naive = 360 * rs + (9 * 4 if prec == "f16" else 0)
        kern["dslash_%s_naive_GBs" % prec] = naive * (V // 2) / (best[1] * 1e-6) / 1e9
        kern["dslash_%s_TFLOPs" % prec] = f1 * (V // 2) / (best[1] * 1e-6) / 1e12
        fin.close()
        fout.close()
    # the library's bandwidth probes over 1 GiB: a copy (bytes read + written)
    # and a read-only stream
    kern["copy_probe_GBs"] = lq.bandwidth_probe(1 << 30, "copy", reps=10)
    kern["read_probe_GBs"] = lq.bandwidth_probe(1 << 30, "read", reps=10)
    if roof is not None:
        roof["frac_of_copy_probe"] = roof["achieved"] / kern["copy_probe_GBs"]
        roof["frac_of_read_probe"] = roof["achieved"] / kern["read_probe_GBs"]
    return kern, roof


def _extras(lq, torch):
    """The other workloads, each timed once after a warm-up call (mixed solves
    with the A_ee^-1-preconditioned inner system):
    - the 12 spin-colour point sources of one propagator on 24^3x48 (clover,
      kappa 0.135, c_sw 1.7) as one 12-RHS solve vs 12 single solves;
    - a ragged batch 8^4, 12^4, 16^3x32, 20^3x40 (4 Gaussian sources each)
      in one batched solve vs separate solves;
    - time to solution on 16^3x32 clover (kappa 0.13, c_sw 1.0): FP64
      BiCGStab and CGNE vs FP32- and FP16-inner BiCGStab;
    - the pseudofermion force on 16^4 Wilson (kappa 0.125), FP64 and FP32;
    - the clover pseudofermion force on 16^3x32 (solve to 1e-10), FP64 and
      FP32 hopping part."""
    from lattice_inputs import (ANTIPERIODIC_T, RAGGED_DIMS, WORKLOADS, gaussian_parity_spinor, gaussian_spinor,
                                point_sources, workload_gauge, workload_source)
    out = {}
    # the batched workloads with their stated FP32 inner solve, and with
    # binary16 storage beside it
    prms = {"f32": lq.SolverParams(tol=1e-10, inner="f32", inner_tol=1e-5, check_every=10, left_precond=True),
            "f16": lq.SolverParams(tol=1e-10, inner="f16", inner_tol=5e-3, check_every=10, left_precond=True)}
    w = WORKLOADS["clover_24x24x24x48"]
    d = w["dims"]
    op = lq.Operator(d, w["kappa"], w["csw"], ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(torch.from_numpy(workload_gauge("clover_24x24x24x48")).cuda())
    op.tune(12, left=True)
    src = torch.from_numpy(point_sources(d)).cuda()
    for inner, prm in prms.items():
        tag = "" if inner == "f16" else "_f32"
        op.solve(src, "D", prm)
        (_, st), ms12 = _timed(torch, lambda: op.solve(src, "D", prm))
        op.solve(src[0], "D", prm)
        ms1 = 0.0
        for k in range(12):
            _, m = _timed(torch, lambda: op.solve(src[k], "D", prm))
            ms1 += m
        out["propagator_24x24x24x48_12rhs%s_ms" % tag] = ms12
        out["propagator_24x24x24x48_12_single%s_ms" % tag] = ms1
        out["propagator_12rhs%s_speedup" % tag] = ms1 / ms12
        out["propagator%s_max_diff" % tag] = max(s.diff for s in st)
        out["propagator%s_iters" % tag] = [s.nconv for s in st]
        print("bench: propagator inner %s %.1f ms (12 RHS) vs %.1f ms (12 single)" % (inner, ms12, ms1),
              file=sys.stderr, flush=True)
    op.close()

    ops, bs = [], []
    for i, dd in enumerate(RAGGED_DIMS):
        o = lq.Operator(dd, 0.135, 1.7, ANTIPERIODIC_T, link_recon=12)
        o.set_gauge(torch.from_numpy(workload_gauge("clover_24x24x24x48", dims=dd)).cuda())
        ops.append(o)
        bs.append(torch.from_numpy(gaussian_spinor(dd, 2003 + 10 * i, 4)).cuda())
    batch = lq.Batch(ops, [4] * len(ops))
    for inner, prm in prms.items():
        tag = "" if inner == "f16" else "_f32"
        batch.solve(bs, prm)
        (_, stb), msb = _timed(torch, lambda: batch.solve(bs, prm))
        mss = 0.0
        for o, b in zip(ops, bs):
            o.solve(b, "D", prm)
            _, m = _timed(torch, lambda: o.solve(b, "D", prm))
            mss += m
        out["ragged_batch%s_ms" % tag] = msb
        out["ragged_separate%s_ms" % tag] = mss
        out["ragged_batch%s_speedup" % tag] = mss / msb
        out["ragged%s_max_diff" % tag] = max(s.diff for s in stb)
        print("bench: ragged batch inner %s %.1f ms vs %.1f ms separate" % (inner, msb, mss), file=sys.stderr,
              flush=True)
    batch.close()
    for o in ops:
        o.close()

    w = WORKLOADS["clover_16x16x16x32"]
    d = w["dims"]
    op = lq.Operator(d, w["kappa"], w["csw"], ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(torch.from_numpy(workload_gauge("clover_16x16x16x32")).cuda())
    b1 = torch.from_numpy(workload_source("clover_16x16x16x32")).cuda()
    x64 = None
    for name, solver, inner, itol in (("fp64", "bicgstab", "f64", 1e-5), ("fp64_cgne", "cgne", "f64", 1e-5),
                                      ("mixed_f32", "bicgstab", "f32", 1e-5), ("mixed_f16", "bicgstab", "f16", 5e-3)):
        p1 = lq.SolverParams(solver=solver, tol=1e-10, inner=inner, inner_tol=itol, check_every=10,
                             left_precond=inner != "f64")
        op.solve(b1, "D", p1)
        (xs, st1), ms = _timed(torch, lambda: op.solve(b1, "D", p1))
        out["clover_16x16x16x32_%s_ms" % name] = ms
        out["clover_16x16x16x32_%s_iters" % name] = st1[0].nconv
        out["clover_16x16x16x32_%s_diff" % name] = st1[0].diff
        if name == "fp64":
            x64 = xs
        else:
            out["clover_16x16x16x32_%s_err_vs_fp64" % name] = float(torch.linalg.vector_norm(xs - x64) /
                                                                    torch.linalg.vector_norm(x64))
        C1_SOLUTIONS[name] = xs.cpu().numpy()
    op.close()
    print("bench: 16x16x16x32 ladder %s" % json.dumps({k: v for k, v in out.items() if k.startswith("clover_16")}),
          file=sys.stderr, flush=True)

    out.update(_forces(lq, torch))
    out.update(_eigs(lq, torch))
    out.update(_solver_variants(lq, torch))
    return out


def _forces(lq, torch):
    """The pseudofermion force (solve + force kernels), each timed once after
    a warm-up call: 16^4 Wilson (kappa 0.125) and 16^3x32 clover (kappa 0.13,
    c_sw 1.0), FP64 and FP32."""
    from lattice_inputs import ANTIPERIODIC_T, WORKLOADS, gaussian_parity_spinor, workload_gauge
    out = {}
    w = WORKLOADS["wilson_16x16x16x16"]
    d = w["dims"]
    op = lq.Operator(d, w["kappa"], 0.0, ANTIPERIODIC_T)
    op.set_gauge(torch.from_numpy(workload_gauge("wilson_16x16x16x16")).cuda())
    phi = torch.from_numpy(gaussian_parity_spinor(d, 2004)).cuda()
    for prec, inner in (("f64", "f64"), ("f32", "f32")):
        fp = lq.SolverParams(solver="cgne", tol=1e-12, inner=inner)
        lq.pf_force(op, phi, fp, "eo", prec)
        (res, ms) = _timed(torch, lambda: lq.pf_force(op, phi, fp, "eo", prec))
        out["force_16x16x16x16_%s_ms" % prec] = ms
        out["force_16x16x16x16_%s_iters" % prec] = res[4].nconv
    op.close()

    w = WORKLOADS["clover_16x16x16x32"]
    d = w["dims"]
    op = lq.Operator(d, w["kappa"], w["csw"], ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(torch.from_numpy(workload_gauge("clover_16x16x16x32")).cuda())
    phi = torch.from_numpy(gaussian_parity_spinor(d, 2005)).cuda()
    for prec, inner in (("f64", "f64"), ("f32", "f32")):
        fp = lq.SolverParams(solver="cgne", tol=1e-10, inner=inner)
        lq.pf_force(op, phi, fp, "eo", prec)
        (res, ms) = _timed(torch, lambda: lq.pf_force(op, phi, fp, "eo", prec))
        out["force_clover_16x16x16x32_%s_ms" % prec] = ms
        out["force_clover_16x16x16x32_%s_iters" % prec] = res[4].nconv
    op.close()
    out.update(_md(lq, torch))
    return out


def _md(lq, torch):
    """One molecular-dynamics trajectory (tau 1, 10 leapfrog steps, Wilson
    gauge action at beta 5.6 plus the even-odd pseudofermion; solves to
    1e-10 with an FP32 inner solve) on 16^4 Wilson and 16^3x32 clover,
    timed once after a warm-up trajectory from the same start."""
    from lattice_inputs import (ANTIPERIODIC_T, WORKLOADS, gaussian_parity_spinor, random_su3_algebra,
                                workload_gauge)
    out = {}
    sp = lq.SolverParams(solver="cgne", tol=1e-10, inner="f32")
    md = lq.MDParams(beta=5.6, tau=1.0, nsteps=10, integrator="leapfrog", fermion=True, force_prec="f32")
    for name in ("wilson_16x16x16x16", "clover_16x16x16x32"):
        w = WORKLOADS[name]
        d = w["dims"]
        op = lq.Operator(d, w["kappa"], w["csw"], ANTIPERIODIC_T, link_recon=12)
        U0 = torch.from_numpy(workload_gauge(name)).cuda()
        P0 = torch.from_numpy(random_su3_algebra(d, 2006)).cuda()
        phi = torch.from_numpy(gaussian_parity_spinor(d, 2007)).cuda()
        for _ in range(2):
            U, P = U0.clone(), P0.clone()
            st, ms = _timed(torch, lambda: lq.md_trajectory(op, U, P, phi, md, sp))
        out["md_%s_traj_ms" % name] = ms
        out["md_%s_dH" % name] = st.dH
        out["md_%s_n_force" % name] = st.n_force
        out["md_%s_iters" % name] = st.iters
        op.close()
    print("bench: md %s" % json.dumps(out), file=sys.stderr, flush=True)
    return out


def _eigs(lq, torch):
    """The 8 lowest eigenpairs of M^dag M on the 16^3x32 clover workload
    (FP64, residuals to 1e-8): thick-restart Lanczos with 64 basis vectors
    per cycle on the degree-8 Chebyshev filter (interval picked
    automatically), and without the filter; each timed once after a
    warm-up call."""
    from lattice_inputs import ANTIPERIODIC_T, WORKLOADS, gaussian_parity_spinor, workload_gauge
    name = "clover_16x16x16x32"
    w = WORKLOADS[name]
    d = w["dims"]
    op = lq.Operator(d, w["kappa"], w["csw"], ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(torch.from_numpy(workload_gauge(name)).cuda())
    v0 = torch.from_numpy(gaussian_parity_spinor(d, 2008)).cuda()
    out = {}
    for tag, degree in (("", 8), ("_plain", 0)):
        for _ in range(2):
            (ev, res, _, st), ms = _timed(torch, lambda: op.eigs(8, 64, v0=v0, tol=1e-8, cheb_degree=degree))
        out["eigs_%s%s_ms" % (name, tag)] = ms
        out["eigs_%s%s_stats" % (name, tag)] = st
        out["eigs_%s%s_max_resid" % (name, tag)] = float(max(res))
        if not tag:
            out["eigs_%s_lowest" % name] = [float(e) for e in ev]
    op.close()
    print("bench: eigs %s" % json.dumps(out), file=sys.stderr, flush=True)
    return out


def _solver_variants(lq, torch):
    """The solver variants on a near-critical Wilson lattice, 16^3x32 with
    smooth links (exp(i 0.1 H), kappa 0.1248, antiperiodic in time), one
    Gaussian source, true residual 1e-10, each timed once after a warm-up
    call: mixed BiCGStab (binary16 and FP32 storage), CG on the normal
    equations with FP32 storage restarted at every FP64 residual or with
    reliable updates, deflated by the 16 lowest eigenpairs of M^dag M, and
    the two-level multigrid (4^4 aggregates, 12 near-null vectors; the setup
    timed separately)."""
    from lattice_inputs import ANTIPERIODIC_T, gauge_exp, gaussian_parity_spinor, gaussian_spinor
    d, kappa = (16, 16, 16, 32), 0.1248
    tag = "wilson_16x16x16x32_k1248"
    op = lq.Operator(d, kappa, 0.0, ANTIPERIODIC_T, link_recon=12)
    op.set_gauge(torch.from_numpy(gauge_exp(d, 0.1, 4242)).cuda())
    b = torch.from_numpy(gaussian_spinor(d, 4243)).cuda()
    out = {}

    def run(name, fn):
        fn()
        (_, st), ms = _timed(torch, fn)
        st = st[0] if isinstance(st, list) else st
        out["%s_%s_ms" % (tag, name)] = ms
        out["%s_%s_iters" % (tag, name)] = st.nconv
        out["%s_%s_diff" % (tag, name)] = st.diff

    run("bicgstab_f16", lambda: op.solve(b, "D", lq.SolverParams(tol=1e-10, inner="f16", inner_tol=5e-3)))
    run("bicgstab_f32", lambda: op.solve(b, "D", lq.SolverParams(tol=1e-10, inner="f32", inner_tol=1e-5)))
    for rel in (False, True):
        run("cgne_f32_itol0.1%s" % ("_reliable" if rel else ""),
            lambda: op.solve(b, "D", lq.SolverParams(solver="cgne", tol=1e-10, inner="f32", inner_tol=0.1,
                                                     reliable=rel)))
    v0 = torch.from_numpy(gaussian_parity_spinor(d, 4245)).cuda()
    (ev, res, X, st), ms = _timed(torch, lambda: op.eigs(16, 64, v0=v0, tol=1e-8, vectors=True))
    out["%s_eigs16_ms" % tag] = ms
    op.set_deflation(ev, X)
    run("cgne_f32_deflated16", lambda: op.solve(b, "D", lq.SolverParams(solver="cgne", tol=1e-10, inner="f32",
                                                                          inner_tol=1e-5, deflate=True)))
    op.set_deflation([], None)
    v0m = torch.from_numpy(gaussian_spinor(d, 4244, 12)).cuda()
    mg, ms = _timed(torch, lambda: lq.Multigrid(op, v0m, lq.MGParams()))
    out["%s_mg_setup_ms" % tag] = ms
    run("mg_gcr", lambda: mg.solve(b, lq.SolverParams(tol=1e-10, inner_tol=1e-5)))
    mg.close()
    op.close()
    print("bench: solver variants %s" % json.dumps(out), file=sys.stderr, flush=True)
    return out


def _profile(lq, torch, args):
    """One workload alone (for rocprofv3 runs; see --profile)."""
    from lattice_inputs import (ANTIPERIODIC_T, RAGGED_DIMS, WORKLOADS, gaussian_spinor, point_sources,
                                workload_gauge, workload_source)
    out = {}
    if args.profile == "mg":
        from lattice_inputs import gauge_exp
        d, kappa = (16, 16, 16, 32), 0.1248
        op = lq.Operator(d, kappa, 0.0, ANTIPERIODIC_T, link_recon=12)
        op.set_gauge(torch.from_numpy(gauge_exp(d, 0.1, 4242)).cuda())
        b = torch.from_numpy(gaussian_spinor(d, 4243)).cuda()
        mg, setup_ms = _timed(torch, lambda: lq.Multigrid(op, torch.from_numpy(gaussian_spinor(d, 4244, 12)).cuda(),
                                                          lq.MGParams()))
        prm = lq.SolverParams(tol=1e-10, inner_tol=1e-5)
        for _ in range(args.warmup):
            mg.solve(b, prm)
        times = []
        for _ in range(args.steps):
            (_, st), ms = _timed(torch, lambda: mg.solve(b, prm))
            times.append(ms)
        out = {"workload": "wilson_16x16x16x32_k1248", "setup_ms": setup_ms, "solve_ms": times, "gcr_iters": st.nconv,
               "diff": st.diff}
        mg.close()
        op.close()
        return out
    if args.profile == "propagator":
        # the 12 spin-colour point sources of one propagator as one solve
        name = "clover_24x24x24x48"
        w = WORKLOADS[name]
        d = w["dims"]
        op = lq.Operator(d, w["kappa"], w["csw"], ANTIPERIODIC_T, link_recon=args.recon)
        op.set_gauge(torch.from_numpy(workload_gauge(name)).cuda())
        if not args.no_tune:
            op.tune(12, left=args.left_precond)
        src = torch.from_numpy(point_sources(d)).cuda()
        inner_tol = args.inner_tol or {"f16": 5e-3, "f32": 1e-5, "f64": 1e-5}[args.inner]
        prm = lq.SolverParams(tol=args.tol, inner=args.inner, inner_tol=inner_tol, check_every=10,
                              left_precond=args.left_precond)
        for _ in range(args.warmup):
            op.solve(src, "D", prm)
        times = []
        for _ in range(args.steps):
            (_, st), ms = _timed(torch, lambda: op.solve(src, "D", prm))
            times.append(ms)
        out = {"workload": name, "nrhs": 12, "inner": args.inner, "solve_ms": times,
               "iters": [s.nconv for s in st], "outer": [s.nouter for s in st]}
        op.close()
        return out
    if args.profile in ("schur_f16", "schur12_f16", "solve"):
        name = args.workload if args.profile != "schur12_f16" else "clover_24x24x24x48"
        w = WORKLOADS[name]
        d = w["dims"]
        op = lq.Operator(d, w["kappa"], w["csw"], ANTIPERIODIC_T, link_recon=args.recon)
        op.set_gauge(torch.from_numpy(workload_gauge(name)).cuda())
        V = d[0] * d[1] * d[2] * d[3]
        if args.profile == "solve":
            b = torch.from_numpy(workload_source(name)).cuda()
            inner_tol = args.inner_tol or {"f16": 5e-3, "f32": 1e-5, "f64": 1e-5}[args.inner]
            prm = lq.SolverParams(solver=args.solver, tol=args.tol, inner=args.inner, inner_tol=inner_tol,
                                  check_every=10, left_precond=args.left_precond)
            for _ in range(args.warmup):
                op.solve(b, "D", prm)
            times = []
            for _ in range(args.steps):
                (_, st), ms = _timed(torch, lambda: op.solve(b, "D", prm))
                times.append(ms)
            out = {"workload": name, "solve_ms": times, "iters": st[0].nconv, "outer": st[0].nouter,
                   "diff": st[0].diff}
        else:
            nrhs = 1 if args.profile == "schur_f16" else 12
            fin, fout = lq.Field(op, "f16", nrhs), lq.Field(op, "f16", nrhs)
            src = torch.from_numpy(workload_source(name, nrhs=nrhs if nrhs > 1 else None)).cuda()
            fin.load(src.reshape(nrhs, -1, 4, 3)[:, : V // 2].contiguous().reshape((nrhs,) + op.parity_shape))
            if not args.no_tune:  # counter runs take a fixed shape (tuning under counters is not timing)
                op.tune(nrhs, left=args.left_precond)
            else:  # the given order, else the automatic shape, made explicit for the report
                op.set_option("xcd_remap_f16", args.xcd_remap if args.xcd_remap is not None else (0 if nrhs == 1 else 2))
                op.set_option("rhs_per_thread_f16", 1 if nrhs == 1 else 4)
            kind = "schur_left" if args.left_precond else "schur"
            us = _graph_time_us(torch, lambda: lq.apply_field(op, kind, fout, fin), args.kernel_reps)
            b2, _ = op.traffic("f16", nrhs, clover=True)
            bps = 2 * b2 + 52.0  # per site and right-hand side: kernel 1 + kernel 2 (+ the axpy operand)
            out = {"workload": name, "nrhs": nrhs, "kind": kind, "avg_apply_us": us,
                   "bytes_per_apply": bps * nrhs * (V // 2),
                   "GBs": bps * nrhs * (V // 2) / (us * 1e-6) / 1e9,
                   "block": op.get_option("hop_block_f16"), "xcd_remap": op.get_option("xcd_remap_f16"),
                   "rhs_per_thread": op.get_option("rhs_per_thread_f16")}
            fin.close()
            fout.close()
            # a copy of known size in the same run (1 GiB read + 1 GiB written per
            # launch, 3 launches): the reference for scaling hardware counters
            out["copy_probe_GBs"] = lq.bandwidth_probe(1 << 30, "copy", reps=2)
        op.close()
    else:
        prm = lq.SolverParams(tol=1e-10, inner=args.inner, inner_tol=args.inner_tol or
                              {"f16": 5e-3, "f32": 1e-5, "f64": 1e-5}[args.inner], check_every=10,
                              left_precond=args.left_precond)
        ops, bs = [], []
        for i, dd in enumerate(RAGGED_DIMS):
            o = lq.Operator(dd, 0.135, 1.7, ANTIPERIODIC_T, link_recon=12)
            o.set_gauge(torch.from_numpy(workload_gauge("clover_24x24x24x48", dims=dd)).cuda())
            ops.append(o)
            bs.append(torch.from_numpy(gaussian_spinor(dd, 2003 + 10 * i, 4)).cuda())
        batch = lq.Batch(ops, [4] * len(ops))
        batch.solve(bs, prm)
        for o, b in zip(ops, bs):
            o.solve(b, "D", prm)
        for _ in range(args.steps):
            (_, stb), msb = _timed(torch, lambda: batch.solve(bs, prm))
            out.setdefault("batch_ms", []).append(msb)
            for k, (o, b) in enumerate(zip(ops, bs)):
                (_, st), m = _timed(torch, lambda: o.solve(b, "D", prm))
                out.setdefault("separate_ms_%dx%dx%dx%d" % tuple(RAGGED_DIMS[k]), []).append(m)
        out["batch_iters"] = [s.nconv for s in stb]
        batch.close()
        for o in ops:
            o.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="clover_32x32x32x64")
    ap.add_argument("--inner", default="f16", choices=["f16", "f32", "f64"])
    ap.add_argument("--solver", default="bicgstab", choices=["bicgstab", "cgne"])
    ap.add_argument("--recon", type=int, default=12, choices=[12, 18])
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="relative residual of each inner solve (default 5e-3 for f16, 1e-5 otherwise)")
    ap.add_argument("--left-precond", action=argparse.BooleanOptionalAction, default=True,
                    help="inner BiCGStab on A_ee^-1 M, the A_ee^-1-preconditioned Schur form (default on; "
                         "the plain form is timed beside it)")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 / FP32-inner reference solves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (default launch shapes)")
    ap.add_argument("--xcd-remap", type=int, default=None,
                    help="--profile with --no-tune: the binary16 workgroup order to use (0 plain, 1 XCD-aware, "
                         "2 XCD-aware with time slices interleaved)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 12-RHS propagator, ragged batch and force measurements")
    ap.add_argument("--force-only", action="store_true",
                    help="only the pseudofermion force and molecular-dynamics measurements; prints their JSON")
    ap.add_argument("--eigs-only", action="store_true",
                    help="only the eigensolver measurement; prints its JSON")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the per-kernel timings (the roofline kernels), no solves; prints their JSON")
    ap.add_argument("--profile", choices=["schur_f16", "schur12_f16", "solve", "propagator", "ragged", "mg"],
                    default=None,
                    help="run one workload alone for a profiler: schur_f16 the roofline kernel pair on the "
                         "workload (kernel-reps graph-replayed applies), schur12_f16 the same operator with the "
                         "12 point sources of 24^3x48, solve the timed mixed solve (warmup + steps solves), propagator "
                         "the 12-RHS solve of those point sources (warmup + steps solves), ragged "
                         "the ragged batch solve and its lattices' separate solves, mg the multigrid solve of the "
                         "near-critical 16^3x32 Wilson lattice (warmup + steps solves); prints its timings as JSON")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2111_04457_amd as lq
    from lattice_inputs import ANTIPERIODIC_T, WORKLOADS, workload_gauge, workload_source

    from paper_2111_04457_amd import build as hip_build
    if not os.path.exists(hip_build.LIB):
        hip_build.build()

    if args.profile:
        torch.cuda.set_device(0)
        print(json.dumps({"profile": _profile(lq, torch, args)}), flush=True)
        return 0
    if args.force_only:
        torch.cuda.set_device(0)
        print(json.dumps({"forces": _forces(lq, torch)}), flush=True)
        return 0
    if args.eigs_only:
        torch.cuda.set_device(0)
        print(json.dumps({"eigs": _eigs(lq, torch)}), flush=True)
        return 0

    w = WORKLOADS[args.workload]
    dims = w["dims"]
    V = int(np.prod(dims))
    t_gen = time.time()
    U = workload_gauge(args.workload)
    b = workload_source(args.workload)
    print("bench: inputs %s generated in %.1f s" % (args.workload, time.time() - t_gen), file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    U_d = torch.from_numpy(U).cuda()
    b_d = torch.from_numpy(b).cuda()
    op = lq.Operator(dims, w["kappa"], w["csw"], ANTIPERIODIC_T, link_recon=args.recon)
    op.set_gauge(U_d)  # first call also allocates the operator's fields
    torch.cuda.synchronize()
    t_set = time.perf_counter()
    op.set_gauge(U_d)  # link packing (all precisions) + clover build and inverse
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t_set)
    del U_d
    tune = None
    if not args.no_tune:
        t_tune = time.time()
        tune = op.tune(1, left=args.left_precond)
        print("bench: tuned in %.1f s: %s" % (time.time() - t_tune, json.dumps(tune)), file=sys.stderr, flush=True)

    if args.kernels_only:
        kern, roof = _kernels(lq, torch, op, b_d, V, args.recon, args.kernel_reps, args.left_precond)
        print(json.dumps({"kernels": kern, "roofline": roof}), flush=True)
        op.close()
        return 0

    inner_tol = args.inner_tol or {"f16": 5e-3, "f32": 1e-5, "f64": 1e-5}[args.inner]
    prm = lq.SolverParams(solver=args.solver, tol=args.tol, inner=args.inner, inner_tol=inner_tol, check_every=10,
                          left_precond=args.left_precond)

    for _ in range(args.warmup):
        op.solve(b_d, "D", prm)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    hop_bytes = 0.0
    stats = []
    t0 = time.perf_counter()
    ev0.record(stream)
    x_d = None
    for _ in range(args.steps):
        x_d, st = op.solve(b_d, "D", prm)
        hop_bytes += st[0].hop_bytes
        stats.append(st[0])
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    value = hop_bytes / wall / 1e9
    print("bench: %d steps, %.1f ms/step, iters %d outer %d diff %.2e" %
          (args.steps, ms_per_step, stats[-1].nconv, stats[-1].nouter, stats[-1].diff), file=sys.stderr, flush=True)

    # time to solution of the reference solves on the same GPU
    tts = {"setup_ms": setup_ms, "mixed_%s_ms" % args.inner: ms_per_step, "mixed_%s_iters" % args.inner: stats[-1].nconv,
           "mixed_%s_outer" % args.inner: stats[-1].nouter, "mixed_%s_diff" % args.inner: stats[-1].diff}
    if not args.no_compare:
        refs = {}
        runs = [("f64", args.solver, "fp64", False), ("f32", args.solver, "mixed_f32", False)]
        if args.solver == "bicgstab":
            runs.append(("f64", "cgne", "fp64_cgne", False))
            # the same mixed solve with inner BiCGStab on A_ee^-1 M (or without, if the main run used it)
            runs.append((args.inner, "bicgstab", "mixed_%s_%s" % (args.inner, "plain" if args.left_precond else "left"),
                         not args.left_precond))
        for inner, solver, name, left in runs:
            if inner == args.inner and solver == args.solver and left == args.left_precond:
                continue
            p2 = lq.SolverParams(solver=solver, tol=args.tol, inner=inner,
                                 inner_tol=inner_tol if inner == args.inner else 1e-5, check_every=10,
                                 left_precond=left)
            op.solve(b_d, "D", p2)  # captures this solver's graphs
            torch.cuda.synchronize()
            ta = time.perf_counter()
            xr, sr = op.solve(b_d, "D", p2)
            torch.cuda.synchronize()
            tts["%s_ms" % name] = 1e3 * (time.perf_counter() - ta)
            tts["%s_iters" % name] = sr[0].nconv
            tts["%s_diff" % name] = sr[0].diff
            if solver == args.solver and not left:
                refs[inner] = xr
        if "f64" in refs:
            x64 = refs["f64"]
            tts["err_vs_fp64_solution"] = float(torch.linalg.vector_norm(x_d - x64) / torch.linalg.vector_norm(x64))
            tts["speedup_vs_fp64"] = tts["fp64_ms"] / ms_per_step
        print("bench: reference solves %s" % json.dumps(tts), file=sys.stderr, flush=True)

    kern, roof = _kernels(lq, torch, op, b_d, V, args.recon, args.kernel_reps, args.left_precond)
    if roof is not None:
        roof["traffic"] = _traffic_from_profile(roof["kernel"])
    print("bench: kernels %s" % json.dumps(kern), file=sys.stderr, flush=True)

    op.close()
    extras = None if args.no_extras else _extras(lq, torch)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ncores = len(os.sched_getaffinity(0))
        oracle.set_num_threads(ncores)
        # a bounded sample: full-lattice FP64 hopping-term applies of the
        # oracle on the same input for about 8 s
        ta = time.perf_counter()
        oracle.hop(dims, U, ANTIPERIODIC_T, b)
        t1 = time.perf_counter() - ta
        reps = max(1, min(200, int(8.0 / max(t1, 1e-3))))
        ta = time.perf_counter()
        for _ in range(reps):
            oracle.hop(dims, U, ANTIPERIODIC_T, b)
        tc = (time.perf_counter() - ta) / reps
        # the oracle applies H on both parities: V output sites, FP64 bytes per site
        cpu = {"value": 1536.0 * V / tc / 1e9, "unit": "GB/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "%d full-lattice FP64 hopping-term applies of the oracle on %s (%d sites each), %.3f s each"
                         % (reps, args.workload, V, tc)}
        if not args.no_extras:
            # time to solution of the oracle's FP64 even-odd BiCGStab on the
            # 16^3 x 32 clover lattice, against the GPU figures in extras
            w1 = WORKLOADS["clover_16x16x16x32"]
            U1 = workload_gauge("clover_16x16x16x32")
            b1 = workload_source("clover_16x16x16x32")
            ta = time.perf_counter()
            ref = oracle.Operator(w1["dims"], U1, w1["kappa"], w1["csw"], ANTIPERIODIC_T)
            x1, it1 = oracle.solve_eo(ref, b1, tol=1e-10)
            cpu["solve_16x16x16x32_fp64_s"] = time.perf_counter() - ta
            cpu["solve_16x16x16x32_fp64_iters"] = it1
            cpu["solve_16x16x16x32_fp64_diff"] = oracle.true_residual(ref, x1, b1)
            # one D apply of the oracle on the same lattice
            ta = time.perf_counter()
            ref.D(b1)
            cpu["dirac_16x16x16x32_s"] = time.perf_counter() - ta
            # the GPU solutions of the ladder against the oracle's solution
            # (solved on to 1e-13: its own error is then far below theirs)
            x1t, _ = oracle.solve_eo(ref, b1, tol=1e-13)
            cpu["c1_err_vs_oracle_solution"] = {
                name: float(np.linalg.norm(xg.reshape(-1) - x1t.reshape(-1)) / np.linalg.norm(x1t.reshape(-1)))
                for name, xg in C1_SOLUTIONS.items()}
            # the FP64 solve on 32^3 x 64 by the oracle, extrapolated (it would
            # take minutes): one BiCGStab iteration applies M twice, i.e. at
            # least two full-lattice hopping terms, times the GPU FP64 solve's
            # iterations (clover site products and vector operations not counted)
            if "fp64_iters" in tts:
                cpu["solve_%s_fp64_extrapolated_s" % args.workload] = 2 * tc * tts["fp64_iters"]
                cpu["solve_%s_fp64_extrapolation" % args.workload] = (
                    "2 full-lattice oracle hops per BiCGStab iteration x %d iterations (GPU FP64 count); "
                    "a lower bound" % tts["fp64_iters"])
        print("bench: cpu baseline %s" % json.dumps(cpu), file=sys.stderr, flush=True)

    line = {
        "metric": "dslash GB/s (% HBM peak); time to 1e-10 residual, mixed vs FP64 solve",
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f16": "f16-storage/f32", "f32": "f32", "f64": "f64"}[args.inner] + "+f64-outer",
        "data": "synthetic",
        "config": {"workload": args.workload, "dims": list(dims), "kappa": w["kappa"], "csw": w["csw"],
                   "links": "exp(i*%.1f*H)" % w["eps"], "solver": args.solver, "inner": args.inner,
                   "link_recon": args.recon, "tol": args.tol, "left_precond": bool(args.left_precond),
                   "parallelism": "single-gpu"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "time_to_solution": tts,
        "kernels": kern,
        "tuning": tune,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
