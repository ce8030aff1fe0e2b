// solver.hip -- propagator solves: FP64 defect correction around a Krylov
// inner solver (BiCGStab on M, or CG on the normal equations) in FP64, FP32
// or FP16 storage, for nrhs systems at once.  This is the mixed-precision
// propagator solve of the paper's Fig. 1 (a double-precision outer
// template over a single-precision inner field type), solving D x = b.
//
// Outer loop (FP64): r = rhs - A x; stop when |r|^2 <= target; else
// r_in = r / |r| in the inner precision, inner solve to a relative residual
// max(inner_tol, sqrt(target) / (2 |r|)), x += |r| e.  For D x = b on the
// even-odd system: A is the Schur operator M, rhs = b_e + kappa H_eo
// A_oo^-1 b_o, the odd half is x_o = A_oo^-1 (b_o + kappa H_oe x_e) and the
// reported diff is the true residual |b - D x| / |b| of the full lattice in
// FP64 (|b - D x| equals the Schur residual in exact arithmetic).
//
// Inner iterations keep every scalar on the device; the host reads the
// scalars back every check_every iterations to stop the loop.
#include "solver.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace lq {

namespace {

// Bump allocator over the operator's solver workspace.
struct Arena {
    char *base = nullptr;
    size_t used = 0;
    char *take(size_t bytes)
    {
        char *p = base + used;
        used += (bytes + 255) & ~size_t(255);
        return p;
    }
};

}  // namespace

// Inner BiCGStab on M e = rin from e = 0 (SC_TARGET2 relative to |rin|).
void bicg_init(SolveCtx &c)
{
    LQ_HIP(launch_zero(c.ix, c.s));
    LQ_HIP(launch_copy(c.ir, c.irin, c.sc, c.sps, false, c.s));
    LQ_HIP(launch_copy(c.irhat, c.irin, c.sc, c.sps, false, c.s));
    LQ_HIP(launch_copy(c.ip, c.irin, c.sc, c.sps, false, c.s));
    c.reduce_finish(c.ir, c.ir, RED_NORM, FIN_INIT_BICG);
}

void bicg_iter(SolveCtx &c)
{
    c.apply_reduce_finish(c.iv, c.ip, c.irhat, RED_DOT, FIN_BICG_ALPHA);  // v = M p, <rhat, v>
    LQ_HIP(launch_bicg_s(c.is, c.ir, c.iv, c.sc, c.sps, c.s));
    c.apply_reduce_finish(c.it, c.is, c.is, RED_DOT_NORM, FIN_BICG_OMEGA);  // t = M s, <s, t>, |t|^2
    LQ_HIP(launch_bicg_xr(c.ix, c.ir, c.ip, c.is, c.it, c.irhat, c.sc, c.sps, c.partial, c.s));
    c.finish(3, FIN_BICG_RHO, c.ir.n);
    LQ_HIP(launch_bicg_p(c.ip, c.ir, c.iv, c.sc, c.sps, c.s));
}

// Inner CG from e = 0 on M^dag M e = M^dag rin (normal_rhs = false) or on
// M^dag M e = rin (normal_rhs = true); SC_TARGET2 relative to the initial
// residual.
void cg_init(SolveCtx &c, bool normal_rhs)
{
    LQ_HIP(launch_zero(c.ix, c.s));
    if (normal_rhs) LQ_HIP(launch_copy(c.ir, c.irin, c.sc, c.sps, false, c.s));
    else c.apply(c.ir, c.irin, true);
    LQ_HIP(launch_copy(c.ip, c.ir, c.sc, c.sps, false, c.s));
    c.reduce_finish(c.ir, c.ir, RED_NORM, FIN_INIT_CG);
}

void cg_iter(SolveCtx &c)
{
    c.apply(c.iw, c.ip, false);
    c.reduce_finish(c.iw, c.iw, RED_NORM, FIN_CG_ALPHA);
    c.apply(c.iv, c.iw, true);
    LQ_HIP(launch_cg_xr(c.ix, c.ir, c.ip, c.iv, c.sc, c.sps, c.partial, c.s));
    c.finish(1, FIN_CG_BETA, c.ir.n);
    LQ_HIP(launch_cg_p(c.ip, c.ir, c.sc, c.sps, c.s));
}

// Reliable-update restarts: the inner residual is replaced by the new
// normalised FP64 residual rin, the inner solution restarts from zero (the
// outer loop has added it to x), and the search directions of the last
// inner solve continue (systems with SC_REINIT set start afresh, as after
// bicg_init / cg_init).  The stored scalars are those of each system's last
// iteration, which ended after its x and r update (a system freezes before
// its search direction is updated).
void bicg_restart(SolveCtx &c)
{
    LQ_HIP(launch_zero(c.ix, c.s));
    LQ_HIP(launch_copy(c.ir, c.irin, c.sc, c.sps, false, c.s));
    LQ_HIP(launch_reinit(c.irhat, c.ip, c.iv, c.irin, c.sc, c.sps, c.s));
    c.reduce_finish(c.irhat, c.ir, RED_DOT_NORM, FIN_BICG_RESTART);  // <rhat, r>, |r|^2
    LQ_HIP(launch_bicg_p(c.ip, c.ir, c.iv, c.sc, c.sps, c.s));     // p = r + beta (p - omega v)
}

void cg_restart(SolveCtx &c, bool normal_rhs)
{
    LQ_HIP(launch_zero(c.ix, c.s));
    if (normal_rhs) LQ_HIP(launch_copy(c.ir, c.irin, c.sc, c.sps, false, c.s));
    else c.apply(c.ir, c.irin, true);
    LQ_HIP(launch_reinit(c.ip, FieldView{}, FieldView{}, c.ir, c.sc, c.sps, c.s));
    c.reduce_finish(c.ip, c.ir, RED_DOT_NORM, FIN_CG_RESTART);  // <p, r>, |r|^2
    LQ_HIP(launch_bicg_p(c.ip, c.ir, c.ir, c.sc, c.sps, c.s));  // p = r + beta (p - omega r)
}

bool all_frozen(const SolveCtx &c)
{
    for (int i = 0; i < c.nsys; ++i) {
        const double *h = c.hsc + i * NSC;
        if (h[SC_DONE] == 0.0 && h[SC_BREAK] == 0.0) return false;
    }
    return true;
}

namespace {

// Run inner iterations in chunks of check_every (captured in a hipGraph),
// reading the scalars back after each chunk, until every system is frozen
// or max_iter iterations were made.
int inner_loop(SolveCtx &c, int kind, int max_iter, ChunkPlan &plan)
{
    std::vector<double> prev(c.nsys, 0.0);
    int it = 0;
    while (it < max_iter) {
        const int chunk = plan.next(max_iter - it);
        c.masked = true;
        try {
            c.run_chunk(kind, chunk, [&]() {
                if (kind == 1) bicg_iter(c);
                else cg_iter(c);
            });
        } catch (...) {
            c.masked = false;
            throw;
        }
        c.masked = false;
        it += chunk;
        c.pull();
        c.count_iterations(prev);
        if (all_frozen(c)) break;
    }
    plan.learn(c);
    return it;
}

int inner_bicgstab(SolveCtx &c, int max_iter, ChunkPlan &plan, bool restart)
{
    if (restart) bicg_restart(c);
    else bicg_init(c);
    return inner_loop(c, 1, max_iter, plan);
}

int inner_cg(SolveCtx &c, bool normal_rhs, int max_iter, ChunkPlan &plan, bool restart)
{
    if (restart) cg_restart(c, normal_rhs);
    else cg_init(c, normal_rhs);
    return inner_loop(c, 2, max_iter, plan);
}

}  // namespace

int bicgstab_solve(SolveCtx &c, int max_iter, int check_every, int &hint)
{
    ChunkPlan plan;
    plan.hint = hint;
    plan.start(check_every);
    const int it = inner_bicgstab(c, max_iter, plan, false);
    if (plan.hint > 0) hint = plan.hint;
    return it;
}

void ChunkPlan::learn(const SolveCtx &c)
{
    int most = 0;
    for (int i = 0; i < c.nsys; ++i) {
        const double *h = c.hsc + i * NSC;
        if (h[SC_ODONE] == 0.0 && h[SC_ITER] > most) most = (int)h[SC_ITER];
    }
    hint = most;
}

// bytes of one padded site of a packed spinor field
static long site_bytes_of(int p) { return spinor_field_bytes(p, SB) / SB; }

FieldView SolveCtx::space(char *base, int p) const
{
    if (bt) {
        FieldView v{base, p, 0, 0, nsys};
        v.tiles = reinterpret_cast<const Tile *>(bt->tiles.ptr);
        v.ntiles = bt->ntiles;
        return v;
    }
    return FieldView{base, p, (long)op->g.vh, fb(p, op->g), nsys * sps};
}

size_t SolveCtx::space_bytes(int p) const
{
    if (bt) return (size_t)site_bytes_of(p) * bt->sites;
    return (size_t)fb(p, op->g) * nsys * sps;
}

FieldView SolveCtx::group_view(const FieldView &v, int g) const
{
    if (!bt) return v;
    const lq_op *o = bt->ops[g];
    return FieldView{v.base + site_bytes_of(v.prec) * bt->site0[g], v.prec, (long)o->g.vh, fb(v.prec, o->g),
                     bt->nrhs[g]};
}

void SolveCtx::count_hops(int prec, int n)
{
    // per output site and system, the links shared by each operator's systems
    for (int g = 0; g < ngroups(); ++g) {
        double b, f;
        lq_op *o = group_op(g);
        lq_op_traffic(o, (lq_prec)prec, group_nsys(g), o->has_clover ? 1 : 0, &b, &f);
        hop_bytes += (double)n * b * o->g.vh * group_nsys(g);
    }
    n_hop += n;
}

void SolveCtx::count_iterations(std::vector<double> &prev)
{
    for (int g = 0; g < ngroups(); ++g) {
        double b, f;
        lq_op *o = group_op(g);
        lq_op_traffic(o, (lq_prec)pin, group_nsys(g), o->has_clover ? 1 : 0, &b, &f);
        for (int i = group_sys0(g); i < group_sys0(g) + group_nsys(g); ++i) {
            const double it = hsc[i * NSC + SC_ITER];
            const double d = it - prev[i];
            prev[i] = it;
            n_hop += (long)(4 * d);
            hop_bytes += 4.0 * d * b * o->g.vh;
        }
    }
}

void SolveCtx::apply_group(int g, const FieldView &out, const FieldView &in, bool dag)
{
    if (!bt) {
        const bool m = masked;
        masked = false;
        try {
            apply(out, in, dag);
        } catch (...) {
            masked = m;
            throw;
        }
        masked = m;
        return;
    }
    lq_op *o = bt->ops[g];
    const int p = in.prec;
    const FieldView t = group_view(space(odd_tmp[p], p), g);
    if (left) schur_left(o, p, out, in, t, s);
    else schur(o, p, out, in, t, dag, s);
    double b, f;
    lq_op_traffic(o, (lq_prec)p, group_nsys(g), o->has_clover ? 1 : 0, &b, &f);
    n_hop += 2;
    hop_bytes += 2.0 * b * o->g.vh * group_nsys(g);
}

void SolveCtx::apply(const FieldView &out, const FieldView &in, bool dag)
{
    if (coarse_apply) {
        if (dag) throw Failure{LQ_ERR_STATE, "the coarse operator has no dagger form here"};
        coarse_apply(*this, out, in);
        return;
    }
    const int p = in.prec;
    if (bt) {
        batch_schur(*this, p, out, in, space(odd_tmp[p], p), dag, eo && left, 0, nullptr);
        if (!masked) count_hops(p, 2);
        return;
    }
    op->hop_mask = masked ? sc : nullptr;
    try {
        const FieldView t{odd_tmp[p], p, (long)op->g.vh, fb(p, op->g), nsys};
        if (eo && left) {
            if (dag) throw Failure{LQ_ERR_STATE, "the preconditioned Schur operator has no dagger form here"};
            schur_left(op, p, out, in, t, s);
        } else if (eo) {
            schur(op, p, out, in, t, dag, s);
        } else {
            dirac_full(op, p, out.base, in.base, nsys, dag, s);
        }
    } catch (...) {
        op->hop_mask = nullptr;
        throw;
    }
    op->hop_mask = nullptr;
    if (!masked) count_hops(p, 2);
}

void SolveCtx::apply_reduce_finish(const FieldView &out, const FieldView &in, const FieldView &w, int mode,
                                   int op_fin)
{
    if (!eo) {
        apply(out, in, false);
        reduce_finish(w, out, mode, op_fin);
        return;
    }
    const int p = in.prec;
    const int red = mode == RED_DOT ? 2 : 3;
    if (bt) {
        batch_schur(*this, p, out, in, space(odd_tmp[p], p), false, left, red, &w);
        if (!masked) count_hops(p, 2);
        LQ_HIP(launch_finish(partial, nsys, 1, 0, red, op_fin, sc, 1e-30, s,
                             reinterpret_cast<const int2 *>(bt->hop_range.ptr)));
        return;
    }
    op->hop_mask = masked ? sc : nullptr;
    try {
        const FieldView t{odd_tmp[p], p, (long)op->g.vh, fb(p, op->g), nsys};
        if (left) schur_left(op, p, out, in, t, s, red, &w);
        else schur(op, p, out, in, t, false, s, red, &w);
    } catch (...) {
        op->hop_mask = nullptr;
        throw;
    }
    op->hop_mask = nullptr;
    if (!masked) count_hops(p, 2);
    // partials: one per 64-site wavefront of the even sites, per system
    const int nw = (op->g.vh + 63) / 64;
    LQ_HIP(launch_finish(partial, nsys, 1, nw, red == 2 ? 2 : 3, op_fin, sc, 1e-30, s));
}

void SolveCtx::reduce_finish(const FieldView &x, const FieldView &y, int mode, int op_fin)
{
    LQ_HIP(launch_reduce(x, y, mode, partial, s, masked ? sc : nullptr, sps));
    const int K = mode == RED_NORM ? 1 : mode == RED_DOT ? 2 : 3;
    finish(K, op_fin, x.n);
}

void SolveCtx::finish(int K, int op_fin, long n)
{
    LQ_HIP(launch_finish(partial, nsys, sps, blas_blocks(n), K, op_fin, sc, 1e-30, s,
                         bt ? reinterpret_cast<const int2 *>(bt->blas_range.ptr) : nullptr));
}

void SolveCtx::pull()
{
    LQ_HIP(hipMemcpyAsync(hsc, sc, sizeof(double) * NSC * nsys, hipMemcpyDeviceToHost, s));
    LQ_HIP(hipStreamSynchronize(s));
}

void SolveCtx::push() { LQ_HIP(hipMemcpyAsync(sc, hsc, sizeof(double) * NSC * nsys, hipMemcpyHostToDevice, s)); }

// The solver's vectors, carved from base in the order solver_ws_bytes counts
// them: x, r, y, t, aux (FP64), three odd temporaries (FP64 size), x and
// M x in the inner solution precision, nine inner vectors.
void carve_vectors(SolveCtx &c, char *base, size_t odd)
{
    const size_t f64b = c.space_bytes(F64), finb = c.space_bytes(c.pin), fxb = c.space_bytes(c.px);
    Arena A;
    A.base = base;
    c.x64 = c.space(A.take(f64b), F64);
    c.r64 = c.space(A.take(f64b), F64);
    c.y64 = c.space(A.take(f64b), F64);
    c.t64 = c.space(A.take(f64b), F64);
    c.aux64 = c.space(A.take(f64b), F64);
    for (int p = 0; p < 3; ++p) c.odd_tmp[p] = A.take(odd);
    c.ix = c.space(A.take(fxb), c.px);
    c.ex = c.space(A.take(fxb), c.px);
    c.ir = c.space(A.take(finb), c.pin);
    c.ip = c.space(A.take(finb), c.pin);
    c.iv = c.space(A.take(finb), c.pin);
    c.is = c.space(A.take(finb), c.pin);
    c.it = c.space(A.take(finb), c.pin);
    c.irhat = c.space(A.take(finb), c.pin);
    c.iw = c.space(A.take(finb), c.pin);
    c.irin = c.space(A.take(finb), c.pin);
}

void make_ctx(SolveCtx &c, lq_op *op, int nsys, bool eo, int inner, hipStream_t s)
{
    const Geom &g = op->g;
    c.op = op;
    c.s = s;
    c.nsys = nsys;
    c.eo = eo;
    c.sps = eo ? 1 : 2;
    c.pin = inner;
    c.px = inner == F64 ? F64 : F32;
    op->solver_ws.ensure(solver_ws_bytes(g, nsys, eo, inner));
    carve_vectors(c, op->solver_ws.ptr, (size_t)fb(F64, g) * nsys);

    op->solver_sc.ensure(sizeof(double) * NSC * nsys);
    c.sc = reinterpret_cast<double *>(op->solver_sc.ptr);
    if (op->host_sc_n < (size_t)NSC * nsys) {
        if (op->host_sc) LQ_HIP(hipHostFree(op->host_sc));
        op->host_sc = nullptr;
        op->host_sc_n = 0;
        LQ_HIP(hipHostMalloc(reinterpret_cast<void **>(&op->host_sc), sizeof(double) * NSC * nsys, 0));
        op->host_sc_n = (size_t)NSC * nsys;
    }
    c.hsc = op->host_sc;
    const long nblk = std::max<long>(hop_blocks(g.vh, 64), blas_blocks(g.vh));
    op->partial.ensure(sizeof(double) * 3 * nblk * nsys * 2);
    c.partial = reinterpret_cast<double *>(op->partial.ptr);
    std::memset(c.hsc, 0, sizeof(double) * NSC * nsys);
    c.push();
}

std::vector<double> norms2(SolveCtx &c, const FieldView &v, int sps)
{
    LQ_HIP(launch_reduce(v, v, RED_NORM, c.partial, c.s));
    LQ_HIP(launch_finish(c.partial, c.nsys, sps, blas_blocks(v.n), 1, FIN_NORM, c.sc, 0, c.s));
    c.pull();
    std::vector<double> out(c.nsys);
    for (int i = 0; i < c.nsys; ++i) out[i] = c.hsc[i * NSC + SC_NORM2];
    return out;
}

OuterStats defect_correction(SolveCtx &c, const lq_solver_params &sp, bool normal, const FieldView &rhs,
                             const std::vector<double> &target2, bool x_zero)
{
    const int nsys = c.nsys;
    OuterStats os;
    os.iters.assign(nsys, 0);
    os.outer.assign(nsys, 0);
    os.restarts.assign(nsys, 0);
    os.r2.assign(nsys, 0.0);
    int total_inner = 0;
    ChunkPlan plan;
    // first chunk of the k-th inner solve: what the k-th inner solve of the
    // previous solve needed (the first inner solve starts from b, the later
    // ones from smaller residuals), else what the last inner solve needed
    std::vector<int> &hints = c.bt ? c.bt->inner_hints : c.op->inner_hints;
    size_t k_inner = 0;
    plan.hint = hints.empty() ? 0 : hints[0];
    // the outer target of each system (FIN_NORM flags systems below it)
    c.pull();
    for (int i = 0; i < nsys; ++i) c.hsc[i * NSC + SC_OTARGET2] = target2[i];
    c.push();
    // The outer loop keeps its decisions per group of systems (the whole
    // solve, or each lattice of a batch, which then runs exactly as it would
    // alone); the inner solves run on every system at once.
    //
    // After an FP64 residual r, the next one may be updated as r - |r| M e
    // with M applied to the inner solution e in e's precision: that apply
    // rounds at ~1e-7 of |r|, a small fraction of the updated residual when
    // the inner solve reduced it by a modest factor (relative target at
    // least 1e-3, as with binary16 storage).  The next residual is FP64
    // again, so the rounding never accumulates, and every convergence
    // decision is taken on an FP64 residual.  It pays only where the FP64
    // apply is bandwidth-bound (at least 2^19 sites per parity over the
    // group's systems): on less work its extra launches and the FP64 check
    // of a converged update cost more than the FP64 apply they replace.
    struct Group {
        bool can_update = false, last_fp64 = true, update = false, all = false, done = false;
        double last_rel = 0.0;  // smallest relative target of the last inner solve
    };
    const int ng = c.ngroups();
    std::vector<Group> gs(ng);
    for (int g = 0; g < ng; ++g)
        gs[g].can_update = !normal && c.eo && c.px != F64 && (long)c.group_op(g)->g.vh * c.group_nsys(g) >= (1L << 19);
    // r = rhs - A x in FP64 (A x = 0 for a zero initial guess), or the
    // update r -= |r| M e, and |r|^2, on group g's systems
    auto residual = [&](int g, bool zero_x, bool update) {
        double *scg = c.sc + (long)c.group_sys0(g) * NSC;
        const FieldView r = c.group_view(c.r64, g);
        if (update) {
            const FieldView ex = c.group_view(c.ex, g);
            c.apply_group(g, ex, c.group_view(c.ix, g), false);
            LQ_HIP(launch_sub_scaled_norm(r, ex, scg, c.sps, c.partial, c.s));  // r -= |r| M e
        } else {
            const FieldView y = c.group_view(c.y64, g), x = c.group_view(c.x64, g);
            if (zero_x) {
                LQ_HIP(launch_zero(y, c.s));
            } else if (normal) {
                const FieldView t = c.group_view(c.t64, g);
                c.apply_group(g, t, x, false);
                c.apply_group(g, y, t, true);
            } else {
                c.apply_group(g, y, x, false);
            }
            LQ_HIP(launch_xmy_norm(r, c.group_view(rhs, g), y, c.partial, c.s));
        }
        LQ_HIP(launch_finish(c.partial, c.group_nsys(g), c.sps, blas_blocks(r.n), 1, FIN_NORM, scg, 1e-30, c.s));
    };
    auto read_norms = [&]() {
        c.pull();
        for (int g = 0; g < ng; ++g) {
            if (gs[g].done) continue;
            gs[g].all = true;
            for (int i = c.group_sys0(g); i < c.group_sys0(g) + c.group_nsys(g); ++i) {
                const double n2 = c.hsc[i * NSC + SC_NORM2];
                os.r2[i] = n2;
                if (!std::isfinite(n2)) throw Failure{LQ_ERR_NONFINITE, "residual is not finite"};
                if (c.hsc[i * NSC + SC_ODONE] == 0.0) gs[g].all = false;
            }
        }
    };
    // the largest |r| / |b| of group g's systems (progress output)
    auto max_rel_residual = [&](int g) {
        double m = 0;
        for (int i = c.group_sys0(g); i < c.group_sys0(g) + c.group_nsys(g); ++i)
            if (target2[i] > 0) m = std::max(m, std::sqrt(os.r2[i] / target2[i]) * sp.tol);
        return m;
    };
    bool first_inner = true;
    // reliable updates: |r| of each system's last inner source (the factor
    // between two normalisations of the inner solve)
    std::vector<double> last_scale(nsys, 0.0);
    for (int step = 0; step <= sp.max_outer; ++step) {
        for (int g = 0; g < ng; ++g) {
            Group &G = gs[g];
            if (G.done) continue;
            G.update = G.can_update && step > 0 && G.last_fp64 && G.last_rel >= 1e-3;
            residual(g, step == 0 && x_zero, G.update);
        }
        read_norms();
        const bool last_step = step == sp.max_outer || total_inner >= sp.max_iter;
        // a converged (or final) updated residual is confirmed in FP64
        bool again = false;
        for (int g = 0; g < ng; ++g)
            if (!gs[g].done && gs[g].update && (gs[g].all || last_step)) {
                residual(g, false, false);
                again = true;
            }
        if (again) read_norms();
        bool finished = true;
        for (int g = 0; g < ng; ++g) {
            Group &G = gs[g];
            if (G.done) continue;
            G.last_fp64 = !G.update || G.all || last_step;
            if (G.all || last_step) G.done = true;
            else finished = false;
        }
        if (finished) break;
        // deflation: the residual loses its components along the deflation
        // space's modes before the inner solve (the solution gains them)
        if (c.deflate) {
            deflate_residual(c, normal);
            read_norms();
        }
        // relative target of this inner solve, per system
        for (int g = 0; g < ng; ++g) {
            Group &G = gs[g];
            if (G.done) continue;
            G.last_rel = 1.0;
            for (int i = c.group_sys0(g); i < c.group_sys0(g) + c.group_nsys(g); ++i) {
                double *h = c.hsc + i * NSC;
                const double rn = std::sqrt(h[SC_NORM2]);
                double rel = 0.5 * std::sqrt(target2[i]) / (rn > 0 ? rn : 1.0);
                if (c.pin != F64) rel = std::max(rel, sp.inner_tol);
                rel = std::min(rel, 0.5);
                if (h[SC_ODONE] == 0.0) G.last_rel = std::min(G.last_rel, rel);
                h[SC_TARGET2] = rel * rel;  // relative; FIN_INIT_* makes it absolute
                h[SC_FORCE_BREAK] = first_inner ? c.force_break : 0;
                // a system continues its Krylov space if its last inner solve
                // converged after at least one iteration
                const bool cont = !first_inner && h[SC_DONE] != 0.0 && h[SC_BREAK] == 0.0 && h[SC_ITER] > 0 &&
                                  last_scale[i] > 0 && rn > 0;
                h[SC_REINIT] = cont ? 0.0 : 1.0;
                h[SC_RESCALE] = cont ? last_scale[i] / rn : 1.0;
                last_scale[i] = rn;
                if (h[SC_ODONE] == 0.0) os.outer[i]++;
            }
            if (c.log >= 2)
                std::fprintf(stderr, "lq: outer step %d, lattice %d: |r| / |b| max %.3e (%s), inner target %.1e\n",
                             step, g, max_rel_residual(g), G.update ? "updated" : "FP64", G.last_rel);
        }
        const bool restart = sp.reliable && !first_inner;
        first_inner = false;
        c.push();
        LQ_HIP(launch_copy(c.irin, c.r64, c.sc, c.sps, true, c.s));
        // left preconditioning of the inner system: A_ee^-1 M e = A_ee^-1 r
        // (the outer loop keeps the true residual of M x = b)
        const bool left = sp.left_precond && c.eo && !normal && sp.solver == LQ_BICGSTAB &&
                          (c.group_op(0)->has_clover || c.group_op(0)->has_twist);
        if (left)
            for (int g = 0; g < ng; ++g)
                if (!gs[g].done) {
                    const FieldView in = c.group_view(c.irin, g);
                    clover_apply(c.group_op(g), c.pin, 0, true, in, in, c.s);
                }
        c.left = left;
        // a stagnating inner solve hands back to the outer loop after
        // kInnerCap iterations (a restart from the current FP64 iterate)
        constexpr int kInnerCap = 1000;
        const int budget = std::min(sp.max_iter - total_inner, kInnerCap);
        if (k_inner < hints.size() && hints[k_inner] > 0) plan.hint = hints[k_inner];
        plan.start(sp.check_every);
        int it;
        if (normal) it = inner_cg(c, true, budget, plan, restart);
        else if (sp.solver == LQ_CGNE) it = inner_cg(c, false, budget, plan, restart);
        else it = inner_bicgstab(c, budget, plan, restart);
        c.left = false;
        total_inner += it;
        if (plan.hint > 0 && k_inner < 64) {
            if (k_inner < hints.size()) hints[k_inner] = plan.hint;
            else hints.push_back(plan.hint);
        }
        ++k_inner;
        for (int i = 0; i < nsys; ++i) {
            const double *h = c.hsc + i * NSC;
            if (h[SC_ODONE] == 0.0) {
                os.iters[i] += (int)h[SC_ITER];
                if (h[SC_BREAK] != 0.0) os.restarts[i]++;
            }
        }
        // x += |r| e
        LQ_HIP(launch_accum(c.x64, c.ix, c.sc, c.sps, true, c.s));
    }
    if (c.log >= 1)
        for (int g = 0; g < ng; ++g) {
            int it = 0, outer = 0, rst = 0;
            for (int i = c.group_sys0(g); i < c.group_sys0(g) + c.group_nsys(g); ++i) {
                it = std::max(it, os.iters[i]);
                outer = std::max(outer, os.outer[i]);
                rst += os.restarts[i];
            }
            const Geom &gg = c.group_op(g)->g;
            std::fprintf(stderr,
                         "lq: solve %dx%dx%dx%d, %d systems: %d outer steps, %d inner iterations (most), %d restarts, "
                         "|r| / |b| max %.3e\n",
                         gg.L[0], gg.L[1], gg.L[2], gg.L[3], c.group_nsys(g), outer, it, rst, max_rel_residual(g));
        }
    return os;
}

// Solve D x = b for nsys systems; b64, x64: full packed FP64 fields
// ([rhs][parity]).  stats[i] filled for each system.
lq_status solve_packed(lq_op *op, const lq_solver_params &sp, int nsys, char *x64, const char *b64, bool use_x0,
                       lq_solve_stats *stats, hipStream_t s)
{
    const Geom &g = op->g;
    SolveCtx c;
    make_ctx(c, op, nsys, sp.even_odd != 0, sp.inner, s);
    c.force_break = op->break_at;
    op->break_at = 0;  // once
    c.deflate = sp.deflate != 0 && op->defl_n > 0;
    c.log = log_level(op);
    const auto t0 = std::chrono::steady_clock::now();

    const FieldView bfull{const_cast<char *>(b64), F64, (long)g.vh, fb(F64, g), 2 * nsys};
    const FieldView xfull{x64, F64, (long)g.vh, fb(F64, g), 2 * nsys};
    const std::vector<double> bn2 = norms2(c, bfull, 2);
    for (int i = 0; i < nsys; ++i)
        if (!std::isfinite(bn2[i])) throw Failure{LQ_ERR_NONFINITE, "right-hand side is not finite"};

    // right-hand side of the solved system and the initial guess
    FieldView rhs = c.aux64;
    if (c.eo) {
        const FieldView be = full_parity_view(const_cast<char *>(b64), F64, g, nsys, 0);
        const FieldView bo = full_parity_view(const_cast<char *>(b64), F64, g, nsys, 1);
        const FieldView t = FieldView{c.odd_tmp[F64], F64, (long)g.vh, fb(F64, g), nsys};
        clover_apply(op, F64, 1, true, t, bo, s);
        hop(op, F64, rhs, t, 0, false, 0, false, &be, op->prm.kappa, 0, nullptr, s);
        c.count_hops(F64, 1);
        if (use_x0) LQ_HIP(launch_copy(c.x64, full_parity_view(x64, F64, g, nsys, 0), c.sc, 1, false, s));
        else LQ_HIP(launch_zero(c.x64, s));
    } else {
        rhs = bfull;
        if (use_x0) LQ_HIP(launch_copy(c.x64, xfull, c.sc, 2, false, s));
        else LQ_HIP(launch_zero(c.x64, s));
    }
    std::vector<double> target2(nsys);
    for (int i = 0; i < nsys; ++i) target2[i] = sp.tol * sp.tol * bn2[i];
    const OuterStats os = defect_correction(c, sp, false, rhs, target2, !use_x0);

    // Full solution.  The reported residual is the FP64 residual the last
    // outer step computed at the final iterate: on the full lattice it is
    // |b - D x| itself; for the even-odd system the reconstructed odd half
    // x_o = A_oo^-1 (b_o + kappa H_oe x_e) satisfies the odd rows of D x = b
    // identically, and the even rows of b - D x are b_hat_e - M x_e, so
    // |b - D x| = |b_hat_e - M x_e| (up to the rounding of x_o).
    if (c.eo) {
        LQ_HIP(launch_copy(full_parity_view(x64, F64, g, nsys, 0), c.x64, c.sc, 1, false, s));
        const FieldView bo = full_parity_view(const_cast<char *>(b64), F64, g, nsys, 1);
        hop(op, F64, full_parity_view(x64, F64, g, nsys, 1), c.x64, 1, false, 2, true, &bo, op->prm.kappa, 0, nullptr,
            s);
        c.count_hops(F64, 1);
    } else {
        LQ_HIP(launch_copy(xfull, c.x64, c.sc, 2, false, s));
    }
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    bool all_conv = true;
    for (int i = 0; i < nsys; ++i) {
        const double r2 = os.r2[i];
        const double diff = bn2[i] > 0 ? std::sqrt(r2 / bn2[i]) : 0.0;
        if (!std::isfinite(diff)) throw Failure{LQ_ERR_NONFINITE, "final residual is not finite"};
        const bool conv = diff <= sp.tol;
        all_conv = all_conv && conv;
        if (stats) {
            lq_solve_stats &st = stats[i];
            st.nconv = os.iters[i];
            st.nouter = os.outer[i];
            st.restarts = os.restarts[i];
            st.converged = conv ? 1 : 0;
            st.diff = diff;
            st.t_solve_ms = ms;
            st.hop_bytes = c.hop_bytes;
            st.n_hop = (int)c.n_hop;
        }
    }
    return all_conv ? LQ_OK : LQ_NOT_CONVERGED;
}

bool valid_solver_params(const lq_solver_params *sp, std::string &why)
{
    if (sp->max_iter < 0 || sp->max_outer < 0 || !(sp->tol > 0) || !(sp->inner_tol > 0) || !(sp->inner_tol < 1)) {
        why = "tol, inner_tol, max_iter or max_outer out of range";
        return false;
    }
    if (sp->solver != LQ_CGNE && sp->solver != LQ_BICGSTAB) {
        why = "unknown solver";
        return false;
    }
    if (sp->inner < LQ_F64 || sp->inner > LQ_F16) {
        why = "unknown inner precision";
        return false;
    }
    if (!sp->even_odd && sp->solver != LQ_CGNE) {
        why = "the full-lattice solve is CGNE only";
        return false;
    }
    if (sp->left_precond != 0 && sp->left_precond != 1) {
        why = "left_precond must be 0 or 1";
        return false;
    }
    if (sp->reliable != 0 && sp->reliable != 1) {
        why = "reliable must be 0 or 1";
        return false;
    }
    if (sp->deflate != 0 && sp->deflate != 1) {
        why = "deflate must be 0 or 1";
        return false;
    }
    if (sp->deflate && !sp->even_odd) {
        why = "deflation needs the even-odd solve";
        return false;
    }
    return true;
}

}  // namespace lq

using namespace lq;

static lq_status solve_device(lq_op *op, const lq_solver_params *sp, lq_kind mode, int nrhs, void *x, const void *b,
                              int use_x0, lq_solve_stats *stats, void *stream);

extern "C" lq_status lq_solve(lq_op *op, const lq_solver_params *sp, lq_kind mode, int nrhs, void *x, const void *b,
                              int use_x0, lq_solve_stats *stats, void *stream)
{
    if (!op || !sp || !x || !b) {
        set_error("lq_solve: null argument");
        return LQ_ERR_ARG;
    }
    return solve_device(op, sp, mode, nrhs, x, b, use_x0, stats, stream);
}

extern "C" lq_status lq_solve_host(lq_op *op, const lq_solver_params *sp, lq_kind mode, int nrhs, void *x,
                                   const void *b, int use_x0, lq_solve_stats *stats, void *stream)
{
    if (!op || !sp || !x || !b) {
        set_error("lq_solve_host: null argument");
        return LQ_ERR_ARG;
    }
    if (nrhs < 1) {
        set_error("lq_solve_host: nrhs < 1");
        return LQ_ERR_ARG;
    }
    if (op->bound_nrhs && nrhs > op->bound_nrhs) {
        set_error("lq_solve_host: the bound workspace holds " + std::to_string(op->bound_nrhs) +
                  " right-hand sides, " + std::to_string(nrhs) + " requested");
        return LQ_ERR_ARG;
    }
    if (!op->gauge_set) {
        set_error("lq_solve_host: gauge field not set");
        return LQ_ERR_STATE;
    }
    try {
        LQ_HIP(hipSetDevice(op->device));
        hipStream_t us = static_cast<hipStream_t>(stream);
        // b and x staged in device buffers on the caller's stream
        const size_t n = (size_t)op->g.vh * 2 * 12 * 16 * nrhs;
        op->tmp[6].ensure(n);
        op->tmp[7].ensure(n);
        LQ_HIP(hipMemcpyAsync(op->tmp[6].ptr, b, n, hipMemcpyHostToDevice, us));
        if (use_x0) LQ_HIP(hipMemcpyAsync(op->tmp[7].ptr, x, n, hipMemcpyHostToDevice, us));
        const lq_status st = solve_device(op, sp, mode, nrhs, op->tmp[7].ptr, op->tmp[6].ptr, use_x0, stats, stream);
        if (st < 0) return st;
        LQ_HIP(hipMemcpyAsync(x, op->tmp[7].ptr, n, hipMemcpyDeviceToHost, us));
        LQ_HIP(hipStreamSynchronize(us));
        return st;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    }
}

// While in scope, the operator's twisted mass has the opposite sign: a
// twisted-mass operator's D^dag is gamma_5 D(-tau) gamma_5.  The hop kernels
// take the twist factor as an argument, and the captured solver graphs key
// on its value, so nothing else needs rebuilding.
struct TwistFlip {
    lq_op *op;
    explicit TwistFlip(lq_op *o) : op(o) { op->prm.twist = -op->prm.twist; }
    ~TwistFlip() { op->prm.twist = -op->prm.twist; }
    TwistFlip(const TwistFlip &) = delete;
    TwistFlip &operator=(const TwistFlip &) = delete;
};

static lq_status solve_device(lq_op *op, const lq_solver_params *sp, lq_kind mode, int nrhs, void *x, const void *b,
                              int use_x0, lq_solve_stats *stats, void *stream)
{
    if (mode != LQ_D && mode != LQ_DDAG && mode != LQ_DDAGD) {
        set_error("lq_solve: mode must be LQ_D, LQ_DDAG or LQ_DDAGD");
        return LQ_ERR_ARG;
    }
    std::string why;
    if (nrhs < 1 || !valid_solver_params(sp, why)) {
        set_error("lq_solve: invalid solver parameters: " + (nrhs < 1 ? std::string("nrhs < 1") : why));
        return LQ_ERR_ARG;
    }
    if (op->bound_nrhs && nrhs > op->bound_nrhs) {
        set_error("lq_solve: the bound workspace holds " + std::to_string(op->bound_nrhs) + " right-hand sides, " +
                  std::to_string(nrhs) + " requested");
        return LQ_ERR_ARG;
    }
    if (op->has_twist && mode != LQ_D && sp->deflate) {
        set_error("lq_solve: deflate = 1 with a twisted-mass operator needs mode LQ_D (the deflation space belongs "
                  "to the Schur operator of +twist, the dagger modes solve with -twist)");
        return LQ_ERR_ARG;
    }
    if (mode == LQ_DDAGD && use_x0) {
        set_error("lq_solve: LQ_DDAGD solves from zero (two solves in sequence); use_x0 must be 0");
        return LQ_ERR_ARG;
    }
    if (!op->gauge_set) {
        set_error("lq_solve: gauge field not set");
        return LQ_ERR_STATE;
    }
    if (sp->deflate && op->defl_n == 0) {
        set_error("lq_solve: deflate = 1 but the operator has no deflation space (lq_op_set_deflation)");
        return LQ_ERR_STATE;
    }
    try {
        set_error("");
        LQ_HIP(hipSetDevice(op->device));
        // the solve runs on the operator's own stream (capturable), ordered
        // after the caller's stream and synchronized before returning
        hipStream_t us = static_cast<hipStream_t>(stream);
        LQ_HIP(hipEventRecord(op->ev_in, us));
        LQ_HIP(hipStreamWaitEvent(op->stream, op->ev_in, 0));
        hipStream_t s = op->stream;
        const Geom &g = op->g;
        if (sp->left_precond && sp->even_odd && sp->solver == LQ_BICGSTAB) ensure_even_inverse(op, s);
        const size_t full = 2 * (size_t)fb(F64, g) * nrhs;
        op->tmp[4].ensure(full);
        op->tmp[5].ensure(full);
        char *bp = op->tmp[4].ptr, *xp = op->tmp[5].ptr;
        const double *bsrc = static_cast<const double *>(b);
        double *xdst = static_cast<double *>(x);
        for (int p = 0; p < 2; ++p) {
            LQ_HIP(launch_pack_spinor(g, p, 0, bsrc, full_parity_view(bp, F64, g, nrhs, p), s));
            if (use_x0) LQ_HIP(launch_pack_spinor(g, p, 0, xdst, full_parity_view(xp, F64, g, nrhs, p), s));
        }
        const FieldView bfull{bp, F64, (long)g.vh, fb(F64, g), 2 * nrhs};
        const FieldView xfull{xp, F64, (long)g.vh, fb(F64, g), 2 * nrhs};
        lq_status st;
        if (mode == LQ_D) {
            st = solve_packed(op, *sp, nrhs, xp, bp, use_x0, stats, s);
        } else if (mode == LQ_DDAG) {
            // D^dag = gamma_5 D gamma_5: x = gamma_5 D^-1 gamma_5 b (twisted
            // mass: D(tau)^dag = gamma_5 D(-tau) gamma_5)
            LQ_HIP(launch_gamma5(bfull, s));
            if (use_x0) LQ_HIP(launch_gamma5(xfull, s));
            {
                const TwistFlip flip(op);
                st = solve_packed(op, *sp, nrhs, xp, bp, use_x0, stats, s);
            }
            LQ_HIP(launch_gamma5(xfull, s));
        } else {
            // D^dag D x = b: y = (D^dag)^-1 b = gamma_5 D^-1 gamma_5 b, then x = D^-1 y.
            // With r1 = b - D^dag y and r2 = y - D x, b - D^dag D x = r1 + D^dag r2,
            // so |b - D^dag D x| <= |r1| + |D| |r2|: the first solve runs to tol / 2
            // and the second to tol |b| / (2 |D| |y|), with the bound
            // |D| <= 1 + 16 kappa + 12 |c_sw| kappa: each of the eight hopping
            // terms is kappa (1 -+ gamma_mu) (norm 2) times a unitary link; each of
            // the six terms of F is c_sw kappa gamma_mu gamma_nu (norm 1) times
            // Fhat, whose norm is at most 2 ((Q - Q^dag) / 8 with Q four unitary
            // plaquettes, and at most as much again for the removed trace).
            // The twisted-mass term i tau gamma_5 adds |tau| to the bound, and
            // the first solve is with D(-tau).
            std::vector<lq_solve_stats> st1(nrhs);
            LQ_HIP(launch_gamma5(bfull, s));
            lq_solver_params sp1 = *sp;
            sp1.tol = sp->tol * 0.5;
            {
                const TwistFlip flip(op);
                st = solve_packed(op, sp1, nrhs, xp, bp, false, st1.data(), s);
            }
            if (st < 0) return st;
            LQ_HIP(launch_gamma5(xfull, s));  // y
            LQ_HIP(launch_gamma5(bfull, s));  // b restored
            SolveCtx c;
            c.op = op;
            c.s = s;
            c.nsys = nrhs;
            c.sc = reinterpret_cast<double *>(op->solver_sc.ptr);
            c.hsc = op->host_sc;
            c.partial = reinterpret_cast<double *>(op->partial.ptr);
            const std::vector<double> bn2 = norms2(c, bfull, 2);
            const std::vector<double> yn2 = norms2(c, xfull, 2);
            const double dnorm =
                1.0 + std::fabs(op->prm.twist) + std::fabs(op->prm.kappa) * (16.0 + 12.0 * std::fabs(op->prm.csw));
            lq_solver_params sp2 = *sp;
            sp2.tol = 0.5 * sp->tol;
            for (int i = 0; i < nrhs; ++i)
                if (yn2[i] > 0) sp2.tol = std::min(sp2.tol, 0.5 * sp->tol * std::sqrt(bn2[i] / yn2[i]) / dnorm);
            LQ_HIP(hipMemcpyAsync(bp, xp, full, hipMemcpyDeviceToDevice, s));  // b slot := y
            st = solve_packed(op, sp2, nrhs, xp, bp, false, stats, s);
            if (st < 0) return st;
            // diff of the normal system |b - D^dag D x| / |b|, b re-packed
            for (int p = 0; p < 2; ++p) LQ_HIP(launch_pack_spinor(g, p, 0, bsrc, full_parity_view(bp, F64, g, nrhs, p), s));
            op->tmp[0].ensure(full);
            op->tmp[1].ensure(full);
            dirac_full(op, F64, op->tmp[0].ptr, xp, nrhs, false, s);
            dirac_full(op, F64, op->tmp[1].ptr, op->tmp[0].ptr, nrhs, true, s);
            const FieldView fy{op->tmp[1].ptr, F64, (long)g.vh, fb(F64, g), 2 * nrhs};
            const FieldView fr{op->tmp[0].ptr, F64, (long)g.vh, fb(F64, g), 2 * nrhs};
            LQ_HIP(launch_xmy_norm(fr, bfull, fy, c.partial, s));
            LQ_HIP(launch_finish(c.partial, nrhs, 2, blas_blocks(g.vh), 1, FIN_NORM, c.sc, 0, s));
            c.pull();
            bool all = true;
            for (int i = 0; i < nrhs; ++i) {
                const double d = bn2[i] > 0 ? std::sqrt(c.hsc[i * NSC + SC_NORM2] / bn2[i]) : 0.0;
                if (stats) {
                    stats[i].diff = d;
                    stats[i].converged = d <= sp->tol;
                    stats[i].nconv += st1[i].nconv;
                    stats[i].nouter += st1[i].nouter;
                    stats[i].restarts += st1[i].restarts;
                    stats[i].t_solve_ms += st1[i].t_solve_ms;
                    stats[i].hop_bytes += st1[i].hop_bytes;
                    stats[i].n_hop += st1[i].n_hop;
                }
                all = all && d <= sp->tol;
            }
            st = all ? LQ_OK : LQ_NOT_CONVERGED;
        }
        if (st < 0) return st;
        for (int p = 0; p < 2; ++p)
            LQ_HIP(launch_unpack_spinor(g, p, 0, full_parity_view(xp, F64, g, nrhs, p), xdst, s));
        LQ_HIP(hipEventRecord(op->ev_out, s));
        LQ_HIP(hipStreamWaitEvent(us, op->ev_out, 0));
        LQ_HIP(hipStreamSynchronize(s));
        return st;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return LQ_ERR_STATE;
    }
}
