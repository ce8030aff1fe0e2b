// solver.hip -- propagator solves: FP64 defect correction around a Krylov
// inner solver (BiCGStab on M, or CG on the normal equations) in FP64, FP32
// or FP16 storage, for nrhs systems at once.  This is the mixed-precision
// propagator solve of the paper's Fig. 1 (a double-precision outer
// template over a single-precision inner field type), solving D x = b.
//
// Outer loop (FP64): r = b_hat - M x; stop when |r| <= tol |b|; else
// r_in = r / |r| in the inner precision, inner solve M e = r_in to a relative
// residual max(inner_tol, tol |b| / (2 |r|)), x += |r| e.  Even-odd: M is the
// Schur operator, b_hat = b_e + kappa H_eo A_oo^-1 b_o, and at the end
// x_o = A_oo^-1 (b_o + kappa H_oe x_e); the reported diff is the true
// residual |b - D x| / |b| of the full lattice in FP64.
//
// Inner iterations keep every scalar on the device; the host reads the
// scalars back every check_every iterations to stop the loop.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "blas.h"
#include "runtime.h"

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

struct Ctx {
    lq_op *op;
    hipStream_t s;
    int nsys;
    bool eo;          // even-odd Schur system (else full lattice)
    int sps;          // slices per system of a solve-space vector
    int pin, px;      // inner storage precision, inner solution precision
    double *sc;       // device scalars [nsys][NSC]
    double *hsc;      // pinned host mirror
    double *partial;  // reduction partials
    char *odd_tmp[3]; // odd scratch per precision (even-odd) / full scratch (full lattice)
    long n_hop = 0;
    double hop_bytes = 0;
    const Geom &g() const { return op->g; }

    // a vector of the solve space (even parity, or full lattice) in precision p
    FieldView space(char *base, int p) const
    {
        return FieldView{base, p, (long)op->g.vh, fb(p, op->g), nsys * sps};
    }
    size_t space_bytes(int p) const { return (size_t)fb(p, op->g) * nsys * sps; }

    void count_hops(int prec, int n)
    {
        double b, f;
        lq_op_traffic(op, (lq_prec)prec, 1, op->has_clover ? 1 : 0, &b, &f);
        n_hop += n;
        hop_bytes += (double)n * b * op->g.vh * nsys;
    }

    // out = M in (dag: M^dag) in precision of the views
    void apply(const FieldView &out, const FieldView &in, bool dag)
    {
        const int p = in.prec;
        if (eo) {
            schur(op, p, out, in, FieldView{odd_tmp[p], p, (long)op->g.vh, fb(p, op->g), nsys}, dag, s);
        } else {
            dirac_full(op, p, out.base, in.base, nsys, dag, s);
        }
        count_hops(p, 2);
    }

    void reduce_finish(const FieldView &x, const FieldView &y, int mode, int op_fin)
    {
        LQ_HIP(launch_reduce(x, y, mode, partial, s));
        const int K = mode == RED_NORM ? 1 : mode == RED_DOT ? 2 : 3;
        LQ_HIP(launch_finish(partial, nsys, sps, blas_blocks(x.n), K, op_fin, sc, 1e-30, s));
    }
    void finish(int K, int op_fin, long n)
    {
        LQ_HIP(launch_finish(partial, nsys, sps, blas_blocks(n), K, op_fin, sc, 1e-30, s));
    }

    void pull()
    {
        LQ_HIP(hipMemcpyAsync(hsc, sc, sizeof(double) * NSC * nsys, hipMemcpyDeviceToHost, s));
        LQ_HIP(hipStreamSynchronize(s));
    }
    void push()
    {
        LQ_HIP(hipMemcpyAsync(sc, hsc, sizeof(double) * NSC * nsys, hipMemcpyHostToDevice, s));
    }
};

struct InnerVecs {
    FieldView x, r, p, v, sv, t, rhat, w;
};

// Inner BiCGStab on M e = rin from e = 0.  Returns when every system is
// done or broken down, or after max_iter iterations.
int inner_bicgstab(Ctx &c, const InnerVecs &V, const FieldView &rin, int max_iter, int check_every)
{
    LQ_HIP(launch_zero(V.x, c.s));
    LQ_HIP(launch_copy(V.r, rin, c.sc, c.sps, false, c.s));
    LQ_HIP(launch_copy(V.rhat, rin, c.sc, c.sps, false, c.s));
    LQ_HIP(launch_copy(V.p, rin, c.sc, c.sps, false, c.s));
    c.reduce_finish(V.r, V.r, RED_NORM, FIN_INIT_BICG);
    int it = 0;
    while (it < max_iter) {
        const int chunk = std::min(check_every, max_iter - it);
        for (int k = 0; k < chunk; ++k) {
            c.apply(V.v, V.p, false);
            c.reduce_finish(V.rhat, V.v, RED_DOT, FIN_BICG_ALPHA);
            LQ_HIP(launch_bicg_s(V.sv, V.r, V.v, c.sc, c.sps, c.s));
            c.apply(V.t, V.sv, false);
            c.reduce_finish(V.sv, V.t, RED_DOT_NORM, FIN_BICG_OMEGA);
            LQ_HIP(launch_bicg_xr(V.x, V.r, V.p, V.sv, V.t, V.rhat, c.sc, c.sps, c.partial, c.s));
            c.finish(3, FIN_BICG_RHO, V.r.n);
            LQ_HIP(launch_bicg_p(V.p, V.r, V.v, c.sc, c.sps, c.s));
        }
        it += chunk;
        c.pull();
        bool all = true;
        for (int i = 0; i < c.nsys; ++i) {
            const double *h = c.hsc + i * NSC;
            if (h[SC_DONE] == 0.0 && h[SC_BREAK] == 0.0) all = false;
        }
        if (all) break;
    }
    return it;
}

// Inner CG on M^dag M e = M^dag rin from e = 0.
int inner_cgne(Ctx &c, const InnerVecs &V, const FieldView &rin, int max_iter, int check_every)
{
    LQ_HIP(launch_zero(V.x, c.s));
    c.apply(V.r, rin, true);
    LQ_HIP(launch_copy(V.p, V.r, c.sc, c.sps, false, c.s));
    c.reduce_finish(V.r, V.r, RED_NORM, FIN_INIT_CG);
    int it = 0;
    while (it < max_iter) {
        const int chunk = std::min(check_every, max_iter - it);
        for (int k = 0; k < chunk; ++k) {
            c.apply(V.w, V.p, false);
            c.reduce_finish(V.w, V.w, RED_NORM, FIN_CG_ALPHA);
            c.apply(V.v, V.w, true);
            LQ_HIP(launch_cg_xr(V.x, V.r, V.p, V.v, c.sc, c.sps, c.partial, c.s));
            c.finish(1, FIN_CG_BETA, V.r.n);
            LQ_HIP(launch_cg_p(V.p, V.r, c.sc, c.sps, c.s));
        }
        it += chunk;
        c.pull();
        bool all = true;
        for (int i = 0; i < c.nsys; ++i) {
            const double *h = c.hsc + i * NSC;
            if (h[SC_DONE] == 0.0 && h[SC_BREAK] == 0.0) all = false;
        }
        if (all) break;
    }
    return it;
}

}  // namespace

// Solve D x = b for nsys systems; b64, x64: full packed FP64 fields.
// stats[i] filled for each system.  Returns LQ_OK or LQ_NOT_CONVERGED.
lq_status solve_packed(lq_op *op, const lq_solver_params &sp, int nsys, char *x64, const char *b64, bool use_x0,
                       lq_solve_stats *stats, hipStream_t s)
{
    const Geom &g = op->g;
    Ctx c{op, s, nsys};
    c.eo = sp.even_odd != 0;
    c.sps = c.eo ? 1 : 2;
    c.pin = sp.inner;
    c.px = sp.inner == F64 ? F64 : F32;

    // workspace
    Arena A;
    const size_t f64b = c.space_bytes(F64), finb = c.space_bytes(c.pin), fxb = c.space_bytes(c.px);
    const size_t odd = (size_t)fb(F64, g) * nsys * (c.eo ? 1 : 2);
    const size_t need = 6 * f64b + 8 * finb + fxb + 3 * (odd + 256) + 2 * (size_t)fb(F64, g) * nsys + 64 * 256;
    op->solver_ws.ensure(need);
    A.base = op->solver_ws.ptr;
    char *bh = A.take(f64b), *xs = A.take(f64b), *r64 = A.take(f64b), *y64 = A.take(f64b);
    char *full_r = A.take(2 * (size_t)fb(F64, g) * nsys), *full_y = A.take(2 * (size_t)fb(F64, g) * nsys);
    for (int p = 0; p < 3; ++p) c.odd_tmp[p] = A.take(odd);
    InnerVecs V;
    V.x = c.space(A.take(fxb), c.px);
    V.r = c.space(A.take(finb), c.pin);
    V.p = c.space(A.take(finb), c.pin);
    V.v = c.space(A.take(finb), c.pin);
    V.sv = c.space(A.take(finb), c.pin);
    V.t = c.space(A.take(finb), c.pin);
    V.rhat = c.space(A.take(finb), c.pin);
    V.w = c.space(A.take(finb), c.pin);
    const FieldView rin = c.space(A.take(finb), c.pin);

    op->solver_sc.ensure(sizeof(double) * NSC * nsys);
    c.sc = reinterpret_cast<double *>(op->solver_sc.ptr);
    if (op->host_sc_n < (size_t)NSC * nsys) {
        if (op->host_sc) LQ_HIP(hipHostFree(op->host_sc));
        op->host_sc = nullptr;
        LQ_HIP(hipHostMalloc(reinterpret_cast<void **>(&op->host_sc), sizeof(double) * NSC * nsys, 0));
        op->host_sc_n = (size_t)NSC * nsys;
    }
    c.hsc = op->host_sc;
    const long nblk = std::max<long>(hop_blocks(g.vh, 64), blas_blocks(g.vh));
    op->partial.ensure(sizeof(double) * 3 * nblk * nsys * 2);
    c.partial = reinterpret_cast<double *>(op->partial.ptr);
    std::memset(c.hsc, 0, sizeof(double) * NSC * nsys);
    c.push();

    const auto t0 = std::chrono::steady_clock::now();

    // |b|^2 of the full lattice, per system
    const FieldView bfull{const_cast<char *>(b64), F64, (long)g.vh, fb(F64, g), 2 * nsys};
    {
        LQ_HIP(launch_reduce(bfull, bfull, RED_NORM, c.partial, s));
        LQ_HIP(launch_finish(c.partial, nsys, 2, blas_blocks(g.vh), 1, FIN_NORM, c.sc, 0, s));
        c.pull();
    }
    std::vector<double> bn2(nsys);
    for (int i = 0; i < nsys; ++i) bn2[i] = c.hsc[i * NSC + SC_NORM2];
    for (int i = 0; i < nsys; ++i)
        if (!std::isfinite(bn2[i])) throw Failure{LQ_ERR_NONFINITE, "right-hand side is not finite"};

    // right-hand side of the solved system and the initial guess
    const FieldView bhv = c.space(bh, F64);
    const FieldView xv = c.space(xs, F64);
    const FieldView r64v = c.space(r64, F64);
    const FieldView y64v = c.space(y64, F64);
    if (c.eo) {
        const FieldView be = full_parity_view(const_cast<char *>(b64), F64, g, nsys, 0);
        const FieldView bo = full_parity_view(const_cast<char *>(b64), F64, g, nsys, 1);
        const FieldView t = FieldView{c.odd_tmp[F64], F64, (long)g.vh, fb(F64, g), nsys};
        clover_apply(op, F64, 1, true, t, bo, s);
        hop(op, F64, bhv, t, 0, false, 0, false, &be, op->prm.kappa, 0, nullptr, s);
        c.count_hops(F64, 1);
        if (use_x0) LQ_HIP(launch_copy(xv, full_parity_view(x64, F64, g, nsys, 0), c.sc, 1, false, s));
        else LQ_HIP(launch_zero(xv, s));
    } else {
        LQ_HIP(launch_copy(bhv, bfull, c.sc, 2, false, s));
        if (use_x0) LQ_HIP(launch_copy(xv, FieldView{x64, F64, (long)g.vh, fb(F64, g), 2 * nsys}, c.sc, 2, false, s));
        else LQ_HIP(launch_zero(xv, s));
    }

    std::vector<int> iters(nsys, 0), outer(nsys, 0), restarts(nsys, 0);
    int total_inner = 0;
    bool ok = false;
    for (int step = 0; step <= sp.max_outer; ++step) {
        // r = b_hat - M x, |r|^2
        c.pull();
        for (int i = 0; i < nsys; ++i) c.hsc[i * NSC + SC_OTARGET2] = sp.tol * sp.tol * bn2[i];
        c.push();
        c.apply(y64v, xv, false);
        LQ_HIP(launch_xmy_norm(r64v, bhv, y64v, c.partial, s));
        c.finish(1, FIN_NORM, g.vh);
        c.pull();
        bool all = true;
        for (int i = 0; i < nsys; ++i) {
            const double n2 = c.hsc[i * NSC + SC_NORM2];
            if (!std::isfinite(n2)) throw Failure{LQ_ERR_NONFINITE, "residual is not finite"};
            if (c.hsc[i * NSC + SC_ODONE] == 0.0) all = false;
        }
        if (all) {
            ok = true;
            break;
        }
        if (step == sp.max_outer || total_inner >= sp.max_iter) break;
        // relative target of this inner solve, per system
        for (int i = 0; i < nsys; ++i) {
            double *h = c.hsc + i * NSC;
            const double rn = std::sqrt(h[SC_NORM2]);
            double rel = 0.5 * sp.tol * std::sqrt(bn2[i]) / (rn > 0 ? rn : 1.0);
            if (c.pin != F64) rel = std::max(rel, sp.inner_tol);
            rel = std::min(rel, 0.5);
            h[SC_TARGET2] = rel * rel;  // relative; FIN_INIT converts it
            if (h[SC_ODONE] == 0.0) outer[i]++;
        }
        // SC_TARGET2 is relative to the initial inner residual (FIN_INIT
        // scales it): |rin| for BiCGStab, |M^dag rin| for CGNE.
        c.push();
        LQ_HIP(launch_copy(rin, r64v, c.sc, c.sps, true, s));
        const int budget = sp.max_iter - total_inner;
        int it = 0;
        if (sp.solver == LQ_CGNE) {
            it = inner_cgne(c, V, rin, budget, std::max(1, sp.check_every));
        } else {
            it = inner_bicgstab(c, V, rin, budget, std::max(1, sp.check_every));
        }
        total_inner += it;
        for (int i = 0; i < nsys; ++i) {
            const double *h = c.hsc + i * NSC;
            if (h[SC_ODONE] == 0.0) {
                iters[i] += (int)h[SC_ITER];
                if (h[SC_BREAK] != 0.0) restarts[i]++;
            }
        }
        // x += |r| e
        LQ_HIP(launch_accum(xv, V.x, c.sc, c.sps, true, s));
    }

    // full solution and true residual
    if (c.eo) {
        LQ_HIP(launch_copy(full_parity_view(x64, F64, g, nsys, 0), xv, c.sc, 1, false, s));
        const FieldView bo = full_parity_view(const_cast<char *>(b64), F64, g, nsys, 1);
        hop(op, F64, full_parity_view(x64, F64, g, nsys, 1), xv, 1, false, 2, true, &bo, op->prm.kappa, 0, nullptr, s);
        c.count_hops(F64, 1);
    } else {
        LQ_HIP(launch_copy(FieldView{x64, F64, (long)g.vh, fb(F64, g), 2 * nsys}, xv, c.sc, 2, false, s));
    }
    dirac_full(op, F64, full_y, x64, nsys, false, s);
    c.count_hops(F64, 2);
    const FieldView fr{full_r, F64, (long)g.vh, fb(F64, g), 2 * nsys};
    const FieldView fy{full_y, F64, (long)g.vh, fb(F64, g), 2 * nsys};
    LQ_HIP(launch_xmy_norm(fr, bfull, fy, c.partial, s));
    LQ_HIP(launch_finish(c.partial, nsys, 2, blas_blocks(g.vh), 1, FIN_NORM, c.sc, 0, s));
    c.pull();
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    bool all_conv = true;
    for (int i = 0; i < nsys; ++i) {
        const double r2 = c.hsc[i * NSC + SC_NORM2];
        const double diff = bn2[i] > 0 ? std::sqrt(r2 / bn2[i]) : 0.0;
        if (!std::isfinite(diff)) throw Failure{LQ_ERR_NONFINITE, "final residual is not finite"};
        const bool conv = diff <= sp.tol;
        all_conv = all_conv && conv;
        if (stats) {
            lq_solve_stats &st = stats[i];
            st.nconv = iters[i];
            st.nouter = outer[i];
            st.restarts = restarts[i];
            st.converged = conv ? 1 : 0;
            st.diff = diff;
            st.t_solve_ms = ms;
            st.hop_bytes = c.hop_bytes;
            st.n_hop = (int)c.n_hop;
        }
    }
    (void)ok;
    return all_conv ? LQ_OK : LQ_NOT_CONVERGED;
}

}  // namespace lq

using namespace lq;

extern "C" lq_status lq_solve(lq_op *op, const lq_solver_params *sp, lq_kind mode, int nrhs, void *x, const void *b,
                              int use_x0, lq_solve_stats *stats, void *stream)
{
    if (!op || !sp || !x || !b) {
        set_error("lq_solve: null argument");
        return LQ_ERR_ARG;
    }
    if (mode != LQ_D && mode != LQ_DDAG && mode != LQ_DDAGD) {
        set_error("lq_solve: mode must be LQ_D, LQ_DDAG or LQ_DDAGD");
        return LQ_ERR_ARG;
    }
    if (nrhs < 1 || sp->max_iter < 0 || sp->max_outer < 0 || !(sp->tol > 0) || !(sp->inner_tol > 0) ||
        (sp->solver != LQ_CGNE && sp->solver != LQ_BICGSTAB) || (sp->inner < LQ_F64 || sp->inner > LQ_F16)) {
        set_error("lq_solve: invalid solver parameters");
        return LQ_ERR_ARG;
    }
    if (!sp->even_odd && sp->solver != LQ_CGNE) {
        set_error("lq_solve: the full-lattice solve is CGNE only");
        return LQ_ERR_ARG;
    }
    if (!op->gauge_set) {
        set_error("lq_solve: gauge field not set");
        return LQ_ERR_STATE;
    }
    try {
        set_error("");
        LQ_HIP(hipSetDevice(op->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const Geom &g = op->g;
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
            // D^dag = gamma_5 D gamma_5: x = gamma_5 D^-1 gamma_5 b
            LQ_HIP(launch_gamma5(bfull, s));
            if (use_x0) LQ_HIP(launch_gamma5(xfull, s));
            st = solve_packed(op, *sp, nrhs, xp, bp, use_x0, stats, s);
            LQ_HIP(launch_gamma5(xfull, s));
            LQ_HIP(launch_gamma5(bfull, s));
        } else {
            // D^dag D x = b: y = (D^dag)^-1 b, then x = D^-1 y
            std::vector<lq_solve_stats> st1(nrhs);
            LQ_HIP(launch_gamma5(bfull, s));
            st = solve_packed(op, *sp, nrhs, xp, bp, false, st1.data(), s);
            if (st < 0) return st;
            LQ_HIP(launch_gamma5(xfull, s));  // y
            LQ_HIP(launch_gamma5(bfull, s));  // b restored
            op->tmp[0].ensure(full);
            char *yp = op->tmp[0].ptr;
            LQ_HIP(hipMemcpyAsync(yp, xp, full, hipMemcpyDeviceToDevice, s));
            lq_solver_params sp2 = *sp;
            sp2.tol = sp->tol * 0.5;
            st = solve_packed(op, sp2, nrhs, xp, yp, false, stats, s);
            // diff of the normal system |b - D^dag D x| / |b|
            op->tmp[1].ensure(full);
            dirac_full(op, F64, yp, xp, nrhs, false, s);
            dirac_full(op, F64, op->tmp[1].ptr, yp, nrhs, true, s);
            const FieldView fy{op->tmp[1].ptr, F64, (long)g.vh, fb(F64, g), 2 * nrhs};
            const FieldView fr{yp, F64, (long)g.vh, fb(F64, g), 2 * nrhs};
            double *partial = reinterpret_cast<double *>(op->partial.ptr);
            double *sc = reinterpret_cast<double *>(op->solver_sc.ptr);
            std::vector<double> bn2(nrhs), rn2(nrhs);
            LQ_HIP(launch_reduce(bfull, bfull, RED_NORM, partial, s));
            LQ_HIP(launch_finish(partial, nrhs, 2, blas_blocks(g.vh), 1, FIN_NORM, sc, 0, s));
            LQ_HIP(hipMemcpyAsync(op->host_sc, sc, sizeof(double) * NSC * nrhs, hipMemcpyDeviceToHost, s));
            LQ_HIP(hipStreamSynchronize(s));
            for (int i = 0; i < nrhs; ++i) bn2[i] = op->host_sc[i * NSC + SC_NORM2];
            LQ_HIP(launch_xmy_norm(fr, bfull, fy, partial, s));
            LQ_HIP(launch_finish(partial, nrhs, 2, blas_blocks(g.vh), 1, FIN_NORM, sc, 0, s));
            LQ_HIP(hipMemcpyAsync(op->host_sc, sc, sizeof(double) * NSC * nrhs, hipMemcpyDeviceToHost, s));
            LQ_HIP(hipStreamSynchronize(s));
            bool all = true;
            for (int i = 0; i < nrhs; ++i) {
                const double d = bn2[i] > 0 ? std::sqrt(op->host_sc[i * NSC + SC_NORM2] / bn2[i]) : 0.0;
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
            st = st < 0 ? st : (all ? LQ_OK : LQ_NOT_CONVERGED);
        }
        if (st < 0) return st;
        for (int p = 0; p < 2; ++p)
            LQ_HIP(launch_unpack_spinor(g, p, 0, full_parity_view(xp, F64, g, nrhs, p), xdst, s));
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
