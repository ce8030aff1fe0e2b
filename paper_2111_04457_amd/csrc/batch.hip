// batch.hip -- one solve over several lattices of different volumes (a
// ragged batch: each an lq_op with its own gauge field, nrhs right-hand
// sides each), with every stage of an inner Krylov iteration ONE launch over
// all lattices' systems.
//
// The solver's vectors are ragged fields: the even-site slices of every
// system, lattice by lattice, back to back.  A table of workgroup tiles
// (system, block of 256 sites) drives the vector kernels over all slices at
// once, and per-system ranges of their partial sums drive the fixed-order
// reductions.  The Schur operator is two launches of the batched hopping
// kernel, whose workgroups run each lattice's tiles with that lattice's
// arguments (geometry, links, clover blocks, slices, scalars).  Each chunk
// of inner iterations is captured once into a hipGraph and replayed.
//
// The outer FP64 loop takes its decisions per lattice, as a solve of that
// lattice alone would (the even-odd preparation and reconstruction, the FP64
// residuals, the choice of residual update), so every system's result
// equals that of a separate lq_solve bit for bit: the per-site arithmetic,
// the partial sums and their order of summation are the same.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "solver.h"

namespace lq {

namespace {

constexpr int kBT = 256;  // sites per workgroup of the vector kernels

int vec_blocks(long n) { return (int)((n + kBT - 1) / kBT); }

// Layout of the batch's systems and its device tables (once per batch: the
// volumes and right-hand-side counts do not change).
void layout(lq_batch *bt, hipStream_t s)
{
    if (bt->nsys) return;
    const int n = (int)bt->ops.size();
    bt->sys0.assign(n, 0);
    bt->site0.assign(n, 0);
    bt->hop_part0.assign(n, 0);
    std::vector<Tile> tiles;
    std::vector<int2> blas, hopr;
    long site = 0, hp = 0;
    int sys = 0;
    for (int i = 0; i < n; ++i) {
        const Geom &g = bt->ops[i]->g;
        bt->sys0[i] = sys;
        bt->site0[i] = site;
        bt->hop_part0[i] = hp;
        const long pad = padded_sites(g.vh);
        const int nw = (g.vh + 63) / 64;
        for (int r = 0; r < bt->nrhs[i]; ++r, ++sys) {
            blas.push_back(int2{(int)tiles.size(), vec_blocks(g.vh)});
            for (int k = 0; k < vec_blocks(g.vh); ++k) tiles.push_back(Tile{sys, k, g.vh, (int)site});
            hopr.push_back(int2{(int)(hp + (long)r * nw), nw});
            site += pad;
        }
        hp += (long)bt->nrhs[i] * nw;
    }
    if (site > 0x7fffffffL || (long)tiles.size() > 0x7fffffffL)
        throw Failure{LQ_ERR_ARG, "lq_batch_solve: the batch holds more than 2^31 sites"};
    bt->nsys = sys;
    bt->sites = site;
    bt->ntiles = (int)tiles.size();
    bt->tiles.ensure(sizeof(Tile) * tiles.size());
    bt->blas_range.ensure(sizeof(int2) * blas.size());
    bt->hop_range.ensure(sizeof(int2) * hopr.size());
    LQ_HIP(hipMemcpyAsync(bt->tiles.ptr, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, s));
    LQ_HIP(hipMemcpyAsync(bt->blas_range.ptr, blas.data(), sizeof(int2) * blas.size(), hipMemcpyHostToDevice, s));
    LQ_HIP(hipMemcpyAsync(bt->hop_range.ptr, hopr.data(), sizeof(int2) * hopr.size(), hipMemcpyHostToDevice, s));
    LQ_HIP(hipStreamSynchronize(s));
}

void make_batch_ctx(SolveCtx &c, lq_batch *bt, int inner, hipStream_t s)
{
    c.op = nullptr;
    c.bt = bt;
    c.s = s;
    c.nsys = bt->nsys;
    c.eo = true;
    c.sps = 1;
    c.pin = inner;
    c.px = inner == F64 ? F64 : F32;
    const size_t f64b = c.space_bytes(F64), finb = c.space_bytes(c.pin), fxb = c.space_bytes(c.px);
    bt->ws.ensure(5 * (f64b + 256) + 9 * (finb + 256) + 2 * (fxb + 256) + 3 * (f64b + 256));
    carve_vectors(c, bt->ws.ptr, f64b);
    bt->sc.ensure(sizeof(double) * NSC * c.nsys);
    c.sc = reinterpret_cast<double *>(bt->sc.ptr);
    if (bt->host_sc_n < (size_t)NSC * c.nsys) {
        if (bt->host_sc) LQ_HIP(hipHostFree(bt->host_sc));
        bt->host_sc = nullptr;
        bt->host_sc_n = 0;
        LQ_HIP(hipHostMalloc(reinterpret_cast<void **>(&bt->host_sc), sizeof(double) * NSC * c.nsys, 0));
        bt->host_sc_n = (size_t)NSC * c.nsys;
    }
    c.hsc = bt->host_sc;
    // partial sums: the vector kernels' (one per tile), the fused hops' (one
    // per 64-site wavefront and system) and the per-lattice norms of the
    // full right-hand sides (two parities)
    long np = bt->ntiles;
    long hop = 0, full = 0;
    for (size_t i = 0; i < bt->ops.size(); ++i) {
        const long vh = bt->ops[i]->g.vh;
        hop += (long)bt->nrhs[i] * ((vh + 63) / 64);
        full = std::max(full, 2L * bt->nrhs[i] * vec_blocks(vh));
    }
    np = std::max(np, std::max(hop, full));
    bt->partial.ensure(sizeof(double) * 3 * (size_t)np);
    c.partial = reinterpret_cast<double *>(bt->partial.ptr);
    std::memset(c.hsc, 0, sizeof(double) * NSC * c.nsys);
    c.push();
}

}  // namespace

void batch_schur(SolveCtx &c, int prec, const FieldView &out, const FieldView &in, const FieldView &odd, bool dag,
                 bool left, int red, const FieldView *w)
{
    lq_batch *bt = c.bt;
    if (left && dag) throw Failure{LQ_ERR_STATE, "the preconditioned Schur operator has no dagger form here"};
    const int n = (int)bt->ops.size();
    const bool clover = bt->ops[0]->has_clover || bt->ops[0]->has_twist;  // a site-local factor
    const int K = red == 2 ? 2 : 3;
    // four right-hand sides per workgroup (links in LDS) where the operators'
    // setting takes them for the fewest right-hand sides of the batch
    int minr = bt->nrhs[0];
    for (int g = 1; g < n; ++g) minr = std::min(minr, bt->nrhs[g]);
    const int R = (prec != F64 && minr >= 4 && eff_nr(bt->ops[0], prec, minr) == 4) ? 4 : 1;
    for (int g0 = 0; g0 < n; g0 += kMaxBatch) {
        HopBatch k1{}, k2{};
        const int nl = std::min(kMaxBatch, n - g0);
        k1.nlat = k2.nlat = nl;
        k1.nr = k2.nr = R;
        for (int j = 0; j < nl; ++j) {
            const int g = g0 + j;
            lq_op *o = bt->ops[g];
            const FieldView in_g = c.group_view(in, g), out_g = c.group_view(out, g), odd_g = c.group_view(odd, g);
            FieldView w_g{};
            if (w) w_g = c.group_view(*w, g);
            const double k = o->prm.kappa;
            // t_o = A_oo^-1 H_oe x_e, then y_e = A_ee x_e - kappa^2 H_eo t_o
            // (left: x_e - kappa^2 A_ee^-1 H_eo t_o), as the operator's schur()
            HopArgs a1 = hop_args(o, prec, odd_g, in_g, 1, 2, true, dag, nullptr, 1.0, nullptr);
            HopArgs a2 = hop_args(o, prec, out_g, odd_g, 0, left ? 3 : 1, left, dag, &in_g, -k * k, w ? &w_g : nullptr);
            if (c.masked) {
                set_hop_mask(a1, c.sc + (long)bt->sys0[g] * NSC);
                set_hop_mask(a2, c.sc + (long)bt->sys0[g] * NSC);
            }
            if (red) a2.partial = c.partial + bt->hop_part0[g] * K;
            k1.a[j] = a1;
            k2.a[j] = a2;
            const int tiles = hop_blocks(o->g.vh, 64) * ((bt->nrhs[g] + R - 1) / R);
            k1.tile_off[j + 1] = k1.tile_off[j] + tiles;
            k2.tile_off[j + 1] = k2.tile_off[j] + tiles;
        }
        const int recon = bt->ops[0]->prm.link_recon;
        const int tw = bt->ops[0]->has_twist ? kTwist : 0;  // every operator of a batch is of one kind
        LQ_HIP(launch_hop_batch(k1, prec, recon, dag, clover ? (2 | tw) : 0, false, 0, c.s));
        LQ_HIP(launch_hop_batch(k2, prec, recon, dag, clover ? ((left ? 3 : 1) | tw) : 0, true, red, c.s));
    }
}

namespace {

// D x = b for every system of the batch: packed b (op->tmp[4]) and x
// (op->tmp[5]) of each lattice, full FP64 fields [rhs][parity].
lq_status solve_batch(lq_batch *bt, const lq_solver_params &sp, lq_solve_stats *stats, hipStream_t s)
{
    const int n = (int)bt->ops.size();
    layout(bt, s);
    // graphs captured for other gauge fields / parameters are dropped
    std::vector<long> gen;
    for (const lq_op *o : bt->ops) gen.push_back(o->generation);
    if (gen != bt->generations) {
        bt->clear_graphs();
        bt->generations = gen;
    }
    SolveCtx c;
    make_batch_ctx(c, bt, sp.inner, s);
    for (lq_op *o : bt->ops) c.log = std::max(c.log, log_level(o));
    const auto t0 = std::chrono::steady_clock::now();
    // |b|^2 per system, lattice by lattice (as a lattice's own solve sums them)
    for (int i = 0; i < n; ++i) {
        lq_op *o = bt->ops[i];
        const FieldView bfull{o->tmp[4].ptr, F64, (long)o->g.vh, fb(F64, o->g), 2 * bt->nrhs[i]};
        LQ_HIP(launch_reduce(bfull, bfull, RED_NORM, c.partial, s));
        LQ_HIP(launch_finish(c.partial, bt->nrhs[i], 2, blas_blocks(o->g.vh), 1, FIN_NORM,
                             c.sc + (long)bt->sys0[i] * NSC, 0, s));
    }
    c.pull();
    std::vector<double> bn2(c.nsys);
    for (int k = 0; k < c.nsys; ++k) {
        bn2[k] = c.hsc[k * NSC + SC_NORM2];
        if (!std::isfinite(bn2[k])) throw Failure{LQ_ERR_NONFINITE, "right-hand side is not finite"};
    }
    // even-odd right-hand sides b_e + kappa H_eo A_oo^-1 b_o; x_e = 0
    const FieldView todd = c.space(c.odd_tmp[F64], F64);
    for (int i = 0; i < n; ++i) {
        lq_op *o = bt->ops[i];
        const int nr = bt->nrhs[i];
        const FieldView be = full_parity_view(o->tmp[4].ptr, F64, o->g, nr, 0);
        const FieldView bo = full_parity_view(o->tmp[4].ptr, F64, o->g, nr, 1);
        const FieldView t = c.group_view(todd, i);
        clover_apply(o, F64, 1, true, t, bo, s);
        hop(o, F64, c.group_view(c.aux64, i), t, 0, false, 0, false, &be, o->prm.kappa, 0, nullptr, s);
    }
    c.count_hops(F64, 1);
    LQ_HIP(launch_zero(c.x64, s));
    std::vector<double> target2(c.nsys);
    for (int k = 0; k < c.nsys; ++k) target2[k] = sp.tol * sp.tol * bn2[k];
    const OuterStats os = defect_correction(c, sp, false, c.aux64, target2, true);
    // x_o = A_oo^-1 (b_o + kappa H_oe x_e), lattice by lattice
    for (int i = 0; i < n; ++i) {
        lq_op *o = bt->ops[i];
        const int nr = bt->nrhs[i];
        const FieldView xe = c.group_view(c.x64, i);
        LQ_HIP(launch_copy(full_parity_view(o->tmp[5].ptr, F64, o->g, nr, 0), xe, c.sc, 1, false, s));
        const FieldView bo = full_parity_view(o->tmp[4].ptr, F64, o->g, nr, 1);
        hop(o, F64, full_parity_view(o->tmp[5].ptr, F64, o->g, nr, 1), xe, 1, false, 2, true, &bo, o->prm.kappa, 0,
            nullptr, s);
    }
    c.count_hops(F64, 1);
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    bool all_conv = true;
    for (int k = 0; k < c.nsys; ++k) {
        const double diff = bn2[k] > 0 ? std::sqrt(os.r2[k] / bn2[k]) : 0.0;
        if (!std::isfinite(diff)) throw Failure{LQ_ERR_NONFINITE, "final residual is not finite"};
        const bool conv = diff <= sp.tol;
        all_conv = all_conv && conv;
        if (stats) {
            lq_solve_stats &st = stats[k];
            st.nconv = os.iters[k];
            st.nouter = os.outer[k];
            st.restarts = os.restarts[k];
            st.converged = conv ? 1 : 0;
            st.diff = diff;
            st.t_solve_ms = ms;
            st.hop_bytes = c.hop_bytes;
            st.n_hop = (int)c.n_hop;
        }
    }
    return all_conv ? LQ_OK : LQ_NOT_CONVERGED;
}

}  // namespace

}  // namespace lq

using namespace lq;

extern "C" lq_status lq_batch_create(lq_op *const *ops, int nops, const int *nrhs, lq_batch **out)
{
    if (!ops || !nrhs || !out || nops < 1) {
        set_error("lq_batch_create: null argument or nops < 1");
        return LQ_ERR_ARG;
    }
    *out = nullptr;
    for (int i = 0; i < nops; ++i) {
        if (!ops[i] || nrhs[i] < 1) {
            set_error("lq_batch_create: null operator or nrhs < 1");
            return LQ_ERR_ARG;
        }
        for (int j = 0; j < i; ++j)
            if (ops[j] == ops[i]) {
                set_error("lq_batch_create: an operator appears twice (use nrhs for several sources)");
                return LQ_ERR_ARG;
            }
        if (ops[i]->device != ops[0]->device) {
            set_error("lq_batch_create: operators on different devices");
            return LQ_ERR_ARG;
        }
        if (ops[i]->prm.link_recon != ops[0]->prm.link_recon) {
            set_error("lq_batch_create: the operators of a batch need one link format (link_recon)");
            return LQ_ERR_ARG;
        }
    }
    lq_batch *b = new (std::nothrow) lq_batch();
    if (!b) {
        set_error("lq_batch_create: host allocation failed");
        return LQ_ERR_NOMEM;
    }
    b->ops.assign(ops, ops + nops);
    b->nrhs.assign(nrhs, nrhs + nops);
    try {
        LQ_HIP(hipSetDevice(ops[0]->device));
        LQ_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        LQ_HIP(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
        LQ_HIP(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    } catch (const Failure &f) {
        delete b;
        set_error(f.msg);
        return f.code;
    }
    set_error("");
    *out = b;
    return LQ_OK;
}

extern "C" void lq_batch_destroy(lq_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->ops[0]->device);
    (void)hipDeviceSynchronize();
    delete b;
}

extern "C" lq_status lq_batch_solve(lq_batch *bt, const lq_solver_params *sp, void *const *x, const void *const *b,
                                    lq_solve_stats *stats, void *stream)
{
    if (!bt || !sp || !x || !b) {
        set_error("lq_batch_solve: null argument");
        return LQ_ERR_ARG;
    }
    std::string why;
    if (!valid_solver_params(sp, why)) {
        set_error("lq_batch_solve: invalid solver parameters: " + why);
        return LQ_ERR_ARG;
    }
    if (sp->deflate) {
        set_error("lq_batch_solve: deflation is a solve of one operator (lq_solve); a batch does not deflate");
        return LQ_ERR_ARG;
    }
    if (!sp->even_odd) {
        set_error("lq_batch_solve: the batched solve runs the even-odd system (even_odd = 1)");
        return LQ_ERR_ARG;
    }
    const int n = (int)bt->ops.size();
    for (int i = 0; i < n; ++i) {
        lq_op *o = bt->ops[i];
        if (!x[i] || !b[i]) {
            set_error("lq_batch_solve: null x or b");
            return LQ_ERR_ARG;
        }
        if (!o->gauge_set) {
            set_error("lq_batch_solve: gauge field not set");
            return LQ_ERR_STATE;
        }
        if (o->has_clover != bt->ops[0]->has_clover || o->has_twist != bt->ops[0]->has_twist) {
            set_error("lq_batch_solve: the operators of a batch must be of one kind (all clover, all twisted-mass or "
                      "all Wilson)");
            return LQ_ERR_ARG;
        }
        if (o->bound_nrhs && bt->nrhs[i] > o->bound_nrhs) {
            set_error("lq_batch_solve: lattice " + std::to_string(i) + ": the bound workspace holds " +
                      std::to_string(o->bound_nrhs) + " right-hand sides");
            return LQ_ERR_ARG;
        }
    }
    try {
        set_error("");
        LQ_HIP(hipSetDevice(bt->ops[0]->device));
        // ordered after the caller's stream, synchronized before returning
        hipStream_t us = static_cast<hipStream_t>(stream);
        LQ_HIP(hipEventRecord(bt->ev_in, us));
        LQ_HIP(hipStreamWaitEvent(bt->stream, bt->ev_in, 0));
        hipStream_t s = bt->stream;
        const bool left = sp->left_precond && sp->solver == LQ_BICGSTAB;
        for (int i = 0; i < n; ++i) {
            lq_op *o = bt->ops[i];
            if (left) ensure_even_inverse(o, s);
            const size_t full = 2 * (size_t)fb(F64, o->g) * bt->nrhs[i];
            o->tmp[4].ensure(full);
            o->tmp[5].ensure(full);
            for (int p = 0; p < 2; ++p)
                LQ_HIP(launch_pack_spinor(o->g, p, 0, static_cast<const double *>(b[i]),
                                          full_parity_view(o->tmp[4].ptr, F64, o->g, bt->nrhs[i], p), s));
        }
        const lq_status st = solve_batch(bt, *sp, stats, s);
        if (st < 0) return st;
        for (int i = 0; i < n; ++i) {
            lq_op *o = bt->ops[i];
            for (int p = 0; p < 2; ++p)
                LQ_HIP(launch_unpack_spinor(o->g, p, 0, full_parity_view(o->tmp[5].ptr, F64, o->g, bt->nrhs[i], p),
                                            static_cast<double *>(x[i]), s));
        }
        LQ_HIP(hipEventRecord(bt->ev_out, s));
        LQ_HIP(hipStreamWaitEvent(us, bt->ev_out, 0));
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
