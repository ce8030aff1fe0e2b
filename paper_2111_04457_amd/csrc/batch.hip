// batch.hip -- one solve over several lattices of different volumes (each
// an lq_op with its own gauge field, nrhs right-hand sides each).
//
// The FP64 defect-correction outer loop runs in lockstep over the lattices.
// Each chunk of inner Krylov iterations of ALL lattices is captured into a
// single hipGraph: the capture forks from the batch's stream into one
// branch per lattice (the lattice's own stream) and joins them again, so one
// graph launch advances every system and the kernels of independent
// lattices may run concurrently on the GPU.  Systems that converge are
// frozen by the kernels' masks; lattices whose systems are all frozen drop
// out of the next chunk's graph.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "solver.h"

struct lq_batch {
    std::vector<lq_op *> ops;
    std::vector<int> nrhs;
    hipStream_t main = nullptr;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    struct G {
        std::vector<long> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<G> graphs;
    ~lq_batch()
    {
        for (auto &g : graphs) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            if (g.graph) (void)hipGraphDestroy(g.graph);
        }
        for (auto e : ev_join) (void)hipEventDestroy(e);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (main) (void)hipStreamDestroy(main);
    }
};

using namespace lq;

namespace {

// Wait on the host for every lattice's stream.
void sync_all(const std::vector<SolveCtx> &cs)
{
    for (const auto &c : cs) LQ_HIP(hipStreamSynchronize(c.s));
}

// One graph launch = `chunk` inner iterations of every active lattice.
void run_batch_chunk(lq_batch *bt, std::vector<SolveCtx> &cs, const std::vector<int> &active, int kind, int chunk)
{
    std::vector<long> key = {kind, chunk};
    for (size_t i = 0; i < cs.size(); ++i) {
        if (!active[i]) continue;
        const lq_op *op = cs[i].op;
        key.insert(key.end(), {(long)i, (long)op, op->generation, (long)op->solver_ws.ptr, (long)op->solver_ws.bytes,
                               (long)cs[i].partial, (long)cs[i].sc, cs[i].nsys, cs[i].pin});
    }
    lq_batch::G *g = nullptr;
    for (auto &e : bt->graphs)
        if (e.key == key) g = &e;
    // the branches may only start after each lattice's eager work
    for (size_t i = 0; i < cs.size(); ++i)
        if (active[i]) {
            LQ_HIP(hipEventRecord(bt->ev_join[i], cs[i].s));
            LQ_HIP(hipStreamWaitEvent(bt->main, bt->ev_join[i], 0));
        }
    if (!g) {
        lq_batch::G ng;
        ng.key = key;
        LQ_HIP(hipStreamBeginCapture(bt->main, hipStreamCaptureModeThreadLocal));
        try {
            LQ_HIP(hipEventRecord(bt->ev_fork, bt->main));
            for (size_t i = 0; i < cs.size(); ++i) {
                if (!active[i]) continue;
                SolveCtx &c = cs[i];
                LQ_HIP(hipStreamWaitEvent(c.s, bt->ev_fork, 0));
                c.masked = true;
                for (int k = 0; k < chunk; ++k) {
                    if (kind == 1) bicg_iter(c);
                    else cg_iter(c);
                }
                c.masked = false;
                LQ_HIP(hipEventRecord(bt->ev_join[i], c.s));
                LQ_HIP(hipStreamWaitEvent(bt->main, bt->ev_join[i], 0));
            }
        } catch (...) {
            for (auto &c : cs) c.masked = false;
            hipGraph_t tmp = nullptr;
            (void)hipStreamEndCapture(bt->main, &tmp);
            if (tmp) (void)hipGraphDestroy(tmp);
            throw;
        }
        LQ_HIP(hipStreamEndCapture(bt->main, &ng.graph));
        LQ_HIP(hipGraphInstantiate(&ng.exec, ng.graph, nullptr, nullptr, 0));
        bt->graphs.push_back(ng);
        g = &bt->graphs.back();
    }
    LQ_HIP(hipGraphLaunch(g->exec, bt->main));
    LQ_HIP(hipStreamSynchronize(bt->main));
}

}  // namespace

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
    }
    try {
        set_error("");
        LQ_HIP(hipSetDevice(ops[0]->device));
        lq_batch *b = new lq_batch();
        b->ops.assign(ops, ops + nops);
        b->nrhs.assign(nrhs, nrhs + nops);
        try {
            LQ_HIP(hipStreamCreateWithFlags(&b->main, hipStreamNonBlocking));
            LQ_HIP(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
            b->ev_join.resize(nops, nullptr);
            for (int i = 0; i < nops; ++i) LQ_HIP(hipEventCreateWithFlags(&b->ev_join[i], hipEventDisableTiming));
        } catch (...) {
            delete b;
            throw;
        }
        *out = b;
        return LQ_OK;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    }
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
    const int n = (int)bt->ops.size();
    for (int i = 0; i < n; ++i) {
        if (!x[i] || !b[i]) {
            set_error("lq_batch_solve: null x or b");
            return LQ_ERR_ARG;
        }
        if (!bt->ops[i]->gauge_set) {
            set_error("lq_batch_solve: gauge field not set");
            return LQ_ERR_STATE;
        }
    }
    try {
        set_error("");
        LQ_HIP(hipSetDevice(bt->ops[0]->device));
        hipStream_t us = static_cast<hipStream_t>(stream);
        const auto t0 = std::chrono::steady_clock::now();
        const bool eo = sp->even_odd != 0;
        std::vector<SolveCtx> cs(n);
        std::vector<std::vector<double>> bn2(n), target2(n);
        std::vector<FieldView> rhs(n), bfull(n);
        std::vector<char *> xp(n), bp(n);
        for (int i = 0; i < n; ++i) {
            lq_op *op = bt->ops[i];
            const Geom &g = op->g;
            const int nr = bt->nrhs[i];
            LQ_HIP(hipEventRecord(op->ev_in, us));
            LQ_HIP(hipStreamWaitEvent(op->stream, op->ev_in, 0));
            hipStream_t s = op->stream;
            const size_t full = 2 * (size_t)fb(F64, g) * nr;
            op->tmp[4].ensure(full);
            op->tmp[5].ensure(full);
            bp[i] = op->tmp[4].ptr;
            xp[i] = op->tmp[5].ptr;
            for (int p = 0; p < 2; ++p)
                LQ_HIP(launch_pack_spinor(g, p, 0, static_cast<const double *>(b[i]),
                                          full_parity_view(bp[i], F64, g, nr, p), s));
            make_ctx(cs[i], op, nr, eo, sp->inner, s);
            SolveCtx &c = cs[i];
            bfull[i] = FieldView{bp[i], F64, (long)g.vh, fb(F64, g), 2 * nr};
            bn2[i] = norms2(c, bfull[i], 2);
            for (double v : bn2[i])
                if (!std::isfinite(v)) throw Failure{LQ_ERR_NONFINITE, "right-hand side is not finite"};
            target2[i].resize(nr);
            for (int k = 0; k < nr; ++k) target2[i][k] = sp->tol * sp->tol * bn2[i][k];
            if (eo) {
                rhs[i] = c.aux64;
                const FieldView be = full_parity_view(bp[i], F64, g, nr, 0);
                const FieldView bo = full_parity_view(bp[i], F64, g, nr, 1);
                const FieldView t{c.odd_tmp[F64], F64, (long)g.vh, fb(F64, g), nr};
                clover_apply(op, F64, 1, true, t, bo, s);
                hop(op, F64, rhs[i], t, 0, false, 0, false, &be, op->prm.kappa, 0, nullptr, s);
                c.count_hops(F64, 1);
            } else {
                rhs[i] = bfull[i];
            }
            LQ_HIP(launch_zero(c.x64, s));
        }
        std::vector<std::vector<int>> iters(n), outer(n), restarts(n);
        for (int i = 0; i < n; ++i) {
            iters[i].assign(bt->nrhs[i], 0);
            outer[i].assign(bt->nrhs[i], 0);
            restarts[i].assign(bt->nrhs[i], 0);
        }
        const int kind = sp->solver == LQ_CGNE ? 2 : 1;
        int total_inner = 0;
        std::vector<int> live(n, 1);
        ChunkPlan plan;  // one chunk length for all lattices: the largest hint
        for (int step = 0; step <= sp->max_outer; ++step) {
            // residuals of the lattices still running
            for (int i = 0; i < n; ++i) {
                if (!live[i]) continue;
                SolveCtx &c = cs[i];
                c.pull();
                for (int k = 0; k < c.nsys; ++k) c.hsc[k * NSC + SC_OTARGET2] = target2[i][k];
                c.push();
                c.apply(c.y64, c.x64, false);
                LQ_HIP(launch_xmy_norm(c.r64, rhs[i], c.y64, c.partial, c.s));
                c.finish(1, FIN_NORM, c.r64.n);
            }
            bool all = true;
            for (int i = 0; i < n; ++i) {
                if (!live[i]) continue;
                SolveCtx &c = cs[i];
                c.pull();
                bool done = true;
                for (int k = 0; k < c.nsys; ++k) {
                    if (!std::isfinite(c.hsc[k * NSC + SC_NORM2])) throw Failure{LQ_ERR_NONFINITE, "residual is not finite"};
                    if (c.hsc[k * NSC + SC_ODONE] == 0.0) done = false;
                }
                if (done) live[i] = 0;
                else all = false;
            }
            if (all || step == sp->max_outer || total_inner >= sp->max_iter) break;
            // inner solves of every live lattice
            for (int i = 0; i < n; ++i) {
                if (!live[i]) continue;
                SolveCtx &c = cs[i];
                for (int k = 0; k < c.nsys; ++k) {
                    double *h = c.hsc + k * NSC;
                    const double rn = std::sqrt(h[SC_NORM2]);
                    double rel = 0.5 * std::sqrt(target2[i][k]) / (rn > 0 ? rn : 1.0);
                    if (c.pin != F64) rel = std::max(rel, sp->inner_tol);
                    h[SC_TARGET2] = std::min(rel, 0.5) * std::min(rel, 0.5);
                    if (h[SC_ODONE] == 0.0) outer[i][k]++;
                }
                c.push();
                LQ_HIP(launch_copy(c.irin, c.r64, c.sc, c.sps, true, c.s));
                if (kind == 1) bicg_init(c);
                else cg_init(c, false);
            }
            constexpr int kInnerCap = 1000;
            const int budget = std::min(sp->max_iter - total_inner, kInnerCap);
            plan.start(sp->check_every);
            std::vector<std::vector<double>> prev(n);
            for (int i = 0; i < n; ++i) prev[i].assign(cs[i].nsys, 0.0);
            std::vector<int> act = live;
            int it = 0;
            sync_all(cs);
            for (int i = 0; i < n; ++i)
                if (act[i] && (cs[i].pull(), all_frozen(cs[i]))) act[i] = 0;
            while (it < budget && std::any_of(act.begin(), act.end(), [](int v) { return v != 0; })) {
                const int chunk = plan.next(budget - it);
                run_batch_chunk(bt, cs, act, kind, chunk);
                it += chunk;
                for (int i = 0; i < n; ++i) {
                    if (!act[i]) continue;
                    cs[i].pull();
                    cs[i].count_iterations(prev[i]);
                    if (all_frozen(cs[i])) act[i] = 0;
                }
            }
            total_inner += it;
            int most = 0;
            for (int i = 0; i < n; ++i) {
                if (!live[i]) continue;
                ChunkPlan one;
                one.learn(cs[i]);
                most = std::max(most, one.hint);
            }
            plan.hint = most;
            for (int i = 0; i < n; ++i) {
                if (!live[i]) continue;
                SolveCtx &c = cs[i];
                for (int k = 0; k < c.nsys; ++k) {
                    const double *h = c.hsc + k * NSC;
                    if (h[SC_ODONE] == 0.0) {
                        iters[i][k] += (int)h[SC_ITER];
                        if (h[SC_BREAK] != 0.0) restarts[i][k]++;
                    }
                }
                LQ_HIP(launch_accum(c.x64, c.ix, c.sc, c.sps, true, c.s));
            }
        }
        // reconstruction, true residual, export
        double hop_bytes = 0;
        long n_hop = 0;
        std::vector<std::vector<double>> diff(n);
        for (int i = 0; i < n; ++i) {
            lq_op *op = bt->ops[i];
            const Geom &g = op->g;
            SolveCtx &c = cs[i];
            const int nr = bt->nrhs[i];
            hipStream_t s = c.s;
            const FieldView xfull{xp[i], F64, (long)g.vh, fb(F64, g), 2 * nr};
            if (eo) {
                LQ_HIP(launch_copy(full_parity_view(xp[i], F64, g, nr, 0), c.x64, c.sc, 1, false, s));
                const FieldView bo = full_parity_view(bp[i], F64, g, nr, 1);
                hop(op, F64, full_parity_view(xp[i], F64, g, nr, 1), c.x64, 1, false, 2, true, &bo, op->prm.kappa, 0,
                    nullptr, s);
                c.count_hops(F64, 1);
            } else {
                LQ_HIP(launch_copy(xfull, c.x64, c.sc, 2, false, s));
            }
            // the residual of the last outer step at the final iterate is
            // |b - D x| (see solve_packed): SC_NORM2 still holds it
            for (int p = 0; p < 2; ++p)
                LQ_HIP(launch_unpack_spinor(g, p, 0, full_parity_view(xp[i], F64, g, nr, p), static_cast<double *>(x[i]), s));
            c.pull();
            diff[i].resize(nr);
            for (int k = 0; k < nr; ++k) {
                const double r2 = c.hsc[k * NSC + SC_NORM2];
                diff[i][k] = bn2[i][k] > 0 ? std::sqrt(r2 / bn2[i][k]) : 0.0;
                if (!std::isfinite(diff[i][k])) throw Failure{LQ_ERR_NONFINITE, "final residual is not finite"};
            }
            hop_bytes += c.hop_bytes;
            n_hop += c.n_hop;
            LQ_HIP(hipEventRecord(op->ev_out, s));
            LQ_HIP(hipStreamWaitEvent(us, op->ev_out, 0));
        }
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        bool all_conv = true;
        int idx = 0;
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < bt->nrhs[i]; ++k, ++idx) {
                const bool conv = diff[i][k] <= sp->tol;
                all_conv = all_conv && conv;
                if (stats) {
                    lq_solve_stats &st = stats[idx];
                    st.nconv = iters[i][k];
                    st.nouter = outer[i][k];
                    st.restarts = restarts[i][k];
                    st.converged = conv ? 1 : 0;
                    st.diff = diff[i][k];
                    st.t_solve_ms = ms;
                    st.hop_bytes = hop_bytes;
                    st.n_hop = (int)n_hop;
                }
            }
        return all_conv ? LQ_OK : LQ_NOT_CONVERGED;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return LQ_ERR_STATE;
    }
}
