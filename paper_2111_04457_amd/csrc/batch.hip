// batch.hip -- one solve over several lattices of different volumes (each
// an lq_op with its own gauge field, nrhs right-hand sides each).
//
// Every lattice's solve runs on its operator's own stream, driven by a host
// thread of its own, so the kernels of independent lattices overlap on the
// GPU: while a small lattice waits for its scalar read-backs or issues its
// short launches, the large lattices keep the compute units busy.  Each
// lattice's solve is the ordinary one (even-odd preparation, FP64 defect
// correction around graph-captured inner iterations, reconstruction), so the
// results equal those of separate lq_solve calls bit for bit.
#include <string>
#include <thread>
#include <vector>

#include "solver.h"

struct lq_batch {
    std::vector<lq_op *> ops;
    std::vector<int> nrhs;
};

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
    }
    lq_batch *b = new (std::nothrow) lq_batch();
    if (!b) {
        set_error("lq_batch_create: host allocation failed");
        return LQ_ERR_NOMEM;
    }
    b->ops.assign(ops, ops + nops);
    b->nrhs.assign(nrhs, nrhs + nops);
    set_error("");
    *out = b;
    return LQ_OK;
}

extern "C" void lq_batch_destroy(lq_batch *b) { delete b; }

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
    // per lattice: its offset in stats, its status and error message
    std::vector<int> off(n, 0);
    for (int i = 1; i < n; ++i) off[i] = off[i - 1] + bt->nrhs[i - 1];
    std::vector<lq_status> st(n, LQ_OK);
    std::vector<std::string> msg(n);
    std::vector<lq_solve_stats> local(off[n - 1] + bt->nrhs[n - 1]);
    auto run = [&](int i) {
        st[i] = lq_solve(bt->ops[i], sp, LQ_D, bt->nrhs[i], x[i], b[i], 0, local.data() + off[i], stream);
        if (st[i] < 0) {
            const char *m = lq_last_error();
            msg[i] = m ? m : "";
        }
    };
    std::vector<std::thread> threads;
    try {
        for (int i = 1; i < n; ++i) threads.emplace_back(run, i);
    } catch (const std::exception &) {
        for (auto &t : threads) t.join();
        set_error("lq_batch_solve: could not start host threads");
        return LQ_ERR_STATE;
    }
    run(0);
    for (auto &t : threads) t.join();
    // the first failure in batch order decides the status
    for (int i = 0; i < n; ++i)
        if (st[i] < 0) {
            set_error("lq_batch_solve: lattice " + std::to_string(i) + ": " + msg[i]);
            return st[i];
        }
    if (stats)
        for (size_t k = 0; k < local.size(); ++k) stats[k] = local[k];
    set_error("");
    bool all = true;
    for (int i = 0; i < n; ++i) all = all && st[i] == LQ_OK;
    return all ? LQ_OK : LQ_NOT_CONVERGED;
}
