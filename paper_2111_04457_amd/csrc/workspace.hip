// workspace.hip -- the operator's device memory as one caller-owned
// workspace: its layout (lq_workspace_bytes, lq_op_workspace_bytes) and
// binding (lq_op_bind).  An operator that is not bound allocates the same
// regions itself, on first use.
#include <algorithm>

#include "blas.h"
#include "solver.h"

namespace lq {

Geom make_geom(const lq_op_params &p)
{
    Geom g{};
    long vol = 1;
    for (int i = 0; i < 4; ++i) {
        g.L[i] = p.dims[i];
        g.bc_re[i] = p.bc[i][0];
        g.bc_im[i] = p.bc[i][1];
        vol *= p.dims[i];
    }
    g.lxh = p.dims[0] / 2;
    g.vh = (int)(vol / 2);
    return g;
}

size_t solver_ws_bytes(const Geom &g, int nsys, bool eo, int inner)
{
    const int sps = eo ? 1 : 2;
    const int px = inner == F64 ? F64 : F32;
    const size_t f64b = (size_t)fb(F64, g) * nsys * sps, finb = (size_t)fb(inner, g) * nsys * sps,
                 fxb = (size_t)fb(px, g) * nsys * sps, odd = (size_t)fb(F64, g) * nsys;
    // x, r, y, t, aux (FP64); three odd temporaries (FP64); x, M x (inner
    // solution precision); nine inner vectors (see make_ctx)
    return 5 * (f64b + 256) + 9 * (finb + 256) + 2 * (fxb + 256) + 3 * (odd + 256);
}

WorkspaceLayout workspace_layout(const lq_op_params &p, int nrhs)
{
    const Geom g = make_geom(p);
    const int nl = p.link_recon;
    const bool clover = p.csw != 0.0;
    const size_t f64 = (size_t)fb(F64, g);
    WorkspaceLayout w;
    using L = WorkspaceLayout;
    w.size[L::LINKS64] = 8 * (size_t)link_bytes(F64, 18, g.vh);
    w.size[L::LINKS32] = 8 * (size_t)link_bytes(F32, nl, g.vh);
    w.size[L::LINKS16] = 8 * (size_t)link_bytes(F16, nl, g.vh);
    w.size[L::LINKS64R] = nl == 12 ? 8 * (size_t)link_bytes(F64, 12, g.vh) : 0;
    for (int q = 0; q < 3; ++q) {
        w.size[L::CLOV64 + q] = clover ? 2 * (size_t)clover_bytes(q, g.vh) : 0;
        w.size[L::CLOVINV64 + q] = clover ? 2 * (size_t)clover_bytes(q, g.vh) : 0;
    }
    w.size[L::FLAG] = 256;
    // 0, 1: temporaries of composite applies and of the D^dag D solve (two
    // full FP64 fields); 2, 3: packed input / output of an apply (a full
    // field, or the force's four parity fields of each kind); 4, 5: packed
    // b and x of a solve; 6, 7: staging of host inputs / outputs (full
    // complex128 fields)
    const size_t full = 2 * f64 * nrhs;
    for (int t = 0; t < 8; ++t) w.size[L::TMP0 + t] = full;
    w.size[L::TMP2] = w.size[L::TMP3] = std::max(full, 8 * f64);
    const size_t nblk = (size_t)std::max<long>(hop_blocks(g.vh, 64), blas_blocks(g.vh));
    w.size[L::PARTIAL] = sizeof(double) * 3 * nblk * nrhs * 2;
    w.size[L::SOLVER_SC] = sizeof(double) * NSC * nrhs;
    // the solver's vectors (largest: an FP64 solve on the full lattice); the
    // same region holds the complex128 gauge field of a host-side set_gauge
    // and the field strengths while the clover term is built
    size_t ws = 0;
    for (int eo = 0; eo < 2; ++eo)
        for (int inner = F64; inner <= F16; ++inner) ws = std::max(ws, solver_ws_bytes(g, nrhs, eo != 0, inner));
    ws = std::max(ws, (size_t)g.vh * 2 * 4 * 9 * 16);
    ws = std::max(ws, clover_fbuf_bytes(g.vh));
    w.size[L::SOLVER_WS] = ws;
    size_t off = 0;
    for (int r = 0; r < L::NREGION; ++r) {
        w.off[r] = off;
        off += (w.size[r] + 255) & ~size_t(255);
    }
    w.total = off;
    return w;
}

}  // namespace lq

using namespace lq;

static lq_status ws_arg_error(const std::string &msg)
{
    set_error(msg);
    return LQ_ERR_ARG;
}

extern "C" {

lq_status lq_workspace_bytes(const lq_op_params *p, int nrhs, size_t *bytes)
{
    if (!p || !bytes) return ws_arg_error("lq_workspace_bytes: null argument");
    if (nrhs < 1) return ws_arg_error("lq_workspace_bytes: nrhs must be >= 1");
    long vol = 1;
    for (int i = 0; i < 4; ++i) {
        if (p->dims[i] < 2 || (p->dims[i] & 1)) return ws_arg_error("lq_workspace_bytes: every dimension must be even and >= 2");
        vol *= p->dims[i];
    }
    if (vol > (1L << 28)) return ws_arg_error("lq_workspace_bytes: volume above 2^28 sites");
    if (p->link_recon != 18 && p->link_recon != 12) return ws_arg_error("lq_workspace_bytes: link_recon must be 12 or 18");
    set_error("");
    *bytes = workspace_layout(*p, nrhs).total;
    return LQ_OK;
}

lq_status lq_op_workspace_bytes(const lq_op *op, int nrhs, size_t *bytes)
{
    if (!op) return ws_arg_error("lq_op_workspace_bytes: null operator");
    return lq_workspace_bytes(&op->prm, nrhs, bytes);
}

lq_status lq_op_bind(lq_op *op, void *dev_mem, size_t bytes)
{
    if (!op) return ws_arg_error("lq_op_bind: null operator");
    if (dev_mem && (reinterpret_cast<uintptr_t>(dev_mem) & 255))
        return ws_arg_error("lq_op_bind: the workspace must start on a 256-byte boundary");
    size_t need1 = workspace_layout(op->prm, 1).total;
    if (dev_mem && bytes < need1)
        return ws_arg_error("lq_op_bind: " + std::to_string(bytes) + " bytes given, at least " + std::to_string(need1) +
                            " needed (lq_op_workspace_bytes for nrhs 1)");
    try {
        set_error("");
        LQ_HIP(hipSetDevice(op->device));
        LQ_HIP(hipDeviceSynchronize());  // no kernel may still use the memory being replaced
        op->clear_graphs();
        op->gauge_set = false;
        op->even_inverted = false;
        Buf *regions[WorkspaceLayout::NREGION] = {
            &op->links[F64], &op->links[F32], &op->links[F16], &op->links64r, &op->clov[F64], &op->clov[F32],
            &op->clov[F16], &op->clovinv[F64], &op->clovinv[F32], &op->clovinv[F16], &op->flag, &op->tmp[0],
            &op->tmp[1], &op->tmp[2], &op->tmp[3], &op->tmp[4], &op->tmp[5], &op->tmp[6], &op->tmp[7],
            &op->partial, &op->solver_sc, &op->solver_ws};
        for (Buf *b : regions) b->release();
        op->bound_nrhs = 0;
        if (!dev_mem) return LQ_OK;  // unbound: the library allocates again on demand
        // the most right-hand sides whose layout fits
        const auto fits = [&](int n) { return workspace_layout(op->prm, n).total <= bytes; };
        int lo = 1, hi = 2;  // lo fits; hi does not (or is past the cap)
        while (hi <= (1 << 20) && fits(hi)) {
            lo = hi;
            hi *= 2;
        }
        while (hi - lo > 1) {
            const int mid = lo + (hi - lo) / 2;
            (fits(mid) ? lo : hi) = mid;
        }
        const WorkspaceLayout w = workspace_layout(op->prm, lo);
        char *base = static_cast<char *>(dev_mem);
        // every region is borrowed, the empty ones too (the clover blocks of
        // a Wilson operator): a later need of one is an error, not an allocation
        for (int r = 0; r < WorkspaceLayout::NREGION; ++r) regions[r]->borrow(base + w.off[r], w.size[r]);
        op->bound_nrhs = lo;
        // the pinned host mirror of the solver scalars (host memory)
        if (op->host_sc_n < (size_t)NSC * lo) {
            if (op->host_sc) LQ_HIP(hipHostFree(op->host_sc));
            op->host_sc = nullptr;
            op->host_sc_n = 0;
            LQ_HIP(hipHostMalloc(reinterpret_cast<void **>(&op->host_sc), sizeof(double) * NSC * lo, 0));
            op->host_sc_n = (size_t)NSC * lo;
        }
        return LQ_OK;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return LQ_ERR_STATE;
    }
}

}  // extern "C"
