// abi.hip -- the extern "C" entry points declared in include/lq.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "runtime.h"

using namespace lq;

// Device memory of lq_op_apply_noalloc: a fixed array in the code object, so
// that the call needs no allocation.  Each GPU the library runs on holds its
// own copy (at its own address) until the process ends; every call on that
// GPU shares it.  Host code never passes the array's name to a kernel or a
// copy: it uses the device address looked up once per device.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up on the
// first call on that device, with that device current).
char *scratch_on_device(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) throw Failure{LQ_ERR_STATE, "device index out of range"};
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        LQ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Failure{LQ_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array"};
        g_scratch_ptr[dev] = static_cast<char *>(p);
    }
    return g_scratch_ptr[dev];
}

size_t round256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

#define LQ_VERSION_STRING "lq-mi355x 0.1 (gfx950)"

// Run body, turning Failure / std exceptions into a status + message.
template <typename F>
static lq_status guarded(F &&body)
{
    try {
        set_error("");
        return body();
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return LQ_ERR_NOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return LQ_ERR_STATE;
    }
}

static lq_status arg_error(const std::string &msg)
{
    set_error(msg);
    return LQ_ERR_ARG;
}

static bool valid_prec(int p) { return p == LQ_F64 || p == LQ_F32 || p == LQ_F16; }

static void select_device(lq_op *op) { LQ_HIP(hipSetDevice(op->device)); }

extern "C" {

void lq_op_params_default(lq_op_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    for (int i = 0; i < 4; ++i) {
        p->dims[i] = 4;
        p->bc[i][0] = 1.0;
        p->bc[i][1] = 0.0;
    }
    p->kappa = 0.125;
    p->csw = 0.0;
    p->clover_traceless = 1;
    p->link_recon = 18;
}

void lq_solver_params_default(lq_solver_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->solver = LQ_BICGSTAB;
    p->tol = 1e-10;
    p->max_iter = 100000;
    p->inner = LQ_F32;
    p->inner_tol = 1e-5;
    p->max_outer = 100;
    p->check_every = 8;
    p->even_odd = 1;
    p->left_precond = 0;
    p->reliable = 0;
    p->deflate = 0;
}

const char *lq_version(void) { return LQ_VERSION_STRING; }

const char *lq_last_error(void) { return get_error(); }

lq_status lq_op_create(const lq_op_params *p, lq_op **out)
{
    if (!p || !out) return arg_error("lq_op_create: null argument");
    *out = nullptr;
    long vol = 1;
    for (int i = 0; i < 4; ++i) {
        if (p->dims[i] < 2 || (p->dims[i] & 1))
            return arg_error("lq_op_create: every dimension must be even and >= 2");
        vol *= p->dims[i];
    }
    if (vol > (1L << 28)) return arg_error("lq_op_create: volume above 2^28 sites");
    if (!std::isfinite(p->kappa) || !std::isfinite(p->csw)) return arg_error("lq_op_create: kappa and csw must be finite");
    for (int i = 0; i < 4; ++i) {
        const double m = std::hypot(p->bc[i][0], p->bc[i][1]);
        if (!(std::fabs(m - 1.0) < 1e-12)) return arg_error("lq_op_create: boundary phases must have modulus 1");
    }
    if (p->link_recon != 18 && p->link_recon != 12) return arg_error("lq_op_create: link_recon must be 12 or 18");
    if (!std::isfinite(p->twist)) return arg_error("lq_op_create: twist must be finite");
    if (p->twist != 0.0 && p->csw != 0.0)
        return arg_error("lq_op_create: the twisted-mass operator is provided without the clover term (csw = 0)");
    return guarded([&]() -> lq_status {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
            (void)hipGetLastError();
            set_error("lq_op_create: no HIP device visible");
            return LQ_ERR_NODEVICE;
        }
        int dev = 0;
        LQ_HIP(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        LQ_HIP(hipGetDeviceProperties(&prop, dev));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            set_error(std::string("lq_op_create: device is ") + prop.gcnArchName + ", this library is built for gfx950");
            return LQ_ERR_NODEVICE;
        }
        lq_op *op = new lq_op();
        op->prm = *p;
        op->device = dev;
        op->g = make_geom(*p);
        op->has_clover = p->csw != 0.0;
        op->has_twist = p->twist != 0.0;
        try {
            // device memory comes later: a bound workspace, or allocations on
            // first use (lq_op_set_gauge)
            LQ_HIP(hipStreamCreateWithFlags(&op->stream, hipStreamNonBlocking));
            LQ_HIP(hipEventCreateWithFlags(&op->ev_in, hipEventDisableTiming));
            LQ_HIP(hipEventCreateWithFlags(&op->ev_out, hipEventDisableTiming));
        } catch (...) {
            delete op;
            throw;
        }
        *out = op;
        return LQ_OK;
    });
}

void lq_op_destroy(lq_op *op)
{
    if (!op) return;
    (void)hipSetDevice(op->device);
    (void)hipDeviceSynchronize();
    delete op;
}

static void build_clover(lq_op *op, hipStream_t s)
{
    const Geom &g = op->g;
    op->even_inverted = false;
    if (!op->has_clover) return;
    for (int p = 0; p < 3; ++p) {
        op->clov[p].ensure(2 * clover_bytes(p, g.vh));
        op->clovinv[p].ensure(2 * clover_bytes(p, g.vh));
    }
    {
        // the field strengths: in the solver's region of a bound workspace,
        // else a buffer freed once the blocks are built
        Buf own;
        char *fbuf;
        if (op->bound_nrhs) {
            op->solver_ws.ensure(clover_fbuf_bytes(g.vh));
            fbuf = op->solver_ws.ptr;
        } else {
            own.ensure(clover_fbuf_bytes(g.vh));
            fbuf = own.ptr;
        }
        LQ_HIP(launch_clover_build(g, op->links[F64].ptr, op->prm.csw, op->prm.kappa, op->prm.clover_traceless,
                                   fbuf, op->clov[F64].ptr, s));
        LQ_HIP(hipStreamSynchronize(s));
    }
    // only A_oo is inverted: the even-odd operators use A_ee and A_oo^-1
    LQ_HIP(hipMemsetAsync(op->flag.ptr, 0, sizeof(int), s));
    LQ_HIP(launch_clover_invert(g, 1, op->clov[F64].ptr, op->clovinv[F64].ptr, reinterpret_cast<int *>(op->flag.ptr),
                                s));
    for (int p = F32; p <= F16; ++p) {
        LQ_HIP(launch_convert_clover(g, op->clov[F64].ptr, p, op->clov[p].ptr, s));
        LQ_HIP(launch_convert_clover(g, op->clovinv[F64].ptr, p, op->clovinv[p].ptr, s, 1, 1));
    }
    int flag = 0;
    LQ_HIP(hipMemcpyAsync(&flag, op->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    LQ_HIP(hipStreamSynchronize(s));
    if (flag) throw Failure{LQ_ERR_SINGULAR, "a clover block A_oo = 1 + F on an odd site is singular"};
}

// Pack the links of the device complex128 gauge field U in every precision
// and build the clover term.
static void set_gauge_device(lq_op *op, const double *U, hipStream_t s)
{
    const Geom &g = op->g;
    op->gauge_set = false;
    op->defl_n = 0;  // the deflation space belonged to the previous gauge field
    op->clear_graphs();
    op->links[F64].ensure(8 * link_bytes(F64, 18, g.vh));
    op->links[F32].ensure(8 * link_bytes(F32, op->prm.link_recon, g.vh));
    op->links[F16].ensure(8 * link_bytes(F16, op->prm.link_recon, g.vh));
    if (op->prm.link_recon == 12) op->links64r.ensure(8 * link_bytes(F64, 12, g.vh));
    op->flag.ensure(sizeof(int));
    LQ_HIP(launch_pack_links_f64(g, U, op->links[F64].ptr, s));
    LQ_HIP(launch_convert_links(g, op->links[F64].ptr, F32, op->prm.link_recon, op->links[F32].ptr, s));
    LQ_HIP(launch_convert_links(g, op->links[F64].ptr, F16, op->prm.link_recon, op->links[F16].ptr, s));
    if (op->prm.link_recon == 12) LQ_HIP(launch_convert_links(g, op->links[F64].ptr, F64, 12, op->links64r.ptr, s));
    build_clover(op, s);
    op->gauge_set = true;
}

lq_status lq_op_set_gauge(lq_op *op, const void *U, void *stream)
{
    if (!op || !U) return arg_error("lq_op_set_gauge: null argument");
    return guarded([&]() -> lq_status {
        select_device(op);
        set_gauge_device(op, static_cast<const double *>(U), static_cast<hipStream_t>(stream));
        return LQ_OK;
    });
}

lq_status lq_op_set_gauge_host(lq_op *op, const void *U, void *stream)
{
    if (!op || !U) return arg_error("lq_op_set_gauge_host: null argument");
    return guarded([&]() -> lq_status {
        select_device(op);
        hipStream_t s = static_cast<hipStream_t>(stream);
        // staged in the solver's region (unused between solves)
        const size_t bytes = (size_t)op->g.vh * 2 * 4 * 9 * 16;
        op->solver_ws.ensure(bytes);
        op->clear_graphs();
        LQ_HIP(hipMemcpyAsync(op->solver_ws.ptr, U, bytes, hipMemcpyHostToDevice, s));
        set_gauge_device(op, reinterpret_cast<const double *>(op->solver_ws.ptr), s);
        return LQ_OK;
    });
}

lq_status lq_op_set_params(lq_op *op, double kappa, double csw, const double bc[4][2], void *stream)
{
    if (!op) return arg_error("lq_op_set_params: null operator");
    if (!std::isfinite(kappa) || !std::isfinite(csw)) return arg_error("lq_op_set_params: kappa and csw must be finite");
    if (bc)
        for (int i = 0; i < 4; ++i)
            if (!(std::fabs(std::hypot(bc[i][0], bc[i][1]) - 1.0) < 1e-12))
                return arg_error("lq_op_set_params: boundary phases must have modulus 1");
    if (op->has_twist && csw != 0.0)
        return arg_error("lq_op_set_params: the twisted-mass operator is provided without the clover term (csw = 0)");
    if (op->bound_nrhs && csw != 0.0 && op->clov[F64].bytes < 2 * (size_t)clover_bytes(F64, op->g.vh)) {
        set_error("lq_op_set_params: the bound workspace has no room for clover blocks (it was laid out with "
                  "csw = 0): bind one of lq_op_workspace_bytes bytes after setting csw");
        return LQ_ERR_NOMEM;
    }
    return guarded([&]() -> lq_status {
        select_device(op);
        op->clear_graphs();
        op->defl_n = 0;  // the deflation space belonged to the previous parameters
        op->prm.kappa = kappa;
        op->prm.csw = csw;
        op->has_clover = csw != 0.0;
        if (bc)
            for (int i = 0; i < 4; ++i) {
                op->prm.bc[i][0] = op->g.bc_re[i] = bc[i][0];
                op->prm.bc[i][1] = op->g.bc_im[i] = bc[i][1];
            }
        if (op->gauge_set) {
            op->gauge_set = false;
            build_clover(op, static_cast<hipStream_t>(stream));
            op->gauge_set = true;
        }
        return LQ_OK;
    });
}

// Bytes of the complex128 boundary-layout field of kind (full or parity) and nrhs.
static size_t io_bytes(const lq_op *op, lq_kind kind, int nrhs)
{
    return (size_t)(kind_is_full(kind) ? 2 : 1) * op->g.vh * 12 * 16 * nrhs;
}

static lq_status check_apply_args(const char *fn, lq_op *op, lq_kind kind, lq_prec prec, const void *out,
                                  const void *in, int nrhs)
{
    const std::string f(fn);
    if (!op || !out || !in) return arg_error(f + ": null argument");
    if (kind < LQ_D || kind > LQ_SCHUR_LEFT) return arg_error(f + ": unknown kind");
    if (!valid_prec(prec)) return arg_error(f + ": unknown precision");
    if (nrhs < 1) return arg_error(f + ": nrhs must be >= 1");
    if (out == in) return arg_error(f + ": out and in must differ");
    if (op->bound_nrhs && nrhs > op->bound_nrhs)
        return arg_error(f + ": the bound workspace holds " + std::to_string(op->bound_nrhs) + " right-hand sides, " +
                         std::to_string(nrhs) + " requested");
    if (!op->gauge_set) {
        set_error(f + ": gauge field not set");
        return LQ_ERR_STATE;
    }
    return LQ_OK;
}

// out = K in on device complex128 fields, through the packed buffers tmp[2], tmp[3].
static void apply_device(lq_op *op, lq_kind kind, lq_prec prec, double *dst, const double *src, int nrhs,
                         hipStream_t s)
{
    const Geom &g = op->g;
    const bool full = kind_is_full(kind);
    const long bytes = (full ? 2 : 1) * fb(prec, g) * nrhs;
    op->tmp[2].ensure(bytes);
    op->tmp[3].ensure(bytes);
    if (full) {
        for (int p = 0; p < 2; ++p)
            LQ_HIP(launch_pack_spinor(g, p, 0, src, full_parity_view(op->tmp[2].ptr, prec, g, nrhs, p), s));
    } else {
        LQ_HIP(launch_pack_spinor(g, 0, 1, src, parity_view(op->tmp[2].ptr, prec, g, nrhs), s));
    }
    apply_packed(op, kind, prec, op->tmp[3].ptr, op->tmp[2].ptr, nrhs, s);
    if (full) {
        for (int p = 0; p < 2; ++p)
            LQ_HIP(launch_unpack_spinor(g, p, 0, full_parity_view(op->tmp[3].ptr, prec, g, nrhs, p), dst, s));
    } else {
        LQ_HIP(launch_unpack_spinor(g, 0, 1, parity_view(op->tmp[3].ptr, prec, g, nrhs), dst, s));
    }
}

lq_status lq_op_apply(lq_op *op, lq_kind kind, lq_prec prec, void *out, const void *in, int nrhs, void *stream)
{
    const lq_status st = check_apply_args("lq_op_apply", op, kind, prec, out, in, nrhs);
    if (st != LQ_OK) return st;
    return guarded([&]() -> lq_status {
        select_device(op);
        apply_device(op, kind, prec, static_cast<double *>(out), static_cast<const double *>(in), nrhs,
                     static_cast<hipStream_t>(stream));
        return LQ_OK;
    });
}

lq_status lq_op_apply_host(lq_op *op, lq_kind kind, lq_prec prec, void *out, const void *in, int nrhs, void *stream)
{
    const lq_status st = check_apply_args("lq_op_apply_host", op, kind, prec, out, in, nrhs);
    if (st != LQ_OK) return st;
    return guarded([&]() -> lq_status {
        select_device(op);
        hipStream_t s = static_cast<hipStream_t>(stream);
        const size_t n = io_bytes(op, kind, nrhs);
        op->tmp[6].ensure(n);
        op->tmp[7].ensure(n);
        LQ_HIP(hipMemcpyAsync(op->tmp[6].ptr, in, n, hipMemcpyHostToDevice, s));
        apply_device(op, kind, prec, reinterpret_cast<double *>(op->tmp[7].ptr),
                     reinterpret_cast<const double *>(op->tmp[6].ptr), nrhs, s);
        LQ_HIP(hipMemcpyAsync(out, op->tmp[7].ptr, n, hipMemcpyDeviceToHost, s));
        LQ_HIP(hipStreamSynchronize(s));
        return LQ_OK;
    });
}

lq_status lq_op_apply_noalloc(lq_op *op, lq_kind kind, lq_prec prec, void *out, const void *in, int nrhs,
                              void *stream)
{
    if (!op || !out || !in) return arg_error("lq_op_apply_noalloc: null argument");
    if (kind < LQ_D || kind > LQ_SCHUR_LEFT) return arg_error("lq_op_apply_noalloc: unknown kind");
    if (!valid_prec(prec)) return arg_error("lq_op_apply_noalloc: unknown precision");
    if (nrhs < 1) return arg_error("lq_op_apply_noalloc: nrhs must be >= 1");
    if (out == in) return arg_error("lq_op_apply_noalloc: out and in must differ");
    if (!op->gauge_set) {
        set_error("lq_op_apply_noalloc: gauge field not set");
        return LQ_ERR_STATE;
    }
    const Geom &g = op->g;
    const bool full = kind_is_full(kind);
    const size_t field = round256((size_t)(full ? 2 : 1) * fb(prec, g) * nrhs);
    size_t t0b, t1b;
    apply_temp_bytes(kind, prec, g, nrhs, t0b, t1b);
    const size_t need = 2 * field + round256(t0b) + round256(t1b);
    if (need > kNoallocScratchBytes)
        return arg_error("lq_op_apply_noalloc: the packed fields of this call need " + std::to_string(need) +
                         " bytes, above the fixed scratch of " + std::to_string(kNoallocScratchBytes) +
                         " bytes (use lq_op_apply)");
    return guarded([&]() -> lq_status {
        select_device(op);
        char *base = scratch_on_device(op->device);
        char *pin = base, *pout = base + field;
        char *t0 = t0b ? pout + field : nullptr;
        char *t1 = t1b ? t0 + round256(t0b) : nullptr;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const double *src = static_cast<const double *>(in);
        double *dst = static_cast<double *>(out);
        if (full) {
            for (int p = 0; p < 2; ++p)
                LQ_HIP(launch_pack_spinor(g, p, 0, src, full_parity_view(pin, prec, g, nrhs, p), s));
        } else {
            LQ_HIP(launch_pack_spinor(g, 0, 1, src, parity_view(pin, prec, g, nrhs), s));
        }
        apply_packed(op, kind, prec, pout, pin, nrhs, s, t0, t1);
        if (full) {
            for (int p = 0; p < 2; ++p)
                LQ_HIP(launch_unpack_spinor(g, p, 0, full_parity_view(pout, prec, g, nrhs, p), dst, s));
        } else {
            LQ_HIP(launch_unpack_spinor(g, 0, 1, parity_view(pout, prec, g, nrhs), dst, s));
        }
        return LQ_OK;
    });
}

lq_status lq_field_create(lq_op *op, lq_prec prec, int nrhs, lq_field **out)
{
    if (!op || !out) return arg_error("lq_field_create: null argument");
    if (!valid_prec(prec)) return arg_error("lq_field_create: unknown precision");
    if (nrhs < 1) return arg_error("lq_field_create: nrhs must be >= 1");
    *out = nullptr;
    return guarded([&]() -> lq_status {
        select_device(op);
        lq_field *f = new lq_field();
        f->op = op;
        f->prec = prec;
        f->nrhs = nrhs;
        try {
            f->data.ensure(fb(prec, op->g) * nrhs);
            LQ_HIP(hipMemset(f->data.ptr, 0, fb(prec, op->g) * nrhs));
        } catch (...) {
            delete f;
            throw;
        }
        *out = f;
        return LQ_OK;
    });
}

void lq_field_destroy(lq_field *f)
{
    if (!f) return;
    (void)hipSetDevice(f->op->device);
    (void)hipDeviceSynchronize();
    delete f;
}

lq_status lq_field_import(lq_field *f, const void *src, void *stream)
{
    if (!f || !src) return arg_error("lq_field_import: null argument");
    return guarded([&]() -> lq_status {
        select_device(f->op);
        LQ_HIP(launch_pack_spinor(f->op->g, 0, 1, static_cast<const double *>(src), f->view(),
                                  static_cast<hipStream_t>(stream)));
        return LQ_OK;
    });
}

lq_status lq_field_export(const lq_field *f, void *dst, void *stream)
{
    if (!f || !dst) return arg_error("lq_field_export: null argument");
    return guarded([&]() -> lq_status {
        select_device(f->op);
        LQ_HIP(launch_unpack_spinor(f->op->g, 0, 1, f->view(), static_cast<double *>(dst),
                                    static_cast<hipStream_t>(stream)));
        return LQ_OK;
    });
}

lq_status lq_op_apply_field(lq_op *op, lq_kind kind, lq_field *out, const lq_field *in, void *stream)
{
    if (!op || !out || !in) return arg_error("lq_op_apply_field: null argument");
    if (kind < LQ_SCHUR || kind > LQ_SCHUR_LEFT) return arg_error("lq_op_apply_field: kind must act on parity fields");
    if (out->op != op || in->op != op) return arg_error("lq_op_apply_field: fields belong to another operator");
    if (out->prec != in->prec || out->nrhs != in->nrhs) return arg_error("lq_op_apply_field: precision or nrhs differ");
    if (out == in) return arg_error("lq_op_apply_field: out and in must differ");
    if (!op->gauge_set) {
        set_error("lq_op_apply_field: gauge field not set");
        return LQ_ERR_STATE;
    }
    return guarded([&]() -> lq_status {
        select_device(op);
        apply_packed(op, kind, in->prec, out->data.ptr, in->data.ptr, in->nrhs, static_cast<hipStream_t>(stream));
        return LQ_OK;
    });
}

lq_status lq_op_set_block(lq_op *op, lq_prec prec, int block)
{
    if (!op) return arg_error("lq_op_set_block: null operator");
    if (!valid_prec(prec)) return arg_error("lq_op_set_block: unknown precision");
    if (block != 64 && block != 128 && block != 256) return arg_error("lq_op_set_block: block must be 64, 128 or 256");
    op->hop_block[prec] = block;
    op->clear_graphs();
    return LQ_OK;
}

lq_status lq_op_set_option(lq_op *op, const char *name, int value)
{
    if (!op || !name) return arg_error("lq_op_set_option: null argument");
    const std::string n(name);
    const bool order_ok = value >= -1 && value <= 2;  // -1: automatic
    const bool nr_ok = value == 0 || value == 1 || value == 2 || value == 4;  // 0: automatic
    if (n == "xcd_remap" && order_ok) op->xcd_remap[0] = op->xcd_remap[1] = op->xcd_remap[2] = value;
    else if (n == "xcd_remap_f64" && order_ok) op->xcd_remap[F64] = value;
    else if (n == "xcd_remap_f32" && order_ok) op->xcd_remap[F32] = value;
    else if (n == "xcd_remap_f16" && order_ok) op->xcd_remap[F16] = value;
    else if (n == "rhs_per_thread" && nr_ok)
        op->rhs_per_thread[0] = op->rhs_per_thread[1] = op->rhs_per_thread[2] = value;
    else if (n == "rhs_per_thread_f64" && nr_ok) op->rhs_per_thread[F64] = value;
    else if (n == "rhs_per_thread_f32" && nr_ok) op->rhs_per_thread[F32] = value;
    else if (n == "rhs_per_thread_f16" && nr_ok) op->rhs_per_thread[F16] = value;
    else if (n == "graphs" && (value == 0 || value == 1)) op->use_graphs = value;
    else if (n == "halo" && (value == 0 || value == 1)) op->halo[0] = op->halo[1] = op->halo[2] = value;
    else if (n == "halo_f16" && (value == 0 || value == 1)) op->halo[F16] = value;
    else if (n == "tune_form" && (value == 0 || value == 1)) op->tune_form = value;
    else if (n == "break_at" && value >= 0) op->break_at = value;
    else if (n == "log_level" && value >= 0 && value <= 2) op->log_level = value;
    else return arg_error("lq_op_set_option: unknown option or value: " + n);
    op->clear_graphs();
    return LQ_OK;
}

lq_status lq_op_get_option(const lq_op *op, const char *name, int *value)
{
    if (!op || !name || !value) return arg_error("lq_op_get_option: null argument");
    const std::string n(name);
    if (n == "xcd_remap" || n == "xcd_remap_f16") *value = op->xcd_remap[F16];
    else if (n == "xcd_remap_f64") *value = op->xcd_remap[F64];
    else if (n == "xcd_remap_f32") *value = op->xcd_remap[F32];
    else if (n == "rhs_per_thread_f64") *value = op->rhs_per_thread[F64];
    else if (n == "rhs_per_thread_f32") *value = op->rhs_per_thread[F32];
    else if (n == "rhs_per_thread" || n == "rhs_per_thread_f16") *value = op->rhs_per_thread[F16];
    else if (n == "graphs") *value = op->use_graphs;
    else if (n == "halo" || n == "halo_f16") *value = op->halo[F16];
    else if (n == "tune_form") *value = op->tune_form;
    else if (n == "break_at") *value = op->break_at;
    else if (n == "log_level") *value = op->log_level;
    else if (n == "hop_block_f64") *value = op->hop_block[F64];
    else if (n == "hop_block_f32") *value = op->hop_block[F32];
    else if (n == "hop_block_f16") *value = op->hop_block[F16];
    else if (n == "work_kib") *value = (int)std::min<size_t>(op->work_bytes() >> 10, 0x7fffffff);
    else if (n == "owned_kib") *value = (int)std::min<size_t>((op->owned_bytes() + 1023) >> 10, 0x7fffffff);
    else if (n == "bound_nrhs") *value = op->bound_nrhs;
    else return arg_error("lq_op_get_option: unknown option: " + n);
    return LQ_OK;
}

lq_status lq_op_traffic(const lq_op *op, lq_prec prec, int nrhs, int clover, double *bytes_per_site,
                        double *flops_per_site)
{
    if (!op || !bytes_per_site || !flops_per_site) return arg_error("lq_op_traffic: null argument");
    if (!valid_prec(prec) || nrhs < 1) return arg_error("lq_op_traffic: bad precision or nrhs");
    const double rs = prec == LQ_F64 ? 8 : prec == LQ_F32 ? 4 : 2;
    const int nl = op->prm.link_recon;
    const double spinor = 24 * rs + (prec == LQ_F16 ? 4 : 0);
    double b = 8.0 * nl * rs / nrhs + 2.0 * spinor;
    double f = 1320.0;
    if (clover) {
        b += 72.0 * rs / nrhs;
        f += 504.0;
    }
    *bytes_per_site = b;
    *flops_per_site = f;
    return LQ_OK;
}

}  // extern "C"
