// deflate.hip -- deflation inside the solve: approximate low modes of
// A = M^dag M (the eigensolver's output, Sec. 4 lists eigensolvers among
// the solver algorithms) kept with the operator in the packed FP64 layout
// (lq_op_set_deflation), and the projection the outer FP64 loop applies to
// each residual before an inner solve:
//
//   c_k = v_k^dag y / lambda_k,  y = M^dag r (or r for M^dag M x = b),
//   e = sum_k c_k v_k,  x += e,  r -= M e (or M^dag M e).
//
// With exact eigenpairs the new residual of M x = b has no component along
// the left singular vectors u_k = M v_k / sqrt(lambda_k), and the remaining
// error none along v_k; the Krylov solver then works on the rest of the
// spectrum.  The update of r is an FP64 apply, so r stays the true residual
// of the updated x whatever the quality of the vectors.
#include <cmath>

#include "solver.h"

namespace lq {

namespace {

constexpr int DT = 256;   // threads per workgroup
constexpr int DKC = 8;    // eigenvectors per workgroup of the dot kernel
constexpr int DNB = 128;  // site blocks of the dot kernel per system (at most)

int dot_blocks(long vh) { return (int)std::min<long>(DNB, (vh + DT - 1) / DT); }

// partial[((sys * nvec) + k) * nb + blk] = (re, im) of this block's share of
// <v_k, y_sys> (sites blk * DT, blk * DT + nb * DT, ...)
__global__ __launch_bounds__(DT) void defl_dot_kernel(const char *__restrict__ V, long vs, int nvec, FieldView y,
                                                      double *__restrict__ partial)
{
    const int nb = gridDim.x, sys = blockIdx.y, k0 = blockIdx.z * DKC;
    const char *ys = y.base + (long)sys * y.rs;
    double re[DKC], im[DKC];
#pragma unroll
    for (int q = 0; q < DKC; ++q) re[q] = im[q] = 0.0;
    for (long i = (long)blockIdx.x * DT + threadIdx.x; i < y.n; i += (long)nb * DT) {
        const Spinor<double> yv = load_spinor<F64>(ys, i, y.n);
#pragma unroll
        for (int q = 0; q < DKC; ++q) {
            if (k0 + q >= nvec) break;
            const Spinor<double> v = load_spinor<F64>(V + (long)(k0 + q) * vs, i, y.n);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                re[q] += v.c[c].re * yv.c[c].re + v.c[c].im * yv.c[c].im;
                im[q] += v.c[c].re * yv.c[c].im - v.c[c].im * yv.c[c].re;
            }
        }
    }
    __shared__ double lds[DT / 64];
    for (int q = 0; q < DKC; ++q) {
        if (k0 + q >= nvec) break;
        const double a = block_sum<DT>(re[q], lds);
        const double b = block_sum<DT>(im[q], lds);
        if (threadIdx.x == 0) {
            double *o = partial + (((long)sys * nvec + k0 + q) * nb + blockIdx.x) * 2;
            o[0] = a;
            o[1] = b;
        }
    }
}

// coef[sys * nvec + k] = (sum over the nb partials, in order) / lambda_k;
// zero for a system whose outer residual already meets its target
__global__ __launch_bounds__(64) void defl_coef_kernel(const double *__restrict__ partial, int nb, int nvec,
                                                       const double *__restrict__ inv_lambda,
                                                       const double *__restrict__ sc, double *__restrict__ coef)
{
    const int sys = blockIdx.x / nvec, k = blockIdx.x % nvec;
    const double *p = partial + ((long)sys * nvec + k) * nb * 2;
    double a = 0, b = 0;
    for (int j = threadIdx.x; j < nb; j += 64) {
        a += p[2 * j];
        b += p[2 * j + 1];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (threadIdx.x == 0) {
        const bool done = sc[(long)sys * NSC + SC_ODONE] != 0.0;
        coef[2 * blockIdx.x] = done ? 0.0 : a * inv_lambda[k];
        coef[2 * blockIdx.x + 1] = done ? 0.0 : b * inv_lambda[k];
    }
}

// e_sys = sum_k coef[sys][k] v_k (k in order) and x_sys += e_sys
__global__ __launch_bounds__(DT) void defl_axpy_kernel(const char *__restrict__ V, long vs, int nvec,
                                                       const double *__restrict__ coef, FieldView e, FieldView x)
{
    const long i = (long)blockIdx.x * DT + threadIdx.x;
    const int sys = blockIdx.y;
    if (i >= e.n) return;
    Spinor<double> acc;
#pragma unroll
    for (int c = 0; c < 12; ++c) acc.c[c] = cx<double>{0.0, 0.0};
    const double *cf = coef + (long)sys * nvec * 2;
    for (int k = 0; k < nvec; ++k) {
        const Spinor<double> v = load_spinor<F64>(V + (long)k * vs, i, e.n);
        const double cr = cf[2 * k], ci = cf[2 * k + 1];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            acc.c[c].re += cr * v.c[c].re - ci * v.c[c].im;
            acc.c[c].im += cr * v.c[c].im + ci * v.c[c].re;
        }
    }
    store_spinor<F64>(e.base + (long)sys * e.rs, i, e.n, acc);
    char *xs = x.base + (long)sys * x.rs;
    Spinor<double> xv = load_spinor<F64>(xs, i, x.n);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        xv.c[c].re += acc.c[c].re;
        xv.c[c].im += acc.c[c].im;
    }
    store_spinor<F64>(xs, i, x.n, xv);
}

// r -= t and the partial |r|^2 of each workgroup (the layout of the
// vector kernels' reductions: one per 256 sites, slice by slice)
__global__ __launch_bounds__(DT) void defl_sub_norm_kernel(FieldView r, FieldView t, double *__restrict__ partial)
{
    const long i = (long)blockIdx.x * DT + threadIdx.x;
    const int sys = blockIdx.y;
    double a = 0;
    if (i < r.n) {
        char *rs = r.base + (long)sys * r.rs;
        Spinor<double> rv = load_spinor<F64>(rs, i, r.n);
        const Spinor<double> tv = load_spinor<F64>(t.base + (long)sys * t.rs, i, t.n);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            rv.c[c].re -= tv.c[c].re;
            rv.c[c].im -= tv.c[c].im;
            a += rv.c[c].re * rv.c[c].re + rv.c[c].im * rv.c[c].im;
        }
        store_spinor<F64>(rs, i, r.n, rv);
    }
    __shared__ double lds[DT / 64];
    const double s = block_sum<DT>(a, lds);
    if (threadIdx.x == 0) partial[(long)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

}  // namespace

void deflate_residual(SolveCtx &c, bool normal)
{
    lq_op *op = c.op;
    const Geom &g = op->g;
    const int nvec = op->defl_n, nsys = c.nsys;
    const long vs = fb(F64, g);
    const int nb = dot_blocks(g.vh);
    op->defl_part.ensure(sizeof(double) * 2 * ((size_t)nsys * nvec * nb + (size_t)nsys * nvec));
    double *part = reinterpret_cast<double *>(op->defl_part.ptr);
    double *coef = part + 2 * (size_t)nsys * nvec * nb;
    const char *V = op->defl_vecs.ptr;
    const double *inv_lambda = reinterpret_cast<const double *>(op->defl_vecs.ptr + (size_t)nvec * vs);
    // y = M^dag r (t64), or r itself for the normal equations
    FieldView y = c.r64;
    if (!normal) {
        c.apply(c.t64, c.r64, true);
        y = c.t64;
    }
    defl_dot_kernel<<<dim3(nb, nsys, (nvec + DKC - 1) / DKC), DT, 0, c.s>>>(V, vs, nvec, y, part);
    LQ_HIP(hipGetLastError());
    defl_coef_kernel<<<nsys * nvec, 64, 0, c.s>>>(part, nb, nvec, inv_lambda, c.sc, coef);
    LQ_HIP(hipGetLastError());
    // e (y64) = sum_k c_k v_k, x += e
    const dim3 grid((unsigned)((g.vh + DT - 1) / DT), (unsigned)nsys);
    defl_axpy_kernel<<<grid, DT, 0, c.s>>>(V, vs, nvec, coef, c.y64, c.x64);
    LQ_HIP(hipGetLastError());
    // r -= M e (t64), or M^dag M e (M e in t64, then M^dag of it in y64)
    c.apply(c.t64, c.y64, false);
    FieldView t = c.t64;
    if (normal) {
        c.apply(c.y64, c.t64, true);
        t = c.y64;
    }
    defl_sub_norm_kernel<<<grid, DT, 0, c.s>>>(c.r64, t, c.partial);
    LQ_HIP(hipGetLastError());
    LQ_HIP(launch_finish(c.partial, nsys, 1, (int)grid.x, 1, FIN_NORM, c.sc, 1e-30, c.s));
}

}  // namespace lq

using namespace lq;

extern "C" lq_status lq_op_set_deflation(lq_op *op, int nvec, const double *evals, const void *evecs, void *stream)
{
    if (!op) {
        set_error("lq_op_set_deflation: null operator");
        return LQ_ERR_ARG;
    }
    if (nvec == 0) {
        set_error("");
        op->defl_n = 0;
        return LQ_OK;
    }
    if (nvec < 0 || nvec > 1024 || !evals || !evecs) {
        set_error("lq_op_set_deflation: nvec outside [0, 1024] or a null array");
        return LQ_ERR_ARG;
    }
    for (int k = 0; k < nvec; ++k)
        if (!(evals[k] > 0) || !std::isfinite(evals[k])) {
            set_error("lq_op_set_deflation: eigenvalues must be finite and positive");
            return LQ_ERR_ARG;
        }
    if (!op->gauge_set) {
        set_error("lq_op_set_deflation: gauge field not set");
        return LQ_ERR_STATE;
    }
    if (op->bound_nrhs > 0) {
        set_error("lq_op_set_deflation: the deflation space needs device memory of its own, and the operator is "
                  "bound to a caller's workspace");
        return LQ_ERR_STATE;
    }
    try {
        set_error("");
        LQ_HIP(hipSetDevice(op->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const Geom &g = op->g;
        const long vs = fb(F64, g);
        op->defl_n = 0;
        // nvec packed FP64 parity fields, then 1 / lambda_k
        op->defl_vecs.ensure((size_t)nvec * vs + sizeof(double) * nvec);
        LQ_HIP(launch_pack_spinor(g, 0, 1, static_cast<const double *>(evecs),
                                  FieldView{op->defl_vecs.ptr, F64, (long)g.vh, vs, nvec}, s));
        std::vector<double> inv(nvec);
        for (int k = 0; k < nvec; ++k) inv[k] = 1.0 / evals[k];
        LQ_HIP(hipMemcpyAsync(op->defl_vecs.ptr + (size_t)nvec * vs, inv.data(), sizeof(double) * nvec,
                              hipMemcpyHostToDevice, s));
        LQ_HIP(hipStreamSynchronize(s));
        op->defl_n = nvec;
        return LQ_OK;
    } catch (const Failure &f) {
        set_error(f.msg);
        return f.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return LQ_ERR_STATE;
    }
}
