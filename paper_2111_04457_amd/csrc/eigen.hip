// eigen.hip -- lowest eigenpairs of the Hermitian positive even-odd normal
// operator M^dag M (M the Schur operator of eq. (1) on the even sites), the
// kind of eigenvalue solver the paper's conclusion lists among the
// framework's algorithms.
//
// Lanczos with full reorthogonalisation, in FP64: from a start vector v_1
// the three-term recurrence w = A v_j - alpha_j v_j - beta_{j-1} v_{j-1},
// with w made orthogonal to every earlier v_i twice (classical Gram-Schmidt
// repeated), builds an orthonormal Krylov basis V_m and the tridiagonal
// T_m = V_m^dag A V_m.  The Ritz pairs of T_m (implicit QR on the host)
// give the approximations theta_k, x_k = V_m y_k; each is checked with its
// true residual |A x_k - theta_k x_k| computed on the GPU.  The basis lives
// on the device in the boundary layout ([V/2][4][3] complex128, contiguous)
// so that the dot products and updates are plain vector kernels; every
// apply packs, applies and unpacks.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "solver.h"

namespace lq {

// per-wavefront partial sums of x^dag y (re, im) over n complex entries
__global__ __launch_bounds__(256) void cdot_kernel(const double *x, const double *y, long n, double *partial)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    double re = 0.0, im = 0.0;
    if (i < n) {
        const double xr = x[2 * i], xi = x[2 * i + 1], yr = y[2 * i], yi = y[2 * i + 1];
        re = xr * yr + xi * yi;
        im = xr * yi - xi * yr;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if ((threadIdx.x & 63) == 0 && i < n) {
        partial[2 * (i >> 6)] = re;
        partial[2 * (i >> 6) + 1] = im;
    }
}

// y <- y + (a_re + i a_im) x over n complex entries
__global__ __launch_bounds__(256) void caxpy_kernel(double *y, const double *x, double ar, double ai, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double xr = x[2 * i], xi = x[2 * i + 1];
    y[2 * i] = y[2 * i] + (ar * xr - ai * xi);
    y[2 * i + 1] = y[2 * i + 1] + (ar * xi + ai * xr);
}

// partial[(i * nw + wave) * 2 + {0,1}] = wavefront sums of V_i^dag w (grid.y = i)
__global__ __launch_bounds__(256) void mdot_kernel(const double *V, const double *w, long n, double *partial)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    const long nw = (n + 63) / 64;
    const double *x = V + (long)blockIdx.y * 2 * n;
    double re = 0.0, im = 0.0;
    if (i < n) {
        const double xr = x[2 * i], xi = x[2 * i + 1], yr = w[2 * i], yi = w[2 * i + 1];
        re = xr * yr + xi * yi;
        im = xr * yi - xi * yr;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if ((threadIdx.x & 63) == 0 && i < n) {
        double *o = partial + ((long)blockIdx.y * nw + (i >> 6)) * 2;
        o[0] = re;
        o[1] = im;
    }
}

// c[i] = sum over the nw partials of vector i, in order (one thread per i)
__global__ __launch_bounds__(64) void msum_kernel(const double *partial, long nw, int k, double *c)
{
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= k) return;
    double re = 0.0, im = 0.0;
    for (long wv = 0; wv < nw; ++wv) {
        re += partial[((long)i * nw + wv) * 2];
        im += partial[((long)i * nw + wv) * 2 + 1];
    }
    c[2 * i] = re;
    c[2 * i + 1] = im;
}

// w <- w - sum_i c_i V_i over the first k vectors
__global__ __launch_bounds__(256) void maxpy_kernel(double *w, const double *V, const double *c, int k, long n)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    double re = w[2 * e], im = w[2 * e + 1];
    for (int i = 0; i < k; ++i) {
        const double cr = c[2 * i], ci = c[2 * i + 1];
        const double xr = V[(long)i * 2 * n + 2 * e], xi = V[(long)i * 2 * n + 2 * e + 1];
        re -= cr * xr - ci * xi;
        im -= cr * xi + ci * xr;
    }
    w[2 * e] = re;
    w[2 * e + 1] = im;
}

// y <- a x (real a)
__global__ __launch_bounds__(256) void rscale_kernel(double *y, const double *x, double a, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < 2 * n) y[i] = a * x[i];
}

namespace {

struct Vec {
    lq_op *op;
    hipStream_t s;
    long n;        // complex entries of one vector
    double *part;  // partial sums
    std::vector<double> host;

    unsigned blocks() const { return (unsigned)((n + 255) / 256); }
    // x^dag y, summed on the host in a fixed order
    void dot(const double *x, const double *y, double &re, double &im)
    {
        cdot_kernel<<<blocks(), 256, 0, s>>>(x, y, n, part);
        LQ_HIP(hipGetLastError());
        const long nw = (n + 63) / 64;
        host.resize(2 * (size_t)nw);
        LQ_HIP(hipMemcpyAsync(host.data(), part, sizeof(double) * 2 * nw, hipMemcpyDeviceToHost, s));
        LQ_HIP(hipStreamSynchronize(s));
        re = im = 0.0;
        for (long w = 0; w < nw; ++w) {
            re += host[2 * w];
            im += host[2 * w + 1];
        }
    }
    double norm(const double *x)
    {
        double re, im;
        dot(x, x, re, im);
        return std::sqrt(std::max(re, 0.0));
    }
    void axpy(double *y, const double *x, double ar, double ai)
    {
        caxpy_kernel<<<blocks(), 256, 0, s>>>(y, x, ar, ai, n);
        LQ_HIP(hipGetLastError());
    }
    // w <- w - V_k (V_k^dag w) for the first k basis vectors (classical
    // Gram-Schmidt: all coefficients from one pass over the basis)
    void project_out(double *w, const double *V, int k, double *mpart, double *c)
    {
        const long nw = (n + 63) / 64;
        mdot_kernel<<<dim3(blocks(), (unsigned)k), 256, 0, s>>>(V, w, n, mpart);
        LQ_HIP(hipGetLastError());
        msum_kernel<<<(unsigned)((k + 63) / 64), 64, 0, s>>>(mpart, nw, k, c);
        LQ_HIP(hipGetLastError());
        maxpy_kernel<<<blocks(), 256, 0, s>>>(w, V, c, k, n);
        LQ_HIP(hipGetLastError());
    }
    void scale(double *y, const double *x, double a)
    {
        rscale_kernel<<<(unsigned)((2 * n + 255) / 256), 256, 0, s>>>(y, x, a, n);
        LQ_HIP(hipGetLastError());
    }
};

// out = M^dag M in (boundary-layout even fields), through the packed scratch fields
void apply_normal(lq_op *op, double *out, const double *in, char *pin, char *pout, hipStream_t s)
{
    const Geom &g = op->g;
    LQ_HIP(launch_pack_spinor(g, 0, 1, in, parity_view(pin, F64, g, 1), s));
    apply_packed(op, LQ_SCHUR_NORMAL, F64, pout, pin, 1, s);
    LQ_HIP(launch_unpack_spinor(g, 0, 1, parity_view(pout, F64, g, 1), out, s));
}

// Eigenpairs of the symmetric tridiagonal T (diagonal alpha, off-diagonal
// beta) by implicitly shifted QR: Wilkinson shift from the trailing 2 x 2 of
// the active block, the bulge chased down by Givens rotations applied as
// similarities (only the few entries of the band they touch), negligible
// off-diagonals deflated.  The rotations accumulate into Z, whose columns
// are the eigenvectors; eigenvalues ascending in w.
void tridiag_eig(const std::vector<double> &alpha, const std::vector<double> &beta, std::vector<double> &w,
                 std::vector<double> &Z)
{
    const int m = (int)alpha.size();
    std::vector<double> A((size_t)m * m, 0.0);
    auto a = [&](int i, int j) -> double & { return A[(size_t)i * m + j]; };
    Z.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) {
        a(i, i) = alpha[i];
        if (i + 1 < m) a(i, i + 1) = a(i + 1, i) = beta[i];
        Z[(size_t)i * m + i] = 1.0;  // transposed while rotating: row k is eigenvector k
    }
    const double eps = std::numeric_limits<double>::epsilon();
    auto negligible = [&](int i) {  // the coupling of i - 1 and i
        return std::fabs(a(i, i - 1)) <= eps * (std::fabs(a(i, i)) + std::fabs(a(i - 1, i - 1)));
    };
    long steps = 0;
    int hi = m - 1;
    while (hi > 0) {
        if (negligible(hi)) {
            a(hi, hi - 1) = a(hi - 1, hi) = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && !negligible(lo)) --lo;
        if (lo > 0) a(lo, lo - 1) = a(lo - 1, lo) = 0.0;
        if (++steps > 30L * m) throw Failure{LQ_ERR_STATE, "tridiagonal QR did not converge"};
        // Wilkinson shift: the eigenvalue of the trailing 2 x 2 nearer its last entry
        const double d = 0.5 * (a(hi - 1, hi - 1) - a(hi, hi)), e = a(hi, hi - 1);
        const double mu = a(hi, hi) - e * e / (d + std::copysign(std::hypot(d, e), d));
        double x = a(lo, lo) - mu, z = a(lo + 1, lo);
        for (int k = lo; k < hi; ++k) {
            const double r = std::hypot(x, z);
            const double c = r > 0 ? x / r : 1.0, s = r > 0 ? z / r : 0.0;
            const int j0 = std::max(lo, k - 1), j1 = std::min(hi, k + 2);
            for (int j = j0; j <= j1; ++j) {  // rows k, k + 1
                const double u = a(k, j), v = a(k + 1, j);
                a(k, j) = c * u + s * v;
                a(k + 1, j) = c * v - s * u;
            }
            for (int j = j0; j <= j1; ++j) {  // columns k, k + 1
                const double u = a(j, k), v = a(j, k + 1);
                a(j, k) = c * u + s * v;
                a(j, k + 1) = c * v - s * u;
            }
            if (k > lo) a(k + 1, k - 1) = a(k - 1, k + 1) = 0.0;  // the bulge just chased out
            double *zk = &Z[(size_t)k * m], *zk1 = &Z[(size_t)(k + 1) * m];
            for (int i = 0; i < m; ++i) {
                const double u = zk[i], v = zk1[i];
                zk[i] = c * u + s * v;
                zk1[i] = c * v - s * u;
            }
            if (k + 2 <= hi) {
                x = a(k + 1, k);
                z = a(k + 2, k);
            }
        }
    }
    std::vector<int> idx(m);
    for (int i = 0; i < m; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int p, int q) { return a(p, p) < a(q, q); });
    std::vector<double> Zs((size_t)m * m);
    w.resize(m);
    for (int j = 0; j < m; ++j) {
        w[j] = a(idx[j], idx[j]);
        for (int i = 0; i < m; ++i) Zs[(size_t)i * m + j] = Z[(size_t)idx[j] * m + i];
    }
    Z.swap(Zs);
}

}  // namespace
}  // namespace lq

using namespace lq;

extern "C" lq_status lq_eigs(lq_op *op, int nev, int m, const void *v0, double *evals, double *resid, void *evecs,
                             int *nconv, double tol, void *stream)
{
    if (!op || !v0 || !evals || nev < 1 || m < nev + 1 || m > 1024 || !(tol > 0)) {
        set_error("lq_eigs: null argument, nev < 1, m outside [nev + 1, 1024] or tol <= 0");
        return LQ_ERR_ARG;
    }
    if (!op->gauge_set) {
        set_error("lq_eigs: gauge field not set");
        return LQ_ERR_STATE;
    }
    try {
        set_error("");
        LQ_HIP(hipSetDevice(op->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const Geom &g = op->g;
        const long n = 12L * g.vh;  // complex entries of an even field
        const size_t vbytes = sizeof(double) * 2 * (size_t)n;
        // basis (m + 1 vectors), a work vector, packed scratch, partial sums
        Buf basis, work, packed, part, mpart, coef;
        basis.ensure(vbytes * (size_t)(m + 1));
        work.ensure(vbytes);
        packed.ensure(2 * (size_t)fb(F64, g));
        part.ensure(sizeof(double) * 2 * (size_t)((n + 63) / 64));
        mpart.ensure(sizeof(double) * 2 * (size_t)((n + 63) / 64) * (size_t)m);
        coef.ensure(sizeof(double) * 2 * (size_t)m);
        auto V = [&](int j) { return reinterpret_cast<double *>(basis.ptr) + (size_t)j * 2 * n; };
        double *w = reinterpret_cast<double *>(work.ptr);
        char *pin = packed.ptr, *pout = packed.ptr + fb(F64, g);
        Vec vec{op, s, n, reinterpret_cast<double *>(part.ptr), {}};

        const double n0 = vec.norm(static_cast<const double *>(v0));
        if (!(n0 > 0) || !std::isfinite(n0)) throw Failure{LQ_ERR_ARG, "the start vector is zero or not finite"};
        vec.scale(V(0), static_cast<const double *>(v0), 1.0 / n0);
        std::vector<double> alpha, beta;
        int steps = 0;
        for (int j = 0; j < m; ++j) {
            apply_normal(op, w, V(j), pin, pout, s);
            double ar, ai;
            vec.dot(V(j), w, ar, ai);
            alpha.push_back(ar);
            vec.axpy(w, V(j), -ar, 0.0);
            if (j > 0) vec.axpy(w, V(j - 1), -beta[j - 1], 0.0);
            // full reorthogonalisation against v_0 .. v_j, twice
            for (int pass = 0; pass < 2; ++pass)
                vec.project_out(w, V(0), j + 1, reinterpret_cast<double *>(mpart.ptr),
                                reinterpret_cast<double *>(coef.ptr));
            const double b = vec.norm(w);
            steps = j + 1;
            if (j == m - 1 || !(b > 1e-14 * std::sqrt(std::fabs(ar) + 1e-300))) break;  // invariant subspace
            beta.push_back(b);
            vec.scale(V(j + 1), w, 1.0 / b);
        }
        alpha.resize(steps);
        beta.resize(std::max(0, steps - 1));
        std::vector<double> theta, Z;
        tridiag_eig(alpha, beta, theta, Z);
        const int k = std::min(nev, steps);
        int conv = 0;
        double *X = evecs ? static_cast<double *>(evecs) : nullptr;
        Buf xtmp;
        xtmp.ensure(vbytes);
        double *x = reinterpret_cast<double *>(xtmp.ptr);
        for (int e = 0; e < k; ++e) {
            // Ritz vector x = V y_e (into evecs[e] if given), its residual
            double *xe = X ? X + (size_t)e * 2 * n : x;
            vec.scale(xe, V(0), Z[(size_t)0 * steps + e]);
            for (int i = 1; i < steps; ++i) vec.axpy(xe, V(i), Z[(size_t)i * steps + e], 0.0);
            apply_normal(op, w, xe, pin, pout, s);
            vec.axpy(w, xe, -theta[e], 0.0);
            const double r = vec.norm(w) / vec.norm(xe);
            evals[e] = theta[e];
            if (resid) resid[e] = r;
            if (r <= tol * std::fabs(theta[e])) ++conv;
        }
        for (int e = k; e < nev; ++e) {
            evals[e] = NAN;
            if (resid) resid[e] = NAN;
        }
        LQ_HIP(hipStreamSynchronize(s));
        if (nconv) *nconv = conv;
        return conv == nev ? LQ_OK : LQ_NOT_CONVERGED;
    } catch (const Failure &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return LQ_ERR_STATE;
    }
}
