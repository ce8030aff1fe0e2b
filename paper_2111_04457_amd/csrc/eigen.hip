// eigen.hip -- lowest eigenpairs of the Hermitian positive even-odd normal
// operator A = M^dag M (M the Schur operator of eq. (1) on the even sites),
// the kind of eigenvalue solver the paper's conclusion lists among the
// framework's algorithms.
//
// Thick-restart Lanczos in FP64 on B = A, or on the Chebyshev filter
// B = T_d(L(A)) with L(A) = ((lo + hi) - 2A) / (hi - lo): T_d stays within
// [-1, 1] on [lo, hi] and grows like cosh(d arccosh L) below lo, so the
// lowest eigenvalues of A become the largest, well separated ones of B.
// Each cycle extends the basis to m vectors: w = B v_j, made orthogonal to
// every basis vector by classical Gram-Schmidt (coefficients from one pass
// over the basis), repeated once when the first pass cancelled most of w,
// the projections kept as column j of the projected matrix S = V^dag B V
// (real symmetric).  The Ritz pairs of S
// (Householder to tridiagonal form, implicitly shifted QR; on the host)
// give Ritz vectors x = V y, checked against A itself: the eigenvalue is
// the Rayleigh quotient x^dag A x, convergence its true residual.  A
// restart keeps the best k Ritz vectors and the last basis vector; their
// couplings to it come from the next column's projections.  The basis lives
// on the device in the boundary layout ([V/2][4][3] complex128); the filter
// recurrence runs on packed fields (one pack and unpack per B).
#include <algorithm>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "solver.h"

namespace lq {

// y <- y + (a_re + i a_im) x over n complex entries
__global__ __launch_bounds__(256) void caxpy_kernel(double *y, const double *x, double ar, double ai, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double xr = x[2 * i], xi = x[2 * i + 1];
    y[2 * i] = y[2 * i] + (ar * xr - ai * xi);
    y[2 * i + 1] = y[2 * i + 1] + (ar * xi + ai * xr);
}

// Workgroups per vector of the inner products: each sums a fixed strided
// subset of the entries, so the order of every sum is fixed.
constexpr int DOT_WG = 256;

// partial[(i * DOT_WG + b) * 2 + {0,1}] = workgroup b's share of V_i^dag w
// (grid (DOT_WG, k), block 256)
__global__ __launch_bounds__(256) void mdot_kernel(const double *V, const double *w, long n, double *partial)
{
    const double *x = V + (long)blockIdx.y * 2 * n;
    double re = 0.0, im = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)DOT_WG * 256) {
        const double xr = x[2 * i], xi = x[2 * i + 1], yr = w[2 * i], yi = w[2 * i + 1];
        re += xr * yr + xi * yi;
        im += xr * yi - xi * yr;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    __shared__ double lds[2][4];
    if ((threadIdx.x & 63) == 0) {
        lds[0][threadIdx.x >> 6] = re;
        lds[1][threadIdx.x >> 6] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *o = partial + ((long)blockIdx.y * DOT_WG + blockIdx.x) * 2;
        o[0] = (lds[0][0] + lds[0][1]) + (lds[0][2] + lds[0][3]);
        o[1] = (lds[1][0] + lds[1][1]) + (lds[1][2] + lds[1][3]);
    }
}

// c[i] = sum of the DOT_WG partials of vector i (one wavefront per i, grid
// k): each lane adds DOT_WG / 64 consecutive partials, then the fixed
// butterfly of wave_sum
__global__ __launch_bounds__(64) void msum_kernel(const double *partial, double *c)
{
    static_assert(DOT_WG % 64 == 0, "partials per lane");
    const int i = blockIdx.x;
    const double *p = partial + ((long)i * DOT_WG + threadIdx.x * (DOT_WG / 64)) * 2;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int b = 0; b < DOT_WG / 64; ++b) {
        re += p[2 * b];
        im += p[2 * b + 1];
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (threadIdx.x == 0) {
        c[2 * i] = re;
        c[2 * i + 1] = im;
    }
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

// out_i = sum_{j < m} Y[j * k + i] V_j for the 8 outputs i0 .. i0 + 7 of
// this grid row (i < k), real coefficients
__global__ __launch_bounds__(256) void combine_kernel(const double *V, long n, int m, const double *Y, int k,
                                                      double *out)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const int i0 = blockIdx.y * 8;
    double re[8], im[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) re[t] = im[t] = 0.0;
    for (int j = 0; j < m; ++j) {
        const double xr = V[(long)j * 2 * n + 2 * e], xi = V[(long)j * 2 * n + 2 * e + 1];
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (i0 + t < k) {
                const double y = Y[(long)j * k + i0 + t];
                re[t] += y * xr;
                im[t] += y * xi;
            }
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
        if (i0 + t < k) {
            out[(long)(i0 + t) * 2 * n + 2 * e] = re[t];
            out[(long)(i0 + t) * 2 * n + 2 * e + 1] = im[t];
        }
}

// y <- a x (real a)
__global__ __launch_bounds__(256) void rscale_kernel(double *y, const double *x, double a, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < 2 * n) y[i] = a * x[i];
}

// one step of the Chebyshev recurrence on nd doubles of packed fields:
// out = cy y + ca (A y) + cp yprev (yprev may be null)
__global__ __launch_bounds__(256) void cheb_kernel(double *out, const double *ay, const double *y,
                                                   const double *yprev, double cy, double ca, double cp, long nd)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= nd) return;
    double v = cy * y[i] + ca * ay[i];
    if (yprev) v += cp * yprev[i];
    out[i] = v;
}

namespace {

struct Vec {
    hipStream_t s;
    long n;        // complex entries of one vector
    double *part;  // partial sums (DOT_WG per vector) and, after them, one result
    double *hres;  // pinned host copy of a result

    unsigned blocks() const { return (unsigned)((n + 255) / 256); }
    // x^dag y
    void dot(const double *x, const double *y, double &re, double &im)
    {
        double *c = part + 2 * DOT_WG;
        mdot_kernel<<<dim3(DOT_WG, 1), 256, 0, s>>>(x, y, n, part);
        LQ_HIP(hipGetLastError());
        msum_kernel<<<1, 64, 0, s>>>(part, c);
        LQ_HIP(hipGetLastError());
        LQ_HIP(hipMemcpyAsync(hres, c, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        LQ_HIP(hipStreamSynchronize(s));
        re = hres[0];
        im = hres[1];
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
    // w <- w - V_k c with c = V_k^dag w (stored at c, device) for the first k
    // basis vectors: one classical Gram-Schmidt pass
    void project_out(double *w, const double *V, int k, double *mpart, double *c)
    {
        mdot_kernel<<<dim3(DOT_WG, (unsigned)k), 256, 0, s>>>(V, w, n, mpart);
        LQ_HIP(hipGetLastError());
        msum_kernel<<<(unsigned)k, 64, 0, s>>>(mpart, c);
        LQ_HIP(hipGetLastError());
        maxpy_kernel<<<blocks(), 256, 0, s>>>(w, V, c, k, n);
        LQ_HIP(hipGetLastError());
    }
    // c <- c + d over k complex entries
    void accumulate(double *c, const double *dd, int k)
    {
        caxpy_kernel<<<(unsigned)((k + 255) / 256), 256, 0, s>>>(c, dd, 1.0, 0.0, k);
        LQ_HIP(hipGetLastError());
    }
    void scale(double *y, const double *x, double a)
    {
        rscale_kernel<<<(unsigned)((2 * n + 255) / 256), 256, 0, s>>>(y, x, a, n);
        LQ_HIP(hipGetLastError());
    }
    // out_i = V_m Y[:, i] for i < k (Y device, m x k row-major)
    void combine(double *out, const double *V, int m, const double *Y, int k)
    {
        combine_kernel<<<dim3(blocks(), (unsigned)((k + 7) / 8)), 256, 0, s>>>(V, n, m, Y, k, out);
        LQ_HIP(hipGetLastError());
    }
};

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


// Eigenpairs of the real symmetric S (m x m, row-major): Householder
// reduction to tridiagonal form S = Q T Q^T, then tridiag_eig on T;
// eigenvalues ascending in w, eigenvectors in the columns of Z = Q Z_T.
void sym_eig(std::vector<double> S, int m, std::vector<double> &w, std::vector<double> &Z)
{
    auto s = [&](int i, int j) -> double & { return S[(size_t)i * m + j]; };
    std::vector<double> Q((size_t)m * m, 0.0), v(m), p(m);
    for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
    for (int k = 0; k + 2 < m; ++k) {
        // reflector P = 1 - tau v v^T with P x = -sign(x_0) |x| e_0, x = S[k+1.., k]
        double xn = 0.0;
        for (int i = k + 1; i < m; ++i) xn += s(i, k) * s(i, k);
        xn = std::sqrt(xn);
        if (xn == 0.0) continue;
        const double x0 = s(k + 1, k), alpha = x0 >= 0 ? -xn : xn;
        for (int i = k + 1; i < m; ++i) v[i] = s(i, k);
        v[k + 1] = x0 - alpha;
        double vn = 0.0;
        for (int i = k + 1; i < m; ++i) vn += v[i] * v[i];
        if (vn == 0.0) continue;
        const double tau = 2.0 / vn;
        // S <- P S P on rows / columns k .. m-1: with p = tau S v and
        // q = p - (tau / 2)(p^T v) v, S <- S - v q^T - q v^T
        for (int i = k; i < m; ++i) {
            double t = 0.0;
            for (int j = k + 1; j < m; ++j) t += s(i, j) * v[j];
            p[i] = tau * t;
        }
        double pv = 0.0;
        for (int i = k + 1; i < m; ++i) pv += p[i] * v[i];
        for (int i = k + 1; i < m; ++i) p[i] -= 0.5 * tau * pv * v[i];
        // column / row k: only the entries k+1.. change, to (alpha, 0, ...)
        s(k + 1, k) = s(k, k + 1) = alpha;
        for (int i = k + 2; i < m; ++i) s(i, k) = s(k, i) = 0.0;
        for (int i = k + 1; i < m; ++i)
            for (int j = k + 1; j < m; ++j) s(i, j) -= v[i] * p[j] + p[i] * v[j];
        // Q <- Q P
        for (int i = 0; i < m; ++i) {
            double t = 0.0;
            for (int j = k + 1; j < m; ++j) t += Q[(size_t)i * m + j] * v[j];
            t *= tau;
            for (int j = k + 1; j < m; ++j) Q[(size_t)i * m + j] -= t * v[j];
        }
    }
    std::vector<double> alpha(m), beta(m > 0 ? m - 1 : 0), Zt;
    for (int i = 0; i < m; ++i) {
        alpha[i] = s(i, i);
        if (i + 1 < m) beta[i] = 0.5 * (s(i + 1, i) + s(i, i + 1));
    }
    tridiag_eig(alpha, beta, w, Zt);
    Z.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i)
        for (int l = 0; l < m; ++l) {
            const double q = Q[(size_t)i * m + l];
            if (q == 0.0) continue;
            for (int j = 0; j < m; ++j) Z[(size_t)i * m + j] += q * Zt[(size_t)l * m + j];
        }
}

// The thick-restart Lanczos run of one lq_eigs call.
struct Lanczos {
    lq_op *op;
    hipStream_t s;
    Vec vec;
    long n;
    int m;
    // the workspace stays with the operator (grown as needed, reused by the
    // next call)
    Buf &basis, &ritz, &work, &packed, &part, &mpart, &coef, &ydev;
    double *hres = nullptr;
    long applies = 0;  // applications of A

    double *V(int j) { return reinterpret_cast<double *>(basis.ptr) + (size_t)j * 2 * n; }
    double *X(int i) { return reinterpret_cast<double *>(ritz.ptr) + (size_t)i * 2 * n; }
    double *P(int i) { return reinterpret_cast<double *>(packed.ptr + (size_t)i * fb(F64, op->g)); }

    Lanczos(lq_op *o, hipStream_t st, int m_)
        : op(o), s(st), n(12L * o->g.vh), m(m_), basis(o->eig_ws[0]), ritz(o->eig_ws[1]), work(o->eig_ws[2]),
          packed(o->eig_ws[3]), part(o->eig_ws[4]), mpart(o->eig_ws[5]), coef(o->eig_ws[6]), ydev(o->eig_ws[7])
    {
        const size_t vbytes = sizeof(double) * 2 * (size_t)n;
        basis.ensure(vbytes * (size_t)(m + 1));
        ritz.ensure(vbytes * (size_t)m);
        work.ensure(vbytes);
        packed.ensure(4 * (size_t)fb(F64, op->g));
        LQ_HIP(hipMemsetAsync(packed.ptr, 0, 4 * (size_t)fb(F64, op->g), s));
        part.ensure(sizeof(double) * 2 * (DOT_WG + 1));
        mpart.ensure(sizeof(double) * 2 * DOT_WG * (size_t)m);
        coef.ensure(sizeof(double) * 2 * 2 * (size_t)m * (size_t)(m + 1));
        ydev.ensure(sizeof(double) * (size_t)m * (size_t)m);
        if (!op->eig_host)
            LQ_HIP(hipHostMalloc(reinterpret_cast<void **>(&op->eig_host), 2 * sizeof(double), hipHostMallocDefault));
        hres = op->eig_host;
        vec = Vec{s, n, reinterpret_cast<double *>(part.ptr), hres};
    }
    Lanczos(const Lanczos &) = delete;
    Lanczos &operator=(const Lanczos &) = delete;

    // packed out = A packed in
    void apply_A_packed(char *out, const char *in)
    {
        apply_packed(op, LQ_SCHUR_NORMAL, F64, out, in, 1, s);
        ++applies;
    }
    // out = A in on boundary-layout vectors
    void apply_A(double *out, const double *in)
    {
        const Geom &g = op->g;
        LQ_HIP(launch_pack_spinor(g, 0, 1, in, parity_view(reinterpret_cast<char *>(P(0)), F64, g, 1), s));
        apply_A_packed(reinterpret_cast<char *>(P(1)), reinterpret_cast<char *>(P(0)));
        LQ_HIP(launch_unpack_spinor(g, 0, 1, parity_view(reinterpret_cast<char *>(P(1)), F64, g, 1), out, s));
    }
    // out = T_d(L(A)) in (d = 0: A in) on boundary-layout vectors
    void apply_B(double *out, const double *in, int d, double lo, double hi)
    {
        if (d == 0) return apply_A(out, in);
        const Geom &g = op->g;
        const long nd = (long)(fb(F64, g) / sizeof(double));
        const unsigned nb = (unsigned)((nd + 255) / 256);
        // L y = c0 y + c1 A y;  T_1 = L T_0, T_{k+1} = 2 L T_k - T_{k-1}
        const double c0 = (lo + hi) / (hi - lo), c1 = -2.0 / (hi - lo);
        int prev = 0, cur = 1, nxt = 2;
        const int ay = 3;
        LQ_HIP(launch_pack_spinor(g, 0, 1, in, parity_view(reinterpret_cast<char *>(P(prev)), F64, g, 1), s));
        apply_A_packed(reinterpret_cast<char *>(P(ay)), reinterpret_cast<char *>(P(prev)));
        cheb_kernel<<<nb, 256, 0, s>>>(P(cur), P(ay), P(prev), nullptr, c0, c1, 0.0, nd);
        LQ_HIP(hipGetLastError());
        for (int k = 1; k < d; ++k) {
            apply_A_packed(reinterpret_cast<char *>(P(ay)), reinterpret_cast<char *>(P(cur)));
            cheb_kernel<<<nb, 256, 0, s>>>(P(nxt), P(ay), P(cur), P(prev), 2.0 * c0, 2.0 * c1, -1.0, nd);
            LQ_HIP(hipGetLastError());
            const int t = prev;
            prev = cur;
            cur = nxt;
            nxt = t;
        }
        LQ_HIP(launch_unpack_spinor(g, 0, 1, parity_view(reinterpret_cast<char *>(P(cur)), F64, g, 1), out, s));
    }

    struct Cycle {
        int meff = 0;          // basis vectors of the cycle
        double beta_last = 0;  // coupling of the last Ritz components to v_meff
        bool invariant = false;
        std::vector<double> theta, Z;  // Ritz values (ascending) and vectors of S
    };

    // Extend the basis from k kept vectors (S holding their Ritz values on
    // its diagonal) to m vectors and diagonalise the projected matrix.
    Cycle extend(int k, std::vector<double> &S, int d, double lo, double hi)
    {
        double *w = reinterpret_cast<double *>(work.ptr);
        double *C = reinterpret_cast<double *>(coef.ptr);
        Cycle cy;
        int j = k;
        for (; j < m; ++j) {
            apply_B(w, V(j), d, lo, hi);
            // the recurrence: w loses its components along the vectors it
            // couples to in exact arithmetic (v_{j-1} and v_j; after a
            // restart, every kept vector); then one Gram-Schmidt pass over
            // the whole basis removes what rounding left, repeated only if
            // that pass cancelled most of w (|w| below 1/sqrt 2 of before)
            double *C0 = C + (size_t)j * 2 * (m + 1), *C1 = C + ((size_t)m + j) * 2 * (m + 1);
            double *mp = reinterpret_cast<double *>(mpart.ptr);
            const int first = j == k ? 0 : j - 1;
            const double bB = vec.norm(w);
            LQ_HIP(hipMemsetAsync(C0, 0, sizeof(double) * 2 * (j + 1), s));
            vec.project_out(w, V(first), j + 1 - first, mp, C0 + 2 * first);
            const double bw = vec.norm(w);
            vec.project_out(w, V(0), j + 1, mp, C1);
            double b = vec.norm(w);
            if (b < 0.7071067811865476 * bw) {
                // the third pass accumulates into the local coefficients
                double *C2 = reinterpret_cast<double *>(ydev.ptr);
                vec.project_out(w, V(0), j + 1, mp, C2);
                vec.accumulate(C0, C2, j + 1);
                b = vec.norm(w);
            }
            cy.beta_last = b;
            if (!(b > 1e-14 * bB)) {  // B v_j lies in the basis: an invariant subspace
                cy.invariant = true;
                ++j;
                break;
            }
            vec.scale(V(j + 1), w, 1.0 / b);
        }
        cy.meff = j;
        // columns k .. meff-1 of S from the two passes' coefficients
        std::vector<double> hc(2 * 2 * (size_t)m * (m + 1));
        LQ_HIP(hipMemcpyAsync(hc.data(), C, sizeof(double) * hc.size(), hipMemcpyDeviceToHost, s));
        LQ_HIP(hipStreamSynchronize(s));
        for (int c = k; c < cy.meff; ++c)
            for (int i = 0; i <= c; ++i) {
                const double v = hc[((size_t)0 * m + c) * 2 * (m + 1) + 2 * i] +
                                 hc[((size_t)1 * m + c) * 2 * (m + 1) + 2 * i];
                S[(size_t)i * m + c] = S[(size_t)c * m + i] = v;
            }
        std::vector<double> Sm((size_t)cy.meff * cy.meff);
        for (int i = 0; i < cy.meff; ++i)
            for (int c = 0; c < cy.meff; ++c) Sm[(size_t)i * cy.meff + c] = S[(size_t)i * m + c];
        sym_eig(Sm, cy.meff, cy.theta, cy.Z);
        if (cy.invariant) cy.beta_last = 0.0;
        return cy;
    }

    // Ritz vectors X_i = V Z[:, sel[i]] for i < cnt (into X or dst)
    void ritz_vectors(const Cycle &cy, const std::vector<int> &sel, int cnt, double *dst)
    {
        std::vector<double> Y((size_t)cy.meff * cnt);
        for (int j = 0; j < cy.meff; ++j)
            for (int i = 0; i < cnt; ++i) Y[(size_t)j * cnt + i] = cy.Z[(size_t)j * cy.meff + sel[i]];
        LQ_HIP(hipMemcpyAsync(ydev.ptr, Y.data(), sizeof(double) * Y.size(), hipMemcpyHostToDevice, s));
        vec.combine(dst, V(0), cy.meff, reinterpret_cast<double *>(ydev.ptr), cnt);
        LQ_HIP(hipStreamSynchronize(s));  // Y is a host temporary
    }
};

}  // namespace
}  // namespace lq

using namespace lq;

extern "C" void lq_eig_params_default(lq_eig_params *p)
{
    if (!p) return;
    p->nev = 8;
    p->m = 64;
    p->max_restarts = 100;
    p->cheb_degree = 8;
    p->cheb_lo = 0.0;
    p->cheb_hi = 0.0;
    p->tol = 1e-8;
}

extern "C" lq_status lq_eigs(lq_op *op, const lq_eig_params *prm, const void *v0, double *evals, double *resid,
                             void *evecs, lq_eig_stats *stats, void *stream)
{
    if (!op || !prm || !v0 || !evals) {
        set_error("lq_eigs: null argument");
        return LQ_ERR_ARG;
    }
    const int nev = prm->nev, m = prm->m, d = prm->cheb_degree;
    if (nev < 1 || m < nev + 1 || m > 1024 || prm->max_restarts < 0 || d < 0 || d > 10000 || !(prm->tol > 0) ||
        !std::isfinite(prm->cheb_lo) || !std::isfinite(prm->cheb_hi) || prm->cheb_lo < 0 ||
        (prm->cheb_hi > 0 && !(prm->cheb_hi > prm->cheb_lo))) {
        set_error("lq_eigs: nev < 1, m outside [nev + 1, 1024], max_restarts < 0, cheb_degree outside [0, 10000], "
                  "tol <= 0, or a filter interval with lo < 0 or hi <= lo");
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
        Lanczos lz(op, s, m);
        const double n0 = lz.vec.norm(static_cast<const double *>(v0));
        if (!(n0 > 0) || !std::isfinite(n0)) throw Failure{LQ_ERR_ARG, "the start vector is zero or not finite"};
        double lo = prm->cheb_lo, hi = prm->cheb_hi;
        if (d > 0 && (lo <= 0 || hi <= 0)) {
            // filter interval from one plain Lanczos cycle: hi above the
            // largest Ritz value by its residual bound, lo the (nev+1)-th
            // smallest Ritz value (not below the (nev+1)-th eigenvalue)
            std::vector<double> S((size_t)m * m, 0.0);
            lz.vec.scale(lz.V(0), static_cast<const double *>(v0), 1.0 / n0);
            auto cy = lz.extend(0, S, 0, 0.0, 0.0);
            const int top = cy.meff - 1;
            const double rtop = std::fabs(cy.beta_last * cy.Z[(size_t)(cy.meff - 1) * cy.meff + top]);
            if (hi <= 0) hi = 1.01 * (cy.theta[top] + rtop);
            if (lo <= 0) lo = cy.theta[std::min(nev, cy.meff - 1)];
            if (!(hi > lo) || !(lo > 0)) throw Failure{LQ_ERR_STATE, "could not bracket the spectrum for the filter"};
        }
        std::vector<double> S((size_t)m * m, 0.0);
        lz.vec.scale(lz.V(0), static_cast<const double *>(v0), 1.0 / n0);
        double *w = reinterpret_cast<double *>(lz.work.ptr);
        if (d > 0 && d * std::acosh((hi + lo) / (hi - lo)) > 600.0)
            throw Failure{LQ_ERR_ARG, "cheb_degree too high for the filter interval: T_d(L(0)) would overflow"};
        int k = 0, restarts = 0, conv = 0, cnt = 0;
        std::vector<double> lam(nev, NAN), res(nev, NAN);
        std::vector<int> order;
        for (;;) {
            auto cy = lz.extend(k, S, d, lo, hi);
            // the wanted end of B's spectrum first: the smallest of A, the largest of T_d(L(A))
            order.resize(cy.meff);
            for (int i = 0; i < cy.meff; ++i) order[i] = d == 0 ? i : cy.meff - 1 - i;
            cnt = std::min(nev, cy.meff);
            lz.ritz_vectors(cy, order, cnt, lz.X(0));
            // true eigenvalue (Rayleigh quotient of A) and residual of each
            conv = 0;
            for (int i = 0; i < cnt; ++i) {
                lz.apply_A(w, lz.X(i));
                double xr, xi, ar, ai;
                lz.vec.dot(lz.X(i), lz.X(i), xr, xi);
                lz.vec.dot(lz.X(i), w, ar, ai);
                lam[i] = ar / xr;
                lz.vec.axpy(w, lz.X(i), -lam[i], 0.0);
                res[i] = lz.vec.norm(w) / std::sqrt(xr);
                // with the filter, a pair above lo is not one of the wanted
                // (lowest) ones: an eigenvalue above hi that T_d amplified
                if (res[i] <= prm->tol * std::fabs(lam[i]) && (d == 0 || lam[i] <= lo)) ++conv;
            }
            if (conv == nev || cy.invariant || restarts >= prm->max_restarts || cy.meff < m) break;
            // thick restart: keep kk Ritz vectors of B and v_m
            const int kk = std::min(m - 1, nev + (m - nev) / 2);
            lz.ritz_vectors(cy, order, kk, lz.X(0));
            LQ_HIP(hipMemcpyAsync(lz.V(kk), lz.V(cy.meff), sizeof(double) * 2 * lz.n, hipMemcpyDeviceToDevice, s));
            LQ_HIP(hipMemcpyAsync(lz.V(0), lz.X(0), sizeof(double) * 2 * lz.n * kk, hipMemcpyDeviceToDevice, s));
            std::fill(S.begin(), S.end(), 0.0);
            for (int i = 0; i < kk; ++i) S[(size_t)i * m + i] = cy.theta[order[i]];
            k = kk;
            ++restarts;
        }
        // the nev pairs ascending in the eigenvalue of A
        std::vector<int> idx(nev);
        for (int i = 0; i < nev; ++i) idx[i] = i;
        std::stable_sort(idx.begin(), idx.begin() + cnt, [&](int a, int b) { return lam[a] < lam[b]; });
        for (int i = 0; i < nev; ++i) {
            evals[i] = lam[idx[i]];
            if (resid) resid[i] = res[idx[i]];
            if (evecs && i < cnt)
                LQ_HIP(hipMemcpyAsync(static_cast<double *>(evecs) + (size_t)i * 2 * lz.n, lz.X(idx[i]),
                                      sizeof(double) * 2 * lz.n, hipMemcpyDeviceToDevice, s));
        }
        LQ_HIP(hipStreamSynchronize(s));
        if (stats) {
            stats->nconv = conv;
            stats->restarts = restarts;
            stats->applies = lz.applies;
            stats->cheb_lo = d > 0 ? lo : 0.0;
            stats->cheb_hi = d > 0 ? hi : 0.0;
        }
        return conv == nev ? LQ_OK : LQ_NOT_CONVERGED;
    } catch (const Failure &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return LQ_ERR_STATE;
    }
}

extern "C" lq_status lq_deflated_guess(lq_op *op, int nvec, const double *evals, const void *evecs, const void *b,
                                       void *x0, void *stream)
{
    if (!op || nvec < 1 || nvec > 4096 || !evals || !evecs || !b || !x0) {
        set_error("lq_deflated_guess: null argument or nvec outside [1, 4096]");
        return LQ_ERR_ARG;
    }
    for (int k = 0; k < nvec; ++k)
        if (!(evals[k] > 0) || !std::isfinite(evals[k])) {
            set_error("lq_deflated_guess: eigenvalues must be finite and positive");
            return LQ_ERR_ARG;
        }
    if (!op->gauge_set) {
        set_error("lq_deflated_guess: gauge field not set");
        return LQ_ERR_STATE;
    }
    try {
        set_error("");
        LQ_HIP(hipSetDevice(op->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const Geom &g = op->g;
        const long n = 12L * g.vh;
        const double kappa = op->prm.kappa;
        const long f = fb(F64, g);
        // packed: b (both parities), x (both parities), t, b_hat, y; then the
        // boundary-layout y and x_e, and the reduction scratch (kept with
        // the operator for the next call)
        Buf &packed = op->defl_ws[0], &bnd = op->defl_ws[1], &part = op->defl_ws[2];
        packed.ensure(7 * (size_t)f);
        bnd.ensure(2 * sizeof(double) * 2 * (size_t)n);
        part.ensure(sizeof(double) * 2 * (DOT_WG * (size_t)nvec + nvec));
        char *bp = packed.ptr, *xp = packed.ptr + 2 * f, *tp = packed.ptr + 4 * f, *bh = packed.ptr + 5 * f,
             *yp = packed.ptr + 6 * f;
        double *ybd = reinterpret_cast<double *>(bnd.ptr), *xbd = ybd + 2 * n;
        double *mp = reinterpret_cast<double *>(part.ptr), *cdev = mp + 2 * DOT_WG * (size_t)nvec;
        for (int p = 0; p < 2; ++p)
            LQ_HIP(launch_pack_spinor(g, p, 0, static_cast<const double *>(b), full_parity_view(bp, F64, g, 1, p), s));
        const FieldView be = full_parity_view(bp, F64, g, 1, 0), bo = full_parity_view(bp, F64, g, 1, 1);
        // b_hat = b_e + kappa H_eo A_oo^-1 b_o, y = M^dag b_hat
        clover_apply(op, F64, 1, true, parity_view(tp, F64, g, 1), bo, s);
        hop(op, F64, parity_view(bh, F64, g, 1), parity_view(tp, F64, g, 1), 0, false, 0, false, &be, kappa, 0, nullptr,
            s);
        apply_packed(op, LQ_SCHUR_DAG, F64, yp, bh, 1, s);
        LQ_HIP(launch_unpack_spinor(g, 0, 1, parity_view(yp, F64, g, 1), ybd, s));
        // c_k = v_k^dag y
        const double *Vv = static_cast<const double *>(evecs);
        mdot_kernel<<<dim3(DOT_WG, (unsigned)nvec), 256, 0, s>>>(Vv, ybd, n, mp);
        LQ_HIP(hipGetLastError());
        msum_kernel<<<(unsigned)nvec, 64, 0, s>>>(mp, cdev);
        LQ_HIP(hipGetLastError());
        std::vector<double> c(2 * (size_t)nvec);
        LQ_HIP(hipMemcpyAsync(c.data(), cdev, sizeof(double) * c.size(), hipMemcpyDeviceToHost, s));
        LQ_HIP(hipStreamSynchronize(s));
        // x_e = sum_k (c_k / lambda_k) v_k, the solution's component in the
        // span of the eigenvectors
        LQ_HIP(hipMemsetAsync(xbd, 0, sizeof(double) * 2 * (size_t)n, s));
        const unsigned nb = (unsigned)((n + 255) / 256);
        for (int k = 0; k < nvec; ++k) {
            caxpy_kernel<<<nb, 256, 0, s>>>(xbd, Vv + (size_t)k * 2 * n, c[2 * k] / evals[k], c[2 * k + 1] / evals[k],
                                            n);
            LQ_HIP(hipGetLastError());
        }
        // x_o = A_oo^-1 (b_o + kappa H_oe x_e), then the full field
        const FieldView xe = full_parity_view(xp, F64, g, 1, 0);
        LQ_HIP(launch_pack_spinor(g, 0, 1, xbd, xe, s));
        hop(op, F64, full_parity_view(xp, F64, g, 1, 1), xe, 1, false, 2, true, &bo, kappa, 0, nullptr, s);
        for (int p = 0; p < 2; ++p)
            LQ_HIP(launch_unpack_spinor(g, p, 0, full_parity_view(xp, F64, g, 1, p), static_cast<double *>(x0), s));
        LQ_HIP(hipStreamSynchronize(s));
        return LQ_OK;
    } catch (const Failure &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return LQ_ERR_STATE;
    }
}
