// hmc.hip -- molecular dynamics of the Monte Carlo gauge-field generation
// (Sec. 2: the fermion-matrix solves recur at every step of it): the Wilson
// plaquette gauge action and its force, the momentum and link updates, the
// kinetic energy, and leapfrog / Omelyan trajectories that combine them
// with the pseudofermion force of force.hip.
//
// Conventions (as for the pseudofermion force): the su(3) force G is
// -TA(U M) for the matrix M with dS = sum Re tr(M dU); the equations of
// motion are dU/dt = P U, dP/dt = -G, which conserve
// H = 1/2 sum tr(P^dag P) + S(U).
//
// Gauge action S_g = beta sum_x sum_{mu<nu} (1 - Re tr P_{mu nu}(x) / 3).
// The link U_mu(x) enters the six plaquettes of the planes (mu, nu) that
// contain it through Re tr(U_mu(x) A_mu(x)), A the sum of the six staples
//   U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu),
// so M = -(beta/3) A and G = (beta/3) TA(U A); summing Re tr(U A) over all
// links counts every plaquette four times.
#include <chrono>
#include <cmath>
#include <algorithm>
#include <string>
#include <vector>

#include "solver.h"
#include "su3.h"

namespace lq {

// -TA(B) into o (18 reals), added to o when acc.
__device__ __forceinline__ void store_minus_ta(const M3 &bm, double scale, double *o, bool acc)
{
    const double tri = (bm.e[0].im + bm.e[4].im + bm.e[8].im) / 3.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const cx<double> bik = bm.e[i * 3 + k], bki = bm.e[k * 3 + i];
            double re = 0.5 * (bki.re - bik.re);
            double im = 0.5 * (-bki.im - bik.im);
            if (i == k) im += tri;
            re = scale * re;
            im = scale * im;
            if (acc) {
                o[(i * 3 + k) * 2] += re;
                o[(i * 3 + k) * 2 + 1] += im;
            } else {
                o[(i * 3 + k) * 2] = re;
                o[(i * 3 + k) * 2 + 1] = im;
            }
        }
}

// One link per thread (grid: site blocks x parity x direction).  G (lex,
// [V][4][18], may be null) receives (or is added) the gauge force;
// partial[(mu * 2 + p) * nw + wave] the wavefront's sum of Re tr(U_mu(x) A_mu(x)).
__global__ __launch_bounds__(128) void gauge_force_kernel(Geom g, const char *links64, double beta, double *G,
                                                          int accumulate, double *partial)
{
    const int cb = blockIdx.x * 128 + threadIdx.x;
    const int p = blockIdx.y;
    const int mu = blockIdx.z;
    double retr = 0.0;
    if (cb < g.vh) {
        int x[4];
        cb_coords(g, p, cb, x);
        const long lex = x[0] + (long)g.L[0] * (x[1] + (long)g.L[1] * (x[2] + (long)g.L[2] * x[3]));
        {
            M3 A;
            for (int i = 0; i < 9; ++i) A.e[i] = cx<double>{0, 0};
#pragma unroll 1
            for (int nu = 0; nu < 4; ++nu) {
                if (nu == mu) continue;
                int xm[4], xn[4], xmn[4];
                shift(g, x, mu, 1, nu, 0, xm);    // x + mu
                shift(g, x, mu, 0, nu, 1, xn);    // x + nu
                shift(g, x, mu, 1, nu, -1, xmn);  // x + mu - nu
                int xb[4];
                shift(g, x, mu, 0, nu, -1, xb);   // x - nu
                A = add(A, mul(mul(link_at(g, links64, xm, nu), dag(link_at(g, links64, xn, mu))),
                               dag(link_at(g, links64, x, nu))));
                A = add(A, mul(mul(dag(link_at(g, links64, xmn, nu)), dag(link_at(g, links64, xb, mu))),
                               link_at(g, links64, xb, nu)));
            }
            const M3 B = mul(link_at(g, links64, x, mu), A);
            retr += B.e[0].re + B.e[4].re + B.e[8].re;
            // G = -TA(U M) with M = -(beta/3) A
            if (G) store_minus_ta(B, -beta / 3.0, G + (lex * 4 + mu) * 18, accumulate != 0);
        }
    }
    const double s = wave_sum(retr);
    if ((threadIdx.x & 63) == 0 && cb < g.vh) partial[(long)(mu * 2 + p) * ((g.vh + 63) / 64) + (cb >> 6)] = s;
}

// 1/2 sum |P|^2 per wavefront of 64 links (P: [nlinks][18] reals).
__global__ __launch_bounds__(256) void kinetic_kernel(const double *P, long nlinks, double *partial)
{
    const long l = (long)blockIdx.x * 256 + threadIdx.x;
    double t = 0.0;
    if (l < nlinks) {
        const double *q = P + l * 18;
#pragma unroll
        for (int k = 0; k < 18; ++k) t += q[k] * q[k];
        t = 0.5 * t;
    }
    const double s = wave_sum(t);
    if ((threadIdx.x & 63) == 0 && l < nlinks) partial[l >> 6] = s;
}

// P <- P - c G over n reals.
__global__ __launch_bounds__(256) void update_p_kernel(double *P, const double *G, double c, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) P[i] = P[i] - c * G[i];
}

// U <- exp(e P) U per link: scaling by 2^-s to a Frobenius norm <= 1/4, a
// Taylor polynomial of degree 12 (truncation below 3e-18), then s squarings.
__global__ __launch_bounds__(128) void update_u_kernel(double *U, const double *P, double e, long nlinks)
{
    const long l = (long)blockIdx.x * 128 + threadIdx.x;
    if (l >= nlinks) return;
    M3 X;
    double nrm = 0.0;
    for (int i = 0; i < 9; ++i) {
        X.e[i] = cx<double>{e * P[l * 18 + 2 * i], e * P[l * 18 + 2 * i + 1]};
        nrm += X.e[i].re * X.e[i].re + X.e[i].im * X.e[i].im;
    }
    nrm = sqrt(nrm);
    int s = 0;
    while (nrm > 0.25 && s < 64) {
        nrm *= 0.5;
        ++s;
    }
    const double sc = ldexp(1.0, -s);
    for (int i = 0; i < 9; ++i) X.e[i] = cx<double>{sc * X.e[i].re, sc * X.e[i].im};
    // Horner: E = I + X/1 (I + X/2 (I + ... (I + X/12)))
    M3 E;
    for (int i = 0; i < 9; ++i) E.e[i] = cx<double>{(i % 4 == 0) ? 1.0 : 0.0, 0.0};
    for (int k = 12; k >= 1; --k) {
        M3 T = mul(X, E);
        const double r = 1.0 / k;
        for (int i = 0; i < 9; ++i) E.e[i] = cx<double>{((i % 4 == 0) ? 1.0 : 0.0) + r * T.e[i].re, r * T.e[i].im};
    }
    for (int k = 0; k < s; ++k) E = mul(E, E);
    M3 u;
    for (int i = 0; i < 9; ++i) u.e[i] = cx<double>{U[l * 18 + 2 * i], U[l * 18 + 2 * i + 1]};
    const M3 n = mul(E, u);
    for (int i = 0; i < 9; ++i) {
        U[l * 18 + 2 * i] = n.e[i].re;
        U[l * 18 + 2 * i + 1] = n.e[i].im;
    }
}

// out = 2 a - b over n reals (linear extrapolation of two solutions).
__global__ __launch_bounds__(256) void extrapolate_kernel(double *out, const double *a, const double *b, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = 2.0 * a[i] - b[i];
}

// ------------------------------------------------------------------ host --

namespace {

long nlinks(const Geom &g) { return 8L * g.vh; }

double host_sum(const double *dev, long n, hipStream_t s)
{
    std::vector<double> h((size_t)n);
    LQ_HIP(hipMemcpyAsync(h.data(), dev, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, s));
    LQ_HIP(hipStreamSynchronize(s));
    double t = 0.0;
    for (long i = 0; i < n; ++i) t += h[(size_t)i];  // fixed order
    return t;
}

// Gauge action (if want_s) and force (added to G when accumulate) at the
// operator's current gauge field.
double gauge_part(lq_op *op, double beta, double *G, bool accumulate, bool want_s, hipStream_t s)
{
    const Geom &g = op->g;
    const long nw = (g.vh + 63) / 64;
    op->md_partial.ensure(sizeof(double) * (size_t)std::max<long>(8 * nw, (nlinks(g) + 63) / 64));
    double *part = reinterpret_cast<double *>(op->md_partial.ptr);
    gauge_force_kernel<<<dim3((unsigned)((g.vh + 127) / 128), 2, 4), 128, 0, s>>>(g, op->links[F64].ptr, beta, G,
                                                                                    accumulate ? 1 : 0, part);
    LQ_HIP(hipGetLastError());
    if (!want_s) return 0.0;
    const double retr = host_sum(part, 8 * nw, s);
    return beta * (6.0 * 2.0 * g.vh - retr / 12.0);
}

double kinetic(lq_op *op, const double *P, hipStream_t s)
{
    const long n = nlinks(op->g);
    op->md_partial.ensure(sizeof(double) * (size_t)std::max<long>(8 * ((op->g.vh + 63) / 64), (n + 63) / 64));
    double *part = reinterpret_cast<double *>(op->md_partial.ptr);
    kinetic_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(P, n, part);
    LQ_HIP(hipGetLastError());
    return host_sum(part, (n + 63) / 64, s);
}

void update_p(lq_op *op, double *P, const double *G, double c, hipStream_t s)
{
    const long n = 18 * nlinks(op->g);
    update_p_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(P, G, c, n);
    LQ_HIP(hipGetLastError());
}

void update_u(lq_op *op, double *U, const double *P, double e, hipStream_t s)
{
    const long n = nlinks(op->g);
    update_u_kernel<<<(unsigned)((n + 127) / 128), 128, 0, s>>>(U, P, e, n);
    LQ_HIP(hipGetLastError());
    const lq_status st = lq_op_set_gauge(op, U, s);
    if (st != LQ_OK) throw Failure{st, std::string("gauge update: ") + lq_last_error()};
}

struct MD {
    lq_op *op;
    const lq_md_params *mp;
    const lq_solver_params *sp;
    const void *phi;
    double *G;
    hipStream_t s;
    int n_force = 0;
    long iters = 0;
    bool converged = true;
    // solution history: buffer indices of the last and the one before, and
    // how many of them hold solutions of this trajectory
    int last = 0, before = 1, nhist = 0;

    double *xbuf(int i) { return reinterpret_cast<double *>(op->md_X[i].ptr); }

    // G(U) at the operator's gauge field; the actions when want_s
    void force(bool want_s, double *Sg, double *Sf)
    {
        ++n_force;
        double sf = 0.0;
        if (mp->fermion) {
            // initial guess from the previous solutions; the new one goes to
            // the buffer that is no longer needed
            const long n = 24L * op->g.vh;
            const double *x0 = nullptr;
            if (mp->chrono >= 2 && nhist >= 2) {
                extrapolate_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(xbuf(2), xbuf(last), xbuf(before), n);
                LQ_HIP(hipGetLastError());
                x0 = xbuf(2);
            } else if (mp->chrono >= 1 && nhist >= 1) {
                x0 = xbuf(last);
            }
            const int out = nhist >= 1 ? before : last;
            lq_solve_stats st{};
            const lq_status rc = pf_force_guess(op, sp, 0, (lq_prec)mp->force_prec, phi, nullptr, G,
                                                mp->chrono ? xbuf(out) : nullptr, &sf, &st, s, x0);
            if (rc < 0) throw Failure{rc, std::string("pseudofermion force: ") + lq_last_error()};
            if (rc == LQ_NOT_CONVERGED) converged = false;
            iters += st.nconv;
            if (mp->chrono) {
                if (nhist >= 1) std::swap(last, before);
                nhist = std::min(nhist + 1, 2);
            }
        }
        const double sg = gauge_part(op, mp->beta, G, mp->fermion != 0, want_s, s);
        if (want_s) {
            *Sg = sg;
            *Sf = sf;
        }
    }
};

}  // namespace
}  // namespace lq

using namespace lq;

extern "C" void lq_md_params_default(lq_md_params *p)
{
    if (!p) return;
    p->beta = 5.6;
    p->tau = 1.0;
    p->nsteps = 10;
    p->integrator = LQ_LEAPFROG;
    p->lambda = 0.1931833275037836;
    p->fermion = 1;
    p->force_prec = LQ_F64;
    p->chrono = 2;
}

extern "C" lq_status lq_gauge_force(lq_op *op, double beta, void *G, double *S, void *stream)
{
    if (!op || (!G && !S)) {
        set_error("lq_gauge_force: null operator, or neither G nor S requested");
        return LQ_ERR_ARG;
    }
    if (!std::isfinite(beta)) {
        set_error("lq_gauge_force: beta must be finite");
        return LQ_ERR_ARG;
    }
    if (!op->gauge_set) {
        set_error("lq_gauge_force: gauge field not set");
        return LQ_ERR_STATE;
    }
    try {
        set_error("");
        LQ_HIP(hipSetDevice(op->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const double sg = gauge_part(op, beta, static_cast<double *>(G), false, true, s);
        if (S) *S = sg;
        return LQ_OK;
    } catch (const Failure &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return LQ_ERR_STATE;
    }
}

extern "C" lq_status lq_md_trajectory(lq_op *op, const lq_md_params *mp, const lq_solver_params *sp, void *U, void *P,
                                      const void *phi, lq_md_stats *stats, void *stream)
{
    if (!op || !mp || !U || !P) {
        set_error("lq_md_trajectory: null argument");
        return LQ_ERR_ARG;
    }
    if (mp->nsteps < 1 || !std::isfinite(mp->tau) || !std::isfinite(mp->beta) || !std::isfinite(mp->lambda) ||
        (mp->integrator != LQ_LEAPFROG && mp->integrator != LQ_OMELYAN) || (mp->fermion != 0 && mp->fermion != 1) ||
        mp->chrono < 0 || mp->chrono > 2) {
        set_error("lq_md_trajectory: invalid parameters (nsteps >= 1, finite tau, beta and lambda, "
                  "integrator LQ_LEAPFROG or LQ_OMELYAN, fermion 0 or 1, chrono 0, 1 or 2)");
        return LQ_ERR_ARG;
    }
    if (mp->fermion && (!sp || !phi)) {
        set_error("lq_md_trajectory: the pseudofermion action needs solver parameters and phi");
        return LQ_ERR_ARG;
    }
    if (mp->fermion && mp->force_prec != LQ_F64 && mp->force_prec != LQ_F32) {
        set_error("lq_md_trajectory: force precision must be LQ_F64 or LQ_F32");
        return LQ_ERR_ARG;
    }
    try {
        set_error("");
        LQ_HIP(hipSetDevice(op->device));
        hipStream_t s = static_cast<hipStream_t>(stream);
        const auto t0 = std::chrono::steady_clock::now();
        double *Ud = static_cast<double *>(U);
        double *Pd = static_cast<double *>(P);
        op->md_G.ensure(sizeof(double) * 18 * (size_t)nlinks(op->g));
        if (mp->fermion && mp->chrono)
            for (int i = 0; i < 3; ++i) op->md_X[i].ensure(sizeof(double) * 24 * (size_t)op->g.vh);
        MD md{op, mp, sp, phi, reinterpret_cast<double *>(op->md_G.ptr), s};
        {
            const lq_status st = lq_op_set_gauge(op, U, s);
            if (st != LQ_OK) throw Failure{st, std::string("initial gauge field: ") + lq_last_error()};
        }
        lq_md_stats out{};
        out.T0 = kinetic(op, Pd, s);
        md.force(true, &out.Sg0, &out.Sf0);
        const double e = mp->tau / mp->nsteps;
        const int n = mp->nsteps;
        if (mp->integrator == LQ_LEAPFROG) {
            // P half step, then per step: U by e, force, P by e (the last by e/2)
            update_p(op, Pd, md.G, 0.5 * e, s);
            for (int k = 0; k < n; ++k) {
                update_u(op, Ud, Pd, e, s);
                const bool last = k == n - 1;
                md.force(last, &out.Sg1, &out.Sf1);
                update_p(op, Pd, md.G, last ? 0.5 * e : e, s);
            }
        } else {
            // per step: P by lam e, U by e/2, P by (1 - 2 lam) e, U by e/2, P by lam e;
            // the P updates of adjacent steps are merged (2 lam e)
            const double lam = mp->lambda;
            update_p(op, Pd, md.G, lam * e, s);
            for (int k = 0; k < n; ++k) {
                update_u(op, Ud, Pd, 0.5 * e, s);
                md.force(false, nullptr, nullptr);
                update_p(op, Pd, md.G, (1.0 - 2.0 * lam) * e, s);
                update_u(op, Ud, Pd, 0.5 * e, s);
                const bool last = k == n - 1;
                md.force(last, &out.Sg1, &out.Sf1);
                update_p(op, Pd, md.G, last ? lam * e : 2.0 * lam * e, s);
            }
        }
        out.T1 = kinetic(op, Pd, s);
        out.H0 = out.T0 + out.Sg0 + out.Sf0;
        out.H1 = out.T1 + out.Sg1 + out.Sf1;
        out.dH = out.H1 - out.H0;
        out.n_force = md.n_force;
        out.iters = md.iters;
        out.converged = md.converged ? 1 : 0;
        out.t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (stats) *stats = out;
        return md.converged ? LQ_OK : LQ_NOT_CONVERGED;
    } catch (const Failure &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return LQ_ERR_STATE;
    }
}
