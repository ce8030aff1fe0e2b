// force.hip -- pseudofermion force: the derivative of
//   S = phi^dag (A)^-1 phi,  A = M^dag M (even-odd Wilson, M = 1 - kappa^2 H_eo H_oe)
//                            or A = D^dag D (full lattice, D = 1 - kappa H)
// with respect to every link, from the hopping term of eq. (1) (Sec. 3).
//
// With X = A^-1 phi: even-odd: Y = M X, Z = H_oe X, W = (H_eo)^dag Y and
//   dS = 2 kappa^2 Re[ Y^dag dH_eo Z + W^dag dH_oe X ];
// full lattice: Y = D X and dS = 2 kappa Re[ Y^dag dH X ].
// For a pair Re[a^dag dH b] the link U_mu(x) receives, as the matrix M with
// dS = sum Re tr(M dU), the forward term  ph sum_s [(1-g)b(x+mu)]_s a(x)_s^dag
// plus the conjugate transpose of  conj(ph) sum_s [(1+g)b(x)]_s a(x+mu)_s^dag.
// In the chiral basis (1 + s gamma_mu)/2 is a rank-2 projector, so each sum
// is an outer product of the two projected half spinors:
//   sum_s [(1+sg) b]_s a_s^dag = sum_{j=0,1} h^b_j (h^a_j)^dag,  h = up + s B dn.
// The kernel writes the gradient M^dag (dS = Re sum conj(M^dag) dU) and the
// su(3) force G = -TA(U M), where
// TA(B) = (B - B^dag)/2 - tr(B - B^dag)/6.
//
// Clover operator (A = 1 + F, F = -c_sw kappa sum_{mu<nu} gamma_mu gamma_nu
// (x) Fhat_{mu nu}, Fhat = (Q - Q^dag)/8 from the four counter-clockwise
// leaves, trace removed if traceless): even-odd with
// M = A_ee - kappa^2 H_eo A_oo^-1 H_oe, Z = A_oo^-1 H_oe X, W = A_oo^-1 H_eo^dag Y,
//   dS = 2 kappa^2 Re[Y^dag dH_eo Z + W^dag dH_oe X] - 2 Re[Y^dag dA_ee X + kappa^2 W^dag dA_oo Z];
// full lattice: dS = 2 kappa Re[Y^dag dH X] - 2 Re[Y^dag dA X].
// For a pair Re[a^dag dA b] at site x, with
// Lambda_{mu nu} = sum_{s s'} (gamma_mu gamma_nu)_{s s'} b_{s'} a_s^dag (3x3) and
// Lt = Lambda - tr(Lambda)/3 (traceless) or Lambda:
//   Re[a^dag dA b] = -c_sw kappa / 8 sum_{mu<nu} Re tr[dQ_{mu nu}(x) (Lt - Lt^dag)],
// so the clover part is sum_x sum_{mu<nu} Re tr[dQ_{mu nu}(x) Gamma_{mu nu}(x)]
// with the insertion Gamma = c (Lt - Lt^dag), c = c_sw kappa / 4 (even sites
// or full lattice) or c_sw kappa^3 / 4 (odd sites).  Each link lies in two
// plaquettes per plane it spans, each of them a leaf of Q at its four
// corners: the link receives, per plaquette, the loop product that follows
// it with Gamma inserted at each corner in turn (its conjugate transpose
// where the loop walks the link backwards).
#include <chrono>
#include <cmath>

#include "solver.h"
#include "stencil.h"
#include "su3.h"

namespace lq {

struct ForceArgs {
    Geom g;
    const char *links;  // packed links of the force precision ([parity][mu])
    // per output parity p: a, c on parity p; b, d on parity 1 - p
    FieldView a[2], b[2], c[2], d[2];
    double coef;
    double *M;  // complex128 [V][4][3][3] (lex) or null
    double *G;
};

template <int P, int NL, int MU>
__device__ __forceinline__ void force_dir(const ForceArgs &f, int p, int cb, const int c[4], double *Mo, double *Go,
                                          long lex)
{
    using R = typename PT<P>::R;
    int d[4] = {c[0], c[1], c[2], c[3]};
    const bool wrap = d[MU] == f.g.L[MU] - 1;
    d[MU] = wrap ? 0 : d[MU] + 1;
    const int nb = cb_index(f.g, d);
    const Spinor<R> av = load_spinor<P>(f.a[p].base, cb, f.a[p].n);
    const Spinor<R> cv = load_spinor<P>(f.c[p].base, cb, f.c[p].n);
    const Spinor<R> bv = load_spinor<P>(f.b[p].base, nb, f.b[p].n);
    const Spinor<R> dv = load_spinor<P>(f.d[p].base, nb, f.d[p].n);
    cx<R> ha[6], hb[6], hc[6], hd[6];
    project<MU, -1>(av, ha);
    project<MU, -1>(bv, hb);
    project<MU, +1>(cv, hc);
    project<MU, +1>(dv, hd);
    cx<R> m[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cx<R> acc = cx<R>{0, 0};
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                acc = acc + cmulc(ha[s * 3 + k], hb[s * 3 + i]);
                acc = acc + cmulc(hc[s * 3 + k], hd[s * 3 + i]);
            }
            m[i * 3 + k] = acc;
        }
    cx<R> ph = cx<R>{(R)f.coef, 0};
    if (wrap) ph = cx<R>{(R)(f.coef * f.g.bc_re[MU]), (R)(f.coef * f.g.bc_im[MU])};
#pragma unroll
    for (int i = 0; i < 9; ++i) m[i] = ph * m[i];
    if (Mo) {
        // the gradient in the convention dS = Re sum conj(grad) dU: grad = M^dag
        double *o = Mo + (lex * 4 + MU) * 18;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                o[2 * (i * 3 + k)] = (double)m[k * 3 + i].re;
                o[2 * (i * 3 + k) + 1] = -(double)m[k * 3 + i].im;
            }
    }
    if (Go) {
        cx<R> u[9];
        load_link<P, NL>(f.links, f.g.vh, p, MU, cb, u);
        cx<R> bm[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                bm[i * 3 + k] = u[i * 3 + 0] * m[0 * 3 + k] + u[i * 3 + 1] * m[1 * 3 + k] + u[i * 3 + 2] * m[2 * 3 + k];
        // G = -TA(B) = (B^dag - B)/2 + tr(B - B^dag)/6
        const R tri = (bm[0].im + bm[4].im + bm[8].im) / (R)3;  // tr(B - B^dag)/6 = i Im tr(B)/3
        double *o = Go + (lex * 4 + MU) * 18;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const cx<R> bik = bm[i * 3 + k], bki = bm[k * 3 + i];
                R re = (R)0.5 * (bki.re - bik.re);
                R im = (R)0.5 * (-bki.im - bik.im);
                if (i == k) im += tri;
                o[(i * 3 + k) * 2] = (double)re;
                o[(i * 3 + k) * 2 + 1] = (double)im;
            }
    }
}

template <int P, int NL>
__global__ __launch_bounds__(128) void force_kernel(ForceArgs f)
{
    const int cb = blockIdx.x * 128 + threadIdx.x;
    const int p = blockIdx.y;
    if (cb >= f.g.vh) return;
    int c[4];
    cb_coords(f.g, p, cb, c);
    const long lex = c[0] + (long)f.g.L[0] * (c[1] + (long)f.g.L[1] * (c[2] + (long)f.g.L[2] * c[3]));
    force_dir<P, NL, 0>(f, p, cb, c, f.M, f.G, lex);
    force_dir<P, NL, 1>(f, p, cb, c, f.M, f.G, lex);
    force_dir<P, NL, 2>(f, p, cb, c, f.M, f.G, lex);
    force_dir<P, NL, 3>(f, p, cb, c, f.M, f.G, lex);
}

// ---------------------------------------------------------------- clover --

// gamma_mu gamma_nu of the chiral basis, plane by plane (mu, nu) = (0,1),
// (0,2), (0,3), (1,2), (1,3), (2,3): block-diagonal over chirality, each
// block s_k i sigma_m, with m and the signs s_0 (spins 0, 1), s_1 (spins 2, 3).
__device__ __forceinline__ void plane_spin(int pid, int &m, int &s0, int &s1)
{
    switch (pid) {
    case 0: m = 3; s0 = 1; s1 = 1; break;    // xy
    case 1: m = 2; s0 = -1; s1 = -1; break;  // xz
    case 2: m = 1; s0 = -1; s1 = 1; break;   // xt
    case 3: m = 1; s0 = 1; s1 = 1; break;    // yz
    case 4: m = 2; s0 = -1; s1 = 1; break;   // yt
    default: m = 3; s0 = -1; s1 = 1; break;  // zt
    }
}

__device__ __forceinline__ int plane_id(int a, int b)
{
    // a < b
    return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}

struct InsertArgs {
    Geom g;
    FieldView a[2], b[2];  // the pair (a, b) on each parity (FP64)
    double c[2];           // insertion coefficient per parity (0: none)
    int traceless;
    char *gam;             // [parity][plane] x 18 reals over vh
};

// One site per thread: Gamma_{mu nu}(x) = c (Lt - Lt^dag) for the six planes.
__global__ __launch_bounds__(128) void clover_insert_kernel(InsertArgs f)
{
    const int cb = blockIdx.x * 128 + threadIdx.x;
    const int p = blockIdx.y;
    if (cb >= f.g.vh) return;
    const double cf = f.c[p];
    Spinor<double> av, bv;
    if (cf != 0.0) {
        av = load_spinor<F64>(f.a[p].base, cb, f.a[p].n);
        bv = load_spinor<F64>(f.b[p].base, cb, f.b[p].n);
    }
    for (int pid = 0; pid < 6; ++pid) {
        int m, s0, s1;
        plane_spin(pid, m, s0, s1);
        // i sigma_m as 2x2: entries (i, j)
        cx<double> is[2][2];
        if (m == 1) { is[0][0] = cx<double>{0, 0}; is[0][1] = cx<double>{0, 1}; is[1][0] = cx<double>{0, 1}; is[1][1] = cx<double>{0, 0}; }
        else if (m == 2) { is[0][0] = cx<double>{0, 0}; is[0][1] = cx<double>{1, 0}; is[1][0] = cx<double>{-1, 0}; is[1][1] = cx<double>{0, 0}; }
        else { is[0][0] = cx<double>{0, 1}; is[0][1] = cx<double>{0, 0}; is[1][0] = cx<double>{0, 0}; is[1][1] = cx<double>{0, -1}; }
        // Lambda_{d c} = sum_{s s'} G_{s s'} b_{s' d} conj(a_{s c})
        cx<double> L[9];
        for (int i = 0; i < 9; ++i) L[i] = cx<double>{0, 0};
        if (cf != 0.0)
            for (int k = 0; k < 2; ++k) {
                const double sk = k == 0 ? s0 : s1;
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < 2; ++j) {
                        const cx<double> gij = sk * is[i][j];
                        if (gij.re == 0.0 && gij.im == 0.0) continue;
                        const int s = 2 * k + i, sp = 2 * k + j;
                        for (int d = 0; d < 3; ++d)
                            for (int c = 0; c < 3; ++c)
                                L[d * 3 + c] = L[d * 3 + c] + gij * cmulc(av.c[s * 3 + c], bv.c[sp * 3 + d]);
                    }
            }
        if (f.traceless) {
            const cx<double> tr = (1.0 / 3.0) * (L[0] + L[4] + L[8]);
            L[0] = L[0] - tr;
            L[4] = L[4] - tr;
            L[8] = L[8] - tr;
        }
        double raw[18];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                // c (L - L^dag)_{ij}
                const cx<double> v = L[i * 3 + j] - conj(L[j * 3 + i]);
                raw[2 * (i * 3 + j)] = cf * v.re;
                raw[2 * (i * 3 + j) + 1] = cf * v.im;
            }
        store_planes<double, 18>(f.gam + (long)(p * 6 + pid) * Planes<double, 18>::field_bytes(f.g.vh), cb, f.g.vh,
                                 raw);
    }
}

__device__ __forceinline__ M3 gamma_at(const Geom &g, const char *gam, const int c[4], int pid)
{
    const int p = (c[0] + c[1] + c[2] + c[3]) & 1;
    double raw[18];
    load_planes<double, 18>(gam + (long)(p * 6 + pid) * Planes<double, 18>::field_bytes(g.vh), cb_index(g, c), g.vh,
                            raw);
    M3 m;
#pragma unroll
    for (int i = 0; i < 9; ++i) m.e[i] = cx<double>{raw[2 * i], raw[2 * i + 1]};
    return m;
}

// R = G0 A B C + A G1 B C + A B G2 C + A B C G3: the loop product that follows
// a link (A, B, C the other three factors in loop order), with the insertion
// of each corner after the link (G0 first, G3 at the link's own start).
// A factor of a loop: the link U_dir(c), conjugate-transposed when dg.
struct LoopFactor {
    const int *c;
    int dir;
    bool dg;
};

__device__ __forceinline__ M3 factor_at(const Geom &g, const char *links64, const LoopFactor &f)
{
    const M3 u = link_at(g, links64, f.c, f.dir);
    return f.dg ? dag(u) : u;
}

// In Horner form, S = G0 A + A G1;  S = S B + (A B) G2;  S = S C + (A B C) G3,
// each factor and insertion loaded when it is needed (few matrices live).
__device__ __forceinline__ M3 loop_insert(const Geom &g, const char *links64, const char *gam, int pid,
                                          const LoopFactor &fa, const LoopFactor &fb, const LoopFactor &fc,
                                          const int *c0, const int *c1, const int *c2, const int *c3)
{
    const M3 A = factor_at(g, links64, fa);
    M3 S = add(mul(gamma_at(g, gam, c0, pid), A), mul(A, gamma_at(g, gam, c1, pid)));
    const M3 B = factor_at(g, links64, fb);
    M3 Q = mul(A, B);
    S = add(mul(S, B), mul(Q, gamma_at(g, gam, c2, pid)));
    const M3 C = factor_at(g, links64, fc);
    Q = mul(Q, C);
    S = add(mul(S, C), mul(Q, gamma_at(g, gam, c3, pid)));
    return S;
}

struct CloverForceArgs {
    Geom g;
    const char *links64;  // packed FP64 links, 18 reals
    const char *gam;
    double *M, *G;        // outputs of the hopping-term kernel, added to (each may be null)
};

// One (site, direction) per thread: the clover part Mc of the link's matrix;
// adds Mc^dag to the gradient and -TA(U Mc) to the force (both linear in M).
__global__ __launch_bounds__(128) void clover_force_kernel(CloverForceArgs f)
{
    const int cb = blockIdx.x * 128 + threadIdx.x;
    const int p = blockIdx.y;
    const int rho = blockIdx.z;
    if (cb >= f.g.vh) return;
    const Geom &g = f.g;
    int y[4];
    cb_coords(g, p, cb, y);
    const long lex = y[0] + (long)g.L[0] * (y[1] + (long)g.L[1] * (y[2] + (long)g.L[2] * y[3]));
    M3 m;
    for (int i = 0; i < 9; ++i) m.e[i] = cx<double>{0, 0};
    // one plane at a time: unrolled, the compiler would hoist the loads of all
    // three planes and run out of registers
#pragma unroll 1
    for (int sg = 0; sg < 4; ++sg) {
        if (sg == rho) continue;
        const int a = rho < sg ? rho : sg, b = rho < sg ? sg : rho;
        const int pid = plane_id(a, b);
        int c1[4], c2[4], c3[4], c4[4];
        if (rho == a) {
            // plaquette based at y: U_a(y) [the link] U_b(y+a) U_a(y+b)^dag U_b(y)^dag
            shift(g, y, a, 1, b, 0, c2);
            shift(g, y, a, 1, b, 1, c3);
            shift(g, y, a, 0, b, 1, c4);
            m = add(m, loop_insert(g, f.links64, f.gam, pid, {c2, b, false}, {c4, a, true}, {y, b, true}, c2, c3, c4,
                                   y));
            // plaquette based at z = y - b, walking the link backwards:
            // U_a(z) U_b(z+a) U_a(y)^dag U_b(z)^dag
            shift(g, y, a, 0, b, -1, c1);  // z
            shift(g, y, a, 1, b, -1, c2);  // z + a
            shift(g, y, a, 1, b, 0, c3);   // y + a
            m = add(m, dag(loop_insert(g, f.links64, f.gam, pid, {c1, b, true}, {c1, a, false}, {c2, b, false}, y,
                                       c1, c2, c3)));
        } else {
            // plaquette based at y, walking the link backwards:
            // U_a(y) U_b(y+a) U_a(y+b)^dag U_b(y)^dag
            shift(g, y, a, 1, b, 0, c2);
            shift(g, y, a, 1, b, 1, c3);
            shift(g, y, a, 0, b, 1, c4);
            m = add(m, dag(loop_insert(g, f.links64, f.gam, pid, {y, a, false}, {c2, b, false}, {c4, a, true}, y,
                                       c2, c3, c4)));
            // plaquette based at z = y - a: U_a(z) U_b(y) [the link] U_a(z+b)^dag U_b(z)^dag
            shift(g, y, a, -1, b, 0, c1);  // z
            shift(g, y, a, 0, b, 1, c3);   // y + b
            shift(g, y, a, -1, b, 1, c4);  // z + b
            m = add(m, loop_insert(g, f.links64, f.gam, pid, {c4, a, true}, {c1, b, true}, {c1, a, false}, c3, c4,
                                   c1, y));
        }
    }
    if (f.M) {
        double *o = f.M + (lex * 4 + rho) * 18;
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) {
                o[2 * (i * 3 + k)] += m.e[k * 3 + i].re;
                o[2 * (i * 3 + k) + 1] -= m.e[k * 3 + i].im;
            }
    }
    if (f.G) {
        const M3 bm = mul(link_at(g, f.links64, y, rho), m);
        const double tri = (bm.e[0].im + bm.e[4].im + bm.e[8].im) / 3.0;
        double *o = f.G + (lex * 4 + rho) * 18;
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) {
                const cx<double> bik = bm.e[i * 3 + k], bki = bm.e[k * 3 + i];
                double re = 0.5 * (bki.re - bik.re);
                double im = 0.5 * (-bki.im - bik.im);
                if (i == k) im += tri;
                o[(i * 3 + k) * 2] += re;
                o[(i * 3 + k) * 2 + 1] += im;
            }
    }
}

static hipError_t launch_clover_force(const InsertArgs &ia, const CloverForceArgs &cf, hipStream_t s)
{
    const unsigned nb = (unsigned)((ia.g.vh + 127) / 128);
    clover_insert_kernel<<<dim3(nb, 2), 128, 0, s>>>(ia);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    clover_force_kernel<<<dim3(nb, 2, 4), 128, 0, s>>>(cf);
    return hipGetLastError();
}

static hipError_t launch_force(const ForceArgs &f, int prec, int nl, hipStream_t s)
{
    const dim3 grid((f.g.vh + 127) / 128, 2);
    if (prec == F64) force_kernel<F64, 18><<<grid, 128, 0, s>>>(f);
    else if (prec == F32 && nl == 18) force_kernel<F32, 18><<<grid, 128, 0, s>>>(f);
    else if (prec == F32 && nl == 12) force_kernel<F32, 12><<<grid, 128, 0, s>>>(f);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace lq

using namespace lq;

namespace lq {

lq_status pf_force_guess(lq_op *op, const lq_solver_params *sp, int variant, lq_prec force_prec, const void *phi,
                         void *dSdU, void *G, void *X_out, double *S, lq_solve_stats *stats, void *stream,
                         const void *X0)
{
    if (!op || !sp || !phi) {
        set_error("lq_pf_force: null argument");
        return LQ_ERR_ARG;
    }
    if (variant != 0 && variant != 1) {
        set_error("lq_pf_force: variant must be 0 (even-odd) or 1 (full lattice)");
        return LQ_ERR_ARG;
    }
    if (force_prec != LQ_F64 && force_prec != LQ_F32) {
        set_error("lq_pf_force: force precision must be LQ_F64 or LQ_F32");
        return LQ_ERR_ARG;
    }
    std::string why;
    if (!lq::valid_solver_params(sp, why) && why != "the full-lattice solve is CGNE only") {
        set_error("lq_pf_force: invalid solver parameters: " + why);
        return LQ_ERR_ARG;
    }
    if (sp->deflate && (variant != 0 || op->defl_n == 0)) {
        set_error("lq_pf_force: deflate = 1 needs the even-odd variant and the operator's deflation space");
        return LQ_ERR_STATE;
    }
    if (!op->gauge_set) {
        set_error("lq_pf_force: gauge field not set");
        return LQ_ERR_STATE;
    }
    try {
        set_error("");
        LQ_HIP(hipSetDevice(op->device));
        hipStream_t us = static_cast<hipStream_t>(stream);
        LQ_HIP(hipEventRecord(op->ev_in, us));
        LQ_HIP(hipStreamWaitEvent(op->stream, op->ev_in, 0));
        hipStream_t s = op->stream;
        const Geom &g = op->g;
        const bool eo = variant == 0;
        const auto t0 = std::chrono::steady_clock::now();
        SolveCtx c;
        make_ctx(c, op, 1, eo, sp->inner, s);
        c.deflate = sp->deflate != 0 && eo;
        // phi packed into the solve space (FP64)
        FieldView phiv = c.aux64;
        if (eo) LQ_HIP(launch_pack_spinor(g, 0, 1, static_cast<const double *>(phi), phiv, s));
        else
            for (int p = 0; p < 2; ++p)
                LQ_HIP(launch_pack_spinor(g, p, 0, static_cast<const double *>(phi),
                                          FieldView{phiv.base + p * fb(F64, g), F64, (long)g.vh, 2 * fb(F64, g), 1},
                                          s));
        const std::vector<double> pn2 = norms2(c, phiv, c.sps);
        if (!std::isfinite(pn2[0])) throw Failure{LQ_ERR_NONFINITE, "phi is not finite"};
        // X = (M^dag M)^-1 phi
        // initial guess: zero, or X0 (the even-odd variant)
        if (X0 && eo) LQ_HIP(launch_pack_spinor(g, 0, 1, static_cast<const double *>(X0), c.x64, s));
        else LQ_HIP(launch_zero(c.x64, s));
        lq_solver_params sp2 = *sp;
        const std::vector<double> target2{sp->tol * sp->tol * pn2[0]};
        const OuterStats os = defect_correction(c, sp2, true, phiv, target2, !(X0 && eo));
        // final normal-system residual
        c.apply(c.t64, c.x64, false);
        c.apply(c.y64, c.t64, true);
        LQ_HIP(launch_xmy_norm(c.r64, phiv, c.y64, c.partial, s));
        LQ_HIP(launch_finish(c.partial, 1, c.sps, blas_blocks(g.vh), 1, FIN_NORM, c.sc, 0, s));
        c.pull();
        const double diff = pn2[0] > 0 ? std::sqrt(c.hsc[SC_NORM2] / pn2[0]) : 0.0;
        // S = Re <phi, X>
        LQ_HIP(launch_reduce(phiv, c.x64, RED_DOT, c.partial, s));
        LQ_HIP(launch_finish(c.partial, 1, c.sps, blas_blocks(g.vh), 2, FIN_DOT, c.sc, 0, s));
        c.pull();
        const double Sval = c.hsc[SC_DOT_RE];

        // Y, Z, W (FP64), in the odd scratch and solve vectors
        const int fp = force_prec;
        ForceArgs f{};
        f.g = g;
        f.links = op->links[fp].ptr;
        f.M = static_cast<double *>(dSdU);
        f.G = static_cast<double *>(G);
        InsertArgs ia{};
        ia.g = g;
        ia.traceless = op->prm.clover_traceless;
        op->tmp[2].ensure(4 * (size_t)fb(F64, g) * 2);
        op->tmp[3].ensure(4 * (size_t)fb(fp, g) * 2);
        if (eo) {
            const FieldView X = c.x64;
            const FieldView Y = c.y64;
            const FieldView Z = parity_view(op->tmp[2].ptr, F64, g, 1);
            const FieldView W = parity_view(op->tmp[2].ptr + fb(F64, g), F64, g, 1);
            c.apply(Y, X, false);
            // Z = A_oo^-1 H_oe X, W = A_oo^-1 H_eo^dag Y (A_oo = 1 without clover)
            hop(op, F64, Z, X, 1, false, 2, true, nullptr, 1.0, 0, nullptr, s);
            hop(op, F64, W, Y, 1, true, 2, true, nullptr, 1.0, 0, nullptr, s);
            if (op->has_clover) {
                ia.a[0] = Y; ia.b[0] = X; ia.c[0] = op->prm.csw * op->prm.kappa / 4;
                ia.a[1] = W; ia.b[1] = Z;
                ia.c[1] = op->prm.csw * op->prm.kappa * op->prm.kappa * op->prm.kappa / 4;
            }
            FieldView Xf = X, Yf = Y, Zf = Z, Wf = W;
            if (fp != F64) {
                char *b = op->tmp[3].ptr;
                Xf = parity_view(b, fp, g, 1);
                Yf = parity_view(b + fb(fp, g), fp, g, 1);
                Zf = parity_view(b + 2 * fb(fp, g), fp, g, 1);
                Wf = parity_view(b + 3 * fb(fp, g), fp, g, 1);
                LQ_HIP(launch_copy(Xf, X, c.sc, 1, false, s));
                LQ_HIP(launch_copy(Yf, Y, c.sc, 1, false, s));
                LQ_HIP(launch_copy(Zf, Z, c.sc, 1, false, s));
                LQ_HIP(launch_copy(Wf, W, c.sc, 1, false, s));
            }
            // even x: P(Y(x), Z(x+mu)) + Q^dag(X(x), W(x+mu)); odd x: Q^dag(Z(x), Y(x+mu)) + P(W(x), X(x+mu))
            f.a[0] = Yf; f.b[0] = Zf; f.c[0] = Xf; f.d[0] = Wf;
            f.a[1] = Wf; f.b[1] = Xf; f.c[1] = Zf; f.d[1] = Yf;
            f.coef = 2.0 * op->prm.kappa * op->prm.kappa;
        } else {
            const FieldView X = c.x64;  // full: [parity] slices
            const FieldView Y = c.y64;
            c.apply(Y, X, false);
            if (op->has_clover)
                for (int p = 0; p < 2; ++p) {
                    ia.a[p] = FieldView{Y.base + p * Y.rs, F64, (long)g.vh, Y.rs, 1};
                    ia.b[p] = FieldView{X.base + p * X.rs, F64, (long)g.vh, X.rs, 1};
                    ia.c[p] = op->prm.csw * op->prm.kappa / 4;
                }
            FieldView Xs = X, Ys = Y;
            if (fp != F64) {
                char *b = op->tmp[3].ptr;
                Xs = FieldView{b, fp, (long)g.vh, fb(fp, g), 2};
                Ys = FieldView{b + 2 * fb(fp, g), fp, (long)g.vh, fb(fp, g), 2};
                LQ_HIP(launch_copy(Xs, X, c.sc, 2, false, s));
                LQ_HIP(launch_copy(Ys, Y, c.sc, 2, false, s));
            }
            for (int p = 0; p < 2; ++p) {
                const FieldView Xp{Xs.base + p * Xs.rs, fp, (long)g.vh, Xs.rs, 1};
                const FieldView Xq{Xs.base + (1 - p) * Xs.rs, fp, (long)g.vh, Xs.rs, 1};
                const FieldView Yp{Ys.base + p * Ys.rs, fp, (long)g.vh, Ys.rs, 1};
                const FieldView Yq{Ys.base + (1 - p) * Ys.rs, fp, (long)g.vh, Ys.rs, 1};
                f.a[p] = Yp; f.b[p] = Xq; f.c[p] = Xp; f.d[p] = Yq;
            }
            f.coef = 2.0 * op->prm.kappa;
        }
        if (dSdU || G) {
            LQ_HIP(launch_force(f, fp, op->nl(fp), s));
            if (op->has_clover) {
                // the clover part, in FP64 whatever the force precision
                op->force_ws.ensure(12 * (size_t)Planes<double, 18>::field_bytes(g.vh));
                ia.gam = op->force_ws.ptr;
                CloverForceArgs cf{};
                cf.g = g;
                cf.links64 = op->links[F64].ptr;
                cf.gam = ia.gam;
                cf.M = f.M;
                cf.G = f.G;
                LQ_HIP(launch_clover_force(ia, cf, s));
            }
        }
        if (X_out) {
            if (eo) LQ_HIP(launch_unpack_spinor(g, 0, 1, c.x64, static_cast<double *>(X_out), s));
            else
                for (int p = 0; p < 2; ++p)
                    LQ_HIP(launch_unpack_spinor(
                        g, p, 0, FieldView{c.x64.base + p * fb(F64, g), F64, (long)g.vh, 2 * fb(F64, g), 1},
                        static_cast<double *>(X_out), s));
        }
        LQ_HIP(hipEventRecord(op->ev_out, s));
        LQ_HIP(hipStreamWaitEvent(us, op->ev_out, 0));
        LQ_HIP(hipStreamSynchronize(s));
        if (S) *S = Sval;
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        const bool conv = diff <= sp->tol;
        if (stats) {
            stats->nconv = os.iters[0];
            stats->nouter = os.outer[0];
            stats->restarts = os.restarts[0];
            stats->converged = conv;
            stats->diff = diff;
            stats->t_solve_ms = ms;
            stats->hop_bytes = c.hop_bytes;
            stats->n_hop = (int)c.n_hop;
        }
        return conv ? LQ_OK : LQ_NOT_CONVERGED;
    } catch (const Failure &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return LQ_ERR_STATE;
    }
}

}  // namespace lq

extern "C" lq_status lq_pf_force(lq_op *op, const lq_solver_params *sp, int variant, lq_prec force_prec,
                                 const void *phi, void *dSdU, void *G, void *X_out, double *S,
                                 lq_solve_stats *stats, void *stream)
{
    return lq::pf_force_guess(op, sp, variant, force_prec, phi, dSdU, G, X_out, S, stats, stream, nullptr);
}
