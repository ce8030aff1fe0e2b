/*
 * lqoracle.c -- plain FP64 CPU reference of the clover (O(a)-improved Wilson)
 * fermion matrix of Akahoshi et al., "General purpose lattice QCD code set
 * Bridge++ 2.0 for high performance computing", Sec. 3, eq. (1):
 *
 *   D_{x,y} = [1 + F(x)] delta_{x,y}
 *           - kappa sum_mu [ (1 - gamma_mu) U_mu(x) delta_{x+mu,y}
 *                          + (1 + gamma_mu) U_mu(x-mu)^dag delta_{x-mu,y} ]
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP path is
 * checked against.  It shares no code with the HIP library; only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * It is deliberately plain: the full 4x4 spin matrices (1 -/+ gamma_mu) are
 * applied to all four spin components (no half-spinor projection), every
 * site is handled independently, and all arithmetic is complex double.  The
 * only parallelism is an OpenMP loop over output sites.
 *
 * Conventions (the paper fixes none of these; the readings are listed in the
 * design notes):
 *  - dims L = (Lx, Ly, Lz, Lt); site index lex = x + Lx*(y + Ly*(z + Lz*t)).
 *  - direction mu = 0..3 is x, y, z, t and uses gamma_{mu+1} of the chiral
 *    basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1,2,3),
 *    gamma_4 = [[0, 1], [1, 0]], gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4.
 *  - gauge field U[site][mu][a][b], (U psi)_a = sum_b U_ab psi_b.
 *  - spinor psi[site][spin][colour]; spin-colour index ic + 3*is.
 *  - boundary condition (the paper: imposed in each direction): a hop
 *    x -> x+mu that crosses the boundary picks up the phase bc[mu]; the
 *    backward hop across the boundary picks up conj(bc[mu]).
 *  - clover term: F(x) = -c_sw kappa sum_{mu<nu} gamma_mu gamma_nu (x) Fhat_{mu nu}(x),
 *    Fhat = (Q - Q^dag)/8 with Q the sum of the four counter-clockwise
 *    plaquettes in the (mu,nu) plane that start and end at x; optionally
 *    made traceless in colour.  The paper only states that F is a 12x12
 *    Hermitian matrix made of the links.
 *  - If L_mu = 2 the forward and backward neighbour are the same site and
 *    both terms are summed.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ---------------------------------------------------------------- gamma -- */

static cplx GAMMA[5][4][4];      /* gamma_1..gamma_4 at [0..3], gamma_5 at [4] */
static cplx ONE_MINUS[4][4][4];  /* 1 - gamma_mu */
static cplx ONE_PLUS[4][4][4];   /* 1 + gamma_mu */

static void build_gammas(void)
{
    const cplx iu = _Complex_I;
    cplx sigma[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -iu}, {iu, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GAMMA, 0, sizeof(GAMMA));
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                GAMMA[k][i][2 + j] = -iu * sigma[k][i][j];
                GAMMA[k][2 + i][j] = iu * sigma[k][i][j];
            }
    for (int i = 0; i < 2; ++i) {
        GAMMA[3][i][2 + i] = 1;
        GAMMA[3][2 + i][i] = 1;
    }
    /* gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 as a plain matrix product */
    cplx t1[4][4], t2[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += GAMMA[0][i][k] * GAMMA[1][k][j];
            t1[i][j] = s;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += t1[i][k] * GAMMA[2][k][j];
            t2[i][j] = s;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx s = 0;
            for (int k = 0; k < 4; ++k) s += t2[i][k] * GAMMA[3][k][j];
            GAMMA[4][i][j] = s;
        }
    for (int mu = 0; mu < 4; ++mu)
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                cplx d = (i == j) ? 1.0 : 0.0;
                ONE_MINUS[mu][i][j] = d - GAMMA[mu][i][j];
                ONE_PLUS[mu][i][j] = d + GAMMA[mu][i][j];
            }
}

__attribute__((constructor)) static void lqo_init(void) { build_gammas(); }

/* Copy gamma_{mu+1} (mu = 0..3) or gamma_5 (mu = 4) into out[4][4]. */
int lqo_gamma(int mu, cplx *out)
{
    if (mu < 0 || mu > 4) return -1;
    memcpy(out, GAMMA[mu], sizeof(GAMMA[mu]));
    return 0;
}

int lqo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void lqo_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------- geometry -- */

static long vol(const int *L) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords_of(const int *L, long s, int c[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int)(s % L[mu]);
        s /= L[mu];
    }
}

static long site_of(const int *L, const int c[4])
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

/* Site reached from c by a step of +1 (dir = +1) or -1 (dir = -1) along mu;
 * *wrapped is set when the step crosses the lattice boundary. */
static long step(const int *L, const int c[4], int mu, int dir, int *wrapped)
{
    int d[4] = {c[0], c[1], c[2], c[3]};
    d[mu] += dir;
    *wrapped = 0;
    if (d[mu] >= L[mu]) { d[mu] -= L[mu]; *wrapped = 1; }
    if (d[mu] < 0) { d[mu] += L[mu]; *wrapped = 1; }
    return site_of(L, d);
}

static const cplx *link(const cplx *U, long s, int mu) { return U + (s * 4 + mu) * 9; }

/* ------------------------------------------------------------------ hop -- */

/* out = sum over 8 neighbours of the hopping term of eq. (1), at one site.
 * dagger = 0: forward hop with (1 - gamma_mu) U_mu(x), backward with
 *             (1 + gamma_mu) U_mu(x-mu)^dag  (the matrix H with D = A - kappa H)
 * dagger = 1: the Hermitian conjugate H^dag: forward hop with
 *             (1 + gamma_mu) U_mu(x), backward with (1 - gamma_mu) U_mu(x-mu)^dag. */
static void hop_site(const int *L, const cplx *U, const cplx *bc, const cplx *in,
                     long x, int dagger, cplx out[12])
{
    int c[4];
    coords_of(L, x, c);
    for (int i = 0; i < 12; ++i) out[i] = 0;
    for (int mu = 0; mu < 4; ++mu) {
        const cplx(*Pf)[4] = dagger ? ONE_PLUS[mu] : ONE_MINUS[mu];
        const cplx(*Pb)[4] = dagger ? ONE_MINUS[mu] : ONE_PLUS[mu];
        int w;
        /* forward: U_mu(x) psi(x + mu) */
        long y = step(L, c, mu, +1, &w);
        cplx ph = w ? bc[mu] : 1.0;
        const cplx *u = link(U, x, mu);
        const cplx *p = in + y * 12;
        cplx t[4][3];
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) {
                cplx acc = 0;
                for (int b = 0; b < 3; ++b) acc += u[a * 3 + b] * p[s * 3 + b];
                t[s][a] = ph * acc;
            }
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) {
                cplx acc = 0;
                for (int r = 0; r < 4; ++r) acc += Pf[s][r] * t[r][a];
                out[s * 3 + a] += acc;
            }
        /* backward: U_mu(x - mu)^dag psi(x - mu) */
        y = step(L, c, mu, -1, &w);
        ph = w ? conj(bc[mu]) : 1.0;
        u = link(U, y, mu);
        p = in + y * 12;
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) {
                cplx acc = 0;
                for (int b = 0; b < 3; ++b) acc += conj(u[b * 3 + a]) * p[s * 3 + b];
                t[s][a] = ph * acc;
            }
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) {
                cplx acc = 0;
                for (int r = 0; r < 4; ++r) acc += Pb[s][r] * t[r][a];
                out[s * 3 + a] += acc;
            }
    }
}

/* out = H in (dagger = 0) or H^dag in (dagger = 1) on the whole lattice. */
void lqo_hop(const int *L, const cplx *U, const cplx *bc, const cplx *in, cplx *out, int dagger)
{
    long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) hop_site(L, U, bc, in, x, dagger, out + x * 12);
}

/* One site of D (dagger = 0) or D^dag (dagger = 1):
 *   D psi     = (1 + F) psi   - kappa H psi
 *   D^dag psi = (1 + F)^dag psi - kappa H^dag psi
 * F may be NULL (Wilson, F = 0). */
static void dirac_site(const int *L, const cplx *U, const cplx *bc, double kappa, const cplx *F,
                       const cplx *in, long x, int dagger, cplx out[12])
{
    cplx h[12];
    hop_site(L, U, bc, in, x, dagger, h);
    const cplx *p = in + x * 12;
    for (int i = 0; i < 12; ++i) {
        cplx diag = p[i];
        if (F) {
            const cplx *f = F + x * 144;
            for (int j = 0; j < 12; ++j)
                diag += (dagger ? conj(f[j * 12 + i]) : f[i * 12 + j]) * p[j];
        }
        out[i] = diag - kappa * h[i];
    }
}

void lqo_dirac(const int *L, const cplx *U, const cplx *bc, double kappa, const cplx *F,
               const cplx *in, cplx *out, int dagger)
{
    long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) dirac_site(L, U, bc, kappa, F, in, x, dagger, out + x * 12);
}

/* D or D^dag at a list of sites only: out[k] = (D in)(sites[k]).  F, if given,
 * is indexed by site like the full field. */
void lqo_dirac_sites(const int *L, const cplx *U, const cplx *bc, double kappa, const cplx *F,
                     const cplx *in, long nsites, const long *sites, cplx *out, int dagger)
{
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nsites; ++k)
        dirac_site(L, U, bc, kappa, F, in, sites[k], dagger, out + k * 12);
}

/* H or H^dag at a list of sites only. */
void lqo_hop_sites(const int *L, const cplx *U, const cplx *bc, const cplx *in,
                   long nsites, const long *sites, cplx *out, int dagger)
{
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nsites; ++k) hop_site(L, U, bc, in, sites[k], dagger, out + k * 12);
}

/* --------------------------------------------------------------- clover -- */

static void mul33(const cplx *a, const cplx *b, cplx *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += a[i * 3 + k] * b[k * 3 + j];
            c[i * 3 + j] = s;
        }
}

static void dag33(const cplx *a, cplx *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c[i * 3 + j] = conj(a[j * 3 + i]);
}

/* product of four 3x3 matrices */
static void mul4(const cplx *a, const cplx *b, const cplx *c, const cplx *d, cplx *out)
{
    cplx t1[9], t2[9];
    mul33(a, b, t1);
    mul33(t1, c, t2);
    mul33(t2, d, out);
}

static long shifted(const int *L, const int c[4], int mu, int dm, int nu, int dn)
{
    int d[4] = {c[0], c[1], c[2], c[3]};
    d[mu] = ((d[mu] + dm) % L[mu] + L[mu]) % L[mu];
    d[nu] = ((d[nu] + dn) % L[nu] + L[nu]) % L[nu];
    return site_of(L, d);
}

/* Q_{mu nu}(x): the sum of the four plaquettes in the (mu, nu) plane that
 * start and end at x, each traversed counter-clockwise (mu to nu). */
static void clover_leaves(const int *L, const cplx *U, long x, int mu, int nu, cplx Q[9])
{
    int c[4];
    coords_of(L, x, c);
    long xpm = shifted(L, c, mu, +1, nu, 0);
    long xpn = shifted(L, c, mu, 0, nu, +1);
    long xmm = shifted(L, c, mu, -1, nu, 0);
    long xmn = shifted(L, c, mu, 0, nu, -1);
    long xmmpn = shifted(L, c, mu, -1, nu, +1);
    long xmmmn = shifted(L, c, mu, -1, nu, -1);
    long xpmmn = shifted(L, c, mu, +1, nu, -1);
    cplx d1[9], d2[9], d3[9], leaf[9];
    for (int i = 0; i < 9; ++i) Q[i] = 0;

    /* x -> x+mu -> x+mu+nu -> x+nu -> x */
    dag33(link(U, xpn, mu), d1);
    dag33(link(U, x, nu), d2);
    mul4(link(U, x, mu), link(U, xpm, nu), d1, d2, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];

    /* x -> x+nu -> x+nu-mu -> x-mu -> x */
    dag33(link(U, xmmpn, mu), d1);
    dag33(link(U, xmm, nu), d2);
    mul4(link(U, x, nu), d1, d2, link(U, xmm, mu), leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];

    /* x -> x-mu -> x-mu-nu -> x-nu -> x */
    dag33(link(U, xmm, mu), d1);
    dag33(link(U, xmmmn, nu), d2);
    mul4(d1, d2, link(U, xmmmn, mu), link(U, xmn, nu), leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];

    /* x -> x-nu -> x-nu+mu -> x+mu -> x */
    dag33(link(U, xmn, nu), d1);
    dag33(link(U, x, mu), d3);
    mul4(d1, link(U, xmn, mu), link(U, xpmmn, nu), d3, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
}

static void clover_site(const int *L, const cplx *U, double csw, double kappa, int traceless,
                        long x, cplx *F /* 144 */)
{
    for (int i = 0; i < 144; ++i) F[i] = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu) {
            cplx Q[9], Fh[9];
            clover_leaves(L, U, x, mu, nu, Q);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Fh[a * 3 + b] = (Q[a * 3 + b] - conj(Q[b * 3 + a])) / 8.0;
            if (traceless) {
                cplx tr = (Fh[0] + Fh[4] + Fh[8]) / 3.0;
                Fh[0] -= tr;
                Fh[4] -= tr;
                Fh[8] -= tr;
            }
            /* gamma_mu gamma_nu */
            cplx gg[4][4];
            for (int s = 0; s < 4; ++s)
                for (int r = 0; r < 4; ++r) {
                    cplx acc = 0;
                    for (int k = 0; k < 4; ++k) acc += GAMMA[mu][s][k] * GAMMA[nu][k][r];
                    gg[s][r] = acc;
                }
            for (int s = 0; s < 4; ++s)
                for (int a = 0; a < 3; ++a)
                    for (int r = 0; r < 4; ++r)
                        for (int b = 0; b < 3; ++b)
                            F[(s * 3 + a) * 12 + r * 3 + b] += -csw * kappa * gg[s][r] * Fh[a * 3 + b];
        }
}

/* F(x) for every site: F[site][12][12], row/column index spin*3 + colour. */
void lqo_clover(const int *L, const cplx *U, double csw, double kappa, int traceless, cplx *F)
{
    long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) clover_site(L, U, csw, kappa, traceless, x, F + x * 144);
}

void lqo_clover_sites(const int *L, const cplx *U, double csw, double kappa, int traceless,
                      long nsites, const long *sites, cplx *F)
{
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nsites; ++k) clover_site(L, U, csw, kappa, traceless, sites[k], F + k * 144);
}

/* ------------------------------------------------------ site matrices --- */

/* out[x] = M[x] in[x] for n sites of 12x12 matrices. */
void lqo_site_apply(long n, const cplx *M, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (long x = 0; x < n; ++x) {
        const cplx *m = M + x * 144;
        const cplx *p = in + x * 12;
        for (int i = 0; i < 12; ++i) {
            cplx acc = 0;
            for (int j = 0; j < 12; ++j) acc += m[i * 12 + j] * p[j];
            out[x * 12 + i] = acc;
        }
    }
}

/* Inverse of each 12x12 matrix by Gauss-Jordan elimination with partial
 * pivoting.  A site whose pivot falls below 1e-14 times the largest entry
 * magnitude is singular: its output is left as zeros.  Returns the number
 * of singular sites. */
long lqo_site_invert(long n, const cplx *M, cplx *Minv)
{
    long nsing = 0;
#pragma omp parallel for schedule(static) reduction(+ : nsing)
    for (long x = 0; x < n; ++x) {
        cplx a[12][24];
        double scale = 0;
        for (int i = 0; i < 12; ++i)
            for (int j = 0; j < 12; ++j) {
                a[i][j] = M[x * 144 + i * 12 + j];
                a[i][12 + j] = (i == j) ? 1.0 : 0.0;
                if (cabs(a[i][j]) > scale) scale = cabs(a[i][j]);
            }
        int sing = 0;
        for (int col = 0; col < 12 && !sing; ++col) {
            int piv = col;
            for (int r = col + 1; r < 12; ++r)
                if (cabs(a[r][col]) > cabs(a[piv][col])) piv = r;
            if (!(cabs(a[piv][col]) > 1e-14 * scale)) { sing = 1; break; }
            if (piv != col)
                for (int j = 0; j < 24; ++j) {
                    cplx t = a[col][j];
                    a[col][j] = a[piv][j];
                    a[piv][j] = t;
                }
            cplx inv = 1.0 / a[col][col];
            for (int j = 0; j < 24; ++j) a[col][j] *= inv;
            for (int r = 0; r < 12; ++r) {
                if (r == col) continue;
                cplx f = a[r][col];
                if (f == 0) continue;
                for (int j = 0; j < 24; ++j) a[r][j] -= f * a[col][j];
            }
        }
        for (int i = 0; i < 12; ++i)
            for (int j = 0; j < 12; ++j) Minv[x * 144 + i * 12 + j] = sing ? 0.0 : a[i][12 + j];
        nsing += sing;
    }
    return nsing;
}

/* ---------------------------------------------------------------- force -- */

/* Derivative of Re[a^dag H b] with respect to every link, as the 3x3 matrix
 * M_mu(x) with  delta Re[a^dag H b] = sum_{x,mu} Re tr( M_mu(x) delta U_mu(x) ).
 * U_mu(x) enters H twice: in the forward hop at x,
 *     a(x)^dag (1 - gamma_mu) U_mu(x) ph b(x+mu),
 * giving  P = ph sum_s [(1 - gamma_mu) b(x+mu)]_s a(x)_s^dag  (colour outer product),
 * and in the backward hop at x+mu,
 *     a(x+mu)^dag (1 + gamma_mu) U_mu(x)^dag conj(ph) b(x),
 * whose real part equals Re tr(delta U  Q^dag) with
 *     Q = conj(ph) sum_s [(1 + gamma_mu) b(x)]_s a(x+mu)_s^dag,
 * so M_mu(x) = P + Q^dag.  The result is added to Macc[site][mu][3][3]
 * scaled by coef. */
void lqo_hop_link_derivative(const int *L, const cplx *bc, const cplx *a, const cplx *b,
                             double coef, cplx *Macc)
{
    long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        int c[4];
        coords_of(L, x, c);
        for (int mu = 0; mu < 4; ++mu) {
            int w;
            long y = step(L, c, mu, +1, &w);
            cplx ph = w ? bc[mu] : 1.0;
            cplx pb[4][3], qb[4][3];
            for (int s = 0; s < 4; ++s)
                for (int col = 0; col < 3; ++col) {
                    cplx accp = 0, accq = 0;
                    for (int r = 0; r < 4; ++r) {
                        accp += ONE_MINUS[mu][s][r] * b[y * 12 + r * 3 + col];
                        accq += ONE_PLUS[mu][s][r] * b[x * 12 + r * 3 + col];
                    }
                    pb[s][col] = accp;
                    qb[s][col] = accq;
                }
            cplx *m = Macc + (x * 4 + mu) * 9;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    /* P_ij = ph sum_s pb[s][i] conj(a(x)[s][j]) */
                    cplx P = 0, Qji = 0;
                    for (int s = 0; s < 4; ++s) {
                        P += pb[s][i] * conj(a[x * 12 + s * 3 + j]);
                        /* Q_ji = conj(ph) sum_s qb[s][j] conj(a(y)[s][i]);
                         * (Q^dag)_ij = conj(Q_ji) */
                        Qji += qb[s][j] * conj(a[y * 12 + s * 3 + i]);
                    }
                    P *= ph;
                    Qji *= conj(ph);
                    m[i * 3 + j] += coef * (P + conj(Qji));
                }
        }
    }
}
