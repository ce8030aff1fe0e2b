/*
 * oracle_driver.c -- runs the C oracle (oracle/lqoracle.c) on one lattice
 * for the host sanitizer test: reads the input file written by the test,
 * computes the clover field, D psi, D^dag psi, H psi and the inverse of the
 * site blocks 1 + F, and writes them to the output file.  Built with
 * AddressSanitizer and UndefinedBehaviorSanitizer together with the oracle,
 * so every out-of-range access or undefined operation in those paths ends
 * the run with a report.
 *
 * Input (little-endian): int dims[4]; double kappa, csw; double bc[4][2];
 * complex double U[V][4][3][3]; complex double psi[V][4][3].
 * Output: F[V][12][12], D psi, D^dag psi, H psi [V][12], (1 + F)^-1 [V][12][12]
 * (complex double), then the number of singular blocks as a long.
 */
#include <complex.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;

void lqo_dirac(const int *L, const cplx *U, const cplx *bc, double kappa, const cplx *F, const cplx *in, cplx *out,
               int dagger);
void lqo_hop(const int *L, const cplx *U, const cplx *bc, const cplx *in, cplx *out, int dagger);
void lqo_clover(const int *L, const cplx *U, double csw, double kappa, int traceless, cplx *F);
long lqo_site_invert(long n, const cplx *M, cplx *Minv);

static void *read_n(FILE *f, size_t bytes)
{
    void *p = malloc(bytes);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 2;
    int L[4];
    double kc[2];
    cplx bc[4];
    if (fread(L, sizeof L, 1, in) != 1 || fread(kc, sizeof kc, 1, in) != 1 || fread(bc, sizeof bc, 1, in) != 1)
        return 2;
    const long V = (long)L[0] * L[1] * L[2] * L[3];
    cplx *U = read_n(in, sizeof(cplx) * V * 36);
    cplx *psi = read_n(in, sizeof(cplx) * V * 12);
    fclose(in);
    cplx *F = calloc((size_t)V * 144, sizeof(cplx));
    cplx *A = calloc((size_t)V * 144, sizeof(cplx));
    cplx *Ainv = calloc((size_t)V * 144, sizeof(cplx));
    cplx *d = calloc((size_t)V * 12, sizeof(cplx));
    cplx *dd = calloc((size_t)V * 12, sizeof(cplx));
    cplx *h = calloc((size_t)V * 12, sizeof(cplx));
    if (!F || !A || !Ainv || !d || !dd || !h) return 3;
    lqo_clover(L, U, kc[1], kc[0], 1, F);
    lqo_dirac(L, U, bc, kc[0], F, psi, d, 0);
    lqo_dirac(L, U, bc, kc[0], F, psi, dd, 1);
    lqo_hop(L, U, bc, psi, h, 0);
    for (long x = 0; x < V; ++x)
        for (int i = 0; i < 12; ++i)
            for (int j = 0; j < 12; ++j) A[x * 144 + i * 12 + j] = F[x * 144 + i * 12 + j] + (i == j ? 1.0 : 0.0);
    const long nsing = lqo_site_invert(V, A, Ainv);
    FILE *out = fopen(argv[2], "wb");
    if (!out) return 2;
    fwrite(F, sizeof(cplx), (size_t)V * 144, out);
    fwrite(d, sizeof(cplx), (size_t)V * 12, out);
    fwrite(dd, sizeof(cplx), (size_t)V * 12, out);
    fwrite(h, sizeof(cplx), (size_t)V * 12, out);
    fwrite(Ainv, sizeof(cplx), (size_t)V * 144, out);
    fwrite(&nsing, sizeof nsing, 1, out);
    fclose(out);
    free(U), free(psi), free(F), free(A), free(Ainv), free(d), free(dd), free(h);
    return 0;
}
