/* Host-only driver for a sanitizer build of the oracle (address and
 * undefined-behaviour checks): calls every exported oracle routine once on a
 * small seeded problem, including the error paths (zero pivot, non-finite
 * norm), and prints a checksum.  Built and run by
 * tests/test_oracle_sanitize.py with gcc; no GPU involved. */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zc;

void orc_lindblad_rhs(int d, const zc *H, int K, const zc *Lk, const zc *rho, zc *out);
void orc_liouvillian(int d, const zc *H, int K, const zc *Lk, zc *Lout);
void orc_matvec(int n, const zc *P, const zc *x, zc *y);
void orc_propagate(int n, const zc *P, int B, zc *rho, long long nsteps, int nthreads);
double orc_norm1(int n, const zc *A);
int orc_scaling_exponent(double norm1, double theta);
void orc_pade13_coefficients(double *b);
int orc_lu_solve(int n, zc *A, zc *B, int nrhs);
int orc_expm_pade13(int n, const zc *A0, double theta, zc *P, int *s_out);
int orc_propagators(int n, int M, const zc *L, const double *dt, double theta, zc *P, int *s_out);
void orc_expm_taylor_ld(int n, const zc *A0, zc *P);
void orc_rk4_ld(int d, const zc *H, int K, const zc *Lk, zc *rho, double dt, long long nsteps, int sub);
void orc_taylor_steps_ld(int d, const zc *H, int K, const zc *Lk, zc *rho, double dt, long long nsteps);
int orc_expm_frechet_blocktri(int n, const zc *A, const zc *E, double theta, zc *expA, zc *Lfr);
int orc_grape(int n, int M, int C, const zc *L0, const zc *Lc, const double *u, double dt, double theta,
              const zc *x0, const zc *w, double *F, double *grad, const unsigned char *mask);
void orc_quantize_q15(long long count, const zc *src, int16_t *re, int16_t *im);
void orc_propagate_q15(int n, const int16_t *Pr, const int16_t *Pi, int B, int16_t *xr, int16_t *xi,
                       long long nsteps);
void orc_quantize_q31(long long count, const zc *src, int32_t *re, int32_t *im);
void orc_propagate_q31(int n, const int32_t *Pr, const int32_t *Pi, int B, int32_t *xr, int32_t *xi,
                       long long nsteps);

static uint64_t rng = 0x9e3779b97f4a7c15ull;
static double urand(void) /* splitmix64 -> [-1, 1) */
{
    uint64_t z = (rng += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

static void fill(zc *a, size_t count, double scale)
{
    for (size_t e = 0; e < count; ++e) a[e] = scale * (urand() + I * urand());
}

int main(void)
{
    const int d = 3, n = 9, K = 2, M = 2, C = 2;
    double sum = 0;
    zc *H = malloc(d * d * sizeof(zc)), *Lk = malloc(K * d * d * sizeof(zc));
    zc *rho = malloc(d * d * sizeof(zc)), *out = malloc(d * d * sizeof(zc));
    zc *L = malloc(n * n * sizeof(zc)), *P = malloc(n * n * sizeof(zc)), *A = malloc(n * n * sizeof(zc));
    fill(H, d * d, 0.5);
    fill(Lk, K * d * d, 0.2);
    fill(rho, d * d, 0.3);
    orc_lindblad_rhs(d, H, K, Lk, rho, out);
    orc_liouvillian(d, H, K, Lk, L);
    for (int e = 0; e < n * n; ++e) A[e] = 0.5 * L[e];
    int s = -1;
    if (orc_expm_pade13(n, A, 0.25, P, &s) != 0) return 1;
    sum += creal(P[3]) + s;
    zc *Ps = malloc(M * n * n * sizeof(zc)), *Ls = malloc(M * n * n * sizeof(zc));
    double dts[2] = {0.5, 1.0};
    int ss[2];
    memcpy(Ls, L, n * n * sizeof(zc));
    memcpy(Ls + n * n, L, n * n * sizeof(zc));
    if (orc_propagators(n, M, Ls, dts, 0.25, Ps, ss) != 0) return 2;
    zc *X = malloc(3 * n * sizeof(zc)), *y = malloc(n * sizeof(zc));
    fill(X, 3 * n, 0.1);
    orc_matvec(n, P, X, y);
    orc_propagate(n, P, 3, X, 5, 2);
    sum += creal(X[4]) + creal(y[2]);
    double b[14];
    orc_pade13_coefficients(b);
    sum += b[13];
    zc *Z = calloc(n * n, sizeof(zc)), *R = malloc(n * n * sizeof(zc));
    fill(R, n * n, 1.0);
    if (orc_lu_solve(n, Z, R, n) != -5) return 3; /* zero pivot */
    Z[4] = NAN;
    if (orc_expm_pade13(n, Z, 0.25, P, &s) != -6) return 4; /* non-finite norm */
    sum += orc_scaling_exponent(orc_norm1(n, A), 0.25);
    orc_expm_taylor_ld(n, A, P);
    sum += cimag(P[7]);
    memcpy(out, rho, d * d * sizeof(zc));
    orc_rk4_ld(d, H, K, Lk, out, 0.1, 3, 4);
    orc_taylor_steps_ld(d, H, K, Lk, rho, 0.1, 3);
    sum += creal(out[0]) + creal(rho[0]);
    zc *E = malloc(n * n * sizeof(zc)), *Lf = malloc(n * n * sizeof(zc));
    fill(E, n * n, 0.1);
    if (orc_expm_frechet_blocktri(n, A, E, 0.25, P, Lf) != 0) return 5;
    sum += creal(Lf[5]);
    zc *Lc = malloc(C * n * n * sizeof(zc));
    fill(Lc, C * n * n, 0.1);
    double u[4] = {0.1, -0.2, 0.05, 0.3}, F = 0, grad[4];
    unsigned char mask[2] = {1, 0};
    zc *x0 = malloc(n * sizeof(zc)), *w = malloc(n * sizeof(zc));
    fill(x0, n, 0.3);
    fill(w, n, 0.3);
    if (orc_grape(n, M, C, L, Lc, u, 0.5, 0.25, x0, w, &F, grad, NULL) != 0) return 6;
    if (orc_grape(n, M, C, L, Lc, u, 0.5, 0.25, x0, w, &F, grad, mask) != 0) return 7;
    sum += F + grad[0];
    int16_t pr[81], pi[81], xr[18], xi[18];
    int32_t qr[81], qi[81], yr[18], yi[18];
    orc_quantize_q15(n * n, Ps, pr, pi);
    orc_quantize_q15(2 * n, X, xr, xi);
    orc_propagate_q15(n, pr, pi, 2, xr, xi, 7);
    orc_quantize_q31(n * n, Ps, qr, qi);
    orc_quantize_q31(2 * n, X, yr, yi);
    orc_propagate_q31(n, qr, qi, 2, yr, yi, 7);
    sum += xr[3] + yr[3] * 0x1.0p-31;
    printf("checksum %.17g\n", sum);
    free(H); free(Lk); free(rho); free(out); free(L); free(P); free(A); free(Ps); free(Ls);
    free(X); free(y); free(Z); free(R); free(E); free(Lf); free(Lc); free(x0); free(w);
    return 0;
}
