/*
 * Plain, slow, obviously correct CPU oracle for dense time-independent
 * Lindblad propagation.  TEST INFRASTRUCTURE ONLY: the test suite, the smoke
 * check and the benchmark's CPU-baseline leg call it; the library never does.
 *
 * Everything is FP64 (C99 `double complex`, row-major, interleaved re/im);
 * the brute-force references are long double.  No BLAS, no blocking, no
 * fusion.  Compile without -ffast-math.
 *
 * Paper: "Hardware-Aware Performance Characterization of Small Dense Lindblad
 * Propagation for Near-Term Quantum Control" (arXiv 2603.18052).
 *   Eq. (1)  Lindblad master equation                       -> orc_lindblad_rhs
 *   Eqs. (2)-(3)  vec rho(t+dt) = P vec rho(t), P = e^{L dt} -> orc_liouvillian
 *   Alg. 1   scaling and squaring of the [13/13] Pade approximant,
 *            theta = 0.25, LU with partial pivoting of the
 *            denominator                                      -> orc_expm_pade13
 *   Alg. 2   row-major dense complex matvec                   -> orc_matvec
 *   Alg. 3   batch of independent states over threads         -> orc_propagate
 *   Alg. 5   fixed-point step (Q1.15, and Q1.31 as in the paper's drift
 *            figure): exact integer sums, floor truncation and
 *            saturation                   -> orc_propagate_q15, orc_propagate_q31
 * The GRAPE gradient (not in the paper) follows the chain rule with the
 * Frechet derivative of exp taken from the block-triangular identity
 * exp([[A, E], [0, A]]) = [[e^A, L(A,E)], [0, e^A]]   (Van Loan 1978).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zc;
typedef long double complex lzc;

#define ORC_OK 0
#define ORC_ENOMEM (-3)
#define ORC_ESINGULAR (-5)
#define ORC_ENONFINITE (-6)

/* ------------------------------------------------------------------ basics */
/* C = A B, n x n.  Every entry is the plain sum over k in ascending order;
 * the loops run k outside j so that rows of B are read contiguously, and
 * rows of C are independent, so they are shared over threads. */
static void mm(int n, const zc *A, const zc *B, zc *C)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if (n >= 128)
#endif
    for (int i = 0; i < n; ++i) {
        zc *c = C + (size_t)i * n;
        for (int j = 0; j < n; ++j) c[j] = 0;
        for (int k = 0; k < n; ++k) {
            const zc a = A[(size_t)i * n + k];
            const zc *b = B + (size_t)k * n;
            for (int j = 0; j < n; ++j) c[j] += a * b[j];
        }
    }
}

/* Eq. (1) applied to one d x d matrix rho, by plain matrix arithmetic:
 *   out = -i (H rho - rho H) + sum_k ( Lk rho Lk^dag - 1/2 Lk^dag Lk rho - 1/2 rho Lk^dag Lk ). */
void orc_lindblad_rhs(int d, const zc *H, int K, const zc *Lk, const zc *rho, zc *out)
{
    size_t dd = (size_t)d * d;
    zc *t1 = malloc(dd * sizeof(zc)), *t2 = malloc(dd * sizeof(zc));
    zc *Ld = malloc(dd * sizeof(zc)), *LdL = malloc(dd * sizeof(zc));
    mm(d, H, rho, t1);
    mm(d, rho, H, t2);
    for (size_t e = 0; e < dd; ++e) out[e] = -I * (t1[e] - t2[e]);
    for (int k = 0; k < K; ++k) {
        const zc *L = Lk + (size_t)k * dd;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) Ld[(size_t)i * d + j] = conj(L[(size_t)j * d + i]);
        mm(d, L, rho, t1);
        mm(d, t1, Ld, t2); /* L rho L^dag */
        for (size_t e = 0; e < dd; ++e) out[e] += t2[e];
        mm(d, Ld, L, LdL);
        mm(d, LdL, rho, t1);
        mm(d, rho, LdL, t2);
        for (size_t e = 0; e < dd; ++e) out[e] -= 0.5 * (t1[e] + t2[e]);
    }
    free(t1); free(t2); free(Ld); free(LdL);
}

/* The superoperator of Eq. (1) in the row-major vectorisation the paper uses
 * (the d x d array is the n-vector, Alg. 2 storage note): column c of L is
 * vec(rhs(E_c)), with E_c the basis matrix that has a single 1 at row c / d,
 * column c % d.  n = d*d; Lout is n x n row-major. */
void orc_liouvillian(int d, const zc *H, int K, const zc *Lk, zc *Lout)
{
    int n = d * d;
    zc *E = calloc((size_t)n, sizeof(zc)), *col = malloc((size_t)n * sizeof(zc));
    for (int c = 0; c < n; ++c) {
        memset(E, 0, (size_t)n * sizeof(zc));
        E[c] = 1.0;
        orc_lindblad_rhs(d, H, K, Lk, E, col);
        for (int r = 0; r < n; ++r) Lout[(size_t)r * n + c] = col[r];
    }
    free(E); free(col);
}

/* Alg. 2: y = P x, one accumulator per output row. */
void orc_matvec(int n, const zc *P, const zc *x, zc *y)
{
    for (int i = 0; i < n; ++i) {
        zc a = 0;
        for (int j = 0; j < n; ++j) a += P[(size_t)i * n + j] * x[j];
        y[i] = a;
    }
}

/* Alg. 3: B independent states (rho is B x n, in place), nsteps applications
 * of Alg. 2 each; the states are split over `nthreads` threads in static
 * chunks, the steps of one state stay sequential. */
void orc_propagate(int n, const zc *P, int B, zc *rho, long long nsteps, int nthreads)
{
#ifdef _OPENMP
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int b = 0; b < B; ++b) {
        zc *x = rho + (size_t)b * n;
        zc *y = malloc((size_t)n * sizeof(zc));
        for (long long t = 0; t < nsteps; ++t) {
            orc_matvec(n, P, x, y);
            memcpy(x, y, (size_t)n * sizeof(zc));
        }
        free(y);
    }
}

/* ------------------------------------------------------------- Alg. 1 */
/* ||A||_1: the largest column sum of complex moduli. */
double orc_norm1(int n, const zc *A)
{
    double best = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += cabs(A[(size_t)i * n + j]);
        if (isnan(s)) return s; /* a NaN column makes the norm undefined */
        if (s > best) best = s;
    }
    return best;
}

/* Scaling exponent of Alg. 1: the smallest s >= 0 with ||A||_1 <= theta 2^s
 * (the ceil(log2(||A||_1/theta)) rule with the exact-power and zero-norm
 * cases taken by exact comparison).  Returns -1 for a non-finite norm. */
int orc_scaling_exponent(double norm1, double theta)
{
    if (!isfinite(norm1)) return -1;
    int s = 0;
    while (norm1 > ldexp(theta, s)) ++s;
    return s;
}

/* Pade [13/13] coefficients b_k = (26-k)! / (k! (13-k)!)  (numerator of the
 * diagonal Pade approximant of exp, scaled so that b_13 = 1), exact integers
 * computed in 128-bit arithmetic and rounded once to double. */
void orc_pade13_coefficients(double *b)
{
    for (int k = 0; k <= 13; ++k) {
        unsigned __int128 num = 1; /* (26-k)! / (13-k)! = prod_{j=14-k}^{26-k} j */
        for (int j = 14 - k; j <= 26 - k; ++j) num *= (unsigned __int128)j;
        unsigned __int128 den = 1; /* k! */
        for (int j = 2; j <= k; ++j) den *= (unsigned __int128)j;
        /* (26-k)!/((13-k)! k!) = num / den ; exact division */
        b[k] = (double)(num / den);
    }
}

/* LU with partial pivoting (largest modulus in the column, lowest row index
 * on ties) of A (n x n, overwritten by unit-lower L and U), applied to the
 * n x nrhs right-hand side B, which is overwritten by the solution of
 * A X = B.  Returns ORC_ESINGULAR on a zero pivot. */
int orc_lu_solve(int n, zc *A, zc *B, int nrhs)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = cabs(A[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = cabs(A[(size_t)i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        if (!(best > 0.0)) return ORC_ESINGULAR;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                zc t = A[(size_t)k * n + j]; A[(size_t)k * n + j] = A[(size_t)p * n + j]; A[(size_t)p * n + j] = t;
            }
            for (int j = 0; j < nrhs; ++j) {
                zc t = B[(size_t)k * nrhs + j]; B[(size_t)k * nrhs + j] = B[(size_t)p * nrhs + j]; B[(size_t)p * nrhs + j] = t;
            }
        }
        zc piv = A[(size_t)k * n + k];
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if (n - k >= 256)
#endif
        for (int i = k + 1; i < n; ++i) { /* rows are independent */
            zc l = A[(size_t)i * n + k] / piv;
            A[(size_t)i * n + k] = l;
            for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
        }
    }
    /* forward substitution with the unit lower factor, then back substitution
     * with U; the right-hand-side columns are independent */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if (nrhs >= 128)
#endif
    for (int j = 0; j < nrhs; ++j) {
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < i; ++k) B[(size_t)i * nrhs + j] -= A[(size_t)i * n + k] * B[(size_t)k * nrhs + j];
        for (int i = n - 1; i >= 0; --i) {
            for (int k = i + 1; k < n; ++k) B[(size_t)i * nrhs + j] -= A[(size_t)i * n + k] * B[(size_t)k * nrhs + j];
            B[(size_t)i * nrhs + j] /= A[(size_t)i * n + i];
        }
    }
    return ORC_OK;
}

/* P = exp(A) for an already scaled generator A = L dt, by the scaling and
 * squaring method of Alg. 1 around the diagonal [13/13] Pade approximant of
 * exp (Higham 2005).  With p(X) = sum_k b_k X^k (coefficients above) the
 * approximant is r(X) = p(-X)^{-1} p(X).  Written as its even part
 * E(X) = sum_j b_{2j} X^{2j} and odd part O(X) = X sum_j b_{2j+1} X^{2j},
 * p(X) = E + O and p(-X) = E - O, so one set of even powers of X serves both
 * polynomials; here they are formed one after another (X^2, X^4, ..., X^12)
 * and summed term by term, the plain definition of the polynomial.  Then
 * X = A / 2^s with s the scaling exponent, P = r(X) solved from
 * (E - O) P = (E + O) by the pivoted LU above, and P squared s times.
 * Returns 0, ORC_ESINGULAR, ORC_ENONFINITE or ORC_ENOMEM; *s_out = s. */
int orc_expm_pade13(int n, const zc *A0, double theta, zc *P, int *s_out)
{
    size_t nn = (size_t)n * n;
    double b[14];
    orc_pade13_coefficients(b);
    int s = orc_scaling_exponent(orc_norm1(n, A0), theta);
    if (s_out) *s_out = s;
    if (s < 0) return ORC_ENONFINITE;
    zc *X = malloc(nn * sizeof(zc)), *X2 = malloc(nn * sizeof(zc)), *Pw = malloc(nn * sizeof(zc));
    zc *T = malloc(nn * sizeof(zc)), *Ev = calloc(nn, sizeof(zc)), *Od = calloc(nn, sizeof(zc));
    zc *Den = malloc(nn * sizeof(zc));
    if (!X || !X2 || !Pw || !T || !Ev || !Od || !Den) {
        free(X); free(X2); free(Pw); free(T); free(Ev); free(Od); free(Den);
        return ORC_ENOMEM;
    }
    for (size_t e = 0; e < nn; ++e) X[e] = ldexp(creal(A0[e]), -s) + I * ldexp(cimag(A0[e]), -s);
    mm(n, X, X, X2);
    /* Pw runs through X^0, X^2, ..., X^12; Ev collects b_{2j} X^{2j} and Od
     * (before the final product with X) b_{2j+1} X^{2j}. */
    memset(Pw, 0, nn * sizeof(zc));
    for (int i = 0; i < n; ++i) Pw[(size_t)i * n + i] = 1.0;
    for (int j = 0; j <= 6; ++j) {
        if (j > 0) {
            mm(n, Pw, X2, T);
            memcpy(Pw, T, nn * sizeof(zc));
        }
        for (size_t e = 0; e < nn; ++e) {
            Ev[e] += b[2 * j] * Pw[e];
            Od[e] += b[2 * j + 1] * Pw[e];
        }
    }
    mm(n, X, Od, T); /* T = O(X) */
    for (size_t e = 0; e < nn; ++e) { Den[e] = Ev[e] - T[e]; P[e] = Ev[e] + T[e]; }
    int rc = orc_lu_solve(n, Den, P, n);
    if (rc == ORC_OK) {
        for (int k = 0; k < s; ++k) {
            mm(n, P, P, T);
            memcpy(P, T, nn * sizeof(zc));
        }
    }
    free(X); free(X2); free(Pw); free(T); free(Ev); free(Od); free(Den);
    return rc;
}

/* P = exp(L dt) for M generators (L is M x n x n), one build per generator
 * (the segment builds of the GRAPE landscape point); s_out has M entries. */
int orc_propagators(int n, int M, const zc *L, const double *dt, double theta, zc *P, int *s_out)
{
    size_t nn = (size_t)n * n;
    zc *A = malloc(nn * sizeof(zc));
    if (!A) return ORC_ENOMEM;
    int rc = ORC_OK;
    for (int m = 0; m < M && rc == ORC_OK; ++m) {
        for (size_t e = 0; e < nn; ++e) A[e] = L[(size_t)m * nn + e] * dt[m];
        rc = orc_expm_pade13(n, A, theta, P + (size_t)m * nn, s_out ? s_out + m : NULL);
    }
    free(A);
    return rc;
}

/* ------------------------------------------------ long-double references */
static double lnorm1(int n, const lzc *A)
{
    long double best = 0;
    for (int j = 0; j < n; ++j) {
        long double s = 0;
        for (int i = 0; i < n; ++i) s += cabsl(A[(size_t)i * n + j]);
        if (s > best) best = s;
    }
    return (double)best;
}

/* exp(A) in long double by the scaled Taylor series: A / 2^k with norm <= 1/2,
 * terms summed until one drops below 1e-22 of the running sum's norm, then
 * k squarings; the result is rounded to double. */
void orc_expm_taylor_ld(int n, const zc *A0, zc *P)
{
    size_t nn = (size_t)n * n;
    lzc *A = malloc(nn * sizeof(lzc)), *S = malloc(nn * sizeof(lzc));
    lzc *Tm = malloc(nn * sizeof(lzc)), *Tn = malloc(nn * sizeof(lzc));
    for (size_t e = 0; e < nn; ++e) A[e] = (lzc)A0[e];
    int k = 0;
    double nrm = lnorm1(n, A);
    while (nrm > 0.5) { nrm *= 0.5; ++k; }
    for (size_t e = 0; e < nn; ++e) A[e] = A[e] / (long double)ldexpl(1.0L, k);
    for (size_t e = 0; e < nn; ++e) { S[e] = 0; Tm[e] = 0; }
    for (int i = 0; i < n; ++i) { S[(size_t)i * n + i] = 1; Tm[(size_t)i * n + i] = 1; }
    for (int m = 1; m < 200; ++m) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                lzc acc = 0;
                for (int q = 0; q < n; ++q) acc += Tm[(size_t)i * n + q] * A[(size_t)q * n + j];
                Tn[(size_t)i * n + j] = acc / (long double)m;
            }
        for (size_t e = 0; e < nn; ++e) { Tm[e] = Tn[e]; S[e] += Tn[e]; }
        if (lnorm1(n, Tm) < 1e-22 * lnorm1(n, S)) break;
    }
    for (int r = 0; r < k; ++r) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                lzc acc = 0;
                for (int q = 0; q < n; ++q) acc += S[(size_t)i * n + q] * S[(size_t)q * n + j];
                Tn[(size_t)i * n + j] = acc;
            }
        memcpy(S, Tn, nn * sizeof(lzc));
    }
    for (size_t e = 0; e < nn; ++e) P[e] = (zc)S[e];
    free(A); free(S); free(Tm); free(Tn);
}

/* Eq. (1) in long double, plain matrix arithmetic. */
static void rhs_ld(int d, const lzc *H, int K, const lzc *Lk, const lzc *rho, lzc *out, lzc *t1, lzc *t2)
{
    size_t dd = (size_t)d * d;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            lzc a = 0;
            for (int q = 0; q < d; ++q) a += H[(size_t)i * d + q] * rho[(size_t)q * d + j] - rho[(size_t)i * d + q] * H[(size_t)q * d + j];
            out[(size_t)i * d + j] = -I * a;
        }
    for (int k = 0; k < K; ++k) {
        const lzc *L = Lk + (size_t)k * dd;
        /* t1 = L rho */
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                lzc a = 0;
                for (int q = 0; q < d; ++q) a += L[(size_t)i * d + q] * rho[(size_t)q * d + j];
                t1[(size_t)i * d + j] = a;
            }
        /* out += t1 L^dag */
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                lzc a = 0;
                for (int q = 0; q < d; ++q) a += t1[(size_t)i * d + q] * conjl(L[(size_t)j * d + q]);
                out[(size_t)i * d + j] += a;
            }
        /* t2 = L^dag L */
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                lzc a = 0;
                for (int q = 0; q < d; ++q) a += conjl(L[(size_t)q * d + i]) * L[(size_t)q * d + j];
                t2[(size_t)i * d + j] = a;
            }
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                lzc a = 0;
                for (int q = 0; q < d; ++q) a += t2[(size_t)i * d + q] * rho[(size_t)q * d + j] + rho[(size_t)i * d + q] * t2[(size_t)q * d + j];
                out[(size_t)i * d + j] -= 0.5L * a;
            }
    }
}

/* Classical RK4 in long double on d rho/dt = rhs(rho) of Eq. (1) directly
 * (no superoperator), nsteps steps of dt, each split into `sub` RK4 steps. */
void orc_rk4_ld(int d, const zc *H, int K, const zc *Lk, zc *rho, double dt, long long nsteps, int sub)
{
    size_t dd = (size_t)d * d;
    lzc *h = malloc(dd * sizeof(lzc)), *L = malloc((size_t)K * dd * sizeof(lzc));
    lzc *x = malloc(dd * sizeof(lzc)), *y = malloc(dd * sizeof(lzc));
    lzc *k1 = malloc(dd * sizeof(lzc)), *k2 = malloc(dd * sizeof(lzc));
    lzc *k3 = malloc(dd * sizeof(lzc)), *k4 = malloc(dd * sizeof(lzc));
    lzc *t1 = malloc(dd * sizeof(lzc)), *t2 = malloc(dd * sizeof(lzc));
    for (size_t e = 0; e < dd; ++e) { h[e] = H[e]; x[e] = rho[e]; }
    for (size_t e = 0; e < (size_t)K * dd; ++e) L[e] = Lk[e];
    long double hs = (long double)dt / sub;
    for (long long t = 0; t < nsteps * sub; ++t) {
        rhs_ld(d, h, K, L, x, k1, t1, t2);
        for (size_t e = 0; e < dd; ++e) y[e] = x[e] + 0.5L * hs * k1[e];
        rhs_ld(d, h, K, L, y, k2, t1, t2);
        for (size_t e = 0; e < dd; ++e) y[e] = x[e] + 0.5L * hs * k2[e];
        rhs_ld(d, h, K, L, y, k3, t1, t2);
        for (size_t e = 0; e < dd; ++e) y[e] = x[e] + hs * k3[e];
        rhs_ld(d, h, K, L, y, k4, t1, t2);
        for (size_t e = 0; e < dd; ++e) x[e] += hs / 6.0L * (k1[e] + 2.0L * k2[e] + 2.0L * k3[e] + k4[e]);
    }
    for (size_t e = 0; e < dd; ++e) rho[e] = (zc)x[e];
    free(h); free(L); free(x); free(y); free(k1); free(k2); free(k3); free(k4); free(t1); free(t2);
}

/* Time stepping of Eq. (1) itself in long double by its Taylor series:
 * rho(t + dt) = sum_k dt^k / k! rhs^k(rho), with rhs applied directly to the
 * d x d matrix (no superoperator, no propagator); the series of each step is
 * summed until a term falls below 1e-24 of the sum (at most 80 terms). */
void orc_taylor_steps_ld(int d, const zc *H, int K, const zc *Lk, zc *rho, double dt, long long nsteps)
{
    size_t dd = (size_t)d * d;
    lzc *h = malloc(dd * sizeof(lzc)), *L = malloc((size_t)K * dd * sizeof(lzc));
    lzc *x = malloc(dd * sizeof(lzc)), *term = malloc(dd * sizeof(lzc)), *nxt = malloc(dd * sizeof(lzc));
    lzc *t1 = malloc(dd * sizeof(lzc)), *t2 = malloc(dd * sizeof(lzc));
    for (size_t e = 0; e < dd; ++e) { h[e] = H[e]; x[e] = rho[e]; }
    for (size_t e = 0; e < (size_t)K * dd; ++e) L[e] = Lk[e];
    for (long long t = 0; t < nsteps; ++t) {
        memcpy(term, x, dd * sizeof(lzc));
        long double xn = 0;
        for (size_t e = 0; e < dd; ++e) xn += cabsl(x[e]);
        for (int k = 1; k <= 80; ++k) {
            rhs_ld(d, h, K, L, term, nxt, t1, t2);
            long double tn = 0;
            for (size_t e = 0; e < dd; ++e) { term[e] = nxt[e] * ((long double)dt / k); tn += cabsl(term[e]); }
            for (size_t e = 0; e < dd; ++e) x[e] += term[e];
            if (tn < 1e-24L * xn) break;
        }
    }
    for (size_t e = 0; e < dd; ++e) rho[e] = (zc)x[e];
    free(h); free(L); free(x); free(term); free(nxt); free(t1); free(t2);
}

/* ------------------------------------------------------------- GRAPE */
/* Frechet derivative L(A, E) of exp at A in direction E, read off the upper
 * right block of exp([[A, E], [0, A]]) computed by orc_expm_pade13 at 2n. */
int orc_expm_frechet_blocktri(int n, const zc *A, const zc *E, double theta, zc *expA, zc *Lfr)
{
    int m = 2 * n;
    zc *Bm = calloc((size_t)m * m, sizeof(zc)), *X = malloc((size_t)m * m * sizeof(zc));
    if (!Bm || !X) { free(Bm); free(X); return ORC_ENOMEM; }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            Bm[(size_t)i * m + j] = A[(size_t)i * n + j];
            Bm[(size_t)(i + n) * m + (j + n)] = A[(size_t)i * n + j];
            Bm[(size_t)i * m + (j + n)] = E[(size_t)i * n + j];
        }
    int rc = orc_expm_pade13(m, Bm, theta, X, NULL);
    if (rc == ORC_OK)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                if (expA) expA[(size_t)i * n + j] = X[(size_t)i * m + j];
                Lfr[(size_t)i * n + j] = X[(size_t)i * m + (j + n)];
            }
    free(Bm); free(X);
    return rc;
}

/* GRAPE fidelity and gradient for piecewise-constant controls:
 *   A_m = dt (L0 + sum_c u[m,c] Lc[c]),  P_m = exp(A_m)  (Alg. 1),
 *   x_m = P_m x_{m-1},  F = Re <w, x_M>  (= Tr(sigma rho_M) for w = vec sigma),
 *   dF/du[m,c] = Re <lambda_m, L(A_m, dt Lc[c]) x_{m-1}>,
 *   lambda_M = w, lambda_{m-1} = P_m^dag lambda_m.
 * Gradients are computed only for slices with mask[m] != 0 (mask NULL = all);
 * the others are left untouched.  L0: n x n; Lc: C x n x n; u: M x C. */
int orc_grape(int n, int M, int C, const zc *L0, const zc *Lc, const double *u, double dt, double theta,
              const zc *x0, const zc *w, double *F, double *grad, const unsigned char *mask)
{
    size_t nn = (size_t)n * n;
    zc *P = malloc((size_t)M * nn * sizeof(zc));
    zc *xs = malloc((size_t)(M + 1) * n * sizeof(zc));
    zc *A = malloc(nn * sizeof(zc)), *E = malloc(nn * sizeof(zc)), *Lf = malloc(nn * sizeof(zc));
    zc *lam = malloc((size_t)n * sizeof(zc)), *tmp = malloc((size_t)n * sizeof(zc));
    int rc = ORC_OK;
    if (!P || !xs || !A || !E || !Lf || !lam || !tmp) { rc = ORC_ENOMEM; goto done; }
    memcpy(xs, x0, (size_t)n * sizeof(zc));
    for (int m = 0; m < M && rc == ORC_OK; ++m) {
        for (size_t e = 0; e < nn; ++e) {
            zc g = L0[e];
            for (int c = 0; c < C; ++c) g += u[(size_t)m * C + c] * Lc[(size_t)c * nn + e];
            A[e] = dt * g;
        }
        rc = orc_expm_pade13(n, A, theta, P + (size_t)m * nn, NULL);
        orc_matvec(n, P + (size_t)m * nn, xs + (size_t)m * n, xs + (size_t)(m + 1) * n);
    }
    if (rc != ORC_OK) goto done;
    {
        zc f = 0;
        for (int i = 0; i < n; ++i) f += conj(w[i]) * xs[(size_t)M * n + i];
        *F = creal(f);
    }
    if (!grad) goto done;
    memcpy(lam, w, (size_t)n * sizeof(zc));
    for (int m = M - 1; m >= 0 && rc == ORC_OK; --m) {
        if (!mask || mask[m]) {
            for (size_t e = 0; e < nn; ++e) {
                zc g = L0[e];
                for (int c = 0; c < C; ++c) g += u[(size_t)m * C + c] * Lc[(size_t)c * nn + e];
                A[e] = dt * g;
            }
            for (int c = 0; c < C && rc == ORC_OK; ++c) {
                for (size_t e = 0; e < nn; ++e) E[e] = dt * Lc[(size_t)c * nn + e];
                rc = orc_expm_frechet_blocktri(n, A, E, theta, NULL, Lf);
                orc_matvec(n, Lf, xs + (size_t)m * n, tmp);
                zc g = 0;
                for (int i = 0; i < n; ++i) g += conj(lam[i]) * tmp[i];
                grad[(size_t)m * C + c] = creal(g);
            }
        }
        /* lambda_{m-1} = P_m^dag lambda_m */
        const zc *Pm = P + (size_t)m * nn;
        for (int j = 0; j < n; ++j) {
            zc a = 0;
            for (int i = 0; i < n; ++i) a += conj(Pm[(size_t)i * n + j]) * lam[i];
            tmp[j] = a;
        }
        memcpy(lam, tmp, (size_t)n * sizeof(zc));
    }
done:
    free(P); free(xs); free(A); free(E); free(Lf); free(lam); free(tmp);
    return rc;
}

/* ------------------------------------------------------------ Alg. 5
 * Q1.15 fixed point: a value v is the 16-bit integer q with v = q / 2^15.
 * Quantisation of P and of the initial state rounds to nearest (ties to even)
 * and saturates to [-2^15, 2^15 - 1] (1.0 itself saturates).  One step forms
 * acc_i = sum_j P_ij x_j exactly in integers (each real product is Q2.30 and
 * the sums need 33 + ceil(log2 n) bits, held in 64-bit integers), then
 * x_i = sat(floor(acc_i / 2^15)) for the real and imaginary parts. */
static int16_t sat16(long long v) { return (int16_t)(v < -32768 ? -32768 : (v > 32767 ? 32767 : v)); }

void orc_quantize_q15(long long count, const zc *src, int16_t *re, int16_t *im)
{
    for (long long e = 0; e < count; ++e) {
        re[e] = (int16_t)fmax(-32768.0, fmin(32767.0, nearbyint(creal(src[e]) * 32768.0)));
        im[e] = (int16_t)fmax(-32768.0, fmin(32767.0, nearbyint(cimag(src[e]) * 32768.0)));
    }
}

static long long floor_div_2_15(long long a)
{
    long long q = a / 32768;
    if (a % 32768 != 0 && a < 0) q -= 1; /* C division truncates toward zero */
    return q;
}

void orc_propagate_q15(int n, const int16_t *Pr, const int16_t *Pi, int B, int16_t *xr, int16_t *xi,
                       long long nsteps)
{
    long long *ar = malloc((size_t)n * sizeof(long long)), *ai = malloc((size_t)n * sizeof(long long));
    for (int b = 0; b < B; ++b) {
        int16_t *vr = xr + (size_t)b * n, *vi = xi + (size_t)b * n;
        for (long long t = 0; t < nsteps; ++t) {
            for (int i = 0; i < n; ++i) {
                long long sr = 0, si = 0;
                for (int j = 0; j < n; ++j) {
                    const long long pr = Pr[(size_t)i * n + j], pi = Pi[(size_t)i * n + j];
                    sr += pr * vr[j] - pi * vi[j];
                    si += pr * vi[j] + pi * vr[j];
                }
                ar[i] = sr;
                ai[i] = si;
            }
            for (int i = 0; i < n; ++i) {
                vr[i] = sat16(floor_div_2_15(ar[i]));
                vi[i] = sat16(floor_div_2_15(ai[i]));
            }
        }
    }
    free(ar);
    free(ai);
}

/* ------------------------------------------------------------ Alg. 5, Q1.31
 * The same step at 31 fractional bits (the paper's Q1.31 drift curve): a
 * value is the 32-bit integer q with v = q / 2^31; quantisation rounds to
 * nearest (ties to even) and saturates to [-2^31, 2^31 - 1].  A real
 * product is Q2.62 and a row's sum needs 66 + ceil(log2 n) bits, so the
 * sums are held in 128-bit integers; then x_i = sat(floor(acc_i / 2^31)). */
static int32_t sat32(__int128 v)
{
    const __int128 lo = -((__int128)1 << 31), hi = ((__int128)1 << 31) - 1;
    return (int32_t)(v < lo ? lo : (v > hi ? hi : v));
}

void orc_quantize_q31(long long count, const zc *src, int32_t *re, int32_t *im)
{
    const double lo = -2147483648.0, hi = 2147483647.0;
    for (long long e = 0; e < count; ++e) {
        re[e] = (int32_t)fmax(lo, fmin(hi, nearbyint(creal(src[e]) * 2147483648.0)));
        im[e] = (int32_t)fmax(lo, fmin(hi, nearbyint(cimag(src[e]) * 2147483648.0)));
    }
}

static __int128 floor_div_2_31(__int128 a)
{
    const __int128 d = (__int128)1 << 31;
    __int128 q = a / d;
    if (a % d != 0 && a < 0) q -= 1; /* C division truncates toward zero */
    return q;
}

void orc_propagate_q31(int n, const int32_t *Pr, const int32_t *Pi, int B, int32_t *xr, int32_t *xi,
                       long long nsteps)
{
    __int128 *ar = malloc((size_t)n * sizeof(__int128)), *ai = malloc((size_t)n * sizeof(__int128));
    for (int b = 0; b < B; ++b) {
        int32_t *vr = xr + (size_t)b * n, *vi = xi + (size_t)b * n;
        for (long long t = 0; t < nsteps; ++t) {
            for (int i = 0; i < n; ++i) {
                __int128 sr = 0, si = 0;
                for (int j = 0; j < n; ++j) {
                    const __int128 pr = Pr[(size_t)i * n + j], pi = Pi[(size_t)i * n + j];
                    sr += pr * vr[j] - pi * vi[j];
                    si += pr * vi[j] + pi * vr[j];
                }
                ar[i] = sr;
                ai[i] = si;
            }
            for (int i = 0; i < n; ++i) {
                vr[i] = sat32(floor_div_2_31(ar[i]));
                vi[i] = sat32(floor_div_2_31(ai[i]));
            }
        }
    }
    free(ar);
    free(ai);
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
