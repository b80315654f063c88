// GRAPE fidelity and gradient for piecewise-constant controls (the
// control-affine segment generator of Eq. (5), propagators by Alg. 1).
//
//   A_m = dt (L0 + sum_c u[m,c] Lc[c]),  P_m = exp(A_m)
//   x_{m+1} = P_m x_m (0-based slices),   F = Re <w, x_M>
//   lambda_M = w,  lambda_m = P_m^dag lambda_{m+1}
//   dF/du[m,c] = Re <lambda_{m+1}, L(A_m, dt Lc[c]) x_m> = dt Re Tr(Lc[c] G_m),
//   G_m = L(A_m, x_m lambda_{m+1}^dag)
// using Tr(L(A,E) B) = Tr(E L(A,B)) for the Frechet derivative of exp, so one
// derivative per slice (in a rank-1 direction) serves every control.
//
// The derivative is evaluated with the Pade [13/13] derivative recurrences
// of scaling and squaring (Al-Mohy & Higham, SIAM J. Matrix Anal. Appl. 30,
// 2009): with X = A/2^s and F = E/2^s, the products and their directional
// derivatives
//   A2 = X X,   M2 = X F + F X;   A4 = A2 A2, M4 = A2 M2 + M2 A2;
//   A6 = A4 A2, M6 = A4 M2 + M4 A2;
//   W1 = b13 A6 + b11 A4 + b9 A2,  W = A6 W1 + b7 A6 + b5 A4 + b3 A2 + b1 I,  U = X W
//   Z1 = b12 A6 + b10 A4 + b8 A2,  V = A6 Z1 + b6 A6 + b4 A4 + b2 A2 + b0 I
//   Lw = A6 (b13 M6 + b11 M4 + b9 M2) + M6 W1 + b7 M6 + b5 M4 + b3 M2
//   Lu = X Lw + F W
//   Lv = A6 (b12 M6 + b10 M4 + b8 M2) + M6 Z1 + b6 M6 + b4 M4 + b2 M2
// one LU of Q = V - U solving Q [X1 | X2 | R] = [Lu + Lv | Lu - Lv | V + U],
// L = X1 + X2 R (the derivative of Q^{-1}(V + U)), then s times
//   L <- R L + L R,  R <- R R.
// All slices of a chunk go through these steps together as batched GEMMs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "lb_internal.hpp"

namespace lb {

namespace grape {

__global__ void outer_kernel(int n, int Mc, const cd *__restrict__ x, const cd *__restrict__ lam,
                             const int *__restrict__ sexp, cd *__restrict__ E) {
    const long long nn = (long long)n * n, total = nn * Mc;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int m = (int)(e / nn);
        const long long r = e - (long long)m * nn;
        const int i = (int)(r / n), j = (int)(r - (long long)i * n);
        const cd a = x[(size_t)m * n + i], b = lam[(size_t)m * n + j];
        const int s = sexp[m];
        E[e] = {ldexp(a.re * b.re + a.im * b.im, -s), ldexp(a.im * b.re - a.re * b.im, -s)};  // a conj(b)
    }
}

// RHS (n x 3n per slice) = [Lu + Lv | Lu - Lv | V + U]
__global__ void rhs3_kernel(int n, int Mc, const cd *__restrict__ Lu, const cd *__restrict__ Lv,
                            const cd *__restrict__ V, const cd *__restrict__ U, cd *__restrict__ R3) {
    const long long nn = (long long)n * n, total = nn * Mc;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long m = e / nn, r = e - m * nn;
        const long long i = r / n, j = r - i * n;
        cd *row = R3 + (size_t)m * 3 * nn + (size_t)i * 3 * n;
        const cd lu = Lu[e], lv = Lv[e], v = V[e], u = U[e];
        row[j] = cadd(lu, lv);
        row[n + j] = csub(lu, lv);
        row[2 * n + j] = cadd(v, u);
    }
}

// dst[m] (n x n, contiguous) = block `blk` (n columns) of src[m] (n x 3n)
__global__ void take_block_kernel(int n, int Mc, const cd *__restrict__ R3, int blk, cd *__restrict__ dst) {
    const long long nn = (long long)n * n, total = nn * Mc;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long m = e / nn, r = e - m * nn;
        const long long i = r / n, j = r - i * n;
        dst[e] = R3[(size_t)m * 3 * nn + (size_t)i * 3 * n + (size_t)blk * n + j];
    }
}

// y = P x (one state), one wavefront per row, lanes over the row
__global__ void __launch_bounds__(256) matvec_kernel(int n, const cd *__restrict__ P, const cd *__restrict__ x,
                                                     cd *__restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (row >= n) return;
    double re = 0.0, im = 0.0;
    for (int j = lane; j < n; j += 64) {
        const cd p = P[(size_t)row * n + j], v = x[j];
        re = fma(p.re, v.re, fma(-p.im, v.im, re));
        im = fma(p.re, v.im, fma(p.im, v.re, im));
    }
    for (int off = 32; off >= 1; off >>= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
    }
    if (lane == 0) y[row] = {re, im};
}

// y = P^dag x in two passes with a fixed summation order.  Pass 1: workgroup
// (jb, r) owns 64 columns j and the r-th of HR row ranges; its four
// wavefronts take every fourth row of the range, lanes run along j (rows of P
// are read contiguously), and the four partial sums meet in LDS.  Pass 2 sums
// the HR partials of each column in order.
constexpr int HR = 16;  // row ranges of the adjoint matvec

__global__ void __launch_bounds__(256) matvec_h_partial_kernel(int n, const cd *__restrict__ P,
                                                               const cd *__restrict__ x, cd *__restrict__ part) {
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    const int r = blockIdx.y;
    const int i0 = (int)(((long long)n * r) / HR), i1 = (int)(((long long)n * (r + 1)) / HR);
    double re = 0.0, im = 0.0;
    if (j < n) {
        for (int i = i0 + g; i < i1; i += 4) {
            const cd p = P[(size_t)i * n + j], v = x[i];
            re = fma(p.re, v.re, fma(p.im, v.im, re));  // conj(p) v
            im = fma(p.re, v.im, fma(-p.im, v.re, im));
        }
    }
    __shared__ double sr[4][64], si[4][64];
    sr[g][c] = re;
    si[g][c] = im;
    __syncthreads();
    if (g == 0 && j < n)
        part[(size_t)r * n + j] = {((sr[0][c] + sr[1][c]) + sr[2][c]) + sr[3][c],
                                   ((si[0][c] + si[1][c]) + si[2][c]) + si[3][c]};
}

__global__ void __launch_bounds__(256) matvec_h_reduce_kernel(int n, const cd *__restrict__ part, cd *__restrict__ y) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double re = 0.0, im = 0.0;
    for (int r = 0; r < HR; ++r) {
        re += part[(size_t)r * n + j].re;
        im += part[(size_t)r * n + j].im;
    }
    y[j] = {re, im};
}

// F = Re sum conj(w_i) x_i, one workgroup, fixed reduction order
__global__ void __launch_bounds__(256) fidelity_kernel(int n, const cd *__restrict__ w, const cd *__restrict__ x,
                                                       double *__restrict__ F) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += w[i].re * x[i].re + w[i].im * x[i].im;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *F = red[0];
}

// LcT[c] = Lc[c]^T
__global__ void transpose_batch_kernel(int n, int C, const cd *__restrict__ Lc, cd *__restrict__ LcT) {
    const long long nn = (long long)n * n, total = nn * C;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long c = e / nn, r = e - c * nn;
        const long long i = r / n, j = r - i * n;
        LcT[c * nn + j * n + i] = Lc[e];
    }
}

constexpr int CMAX = 16;
constexpr int CHUNK = 4096;  // elements per contraction workgroup

// partial[(b * Mc + m) * C + c] = Re sum_{e in chunk b} LcT[c][e] G[m][e]
__global__ void __launch_bounds__(256) contract_kernel(long long nn, int C, const cd *__restrict__ LcT,
                                                       const cd *__restrict__ G, int Mc, double *__restrict__ partial) {
    const int b = blockIdx.x, m = blockIdx.y;
    double acc[CMAX];
#pragma unroll
    for (int c = 0; c < CMAX; ++c) acc[c] = 0.0;
    const long long e0 = (long long)b * CHUNK;
    const cd *Gm = G + (size_t)m * nn;
    for (long long e = e0 + threadIdx.x; e < e0 + CHUNK && e < nn; e += 256) {
        const cd g = Gm[e];
#pragma unroll
        for (int c = 0; c < CMAX; ++c)
            if (c < C) {
                const cd l = LcT[(size_t)c * nn + e];
                acc[c] = fma(l.re, g.re, fma(-l.im, g.im, acc[c]));
            }
    }
    __shared__ double red[256];
    for (int c = 0; c < C; ++c) {
        red[threadIdx.x] = acc[c];
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[((size_t)b * Mc + m) * C + c] = red[0];
        __syncthreads();
    }
}

__global__ void contract_reduce_kernel(int nblk, int Mc, int C, double dt, const double *__restrict__ partial,
                                       double *__restrict__ grad) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Mc * C) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(size_t)b * Mc * C + t];
    grad[t] = dt * s;
}

static int grid1(long long work) {
    long long g = (work + 255) / 256;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

constexpr int FRECHET_MATS = 26;  // n x n temporaries per slice (RHS3 counts 3)

// Products of the forward build kept per slice for the derivative: the
// E-independent half of the recurrences (A2, A4, A6, W1, Z1, W, U, V) and the
// first KEEP_SQ squaring levels R_0 = r13(X), R_{k+1} = R_k R_k.  Matrix kind j
// of slice m sits at cache + (j M + m) n^2, so each kind is one batched operand.
constexpr int KEEP_SQ = 6;
constexpr int KEEP_MATS = 8 + KEEP_SQ;
struct Keep {
    cd *A2, *A4, *A6, *W1, *Z1, *W, *U, *V;
    cd *R[KEEP_SQ];
};
static Keep keep_view(cd *cache, int M, int m0, size_t nn) {
    auto kind = [&](int j) { return cache + ((size_t)j * M + m0) * nn; };
    Keep k;
    k.A2 = kind(0), k.A4 = kind(1), k.A6 = kind(2), k.W1 = kind(3);
    k.Z1 = kind(4), k.W = kind(5), k.U = kind(6), k.V = kind(7);
    for (int l = 0; l < KEEP_SQ; ++l) k.R[l] = kind(8 + l);
    return k;
}

static size_t frechet_bytes(int n, int Mc) {
    const size_t mat = align256((size_t)n * n * sizeof(cd) * Mc);
    return FRECHET_MATS * mat + 4 * align256(Mc * sizeof(double)) + align256((size_t)Mc * n * sizeof(int)) +
           2 * align256(Mc * sizeof(int)) + 2 * align256((size_t)zgemm_mask_bytes(n, n) * Mc);
}

// G[m] = L(A_m, x_m lam_m^dag) for a chunk of Mc slices; A_m = dt Lg[m].
// With keep, the E-independent products and the kept squaring levels come
// from the forward build instead of being recomputed (same operations, same
// operands, so the same values).
static int frechet_chunk(int n, int Mc, const cd *Lg, const double *dt_host, const cd *x, const cd *lam, double theta,
                         cd *G, Workspace *ws, hipStream_t s, const Keep *keep = nullptr) {
    const size_t nn = (size_t)n * n, mat = nn * sizeof(cd) * Mc;
    LB_TRY(ws_ensure(ws, frechet_bytes(n, Mc)));
    const size_t mark = ws->used;
    struct Release {
        Workspace *w;
        size_t m;
        ~Release() { w->used = m; }
    } release{ws, mark};
    cd *A = (cd *)ws_take(ws, mat), *E = (cd *)ws_take(ws, mat);
    cd *A2 = (cd *)ws_take(ws, mat), *A4 = (cd *)ws_take(ws, mat), *A6 = (cd *)ws_take(ws, mat);
    cd *M2 = (cd *)ws_take(ws, mat), *M4 = (cd *)ws_take(ws, mat), *M6 = (cd *)ws_take(ws, mat);
    cd *W1 = (cd *)ws_take(ws, mat), *Z1 = (cd *)ws_take(ws, mat), *T = (cd *)ws_take(ws, mat);
    cd *W = (cd *)ws_take(ws, mat), *U = (cd *)ws_take(ws, mat), *V = (cd *)ws_take(ws, mat);
    cd *Lw = (cd *)ws_take(ws, mat), *Lu = (cd *)ws_take(ws, mat), *Lv = (cd *)ws_take(ws, mat);
    cd *Q = (cd *)ws_take(ws, mat), *R = (cd *)ws_take(ws, mat), *Rt = (cd *)ws_take(ws, mat);
    cd *Lt = (cd *)ws_take(ws, mat);
    cd *R3 = (cd *)ws_take(ws, 3 * mat);
    double *d_dt = (double *)ws_take(ws, Mc * sizeof(double));
    unsigned long long *d_norm = (unsigned long long *)ws_take(ws, Mc * sizeof(double));
    int *d_s = (int *)ws_take(ws, Mc * sizeof(int));
    int *d_info = (int *)ws_take(ws, Mc * sizeof(int));
    int *d_ipiv = (int *)ws_take(ws, (size_t)Mc * n * sizeof(int));
    const long long mb = zgemm_mask_bytes(n, n);
    unsigned char *mA = (unsigned char *)ws_take(ws, (size_t)mb * Mc);
    unsigned char *mA2 = (unsigned char *)ws_take(ws, (size_t)mb * Mc);

    LB_TRY(fill_i32_launch(d_info, Mc, s));
    std::vector<int> sv(Mc);
    LB_TRY(scaling_stage(n, Mc, Lg, dt_host, theta, d_dt, d_norm, d_s, sv.data(), s));
    int smax = 0;
    for (int m = 0; m < Mc; ++m) smax = sv[m] > smax ? sv[m] : smax;
    LB_TRY(scale_launch(n, Mc, Lg, d_dt, d_s, A, s));
    outer_kernel<<<grid1((long long)nn * Mc), 256, 0, s>>>(n, Mc, x, lam, d_s, E);
    LB_TRY(check_launch("outer"));

    double b[14];
    pade13_coefficients(b);
    ZgemmBatch g;
    g.M = g.N = g.K = n;
    g.batch = Mc;
    g.lda = g.ldb = g.ldd = g.ldc = g.ldx = n;
    g.sA = g.sB = g.sD = g.sC = g.sX = (long long)nn;
    // zero 64 x 16 tiles of the sparse left factors A and A2 are skipped
    auto mul = [&](const cd *X, const cd *Y, cd *Z, bool acc, const unsigned char *mask = nullptr) {
        ZgemmBatch h = g;
        h.A = X, h.B = Y, h.D = Z;
        if (acc) h.beta = 1.0, h.Cin = Z;
        h.amask = mask;
        h.sMask = mb;
        return zgemm_batched(h, s);
    };
    auto mul_lc = [&](const cd *X, const cd *Y, cd *Z, const cd *x0, const cd *x1, const cd *x2, double c0,
                      double c1, double c2, double gamma) {
        ZgemmBatch h = g;
        h.A = X, h.B = Y, h.D = Z;
        h.nx = 3;
        h.X[0] = x0, h.X[1] = x1, h.X[2] = x2;
        h.coef[0] = c0, h.coef[1] = c1, h.coef[2] = c2;
        h.gamma = gamma;
        return zgemm_batched(h, s);
    };
    auto lin3 = [&](const cd *x0, const cd *x1, const cd *x2, double c0, double c1, double c2, cd *D) {
        const cd *X[3] = {x0, x1, x2};
        const double c[3] = {c0, c1, c2};
        return zlincomb(n, Mc, 3, X, c, 0.0, D, s);
    };
    if (keep) {
        A2 = keep->A2, A4 = keep->A4, A6 = keep->A6, W1 = keep->W1;
        Z1 = keep->Z1, W = keep->W, U = keep->U, V = keep->V;
    }
    LB_TRY(zgemm_tile_mask(n, n, Mc, A, n, (long long)nn, mA, s));
    if (!keep) LB_TRY(mul(A, A, A2, false, mA));
    LB_TRY(zgemm_tile_mask(n, n, Mc, A2, n, (long long)nn, mA2, s));
    LB_TRY(mul(A, E, M2, false, mA));
    LB_TRY(mul(E, A, M2, true));
    if (!keep) LB_TRY(mul(A2, A2, A4, false, mA2));
    LB_TRY(mul(A2, M2, M4, false, mA2));
    LB_TRY(mul(M2, A2, M4, true));
    if (!keep) LB_TRY(mul(A4, A2, A6, false));  // the operand order of the propagator build
    LB_TRY(mul(A4, M2, M6, false));
    LB_TRY(mul(M4, A2, M6, true));
    if (!keep) {
        LB_TRY(lin3(A6, A4, A2, b[13], b[11], b[9], W1));
        LB_TRY(mul_lc(A6, W1, W, A6, A4, A2, b[7], b[5], b[3], b[1]));
        LB_TRY(mul(A, W, U, false, mA));
        LB_TRY(lin3(A6, A4, A2, b[12], b[10], b[8], Z1));
        LB_TRY(mul_lc(A6, Z1, V, A6, A4, A2, b[6], b[4], b[2], b[0]));
    }
    LB_TRY(lin3(M6, M4, M2, b[13], b[11], b[9], T));
    LB_TRY(mul_lc(A6, T, Lw, M6, M4, M2, b[7], b[5], b[3], 0.0));
    LB_TRY(mul(M6, W1, Lw, true));
    LB_TRY(mul(A, Lw, Lu, false, mA));
    LB_TRY(mul(E, W, Lu, true));
    LB_TRY(lin3(M6, M4, M2, b[12], b[10], b[8], T));
    LB_TRY(mul_lc(A6, T, Lv, M6, M4, M2, b[6], b[4], b[2], 0.0));
    LB_TRY(mul(M6, Z1, Lv, true));
    {
        const cd *X[2] = {V, U};
        const double c[2] = {1.0, -1.0};
        LB_TRY(zlincomb(n, Mc, 2, X, c, 0.0, Q, s));
    }
    rhs3_kernel<<<grid1((long long)nn * Mc), 256, 0, s>>>(n, Mc, Lu, Lv, V, U, R3);
    LB_TRY(check_launch("rhs3"));
    LB_TRY(lu_solve_batched(n, 3 * n, Mc, Q, R3, d_ipiv, d_info, s));
    take_block_kernel<<<grid1((long long)nn * Mc), 256, 0, s>>>(n, Mc, R3, 2, R);
    LB_TRY(check_launch("take_block"));
    {  // L = X1 + X2 R  into G
        ZgemmBatch h = g;
        h.A = R3 + n;  // X2
        h.lda = 3 * n;
        h.sA = 3 * (long long)nn;
        h.B = R;
        h.D = G;
        h.beta = 1.0;
        h.Cin = R3;  // X1
        h.ldc = 3 * n;
        h.sC = 3 * (long long)nn;
        LB_TRY(zgemm_batched(h, s));
    }
    // squarings, masked by each slice's s: level k reads (k even ? G : Lt) and
    // R_k, which is kept (k < KEEP_SQ with keep) or else in (k even ? R : Rt)
    for (int k = 0; k < smax; ++k) {
        const cd *Ls = (k & 1) ? Lt : G;
        cd *Ld = (k & 1) ? G : Lt;
        const bool kept = keep && k < KEEP_SQ;
        const int q = keep ? k - KEEP_SQ : k;  // parity of the ping-pong position
        const cd *Rs = kept ? keep->R[k] : ((q & 1) ? Rt : R);
        cd *Rd = ((q + 1) & 1) ? Rt : R;
        ZgemmBatch h = g;
        h.active = d_s;
        h.level = k;
        h.A = Rs, h.B = Ls, h.D = Ld;
        LB_TRY(zgemm_batched(h, s));
        h.A = Ls, h.B = Rs, h.beta = 1.0, h.Cin = Ld;
        LB_TRY(zgemm_batched(h, s));
        if (k + 1 < smax && !(keep && k + 1 < KEEP_SQ)) {  // R_{k+1}, needed and not kept
            h.A = Rs, h.B = Rs, h.D = Rd, h.beta = 0.0, h.Cin = nullptr;
            LB_TRY(zgemm_batched(h, s));
        }
    }
    if (smax > 0) LB_TRY(odd_copy_launch(n, Mc, d_s, Lt, G, s));
    std::vector<int> info(Mc);
    LB_HIP(hipMemcpyAsync(info.data(), d_info, Mc * sizeof(int), hipMemcpyDeviceToHost, s));
    LB_HIP(hipStreamSynchronize(s));
    for (int m = 0; m < Mc; ++m)
        if (info[m]) return fail(LB_ESINGULAR, "grape_gradient: zero pivot in V - U of a slice");
    return LB_OK;
}

// ---- low-rank derivative (kept path, n >= kLowRankMinN = 64)
// The direction F = u0 v0^H (u0 = x 2^-s, v0 = lambda) has rank one, so every
// derivative matrix of the Pade half is a short sum of rank-one terms, kept
// as a factor pair U Vh (U: n x r, Vh: r x n, both row-major):
//   P0 = [X u0 | u0], P1 = A2 P0, P2 = A4 P0;  Q0 = [v0^H ; v0^H X],
//   Q1 = Q0 A2, Q2 = Q1 A2;  M2 = P0 Q0, M4 = P0 Q1 + P1 Q0,
//   M6 = P0 Q2 + P1 Q1 + P2 Q0 = [P0 P1 P2] [Q2; Q1; Q0],
//   c6 M6 + c4 M4 + c2 M2 = [P0 P1 P2] Vc(c),
//   Vc(c) = [c6 Q2 + c4 Q1 + c2 Q0 ; c6 Q1 + c4 Q0 ; c6 Q0]
// so with U6 = [P0 P1 P2], Uw = [A6 U6 | U6]:
//   Lw = Uw [Vc(b13, b11, b9) ; Vc(b7, b5, b3) + Vh6 W1]
//   Lv = Uw [Vc(b12, b10, b8) ; Vc(b6, b4, b2) + Vh6 Z1]
//   Lu = X Lw + F W = [X Uw | u0] [Vh_Lw ; v0^H W]
//   Lu +- Lv = [X Uw | u0 | +-Uw] Vh_all,  Vh_all = [Vh_Lw ; v0^H W ; Vh_Lv]  (25 rows).
// One LU solve with 25 right-hand sides gives Y = (V - U)^{-1} [X Uw | u0 | Uw];
// L = X1 + X2 R_0 = [Y | Ya, -Yc] [Vh_all ; Vh_all R_0] (rank 50), and each
// squaring level L <- R_k L + L R_k = [U | R_k U] [Vh R_k ; Vh] doubles the
// rank; while every slice is still active and the rank stays <= n / 2 the
// levels run on the factors, then L = U Vh is formed and the remaining
// levels run dense as in frechet_chunk.  Same mathematics as frechet_chunk,
// other rounding.
constexpr int kLowRankMinN = 64;
constexpr int LR_NV = 25;  // columns of the solve
constexpr int LR_R0 = 50;  // rank of L before the squarings

// dst[m][i][j] = sign * src[m][i][j] for i < rows, j < w (row-major blocks)
__global__ void copy2d_kernel(int rows, int w, int Mc, const cd *__restrict__ src, long long lds, long long sS,
                              cd *__restrict__ dst, long long ldd, long long sD, double sign) {
    const long long per = (long long)rows * w, total = per * Mc;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long m = e / per, r = e - m * per;
        const long long i = r / w, j = r - i * w;
        const cd v = src[m * sS + i * lds + j];
        dst[m * sD + i * ldd + j] = {sign * v.re, sign * v.im};
    }
}

// P column 1 = u0 = x 2^-s (P: n x 6 per slice), Qv row 4 = v0^H = conj(lambda)
__global__ void lr_init_kernel(int n, int Mc, const cd *__restrict__ x, const cd *__restrict__ lam,
                               const int *__restrict__ sexp, cd *__restrict__ P, cd *__restrict__ Qv) {
    const long long total = (long long)n * Mc;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long m = e / n, i = e - m * n;
        const cd a = x[e], b = lam[e];
        const int s = sexp[m];
        P[m * 6 * n + i * 6 + 1] = {ldexp(a.re, -s), ldexp(a.im, -s)};
        Qv[m * 6 * n + 4 * n + i] = {b.re, -b.im};
    }
}

// dst (6 x n block, row stride n) = Vc(c6, c4, c2) of Qv = [Q2; Q1; Q0] (2 rows each)
__global__ void vcomb_kernel(int n, int Mc, const cd *__restrict__ Qv, double c6, double c4, double c2,
                             cd *__restrict__ dst, long long sD) {
    const long long per = 6LL * n, total = per * Mc;
    const double c[3] = {c6, c4, c2};
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long m = e / per, r = e - m * per;
        const int row = (int)(r / n), blk = row >> 1, k = row & 1;
        const long long col = r - (long long)row * n;
        double re = 0.0, im = 0.0;
        for (int t = 0; blk + t < 3; ++t) {
            const cd q = Qv[m * per + (long long)(2 * (blk + t) + k) * n + col];
            re = fma(c[t], q.re, re);
            im = fma(c[t], q.im, im);
        }
        dst[m * sD + (long long)row * n + col] = {re, im};
    }
}

// slices whose level count past k0 is odd hold their result in src
__global__ void parity_copy_kernel(long long nn, int Mc, const int *__restrict__ sexp, int k0,
                                   const cd *__restrict__ src, cd *__restrict__ dst) {
    const long long total = nn * Mc;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int m = (int)(e / nn);
        if ((sexp[m] - k0) & 1) dst[e] = src[e];
    }
}

// low-rank levels for a chunk whose smallest s is smin: while the rank r
// allows 2 r <= n, every slice is active and R_k is kept
static int lowrank_levels(int n, int smin) {
    int k = 0, r = LR_R0;
    while (k < smin && k < KEEP_SQ - 1 && 2 * r <= n) ++k, r *= 2;
    return k;
}

static size_t frechet_lowrank_bytes(int n, int Mc, int rmax) {
    const size_t mat = align256((size_t)n * n * sizeof(cd) * Mc);
    auto tb = [&](size_t cols) { return align256((size_t)n * cols * sizeof(cd) * Mc); };
    return 4 * mat + tb(6) + tb(6) + tb(12) + tb(LR_NV) + 2 * tb(rmax) + 4 * align256(Mc * sizeof(double)) +
           align256((size_t)Mc * n * sizeof(int)) + 2 * align256(Mc * sizeof(int)) +
           2 * align256((size_t)zgemm_mask_bytes(n, n) * Mc);
}
static int lowrank_rmax(int n) {
    int r = LR_R0;
    for (int k = 0; k < KEEP_SQ - 1 && 2 * r <= n; ++k) r *= 2;
    return r;
}

// k.U holds the kept factorization of V - U (exchanges in ipiv).
static int frechet_lowrank_chunk(int n, int Mc, const cd *Lg, const double *dt_host, const cd *x, const cd *lam,
                                 double theta, cd *G, Workspace *ws, hipStream_t s, const Keep &k, const int *ipiv) {
    const size_t nn = (size_t)n * n, mat = nn * sizeof(cd) * Mc;
    const int rmax = lowrank_rmax(n);
    LB_TRY(ws_ensure(ws, frechet_lowrank_bytes(n, Mc, rmax)));
    const size_t mark = ws->used;
    struct Release {
        Workspace *w;
        size_t m;
        ~Release() { w->used = m; }
    } release{ws, mark};
    auto thin = [&](size_t cols) { return (cd *)ws_take(ws, (size_t)n * cols * sizeof(cd) * Mc); };
    cd *A = (cd *)ws_take(ws, mat), *Q = (cd *)ws_take(ws, mat);
    cd *Lt = (cd *)ws_take(ws, mat), *Rx[2] = {(cd *)ws_take(ws, mat), nullptr};
    cd *P = thin(6), *Qv = thin(6), *Uw = thin(12), *Y = thin(LR_NV);
    cd *Ub = thin(rmax), *Vb = thin(rmax);
    Rx[1] = Q;  // spare n x n per slice for the squaring levels past the kept ones
    double *d_dt = (double *)ws_take(ws, Mc * sizeof(double));
    unsigned long long *d_norm = (unsigned long long *)ws_take(ws, Mc * sizeof(double));
    int *d_s = (int *)ws_take(ws, Mc * sizeof(int));
    int *d_info = (int *)ws_take(ws, Mc * sizeof(int));
    int *d_ipiv = (int *)ws_take(ws, (size_t)Mc * n * sizeof(int));
    const long long mb = zgemm_mask_bytes(n, n);
    unsigned char *mA = (unsigned char *)ws_take(ws, (size_t)mb * Mc);
    unsigned char *mA2 = (unsigned char *)ws_take(ws, (size_t)mb * Mc);

    LB_TRY(fill_i32_launch(d_info, Mc, s));
    std::vector<int> sv(Mc);
    LB_TRY(scaling_stage(n, Mc, Lg, dt_host, theta, d_dt, d_norm, d_s, sv.data(), s));
    int smax = 0, smin = 1 << 30;
    for (int m = 0; m < Mc; ++m) smax = std::max(smax, sv[m]), smin = std::min(smin, sv[m]);
    LB_TRY(scale_launch(n, Mc, Lg, d_dt, d_s, A, s));
    LB_TRY(zgemm_tile_mask(n, n, Mc, A, n, (long long)nn, mA, s));
    LB_TRY(zgemm_tile_mask(n, n, Mc, k.A2, n, (long long)nn, mA2, s));

    double b[14];
    pade13_coefficients(b);
    const long long sT6 = 6LL * n, sT12 = 12LL * n, sTY = (long long)LR_NV * n, sTR = (long long)rmax * n;
    // D (M x N, ldd, stride sD) = A (M x K) B (K x N) [+ D]
    auto gemm = [&](int M, int N, int K, const cd *Am, long long lda, long long sA, const unsigned char *mask,
                    const cd *Bm, long long ldb, long long sB, cd *D, long long ldd, long long sD, bool acc) {
        ZgemmBatch h;
        h.M = M, h.N = N, h.K = K, h.batch = Mc;
        h.A = Am, h.lda = lda, h.sA = sA;
        h.B = Bm, h.ldb = ldb, h.sB = sB;
        h.D = D, h.ldd = ldd, h.sD = sD;
        if (acc) h.beta = 1.0, h.Cin = D, h.ldc = ldd, h.sC = sD;
        h.amask = mask;
        h.sMask = mb;
        return zgemm_batched(h, s);
    };
    auto copy2d = [&](int rows, int w, const cd *src, long long lds, long long sS, cd *dst, long long ldd,
                      long long sD, double sign) {
        copy2d_kernel<<<grid1((long long)rows * w * Mc), 256, 0, s>>>(rows, w, Mc, src, lds, sS, dst, ldd, sD, sign);
        return check_launch("copy2d");
    };
    const long long NN = (long long)nn;
    lr_init_kernel<<<grid1((long long)n * Mc), 256, 0, s>>>(n, Mc, x, lam, d_s, P, Qv);
    LB_TRY(check_launch("lr_init"));
    // P0 = [X u0 | u0], Q0 = [v0^H ; v0^H X]
    LB_TRY(gemm(n, 1, n, A, n, NN, mA, P + 1, 6, sT6, P, 6, sT6, false));
    LB_TRY(gemm(1, n, n, Qv + 4 * n, n, sT6, nullptr, A, n, NN, Qv + 5 * n, n, sT6, false));
    // P1 = A2 P0, P2 = A4 P0, Q1 = Q0 A2, Q2 = Q1 A2
    LB_TRY(gemm(n, 2, n, k.A2, n, NN, mA2, P, 6, sT6, P + 2, 6, sT6, false));
    LB_TRY(gemm(n, 2, n, k.A4, n, NN, nullptr, P, 6, sT6, P + 4, 6, sT6, false));
    LB_TRY(gemm(2, n, n, Qv + 4 * n, n, sT6, nullptr, k.A2, n, NN, Qv + 2 * n, n, sT6, false));
    LB_TRY(gemm(2, n, n, Qv + 2 * n, n, sT6, nullptr, k.A2, n, NN, Qv, n, sT6, false));
    // Uw = [A6 U6 | U6]
    LB_TRY(gemm(n, 6, n, k.A6, n, NN, nullptr, P, 6, sT6, Uw, 12, sT12, false));
    LB_TRY(copy2d(n, 6, P, 6, sT6, Uw + 6, 12, sT12, 1.0));
    // Vh_all, built in rows 0 .. 24 of Vb: [Vc(b13..) ; Vc(b7..) + Vh6 W1 ; v0^H W ; Vc(b12..) ; Vc(b6..) + Vh6 Z1]
    auto vcomb = [&](double c6, double c4, double c2, cd *dst) {
        vcomb_kernel<<<grid1(6LL * n * Mc), 256, 0, s>>>(n, Mc, Qv, c6, c4, c2, dst, sTR);
        return check_launch("vcomb");
    };
    LB_TRY(vcomb(b[13], b[11], b[9], Vb));
    LB_TRY(vcomb(b[7], b[5], b[3], Vb + 6 * n));
    LB_TRY(gemm(6, n, n, Qv, n, sT6, nullptr, k.W1, n, NN, Vb + 6 * n, n, sTR, true));
    LB_TRY(gemm(1, n, n, Qv + 4 * n, n, sT6, nullptr, k.W, n, NN, Vb + 12 * n, n, sTR, false));
    LB_TRY(vcomb(b[12], b[10], b[8], Vb + 13 * n));
    LB_TRY(vcomb(b[6], b[4], b[2], Vb + 19 * n));
    LB_TRY(gemm(6, n, n, Qv, n, sT6, nullptr, k.Z1, n, NN, Vb + 19 * n, n, sTR, true));
    // Y = (V - U)^{-1} [X Uw | u0 | Uw]
    LB_TRY(gemm(n, 12, n, A, n, NN, mA, Uw, 12, sT12, Y, LR_NV, sTY, false));
    LB_TRY(copy2d(n, 1, P + 1, 6, sT6, Y + 12, LR_NV, sTY, 1.0));
    LB_TRY(copy2d(n, 12, Uw, 12, sT12, Y + 13, LR_NV, sTY, 1.0));
    LB_TRY(lu_resolve_batched(n, LR_NV, Mc, k.U, Y, ipiv, s));  // the forward build's factorization
    // L = [Y | Ya, -Yc] [Vh_all ; Vh_all R_0]
    LB_TRY(copy2d(n, LR_NV, Y, LR_NV, sTY, Ub, rmax, sTR, 1.0));
    LB_TRY(copy2d(n, 13, Y, LR_NV, sTY, Ub + LR_NV, rmax, sTR, 1.0));
    LB_TRY(copy2d(n, 12, Y + 13, LR_NV, sTY, Ub + LR_NV + 13, rmax, sTR, -1.0));
    LB_TRY(gemm(LR_NV, n, n, Vb, n, sTR, nullptr, k.R[0], n, NN, Vb + (long long)LR_NV * n, n, sTR, false));
    // low-rank squaring levels: L <- [U | R_k U] [Vh R_k ; Vh]
    const int klr = lowrank_levels(n, smin);
    int r = LR_R0;
    for (int l = 0; l < klr; ++l, r *= 2) {
        LB_TRY(copy2d(r, n, Vb, n, sTR, Vb + (long long)r * n, n, sTR, 1.0));
        LB_TRY(gemm(r, n, n, Vb + (long long)r * n, n, sTR, nullptr, k.R[l], n, NN, Vb, n, sTR, false));
        LB_TRY(gemm(n, r, n, k.R[l], n, NN, nullptr, Ub, rmax, sTR, Ub + r, rmax, sTR, false));
    }
    // L = U Vh, then the remaining levels dense (level l reads ((l - klr) even ? G : Lt))
    LB_TRY(gemm(n, n, r, Ub, rmax, sTR, nullptr, Vb, n, sTR, G, n, NN, false));
    ZgemmBatch g;
    g.M = g.N = g.K = n;
    g.batch = Mc;
    g.lda = g.ldb = g.ldd = g.ldc = n;
    g.sA = g.sB = g.sD = g.sC = NN;
    for (int l = klr; l < smax; ++l) {
        const int q = l - klr;
        const cd *Ls = (q & 1) ? Lt : G;
        cd *Ld = (q & 1) ? G : Lt;
        const int qr = l - KEEP_SQ;  // R_l past the kept levels ping-pongs in Rx
        const cd *Rs = l < KEEP_SQ ? k.R[l] : Rx[qr & 1];
        ZgemmBatch h = g;
        h.active = d_s;
        h.level = l;
        h.A = Rs, h.B = Ls, h.D = Ld;
        LB_TRY(zgemm_batched(h, s));
        h.A = Ls, h.B = Rs, h.beta = 1.0, h.Cin = Ld;
        LB_TRY(zgemm_batched(h, s));
        if (l + 1 < smax && l + 1 >= KEEP_SQ) {  // R_{l+1}
            h.A = Rs, h.B = Rs, h.D = Rx[(qr + 1) & 1], h.beta = 0.0, h.Cin = nullptr;
            LB_TRY(zgemm_batched(h, s));
        }
    }
    if (smax > klr) {
        parity_copy_kernel<<<grid1((long long)nn * Mc), 256, 0, s>>>((long long)nn, Mc, d_s, klr, Lt, G);
        LB_TRY(check_launch("parity_copy"));
    }
    std::vector<int> info(Mc);
    LB_HIP(hipMemcpyAsync(info.data(), d_info, Mc * sizeof(int), hipMemcpyDeviceToHost, s));
    LB_HIP(hipStreamSynchronize(s));
    for (int m = 0; m < Mc; ++m)
        if (info[m]) return fail(LB_ESINGULAR, "grape_gradient: zero pivot in V - U of a slice");
    return LB_OK;
}

// Forward build of a chunk for the kept path: the same products as the
// derivative's E-independent half (written into the cache), one LU solve of
// (V - U) R_0 = V + U, the squarings R_{k+1} = R_k R_k (kept levels into the
// cache, later ones ping-ponging in the workspace) and P_m = R_{s_m}.
static size_t forward_keep_bytes(int n, int Mc) {
    const size_t mat = align256((size_t)n * n * sizeof(cd) * Mc);
    return 4 * mat + 4 * align256(Mc * sizeof(double)) + align256((size_t)Mc * n * sizeof(int)) +
           2 * align256(Mc * sizeof(int)) + 2 * align256((size_t)zgemm_mask_bytes(n, n) * Mc);
}

// With ipiv_keep (the low-rank derivative's path) V - U is factored in the
// slot of U and the factorization kept, with its exchanges in ipiv_keep.
static int forward_keep_chunk(int n, int Mc, const cd *Lg, const double *dt_host, double theta, const Keep &k,
                              cd *P, Workspace *ws, hipStream_t s, int *ipiv_keep = nullptr) {
    const size_t nn = (size_t)n * n, mat = nn * sizeof(cd) * Mc;
    LB_TRY(ws_ensure(ws, forward_keep_bytes(n, Mc)));
    const size_t mark = ws->used;
    struct Release {
        Workspace *w;
        size_t m;
        ~Release() { w->used = m; }
    } release{ws, mark};
    cd *A = (cd *)ws_take(ws, mat), *Q = (cd *)ws_take(ws, mat);
    cd *Rp[2] = {(cd *)ws_take(ws, mat), (cd *)ws_take(ws, mat)};
    double *d_dt = (double *)ws_take(ws, Mc * sizeof(double));
    unsigned long long *d_norm = (unsigned long long *)ws_take(ws, Mc * sizeof(double));
    int *d_s = (int *)ws_take(ws, Mc * sizeof(int));
    int *d_info = (int *)ws_take(ws, Mc * sizeof(int));
    int *d_ipiv = (int *)ws_take(ws, (size_t)Mc * n * sizeof(int));
    const long long mb = zgemm_mask_bytes(n, n);
    unsigned char *mA = (unsigned char *)ws_take(ws, (size_t)mb * Mc);
    unsigned char *mA2 = (unsigned char *)ws_take(ws, (size_t)mb * Mc);

    LB_TRY(fill_i32_launch(d_info, Mc, s));
    std::vector<int> sv(Mc);
    LB_TRY(scaling_stage(n, Mc, Lg, dt_host, theta, d_dt, d_norm, d_s, sv.data(), s));
    int smax = 0;
    for (int m = 0; m < Mc; ++m) smax = sv[m] > smax ? sv[m] : smax;
    LB_TRY(scale_launch(n, Mc, Lg, d_dt, d_s, A, s));

    double b[14];
    pade13_coefficients(b);
    ZgemmBatch g;
    g.M = g.N = g.K = n;
    g.batch = Mc;
    g.lda = g.ldb = g.ldd = g.ldc = g.ldx = n;
    g.sA = g.sB = g.sD = g.sC = g.sX = (long long)nn;
    auto mul = [&](const cd *X, const cd *Y, cd *Z, const unsigned char *mask) {
        ZgemmBatch h = g;
        h.A = X, h.B = Y, h.D = Z;
        h.amask = mask;
        h.sMask = mb;
        return zgemm_batched(h, s);
    };
    auto mul_lc = [&](const cd *X, const cd *Y, cd *Z, double c0, double c1, double c2, double gamma) {
        ZgemmBatch h = g;
        h.A = X, h.B = Y, h.D = Z;
        h.nx = 3;
        h.X[0] = k.A6, h.X[1] = k.A4, h.X[2] = k.A2;
        h.coef[0] = c0, h.coef[1] = c1, h.coef[2] = c2;
        h.gamma = gamma;
        return zgemm_batched(h, s);
    };
    auto lin3 = [&](double c0, double c1, double c2, cd *D) {
        const cd *X[3] = {k.A6, k.A4, k.A2};
        const double c[3] = {c0, c1, c2};
        return zlincomb(n, Mc, 3, X, c, 0.0, D, s);
    };
    // the operations and operand order of frechet_chunk and of the propagator
    // build, so that P_m and every kept product are those of the other paths
    LB_TRY(zgemm_tile_mask(n, n, Mc, A, n, (long long)nn, mA, s));
    LB_TRY(mul(A, A, k.A2, mA));
    LB_TRY(zgemm_tile_mask(n, n, Mc, k.A2, n, (long long)nn, mA2, s));
    LB_TRY(mul(k.A2, k.A2, k.A4, mA2));
    LB_TRY(mul(k.A4, k.A2, k.A6, nullptr));
    LB_TRY(lin3(b[13], b[11], b[9], k.W1));
    LB_TRY(mul_lc(k.A6, k.W1, k.W, b[7], b[5], b[3], b[1]));
    LB_TRY(mul(A, k.W, k.U, mA));
    LB_TRY(lin3(b[12], b[10], b[8], k.Z1));
    LB_TRY(mul_lc(k.A6, k.Z1, k.V, b[6], b[4], b[2], b[0]));
    {
        const cd *X[2] = {k.V, k.U};
        const double cm[2] = {1.0, -1.0}, cp[2] = {1.0, 1.0};
        LB_TRY(zlincomb(n, Mc, 2, X, cp, 0.0, k.R[0], s));
        cd *Qd = ipiv_keep ? k.U : Q;  // elementwise, so V - U may overwrite U
        LB_TRY(zlincomb(n, Mc, 2, X, cm, 0.0, Qd, s));
        LB_TRY(lu_solve_batched(n, n, Mc, Qd, k.R[0], ipiv_keep ? ipiv_keep : d_ipiv, d_info, s));
    }
    auto level = [&](int l) -> cd * { return l < KEEP_SQ ? k.R[l] : Rp[(l - KEEP_SQ) & 1]; };
    for (int l = 0; l < smax; ++l) {
        ZgemmBatch h = g;
        h.active = d_s;
        h.level = l;
        h.A = level(l), h.B = level(l), h.D = level(l + 1);
        LB_TRY(zgemm_batched(h, s));
    }
    for (int m = 0; m < Mc; ++m)  // P_m = R_{s_m}
        LB_HIP(hipMemcpyAsync(P + (size_t)m * nn, level(sv[m]) + (size_t)m * nn, nn * sizeof(cd),
                              hipMemcpyDeviceToDevice, s));
    std::vector<int> info(Mc);
    LB_HIP(hipMemcpyAsync(info.data(), d_info, Mc * sizeof(int), hipMemcpyDeviceToHost, s));
    LB_HIP(hipStreamSynchronize(s));
    for (int m = 0; m < Mc; ++m)
        if (info[m]) return fail(LB_ESINGULAR, "grape_gradient: zero pivot in V - U of a slice");
    return LB_OK;
}

}  // namespace grape

int generators_launch(int n, int M, int C, const cd *L0, const cd *Lc, const double *u, cd *Lout, hipStream_t s);

// Default cap of the gradient's workspace reservation (slices are processed
// in chunks that fit it; the library workspace's own cap applies as well).
constexpr size_t kGrapeChunkBudget = 24ull << 30;
// Reservation cap when the forward build's products are kept for the
// derivative (about 14 n x n matrices per slice on top of the above).
constexpr size_t kGrapeKeepBudget = 60ull << 30;

static int grape_run(int n, int M, int C, const cd *L0, const cd *Lc, const double *u, double dt, double theta,
                     const cd *x0, const cd *w, double *F, double *grad, long long checkpoint_bytes, Workspace *ws,
                     hipStream_t s) {
    using namespace grape;
    const size_t nn = (size_t)n * n;
    const size_t matb = nn * sizeof(cd);
    bool keepP = checkpoint_bytes <= 0 || (double)M * (double)matb <= (double)checkpoint_bytes;
    const int nblk = (int)((nn + CHUNK - 1) / CHUNK);
    // Kept path: the propagators and the build's E-independent products of
    // every slice stay resident for the derivative, when the checkpoint
    // budget (if any) and the reservation cap allow it.
    const bool lowrank = n >= kLowRankMinN;  // (with keep) the derivative on low-rank factors
    const size_t cache_bytes = align256((size_t)KEEP_MATS * M * matb) +
                               (lowrank ? align256((size_t)M * n * sizeof(int)) : 0);  // + the LU exchanges
    bool keep = checkpoint_bytes <= 0 || (double)(KEEP_MATS + 1) * M * (double)matb <= (double)checkpoint_bytes;
    // ---- reservation: persistent buffers + the larger of the chunk phases
    auto reservation = [&](int mc) {
        const size_t persistent = align256((size_t)(M + 1) * n * sizeof(cd)) * 2 +
                                  align256((size_t)HR * n * sizeof(cd)) + align256((size_t)C * matb) +
                                  align256(sizeof(double)) + align256((size_t)nblk * mc * C * sizeof(double)) +
                                  (keepP ? align256((size_t)M * matb) : 0);
        if (keep) {  // + the cache, the generators of a chunk and the larger phase
            size_t phase = forward_keep_bytes(n, mc);
            const size_t fr = (lowrank ? frechet_lowrank_bytes(n, mc, lowrank_rmax(n)) : frechet_bytes(n, mc)) +
                              align256((size_t)mc * matb);
            if (fr > phase) phase = fr;
            return persistent + cache_bytes + align256((size_t)mc * matb) + phase;
        }
        const size_t chunkp = 2 * align256((size_t)mc * matb);  // generators + propagators of a chunk
        size_t phase = build_workspace_bytes(n, mc);
        const size_t fr = frechet_bytes(n, mc) + align256((size_t)mc * matb);
        if (fr > phase) phase = fr;
        return persistent + chunkp + phase;
    };
    // Slices per batched chunk: the most that fit the budget (larger chunks
    // fill the device better and run fewer sequential LU panel rounds).
    // Results do not depend on the chunking as long as every chunk holds 8
    // or more slices, or every one fewer (the batched LU blocks differently
    // below 8 matrices); chunks are equal in size.
    if (keep) {
        keepP = true;
        if (reservation(1) > std::min(ws->cap, kGrapeKeepBudget)) keep = false;
        keepP = keep || checkpoint_bytes <= 0 || (double)M * (double)matb <= (double)checkpoint_bytes;
    }
    const size_t budget = std::min(ws->cap, keep ? kGrapeKeepBudget : kGrapeChunkBudget);
    int Mc = M < 1024 ? M : 1024;
    while (Mc > 1 && reservation(Mc) > budget) Mc = Mc > 16 ? Mc * 3 / 4 : Mc - 1;
    Mc = (M + (M + Mc - 1) / Mc - 1) / ((M + Mc - 1) / Mc);  // equal chunks, no short tail
    const size_t total = reservation(Mc);
    LB_TRY(ws_ensure(ws, total));
    cd *xs = (cd *)ws_take(ws, (size_t)(M + 1) * n * sizeof(cd));
    cd *lams = (cd *)ws_take(ws, (size_t)(M + 1) * n * sizeof(cd));
    cd *hpart = (cd *)ws_take(ws, (size_t)HR * n * sizeof(cd));
    cd *LcT = (cd *)ws_take(ws, (size_t)C * matb);
    double *d_F = (double *)ws_take(ws, sizeof(double));
    double *partial = (double *)ws_take(ws, (size_t)nblk * Mc * C * sizeof(double));
    cd *Pall = keepP ? (cd *)ws_take(ws, (size_t)M * matb) : nullptr;
    cd *cache = keep ? (cd *)ws_take(ws, (size_t)KEEP_MATS * M * matb) : nullptr;
    int *ipiv_keep = keep && lowrank ? (int *)ws_take(ws, (size_t)M * n * sizeof(int)) : nullptr;
    cd *Lg = (cd *)ws_take(ws, (size_t)Mc * matb);
    cd *Pc = keep ? nullptr : (cd *)ws_take(ws, (size_t)Mc * matb);
    std::vector<double> dts(Mc, dt);

    if (C > 0) {
        transpose_batch_kernel<<<grid1((long long)nn * C), 256, 0, s>>>(n, C, Lc, LcT);
        LB_TRY(check_launch("transpose_batch"));
    }
    LB_HIP(hipMemcpyAsync(xs, x0, n * sizeof(cd), hipMemcpyDeviceToDevice, s));
    auto chunk_props = [&](int m0, int mc, cd *dst) -> int {
        LB_TRY(generators_launch(n, mc, C, L0, Lc, u + (size_t)m0 * C, Lg, s));
        return build_propagators(n, mc, Lg, dts.data(), theta, dst, nullptr, ws, s);
    };
    // ---- forward: propagators (kept if they fit the budget) and states
    for (int m0 = 0; m0 < M; m0 += Mc) {
        const int mc = M - m0 < Mc ? M - m0 : Mc;
        cd *Pdst = keepP ? Pall + (size_t)m0 * nn : Pc;
        if (keep) {
            LB_TRY(generators_launch(n, mc, C, L0, Lc, u + (size_t)m0 * C, Lg, s));
            LB_TRY(forward_keep_chunk(n, mc, Lg, dts.data(), theta, keep_view(cache, M, m0, nn), Pdst, ws, s,
                                      ipiv_keep ? ipiv_keep + (size_t)m0 * n : nullptr));
        } else {
            LB_TRY(chunk_props(m0, mc, Pdst));
        }
        for (int m = 0; m < mc; ++m) {
            matvec_kernel<<<(n * 64 + 255) / 256, 256, 0, s>>>(n, Pdst + (size_t)m * nn, xs + (size_t)(m0 + m) * n,
                                                              xs + (size_t)(m0 + m + 1) * n);
        }
        LB_TRY(check_launch("matvec"));
    }
    fidelity_kernel<<<1, 256, 0, s>>>(n, w, xs + (size_t)M * n, d_F);
    LB_TRY(check_launch("fidelity"));
    LB_HIP(hipMemcpyAsync(F, d_F, sizeof(double), hipMemcpyDeviceToHost, s));
    if (!grad) {
        LB_HIP(hipStreamSynchronize(s));
        return LB_OK;
    }
    // ---- backward, chunks from the last slice
    LB_HIP(hipMemcpyAsync(lams + (size_t)M * n, w, n * sizeof(cd), hipMemcpyDeviceToDevice, s));
    const int nchunks = (M + Mc - 1) / Mc;
    for (int ci = nchunks - 1; ci >= 0; --ci) {
        const int m0 = ci * Mc, mc = M - m0 < Mc ? M - m0 : Mc;
        const cd *Pch = keepP ? Pall + (size_t)m0 * nn : Pc;
        if (!keepP) LB_TRY(chunk_props(m0, mc, Pc));
        for (int m = mc - 1; m >= 0; --m) {
            matvec_h_partial_kernel<<<dim3((n + 63) / 64, HR), 256, 0, s>>>(n, Pch + (size_t)m * nn,
                                                                            lams + (size_t)(m0 + m + 1) * n, hpart);
            matvec_h_reduce_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, hpart, lams + (size_t)(m0 + m) * n);
        }
        LB_TRY(check_launch("matvec_h"));
        // generators of the chunk, then the batched Frechet derivatives
        LB_TRY(generators_launch(n, mc, C, L0, Lc, u + (size_t)m0 * C, Lg, s));
        const size_t mark = ws->used;
        cd *G = (cd *)ws_take(ws, (size_t)mc * matb);
        const Keep kv = keep ? keep_view(cache, M, m0, nn) : Keep{};
        if (keep && lowrank)
            LB_TRY(frechet_lowrank_chunk(n, mc, Lg, dts.data(), xs + (size_t)m0 * n, lams + (size_t)(m0 + 1) * n,
                                         theta, G, ws, s, kv, ipiv_keep + (size_t)m0 * n));
        else
            LB_TRY(frechet_chunk(n, mc, Lg, dts.data(), xs + (size_t)m0 * n, lams + (size_t)(m0 + 1) * n, theta, G,
                                 ws, s, keep ? &kv : nullptr));
        if (C > 0) {
            dim3 cg(nblk, mc);
            contract_kernel<<<cg, 256, 0, s>>>((long long)nn, C, LcT, G, mc, partial);
            LB_TRY(check_launch("contract"));
            contract_reduce_kernel<<<(mc * C + 255) / 256, 256, 0, s>>>(nblk, mc, C, dt, partial,
                                                                        grad + (size_t)m0 * C);
            LB_TRY(check_launch("contract_reduce"));
        }
        ws->used = mark;
    }
    LB_HIP(hipStreamSynchronize(s));
    return LB_OK;
}

}  // namespace lb

using namespace lb;

extern "C" int grape_gradient(int n, int M, int C, const void *L0, const void *Lc, const double *u, double dt,
                              double theta, const void *x0, const void *w, double *F, double *grad,
                              long long checkpoint_bytes, lb_workspace *ws, hipStream_t stream) {
    if (n < 1 || n > 4096) return fail(LB_ESHAPE, "grape_gradient: n must be in [1, 4096]");
    if (M < 1 || C < 0 || C > grape::CMAX) return fail(LB_ESHAPE, "grape_gradient: need M >= 1, 0 <= C <= 16");
    if (!L0 || !x0 || !w || !F || (C > 0 && (!Lc || !u))) return fail(LB_EINVAL, "grape_gradient: NULL pointer");
    if (!std::isfinite(dt) || !(theta > 0.0)) return fail(LB_EINVAL, "grape_gradient: bad dt or theta");
    Workspace *wsp = ws_resolve(ws);
    ws_begin(wsp, stream);
    return grape_run(n, M, C, static_cast<const cd *>(L0), static_cast<const cd *>(Lc), u, dt, theta,
                     static_cast<const cd *>(x0), static_cast<const cd *>(w), F, grad, checkpoint_bytes, wsp, stream);
}
