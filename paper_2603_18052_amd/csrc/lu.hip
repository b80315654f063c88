// Batched solve D X = N (n x n, nrhs right-hand sides) by LU with partial
// pivoting -- the denominator solve of Alg. 1, where D = V - U and N = V + U.
//
// Right-looking factorisation blocked on two levels: outer blocks J of
// NBO = 64 columns (batches of 8 or more matrices; single panels below, where
// launch latency rules), each factored as four panels of NB = 16 columns.  The
// right-hand sides ride along as extra columns of the trailing matrix, so the
// forward substitution L^{-1} Pi N happens inside the factorisation's
// updates.  Per outer block J:
//   per panel, with updates confined to J's columns (all rows):
//     1. lu_panel: one workgroup per matrix (256 threads up to 768 rows,
//        1024 beyond), each thread holds whole rows of the panel in
//        registers; per column a block-wide argmax of |a|^2 (lowest row on
//        ties), a row exchange through LDS, the multipliers and the rank-1
//        update of the rest of the panel;
//     2. the panel's row exchanges on the earlier panels' L columns of J (so
//        that J's L ends in the final row order), and exchanges plus the
//        unit-lower solve of the panel rows on J's later columns;
//     3. a batched MFMA GEMM A22 -= L21 U12 on J's later columns;
//   then on every column right of J (D's trailing columns and all of N): all
//   of J's exchanges in order, the unit-lower solve of J's rows (per panel,
//   a 16-row solve and a GEMM on J's rows below it), and one rank-64 GEMM
//   update of the rows below J -- a quarter of the trailing-matrix traffic of
//   one rank-16 update per panel.  Factored columns left of J are not
//   exchanged (they are not needed again).
// Then back substitution with U, blocked the same way: per outer block of
// rows from the bottom, NB-row solves (trsm_upper) with their updates kept to
// the outer block's rows, then one rank-NBO update N_above -= U_above,J X_J.
#include <climits>
#include <utility>

#include "lb_internal.hpp"

namespace lb {

constexpr int NB = 16;
constexpr int NBO = 64;  // outer block: 4 panels, one rank-64 trailing update
constexpr int kOuterMinBatch = 8;  // below this many matrices: NB-wide blocks
constexpr int PANEL_THREADS = 1024;

template <int R>
__global__ void __launch_bounds__(PANEL_THREADS) lu_panel_kernel(cd *D, int n, long long sD, int k0, int *ipiv,
                                                                 int *info) {
    const int b = blockIdx.x;
    cd *A = D + (size_t)b * sD;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nrows = n - k0;
    const int ncols = min(NB, n - k0);

    __shared__ double red_v[PANEL_THREADS / 64];
    __shared__ int red_i[PANEL_THREADS / 64];
    __shared__ cd rowbuf[2][NB];
    __shared__ int s_piv;

    cd a[R][NB];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + PANEL_THREADS * q;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            a[q][c] = (r < nrows && c < ncols) ? A[(size_t)(k0 + r) * n + k0 + c] : cd{0.0, 0.0};
    }

#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j < ncols) {
        // ---- pivot search: largest |a|^2 in column j among rows >= j
        double bv = -1.0;
        int bi = INT_MAX;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = tid + PANEL_THREADS * q;
            if (r >= j && r < nrows) {
                const double v = a[q][j].re * a[q][j].re + a[q][j].im * a[q][j].im;
                if (v > bv) {
                    bv = v;
                    bi = r;
                }
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double ov = __shfl_xor(bv, off);
            const int oi = __shfl_xor(bi, off);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0) {
            red_v[wave] = bv;
            red_i[wave] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            double v = red_v[0];
            int i = red_i[0];
            for (int w = 1; w < PANEL_THREADS / 64; ++w)
                if (red_v[w] > v || (red_v[w] == v && red_i[w] < i)) {
                    v = red_v[w];
                    i = red_i[w];
                }
            if (!(v > 0.0)) {  // zero (or NaN) pivot: flag, keep going on the diagonal
                info[b] = 1;
                i = j;
            }
            s_piv = i;
            ipiv[(size_t)b * n + k0 + j] = k0 + i;
        }
        __syncthreads();
        const int p = s_piv;
        // ---- row exchange j <-> p through LDS; rowbuf[0] ends up holding the pivot row
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = tid + PANEL_THREADS * q;
            if (r == p) {
#pragma unroll
                for (int c = 0; c < NB; ++c) rowbuf[0][c] = a[q][c];
            }
            if (r == j && p != j) {
#pragma unroll
                for (int c = 0; c < NB; ++c) rowbuf[1][c] = a[q][c];
            }
        }
        __syncthreads();
        if (p != j) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int r = tid + PANEL_THREADS * q;
                if (r == j) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) a[q][c] = rowbuf[0][c];
                } else if (r == p) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) a[q][c] = rowbuf[1][c];
                }
            }
        }
        // ---- multipliers and rank-1 update of the remaining panel columns
        const cd u = rowbuf[0][j];
        const double den = u.re * u.re + u.im * u.im;
        const cd inv = {u.re / den, -u.im / den};
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = tid + PANEL_THREADS * q;
            if (r > j && r < nrows) {
                const cd l = cmul(a[q][j], inv);
                a[q][j] = l;
#pragma unroll
                for (int c = j + 1; c < NB; ++c) {
                    const cd uc = rowbuf[0][c];
                    a[q][c].re = fma(-l.re, uc.re, fma(l.im, uc.im, a[q][c].re));
                    a[q][c].im = fma(-l.re, uc.im, fma(-l.im, uc.re, a[q][c].im));
                }
            }
        }
        __syncthreads();  // rowbuf is rewritten by the next column
        }
    }

#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + PANEL_THREADS * q;
        if (r < nrows) {
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < ncols) A[(size_t)(k0 + r) * n + k0 + c] = a[q][c];
        }
    }
}

// The same panel factorisation for panels of at most 3 x 256 rows, by four
// wavefronts: each thread holds R rows; per column a wavefront argmax by
// shuffles, the four wavefront results through LDS and resolved by every
// thread (one barrier), then the pivot row and row j through LDS (a second
// barrier).  LDS is double-buffered by column parity, so two barriers per
// column suffice.  The same pivot rule and the same per-element arithmetic as
// lu_panel_kernel.  The column index is a template argument
// (spanel_col<R, J>), so every register-array index is static and the rows
// stay in registers for every R.
constexpr int SPANEL_THREADS = 256;
constexpr int SPANEL_MAX_ROWS = 3 * SPANEL_THREADS;
constexpr int SPANEL_WAVES = SPANEL_THREADS / 64;

struct SpanelLds {
    double red_v[2][SPANEL_WAVES];
    int red_i[2][SPANEL_WAVES];
    cd rowbuf[2][2][NB];  // [column parity][pivot row, row j]
};

template <int R, int J>
__device__ __forceinline__ void spanel_col(cd (&a)[R][NB], SpanelLds &sm, int tid, int nrows, int ncols, int n,
                                           int k0, int b, int *ipiv, int *info) {
    if (J >= ncols) return;  // uniform
    constexpr int par = J & 1;
    const int lane = tid & 63, wave = tid >> 6;
    // ---- pivot search: largest |a|^2 in column J among rows >= J (lowest row on ties)
    double bv = -1.0;
    int bi = INT_MAX;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + SPANEL_THREADS * q;
        if (r >= J && r < nrows) {
            const double v = a[q][J].re * a[q][J].re + a[q][J].im * a[q][J].im;
            if (v > bv) {
                bv = v;
                bi = r;
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    if (lane == 0) {
        sm.red_v[par][wave] = bv;
        sm.red_i[par][wave] = bi;
    }
    __syncthreads();
    double v = sm.red_v[par][0];
    int p = sm.red_i[par][0];
#pragma unroll
    for (int w = 1; w < SPANEL_WAVES; ++w)
        if (sm.red_v[par][w] > v || (sm.red_v[par][w] == v && sm.red_i[par][w] < p)) {
            v = sm.red_v[par][w];
            p = sm.red_i[par][w];
        }
    const bool zero = !(v > 0.0);  // zero (or NaN) pivot: flag, keep going on the diagonal
    if (zero) p = J;
    if (tid == 0) {
        if (zero) info[b] = 1;
        ipiv[(size_t)b * n + k0 + J] = k0 + p;
    }
    // ---- row exchange J <-> p through LDS; rowbuf[par][0] holds the pivot row
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + SPANEL_THREADS * q;
        if (r == p) {
#pragma unroll
            for (int c = 0; c < NB; ++c) sm.rowbuf[par][0][c] = a[q][c];
        }
        if (r == J && p != J) {
#pragma unroll
            for (int c = 0; c < NB; ++c) sm.rowbuf[par][1][c] = a[q][c];
        }
    }
    __syncthreads();
    if (p != J) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = tid + SPANEL_THREADS * q;
            if (r == J) {
#pragma unroll
                for (int c = 0; c < NB; ++c) a[q][c] = sm.rowbuf[par][0][c];
            } else if (r == p) {
#pragma unroll
                for (int c = 0; c < NB; ++c) a[q][c] = sm.rowbuf[par][1][c];
            }
        }
    }
    // ---- multipliers and rank-1 update of the remaining panel columns (the
    // pivot row read from LDS once, into registers)
    cd ur[NB];
#pragma unroll
    for (int c = J; c < NB; ++c) ur[c] = sm.rowbuf[par][0][c];
    const cd u = ur[J];
    const double den = u.re * u.re + u.im * u.im;
    const cd inv = {u.re / den, -u.im / den};
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + SPANEL_THREADS * q;
        if (r > J && r < nrows) {
            const cd l = cmul(a[q][J], inv);
            a[q][J] = l;
#pragma unroll
            for (int c = J + 1; c < NB; ++c) {
                a[q][c].re = fma(-l.re, ur[c].re, fma(l.im, ur[c].im, a[q][c].re));
                a[q][c].im = fma(-l.re, ur[c].im, fma(-l.im, ur[c].re, a[q][c].im));
            }
        }
    }
}

template <int R, int... J>
__device__ __forceinline__ void spanel_cols(std::integer_sequence<int, J...>, cd (&a)[R][NB], SpanelLds &sm, int tid,
                                            int nrows, int ncols, int n, int k0, int b, int *ipiv, int *info) {
    (spanel_col<R, J>(a, sm, tid, nrows, ncols, n, k0, b, ipiv, info), ...);
}

template <int R>
__global__ void __launch_bounds__(SPANEL_THREADS) lu_panel_small_kernel(cd *D, int n, long long sD, int k0,
                                                                        int *ipiv, int *info) {
    const int b = blockIdx.x;
    cd *A = D + (size_t)b * sD;
    const int tid = threadIdx.x;
    const int nrows = n - k0;
    const int ncols = min(NB, n - k0);
    __shared__ SpanelLds sm;

    cd a[R][NB];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + SPANEL_THREADS * q;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            a[q][c] = (r < nrows && c < ncols) ? A[(size_t)(k0 + r) * n + k0 + c] : cd{0.0, 0.0};
    }
    spanel_cols<R>(std::make_integer_sequence<int, NB>{}, a, sm, tid, nrows, ncols, n, k0, b, ipiv, info);
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + SPANEL_THREADS * q;
        if (r < nrows) {
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < ncols) A[(size_t)(k0 + r) * n + k0 + c] = a[q][c];
        }
    }
}

// Row exchanges of the panel k0 (rows k0 .. k0 + nb) and X1 = L11^{-1} X1
// (its unit-lower block) on D columns [dc0, dc0 + dcount) and the first
// ncount columns of N, one column per thread; either step can be skipped.
// The panel's exchanges (row k0 + jj with row ipiv[jj], in order) are first
// composed into one permutation of at most 2 NB rows (the panel's rows and
// the pivot rows below it), so each column reads every moved row once and
// writes it once: one memory round trip instead of one per exchange.
__global__ void __launch_bounds__(256) swap_trsm_lower_kernel(cd *D, cd *N, int n, int nrhs, long long sD,
                                                              long long sN, int k0, int nb, const int *ipiv, int dc0,
                                                              int dcount, int ncount, int do_swap, int do_solve) {
    const int b = blockIdx.y;
    cd *Dm = D + (size_t)b * sD;
    cd *Nm = N ? N + (size_t)b * sN : nullptr;
    __shared__ cd L11[NB][NB];
    // rows touched: the panel's nb rows (pos = k0 + i), then the pivot rows
    // below it; src = the original row whose values end in that row.  Unused
    // entries name row k0 on both sides (a read of row k0 and a write of its
    // own value, before the panel rows are written): every column then reads
    // and writes a fixed count of rows with no branches, so the reads issue
    // together.
    __shared__ int pos[2 * NB], src[2 * NB], pv[NB];
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        L11[i][j] = (do_solve && i < nb && j < nb) ? Dm[(size_t)(k0 + i) * n + k0 + j] : cd{0.0, 0.0};
    }
    if (threadIdx.x < NB) pv[threadIdx.x] = do_swap && threadIdx.x < nb ? ipiv[(size_t)b * n + k0 + threadIdx.x] : 0;
    __syncthreads();
    if (threadIdx.x == 0) {  // from LDS only: no global-memory round trip in this serial part
        for (int i = 0; i < 2 * NB; ++i) pos[i] = src[i] = k0 + (i < nb ? i : 0);
        int m = NB;  // next entry for a row below the panel
        if (do_swap) {
            for (int jj = 0; jj < nb; ++jj) {
                const int p = pv[jj];
                bool seen = p < k0 + nb;
                for (int i = NB; i < m && !seen; ++i) seen = pos[i] == p;
                if (!seen) pos[m] = src[m] = p, ++m;
            }
            for (int jj = 0; jj < nb; ++jj) {  // the exchanges in order, on the contents
                const int p = pv[jj];
                if (p != k0 + jj) {
                    int ip = p - k0;  // index of row p (a panel row, or one below it)
                    if (p >= k0 + nb)
                        for (int i = NB; i < m; ++i)
                            if (pos[i] == p) ip = i;
                    const int t = src[jj];
                    src[jj] = src[ip];
                    src[ip] = t;
                }
            }
        }
    }
    __syncthreads();
    const int v = blockIdx.x * blockDim.x + threadIdx.x;  // one column per thread (grid covers all)
    if (v < dcount + ncount) {
        cd *col = v < dcount ? Dm + (dc0 + v) : Nm + (v - dcount);
        const size_t ld = v < dcount ? (size_t)n : (size_t)nrhs;
        // every read before any write (the row indices first: a write through
        // col could alias the LDS tables as far as the compiler knows)
        int rs[2 * NB], rd[NB];
#pragma unroll
        for (int i = 0; i < 2 * NB; ++i) rs[i] = src[i];
#pragma unroll
        for (int i = 0; i < NB; ++i) rd[i] = pos[NB + i];
        cd x[NB], w[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) x[i] = col[(size_t)rs[i] * ld];
#pragma unroll
        for (int i = 0; i < NB; ++i) w[i] = col[(size_t)rs[NB + i] * ld];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            double *q = reinterpret_cast<double *>(col + (size_t)rd[i] * ld);
            q[0] = w[i].re;
            q[1] = w[i].im;
        }
        if (do_solve) {
#pragma unroll
            for (int i = 1; i < NB; ++i) {
                if (i < nb) {
                    cd acc = x[i];
#pragma unroll
                    for (int j = 0; j < i; ++j) {
                        const cd l = L11[i][j];
                        acc.re = fma(-l.re, x[j].re, fma(l.im, x[j].im, acc.re));
                        acc.im = fma(-l.re, x[j].im, fma(-l.im, x[j].re, acc.im));
                    }
                    x[i] = acc;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i)
            if (i < nb) col[(size_t)(k0 + i) * ld] = x[i];
    }
}

// X_block = U_block^{-1} X_block for the rows [b0, b0 + nb) of every column of N.
__global__ void __launch_bounds__(256) trsm_upper_kernel(const cd *D, cd *N, int n, int nrhs, long long sD, long long sN,
                                                         int b0, int nb) {
    const int b = blockIdx.y;
    const cd *Dm = D + (size_t)b * sD;
    cd *Nm = N + (size_t)b * sN;
    __shared__ cd U[NB][NB];
    __shared__ cd Ur[NB];  // 1 / U[i][i], so that the per-column chain holds no division
    for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        U[i][j] = (i < nb && j < nb) ? Dm[(size_t)(b0 + i) * n + b0 + j] : cd{1.0, 0.0};
    }
    __syncthreads();
    if (threadIdx.x < NB) {
        const cd d = U[threadIdx.x][threadIdx.x];
        const double den = d.re * d.re + d.im * d.im;
        Ur[threadIdx.x] = {d.re / den, -d.im / den};
    }
    __syncthreads();
    const int c = blockIdx.x * blockDim.x + threadIdx.x;  // one column per thread (grid covers all)
    if (c < nrhs) {
        cd x[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) x[i] = i < nb ? Nm[(size_t)(b0 + i) * nrhs + c] : cd{0.0, 0.0};
#pragma unroll
        for (int i = NB - 1; i >= 0; --i) {
            if (i < nb) {
                cd acc = x[i];
#pragma unroll
                for (int j = i + 1; j < NB; ++j)
                    if (j < nb) {
                        const cd u = U[i][j];
                        acc.re = fma(-u.re, x[j].re, fma(u.im, x[j].im, acc.re));
                        acc.im = fma(-u.re, x[j].im, fma(-u.im, x[j].re, acc.im));
                    }
                x[i] = cmul(acc, Ur[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i)
            if (i < nb) Nm[(size_t)(b0 + i) * nrhs + c] = x[i];
    }
}

static int swap_trsm(cd *D, cd *N, int n, int nrhs, int batch, int k0, int nb, const int *ipiv, int dc0, int dcount,
                     int ncount, bool do_swap, bool do_solve, hipStream_t s) {
    if (dcount + ncount <= 0) return LB_OK;
    const long long sD = (long long)n * n, sN = (long long)n * nrhs;
    dim3 grid((dcount + ncount + 255) / 256, batch);
    swap_trsm_lower_kernel<<<grid, 256, 0, s>>>(D, N, n, nrhs, sD, sN, k0, nb, ipiv, dc0, dcount, ncount,
                                                do_swap ? 1 : 0, do_solve ? 1 : 0);
    return check_launch("swap_trsm_lower");
}

// C[b] -= A[b] B[b] on sub-blocks (row-major, leading dimensions la, lb, lc)
static int gemm_sub(int M, int N, int K, int batch, const cd *A, long long la, long long sA, const cd *B, long long lb,
                    long long sB, cd *C, long long lc, long long sC, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return LB_OK;
    ZgemmBatch g;
    g.M = M, g.N = N, g.K = K, g.batch = batch;
    g.A = A, g.lda = la, g.sA = sA;
    g.B = B, g.ldb = lb, g.sB = sB;
    g.D = C, g.ldd = lc, g.sD = sC;
    g.Cin = C, g.ldc = lc, g.sC = sC;
    g.alpha = -1.0, g.beta = 1.0;
    return zgemm_batched(g, s);
}

static int back_subst(int n, int nrhs, int batch, const cd *D, cd *N, int nbo, hipStream_t s);

// The right-hand-side steps of outer block J = [K0, KE) after its panels are
// factored: all of J's exchanges, the unit-lower solve of J's rows (per
// panel, a 16-row solve and a GEMM on J's rows below it), one update of the
// rows below J.  D's trailing columns (dtr of them, right of J) ride along.
static int rhs_block(int n, int nrhs, int batch, cd *D, cd *N, const int *ipiv, int K0, int KE, int dtr,
                     hipStream_t s) {
    const long long sD = (long long)n * n, sN = (long long)n * nrhs;
    const int W = KE - K0;
    const bool one = W <= NB;  // a single panel: exchanges and solve in one pass
    for (int k0 = K0; k0 < KE && !one; k0 += NB) {
        const int nb = KE - k0 < NB ? KE - k0 : NB;
        LB_TRY(swap_trsm(D, N, n, nrhs, batch, k0, nb, ipiv, KE, dtr, nrhs, true, false, s));
    }
    for (int k0 = K0; k0 < KE; k0 += NB) {
        const int nb = KE - k0 < NB ? KE - k0 : NB;
        LB_TRY(swap_trsm(D, N, n, nrhs, batch, k0, nb, ipiv, KE, dtr, nrhs, one, true, s));
        const int mrows = KE - k0 - nb;  // rows of J below the panel
        LB_TRY(gemm_sub(mrows, dtr, nb, batch, D + (size_t)(k0 + nb) * n + k0, n, sD, D + (size_t)k0 * n + KE, n, sD,
                        D + (size_t)(k0 + nb) * n + KE, n, sD, s));
        LB_TRY(gemm_sub(mrows, nrhs, nb, batch, D + (size_t)(k0 + nb) * n + k0, n, sD, N + (size_t)k0 * nrhs, nrhs,
                        sN, N + (size_t)(k0 + nb) * nrhs, nrhs, sN, s));
    }
    LB_TRY(gemm_sub(n - KE, dtr, W, batch, D + (size_t)KE * n + K0, n, sD, D + (size_t)K0 * n + KE, n, sD,
                    D + (size_t)KE * n + KE, n, sD, s));
    return gemm_sub(n - KE, nrhs, W, batch, D + (size_t)KE * n + K0, n, sD, N + (size_t)K0 * nrhs, nrhs, sN,
                    N + (size_t)KE * nrhs, nrhs, sN, s);
}

int lu_solve_batched(int n, int nrhs, int batch, cd *D, cd *N, int *ipiv, int *info, hipStream_t s) {
    const long long sD = (long long)n * n, sN = (long long)n * nrhs;
    if (batch > 65535) return fail(LB_ESHAPE, "lu_solve: batch > 65535");
    // small batches are bound by launch latency: one panel per block there
    const int nbo = batch >= kOuterMinBatch ? NBO : NB;
    for (int K0 = 0; K0 < n; K0 += nbo) {
        const int W = n - K0 < nbo ? n - K0 : nbo, KE = K0 + W;
        // ---- the outer block J = [K0, KE): 16-column panels, updates kept to J
        for (int k0 = K0; k0 < KE; k0 += NB) {
            const int nb = KE - k0 < NB ? KE - k0 : NB;
            if (n - k0 <= SPANEL_THREADS)
                lu_panel_small_kernel<1><<<batch, SPANEL_THREADS, 0, s>>>(D, n, sD, k0, ipiv, info);
            else if (n - k0 <= 2 * SPANEL_THREADS)
                lu_panel_small_kernel<2><<<batch, SPANEL_THREADS, 0, s>>>(D, n, sD, k0, ipiv, info);
            else if (n - k0 <= SPANEL_MAX_ROWS)
                lu_panel_small_kernel<3><<<batch, SPANEL_THREADS, 0, s>>>(D, n, sD, k0, ipiv, info);
            else if (n - k0 <= PANEL_THREADS)
                lu_panel_kernel<1><<<batch, PANEL_THREADS, 0, s>>>(D, n, sD, k0, ipiv, info);
            else if (n - k0 <= 2 * PANEL_THREADS)
                lu_panel_kernel<2><<<batch, PANEL_THREADS, 0, s>>>(D, n, sD, k0, ipiv, info);
            else
                lu_panel_kernel<4><<<batch, PANEL_THREADS, 0, s>>>(D, n, sD, k0, ipiv, info);
            LB_TRY(check_launch("lu_panel"));
            // the panel's exchanges also reach the earlier panels' L columns of J
            LB_TRY(swap_trsm(D, nullptr, n, nrhs, batch, k0, nb, ipiv, K0, k0 - K0, 0, true, false, s));
            // and the rest of J: exchanges, U12 = L11^{-1} A12, A22 -= L21 U12
            LB_TRY(swap_trsm(D, nullptr, n, nrhs, batch, k0, nb, ipiv, k0 + nb, KE - k0 - nb, 0, true, true, s));
            LB_TRY(gemm_sub(n - k0 - nb, KE - k0 - nb, nb, batch, D + (size_t)(k0 + nb) * n + k0, n, sD,
                            D + (size_t)k0 * n + k0 + nb, n, sD, D + (size_t)(k0 + nb) * n + k0 + nb, n, sD, s));
        }
        // ---- the columns right of J (of D and all of N): all of J's exchanges,
        // the unit-lower solve of J's rows, then one update of the rows below
        LB_TRY(rhs_block(n, nrhs, batch, D, N, ipiv, K0, KE, n - KE, s));
    }
    return back_subst(n, nrhs, batch, D, N, nbo, s);
}

// Back substitution with U (above the diagonal of the factored D), blocked
// like the factorization: per outer block of rows from the bottom, NB-row
// solves with updates kept to the block, then one update of every row above.
static int back_subst(int n, int nrhs, int batch, const cd *D, cd *N, int nbo, hipStream_t s) {
    const long long sD = (long long)n * n, sN = (long long)n * nrhs;
    const int nblk = (n + NB - 1) / NB;
    const int per_outer = nbo / NB;
    for (int ob = (nblk - 1) / per_outer; ob >= 0; --ob) {
        const int B0 = ob * nbo, BE = n < B0 + nbo ? n : B0 + nbo;
        for (int blk = (BE - 1) / NB; blk >= B0 / NB; --blk) {
            const int b0 = blk * NB;
            const int nb = n - b0 < NB ? n - b0 : NB;
            dim3 grid((nrhs + 255) / 256, batch);
            trsm_upper_kernel<<<grid, 256, 0, s>>>(D, N, n, nrhs, sD, sN, b0, nb);
            LB_TRY(check_launch("trsm_upper"));
            // rows [B0, b0) -= U[B0:b0, b0:b0+nb] X[b0:b0+nb]
            LB_TRY(gemm_sub(b0 - B0, nrhs, nb, batch, D + (size_t)B0 * n + b0, n, sD, N + (size_t)b0 * nrhs, nrhs, sN,
                            N + (size_t)B0 * nrhs, nrhs, sN, s));
        }
        // rows [0, B0) -= U[0:B0, B0:BE] X[B0:BE]
        LB_TRY(gemm_sub(B0, nrhs, BE - B0, batch, D + B0, n, sD, N + (size_t)B0 * nrhs, nrhs, sN, N, nrhs, sN, s));
    }
    return LB_OK;
}

// Solve with a factorization lu_solve_batched left in D (and ipiv): the
// right-hand-side steps of every outer block in the factorization's order,
// then the back substitution.  The same operations on the right-hand sides
// as solving them during the factorization (each column is independent), so
// the same results, provided batch is on the same side of kOuterMinBatch.
int lu_resolve_batched(int n, int nrhs, int batch, const cd *D, cd *N, const int *ipiv, hipStream_t s) {
    if (batch > 65535) return fail(LB_ESHAPE, "lu_resolve: batch > 65535");
    const int nbo = batch >= kOuterMinBatch ? NBO : NB;
    cd *Dm = const_cast<cd *>(D);  // only read: no trailing D columns are passed
    for (int K0 = 0; K0 < n; K0 += nbo) {
        const int KE = n - K0 < nbo ? n : K0 + nbo;
        LB_TRY(rhs_block(n, nrhs, batch, Dm, N, ipiv, K0, KE, 0, s));
    }
    return back_subst(n, nrhs, batch, D, N, nbo, s);
}

}  // namespace lb
