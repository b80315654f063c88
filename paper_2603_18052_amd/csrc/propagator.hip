// Alg. 1: P = exp(L dt) by Pade [13/13] scaling and squaring, batched over M
// generators, FP64 throughout.
//   norm1_kernel     ||L dt||_1 per matrix (column sums of moduli, max)
//   sexp_kernel      s = smallest s >= 0 with ||A||_1 <= theta 2^s (exact), on
//                    the device (the internal synchronous builds of the GRAPE
//                    gradient and the mixed batch take it on the host)
//   scale_kernel     A = (L dt) 2^-s
//   zgemm            A2, A4, A6; V, W' with fused linear-combination epilogues; U
//   zlincomb         V - U, V + U
//   lu_solve         (V - U) P = (V + U)
//   zgemm (masked)   s squarings, ping-pong between two buffers
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "lb_internal.hpp"

namespace lb {

// Pade [13/13] coefficients, b_13 = 1 and b_k = b_{k+1} (26 - k)(k + 1) / (13 - k):
// the ratio of consecutive terms of (26 - k)! / (k! (13 - k)!).  Exact in 64-bit
// integers (the largest intermediate is 8.4e17), each converted once to double.
void pade13_coefficients(double b[14]) {
    unsigned long long c = 1;
    b[13] = 1.0;
    for (int k = 12; k >= 0; --k) {
        c = c * (unsigned long long)(26 - k) * (unsigned long long)(k + 1) / (unsigned long long)(13 - k);
        b[k] = (double)c;
    }
}

// Column sums of |L dt| over all rows, max over the columns of each matrix,
// merged across workgroups with an integer atomic max on the bit pattern
// (non-negative doubles order like their bits; NaN wins).  A workgroup takes
// 16 columns: per block of 256 rows all its threads compute the moduli
// (coalesced 256-byte row pieces) into LDS, then 16 threads add them to their
// column's sum in row order, so every column is summed in the order of a
// plain loop over the rows.
constexpr int N1_COLS = 16, N1_ROWS = 256;
__global__ void __launch_bounds__(256) norm1_kernel(int n, const cd *__restrict__ L, const double *__restrict__ dt,
                                                    unsigned long long *__restrict__ normbits) {
    const int m = blockIdx.y;
    const cd *Lm = L + (size_t)m * n * n;
    const double h = dt[m];
    const int j0 = blockIdx.x * N1_COLS, tid = threadIdx.x;
    __shared__ double mag[N1_ROWS][N1_COLS + 1];
    double s = 0.0;  // the column sum of thread tid < N1_COLS
    for (int i0 = 0; i0 < n; i0 += N1_ROWS) {
        for (int e = tid; e < N1_ROWS * N1_COLS; e += 256) {
            const int r = e / N1_COLS, c = e - r * N1_COLS;
            const int i = i0 + r, j = j0 + c;
            double v = 0.0;
            if (i < n && j < n) {
                const cd x = Lm[(size_t)i * n + j];
                v = hypot(x.re * h, x.im * h);
            }
            mag[r][c] = v;
        }
        __syncthreads();
        if (tid < N1_COLS) {
            const int rows = min(N1_ROWS, n - i0);
            for (int r = 0; r < rows; ++r) s += mag[r][tid];
        }
        __syncthreads();
    }
    if (tid < N1_COLS) mag[0][tid] = s;  // the last barrier ended every read of mag
    __syncthreads();
    if (tid == 0) {
        double best = 0.0;
        for (int c = 0; c < N1_COLS; ++c) {
            const double o = mag[0][c];
            if (isnan(o) || (!isnan(best) && o > best)) best = o;  // NaN wins
        }
        atomicMax(normbits + m, (unsigned long long)__double_as_longlong(best));
    }
}

__global__ void fill_u64_kernel(unsigned long long *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0ull;
}

__global__ void fill_i32_kernel(int *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// A = (L dt) 2^-s, elementwise (the dt product is rounded first, the power of
// two is exact).
__global__ void __launch_bounds__(256) scale_kernel(long long nn, int M, const cd *__restrict__ L,
                                                    const double *__restrict__ dt, const int *__restrict__ sexp,
                                                    cd *__restrict__ A) {
    const long long total = nn * M;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int m = (int)(e / nn);
        const double h = dt[m];
        const int s = sexp[m];
        const cd v = L[e];
        A[e] = {ldexp(v.re * h, -s), ldexp(v.im * h, -s)};
    }
}

// Copy src -> dst for the matrices whose squaring count is odd (their last
// squaring landed in the scratch buffer).
__global__ void __launch_bounds__(256) odd_copy_kernel(long long nn, int M, const int *__restrict__ sexp,
                                                       const cd *__restrict__ src, cd *__restrict__ dst) {
    const long long total = nn * M;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int m = (int)(e / nn);
        if (sexp[m] & 1) dst[e] = src[e];
    }
}

static int grid_1d(long long work) {
    long long g = (work + 255) / 256;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

int scaling_exponent(double norm, double theta) {
    if (!std::isfinite(norm)) return -1;
    int s = 0;
    while (norm > std::ldexp(theta, s)) ++s;
    return s;
}

int scaling_stage(int n, int M, const cd *L, const double *dt_host, double theta, double *d_dt,
                  unsigned long long *d_norm, int *d_s, int *s_host, hipStream_t s) {
    LB_HIP(hipMemcpyAsync(d_dt, dt_host, M * sizeof(double), hipMemcpyHostToDevice, s));
    fill_u64_kernel<<<(M + 255) / 256, 256, 0, s>>>(d_norm, M);
    {
        dim3 grid((n + N1_COLS - 1) / N1_COLS, M);
        norm1_kernel<<<grid, 256, 0, s>>>(n, L, d_dt, d_norm);
        LB_TRY(check_launch("norm1"));
    }
    std::vector<unsigned long long> nb(M);
    std::vector<int> sv(M);
    LB_HIP(hipMemcpyAsync(nb.data(), d_norm, M * sizeof(double), hipMemcpyDeviceToHost, s));
    LB_HIP(hipStreamSynchronize(s));
    for (int m = 0; m < M; ++m) {
        double v;
        std::memcpy(&v, &nb[m], sizeof v);
        sv[m] = scaling_exponent(v, theta);
        if (s_host) s_host[m] = sv[m];
        if (sv[m] < 0)
            return fail(LB_ENONFINITE, "lindblad_propagator: ||L dt||_1 of generator " + std::to_string(m) +
                                           " is not finite");
    }
    LB_HIP(hipMemcpyAsync(d_s, sv.data(), M * sizeof(int), hipMemcpyHostToDevice, s));
    LB_HIP(hipStreamSynchronize(s));  // sv leaves scope
    return LB_OK;
}

int fill_i32_launch(int *p, int count, hipStream_t s) {
    if (count <= 0) return LB_OK;
    fill_i32_kernel<<<(count + 255) / 256, 256, 0, s>>>(p, count);
    return check_launch("fill");
}

int scale_launch(int n, int M, const cd *L, const double *d_dt, const int *d_s, cd *A, hipStream_t s) {
    const size_t nn = (size_t)n * n;
    scale_kernel<<<grid_1d((long long)nn * M), 256, 0, s>>>((long long)nn, M, L, d_dt, d_s, A);
    return check_launch("scale");
}

int odd_copy_launch(int n, int M, const int *d_s, const cd *src, cd *dst, hipStream_t s) {
    const size_t nn = (size_t)n * n;
    odd_copy_kernel<<<grid_1d((long long)nn * M), 256, 0, s>>>((long long)nn, M, d_s, src, dst);
    return check_launch("odd_copy");
}

static size_t mask_bytes(int n, int M) { return align256((size_t)zgemm_mask_bytes(n, n) * M); }

static size_t chunk_bytes(int n, int M) {
    const size_t mat = (size_t)n * n * sizeof(cd) * M;
    return 8 * align256(mat) + 4 * align256(M * sizeof(double)) + align256((size_t)M * n * sizeof(int)) +
           2 * align256(M * sizeof(int)) + 2 * mask_bytes(n, M);
}

size_t build_async_bytes(int n, int M) {
    const size_t mat = (size_t)n * n * sizeof(cd) * M;
    return 8 * align256(mat) + align256((size_t)M * n * sizeof(int)) + 2 * mask_bytes(n, M);
}

// Alg. 1 after its scaling stage, for M matrices whose d_dt and d_s are on
// the device (smax = max s on the host): products, LU solve, squarings.
// Enqueue only, no host synchronisation; zero pivots are flagged in d_info.
int build_chunk_async(int n, int M, const cd *L, const double *d_dt, const int *d_s, int smax, cd *P, int *d_info,
                      Workspace *ws, hipStream_t s, StageClock *clk) {
    auto stage = [&](int i) { return clk ? hipEventRecord(clk->ev[i], s) : hipSuccess; };
    const size_t nn = (size_t)n * n;
    const size_t mat = nn * sizeof(cd) * M;
    LB_TRY(ws_ensure(ws, build_async_bytes(n, M)));
    const size_t mark = ws->used;
    cd *A = (cd *)ws_take(ws, mat);
    cd *A2 = (cd *)ws_take(ws, mat);
    cd *A4 = (cd *)ws_take(ws, mat);
    cd *A6 = (cd *)ws_take(ws, mat);
    cd *T = (cd *)ws_take(ws, mat);
    cd *V = (cd *)ws_take(ws, mat);
    cd *Wp = (cd *)ws_take(ws, mat);
    cd *U = (cd *)ws_take(ws, mat);
    int *d_ipiv = (int *)ws_take(ws, (size_t)M * n * sizeof(int));
    const long long mb = zgemm_mask_bytes(n, n);
    unsigned char *mA = (unsigned char *)ws_take(ws, (size_t)mb * M);
    unsigned char *mA2 = (unsigned char *)ws_take(ws, (size_t)mb * M);
    struct Release {
        Workspace *w;
        size_t m;
        ~Release() { w->used = m; }
    } release{ws, mark};

    LB_TRY(scale_launch(n, M, L, d_dt, d_s, A, s));
    // zero 64 x 16 tiles of the sparse left factors A and A2 are skipped
    LB_TRY(zgemm_tile_mask(n, n, M, A, n, (long long)nn, mA, s));
    LB_HIP(stage(1));
    double b[14];
    pade13_coefficients(b);
    ZgemmBatch g;
    g.M = g.N = g.K = n;
    g.batch = M;
    g.lda = g.ldb = g.ldd = g.ldc = g.ldx = n;
    g.sA = g.sB = g.sD = g.sC = g.sX = (long long)nn;
    auto mul = [&](const cd *X, const cd *Y, cd *Z, const unsigned char *mask = nullptr) {
        ZgemmBatch h = g;
        h.A = X;
        h.B = Y;
        h.D = Z;
        h.amask = mask;
        h.sMask = mb;
        return zgemm_batched(h, s);
    };
    LB_TRY(mul(A, A, A2, mA));
    LB_TRY(zgemm_tile_mask(n, n, M, A2, n, (long long)nn, mA2, s));
    LB_TRY(mul(A2, A2, A4, mA2));
    LB_TRY(mul(A4, A2, A6));
    {  // V = A6 (b12 A6 + b10 A4 + b8 A2) + b6 A6 + b4 A4 + b2 A2 + b0 I
        const cd *X[3] = {A6, A4, A2};
        const double c[3] = {b[12], b[10], b[8]};
        LB_TRY(zlincomb(n, M, 3, X, c, 0.0, T, s));
        ZgemmBatch h = g;
        h.A = A6;
        h.B = T;
        h.D = V;
        h.nx = 3;
        h.X[0] = A6, h.X[1] = A4, h.X[2] = A2;
        h.coef[0] = b[6], h.coef[1] = b[4], h.coef[2] = b[2];
        h.gamma = b[0];
        LB_TRY(zgemm_batched(h, s));
    }
    {  // W' = A6 (b13 A6 + b11 A4 + b9 A2) + b7 A6 + b5 A4 + b3 A2 + b1 I;  U = A W'
        const cd *X[3] = {A6, A4, A2};
        const double c[3] = {b[13], b[11], b[9]};
        LB_TRY(zlincomb(n, M, 3, X, c, 0.0, T, s));
        ZgemmBatch h = g;
        h.A = A6;
        h.B = T;
        h.D = Wp;
        h.nx = 3;
        h.X[0] = A6, h.X[1] = A4, h.X[2] = A2;
        h.coef[0] = b[7], h.coef[1] = b[5], h.coef[2] = b[3];
        h.gamma = b[1];
        LB_TRY(zgemm_batched(h, s));
        LB_TRY(mul(A, Wp, U, mA));
    }
    LB_HIP(stage(2));
    {  // denominator V - U into A2, numerator V + U into P
        const cd *X[2] = {V, U};
        const double cm[2] = {1.0, -1.0}, cp[2] = {1.0, 1.0};
        LB_TRY(zlincomb(n, M, 2, X, cm, 0.0, A2, s));
        LB_TRY(zlincomb(n, M, 2, X, cp, 0.0, P, s));
    }
    LB_HIP(stage(3));
    LB_TRY(lu_solve_batched(n, n, M, A2, P, d_ipiv, d_info, s));
    LB_HIP(stage(4));
    // squarings: level k reads buffer (k even ? P : A4) and writes the other;
    // matrices with s <= k are skipped.
    for (int k = 0; k < smax; ++k) {
        ZgemmBatch h = g;
        const cd *src = (k & 1) ? A4 : P;
        cd *dst = (k & 1) ? P : A4;
        h.A = src;
        h.B = src;
        h.D = dst;
        h.active = d_s;
        h.level = k;
        LB_TRY(zgemm_batched(h, s));
    }
    LB_HIP(stage(5));
    if (smax > 0) LB_TRY(odd_copy_launch(n, M, d_s, A4, P, s));
    return LB_OK;
}

// One chunk of matrices (all buffers sized for `M` matrices): scaling stage,
// the asynchronous build, then the pivot check (two host synchronisations).
static int build_chunk(int n, int M, const cd *L, const double *dt_host, double theta, cd *P, int *s_host,
                       Workspace *ws, hipStream_t s, StageClock *clk) {
    LB_TRY(ws_ensure(ws, chunk_bytes(n, M)));
    const size_t mark = ws->used;
    double *d_dt = (double *)ws_take(ws, M * sizeof(double));
    unsigned long long *d_norm = (unsigned long long *)ws_take(ws, M * sizeof(double));
    int *d_s = (int *)ws_take(ws, M * sizeof(int));
    int *d_info = (int *)ws_take(ws, M * sizeof(int));
    struct Release {
        Workspace *w;
        size_t m;
        ~Release() { w->used = m; }
    } release{ws, mark};

    if (clk) LB_HIP(hipEventRecord(clk->ev[0], s));
    fill_i32_kernel<<<(M + 255) / 256, 256, 0, s>>>(d_info, M);
    std::vector<int> sv(M);
    LB_TRY(scaling_stage(n, M, L, dt_host, theta, d_dt, d_norm, d_s, sv.data(), s));
    if (s_host) std::memcpy(s_host, sv.data(), M * sizeof(int));
    int smax = 0;
    for (int m = 0; m < M; ++m) smax = sv[m] > smax ? sv[m] : smax;
    LB_TRY(build_chunk_async(n, M, L, d_dt, d_s, smax, P, d_info, ws, s, clk));
    if (clk) LB_HIP(hipEventRecord(clk->ev[6], s));
    std::vector<int> info(M);
    LB_HIP(hipMemcpyAsync(info.data(), d_info, M * sizeof(int), hipMemcpyDeviceToHost, s));
    LB_HIP(hipStreamSynchronize(s));
    if (clk) {
        float t[6];
        for (int i = 0; i < 6; ++i) LB_HIP(hipEventElapsedTime(&t[i], clk->ev[i], clk->ev[i + 1]));
        clk->ms[0] += t[3];                // LU solve
        clk->ms[1] += t[1];                // Pade products
        clk->ms[2] += t[4];                // squarings
        clk->ms[3] += t[0] + t[2] + t[5];  // scaling stage, V -/+ U, odd-s copy
    }
    for (int m = 0; m < M; ++m)
        if (info[m]) return fail(LB_ESINGULAR, "lindblad_propagator: zero pivot in V - U of generator " + std::to_string(m));
    return LB_OK;
}

// ------------------------------------------------- stream-ordered build
// Step lengths reach the device as kernel arguments (captured at launch), so
// the host array may be reused as soon as the call returns.
constexpr int kDtPerLaunch = 256;
struct DtArgs {
    double v[kDtPerLaunch];
};
__global__ void set_dt_kernel(DtArgs a, int count, double *__restrict__ d_dt) {
    const int i = threadIdx.x;
    if (i < count) d_dt[i] = a.v[i];
}

// s[m] from ||A_m||_1 by exact comparison with theta 2^s; a non-finite norm
// leaves s = 0 (the build then runs on non-finite values) and flags
// LB_ENONFINITE, an s beyond the squaring cap flags LB_ENOTSUP.  The status
// word keeps the smallest code (atomic min: order independent).
__global__ void sexp_kernel(int M, double theta, const unsigned long long *__restrict__ normbits, int *__restrict__ d_s,
                            int *__restrict__ s_out, int *__restrict__ status) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const double v = __longlong_as_double((long long)normbits[m]);
    int sv = 0, code = LB_OK;
    if (!isfinite(v)) {
        code = LB_ENONFINITE;
    } else {
        while (v > ldexp(theta, sv)) ++sv;
        if (sv > kMaxSquarings) code = LB_ENOTSUP;
    }
    d_s[m] = sv;
    if (s_out) s_out[m] = sv;
    if (code != LB_OK && status) atomicMin(status, code);
}

// Zero pivots (info[m] != 0) -> LB_ESINGULAR in the status word.
__global__ void pivot_status_kernel(int M, const int *__restrict__ info, int *__restrict__ status) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < M && info[m] && status) atomicMin(status, LB_ESINGULAR);
}

size_t build_async_chunk_bytes(int n, int M) {
    return build_async_bytes(n, M) + 3 * align256(M * sizeof(double)) + align256(M * sizeof(int));
}

static int build_chunk_stream_ordered(int n, int M, const cd *L, const double *dt_host, double theta, cd *P,
                                      int *d_s_out, int *d_status, Workspace *ws, hipStream_t s) {
    LB_TRY(ws_ensure(ws, build_async_chunk_bytes(n, M)));
    const size_t mark = ws->used;
    double *d_dt = (double *)ws_take(ws, M * sizeof(double));
    unsigned long long *d_norm = (unsigned long long *)ws_take(ws, M * sizeof(double));
    int *d_s = (int *)ws_take(ws, M * sizeof(int));
    int *d_info = (int *)ws_take(ws, M * sizeof(double));
    struct Release {
        Workspace *w;
        size_t m;
        ~Release() { w->used = m; }
    } release{ws, mark};
    for (int m0 = 0; m0 < M; m0 += kDtPerLaunch) {
        DtArgs a;
        const int c = M - m0 < kDtPerLaunch ? M - m0 : kDtPerLaunch;
        for (int i = 0; i < c; ++i) a.v[i] = dt_host[m0 + i];
        set_dt_kernel<<<1, kDtPerLaunch, 0, s>>>(a, c, d_dt + m0);
        LB_TRY(check_launch("set_dt"));
    }
    fill_u64_kernel<<<(M + 255) / 256, 256, 0, s>>>(d_norm, M);
    fill_i32_kernel<<<(M + 255) / 256, 256, 0, s>>>(d_info, M);
    {
        dim3 grid((n + N1_COLS - 1) / N1_COLS, M);
        norm1_kernel<<<grid, 256, 0, s>>>(n, L, d_dt, d_norm);
        LB_TRY(check_launch("norm1"));
    }
    sexp_kernel<<<(M + 255) / 256, 256, 0, s>>>(M, theta, d_norm, d_s, d_s_out, d_status);
    LB_TRY(check_launch("sexp"));
    // the squaring levels run up to the cap; a level skips (on the device,
    // per workgroup) every matrix whose s it exceeds
    LB_TRY(build_chunk_async(n, M, L, d_dt, d_s, kMaxSquarings, P, d_info, ws, s));
    pivot_status_kernel<<<(M + 255) / 256, 256, 0, s>>>(M, d_info, d_status);
    return check_launch("pivot_status");
}

int build_propagators_async(int n, int M, const cd *L, const double *dt_host, double theta, cd *P, int *d_s_out,
                            int *d_status, Workspace *ws, hipStream_t s) {
    const size_t avail = ws->fixed ? (ws->size > ws->used ? ws->size - ws->used : 0)
                                   : (ws->used == 0 ? ws->cap : (ws->size > ws->used ? ws->size - ws->used : 0));
    long long chunk = M;
    while (chunk > 1 && build_async_chunk_bytes(n, (int)chunk) > avail) chunk = (chunk + 1) / 2;
    if (chunk > 4096) chunk = 4096;
    if (build_async_chunk_bytes(n, (int)chunk) > avail)
        return fail(LB_ENOMEM, "lindblad_propagator: scratch of " + std::to_string(avail) +
                                   " bytes is too small for one n x n build (" +
                                   std::to_string(build_async_chunk_bytes(n, 1)) + " bytes at n = " +
                                   std::to_string(n) + ")");
    const size_t nn = (size_t)n * n;
    for (int m0 = 0; m0 < M; m0 += (int)chunk) {
        const int mc = (int)((M - m0) < chunk ? (M - m0) : chunk);
        LB_TRY(build_chunk_stream_ordered(n, mc, L + nn * m0, dt_host + m0, theta, P + nn * m0,
                                          d_s_out ? d_s_out + m0 : nullptr, d_status, ws, s));
    }
    return LB_OK;
}

static long long build_chunk_size(int n, int M, size_t avail) {
    long long chunk = M;
    while (chunk > 1 && chunk_bytes(n, (int)chunk) > avail) chunk = (chunk + 1) / 2;
    if (chunk > 4096) chunk = 4096;
    return chunk;
}

size_t build_workspace_bytes(int n, int M) { return chunk_bytes(n, M); }

int build_propagators(int n, int M, const cd *L, const double *dt_host, double theta, cd *P, int *s_host,
                      Workspace *ws, hipStream_t s, StageClock *clk) {
    // Chunk the batch so that the eight n x n temporaries per matrix fit in
    // what the workspace can still give (its cap when nothing is taken yet).
    const size_t avail = ws->used == 0 ? ws->cap : (ws->size > ws->used ? ws->size - ws->used : 0);
    const long long chunk = build_chunk_size(n, M, avail);
    if (chunk_bytes(n, (int)chunk) > avail)
        return fail(LB_ENOMEM, "lindblad_propagator: workspace too small for one n x n build");
    const size_t nn = (size_t)n * n;
    for (int m0 = 0; m0 < M; m0 += (int)chunk) {
        const int mc = (int)((M - m0) < chunk ? (M - m0) : chunk);
        LB_TRY(build_chunk(n, mc, L + nn * m0, dt_host + m0, theta, P + nn * m0, s_host ? s_host + m0 : nullptr, ws,
                           s, clk));
    }
    return LB_OK;
}


int propagator_args(const char *who, int n, int M, const void *L, const double *dt, double theta,
                           const void *P) {
    const std::string w(who);
    if (n < 1 || n > 4096) return fail(LB_ESHAPE, w + ": n must be in [1, 4096]");
    if (M < 1) return fail(LB_ESHAPE, w + ": M must be >= 1");
    if (!L || !dt || !P) return fail(LB_EINVAL, w + ": NULL pointer");
    if (!(theta > 0.0) || !std::isfinite(theta)) return fail(LB_EINVAL, w + ": theta must be > 0");
    for (int m = 0; m < M; ++m)
        if (!std::isfinite(dt[m])) return fail(LB_EINVAL, w + ": dt must be finite");
    return LB_OK;
}

}  // namespace lb

using namespace lb;

extern "C" int lindblad_propagator(int n, int M, const void *L, const double *dt, double theta, void *P, int *s_used,
                                   int *status, lb_workspace *ws, hipStream_t stream) {
    LB_TRY(propagator_args("lindblad_propagator", n, M, L, dt, theta, P));
    Workspace *w = ws_resolve(ws);
    ws_begin(w, stream);
    return build_propagators_async(n, M, static_cast<const cd *>(L), dt, theta, static_cast<cd *>(P), s_used, status,
                                   w, stream);
}

extern "C" int lindblad_propagator_stages(int n, int M, const void *L, const double *dt, double theta, void *P,
                                          int *s_host, double *stage_ms, lb_workspace *ws, hipStream_t stream) {
    LB_TRY(propagator_args("lindblad_propagator_stages", n, M, L, dt, theta, P));
    if (!stage_ms) return fail(LB_EINVAL, "lindblad_propagator_stages: stage_ms is NULL");
    Workspace *w = ws_resolve(ws);
    ws_begin(w, stream);
    StageClock clk;
    int created = 0, rc = LB_OK;
    for (; created < 7; ++created)
        if (hipEventCreate(&clk.ev[created]) != hipSuccess) {
            rc = fail(LB_EHIP, "lindblad_propagator_stages: hipEventCreate failed");
            break;
        }
    if (rc == LB_OK)
        rc = build_propagators(n, M, static_cast<const cd *>(L), dt, theta, static_cast<cd *>(P), s_host, w, stream,
                               &clk);
    if (rc != LB_OK) (void)hipStreamSynchronize(stream);  // events may still be pending
    for (int i = 0; i < created; ++i) (void)hipEventDestroy(clk.ev[i]);
    if (rc == LB_OK)
        for (int i = 0; i < 4; ++i) stage_ms[i] = clk.ms[i];
    return rc;
}


// ------------------------------------------------- allocation-free build
// lindblad_propagator_noalloc runs the stream-ordered build above on a fixed
// scratch: a file-scope device array (one copy per device, held until the
// process ends).  Its device address is looked up once per device with
// hipGetSymbolAddress and kept; host code only ever passes that address
// (the array's own name is a host-side stand-in).  Every call on a device
// shares the array, so calls that overlap on one device race.
namespace lb {
constexpr size_t kNoAllocScratchBytes = size_t(80) << 20;
constexpr int kNoAllocMaxDevices = 64;
}  // namespace lb

static __device__ __align__(256) char scratch[lb::kNoAllocScratchBytes];

namespace lb {
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kNoAllocMaxDevices] = {};

static int noalloc_scratch(char **out) {
    int dev = 0;
    LB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return fail(LB_ENOTSUP, "lindblad_propagator_noalloc: device index " + std::to_string(dev) +
                                    " beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        LB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LB_EHIP, "lindblad_propagator_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return LB_OK;
}
}  // namespace lb

extern "C" size_t lindblad_propagator_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

extern "C" int lindblad_propagator_noalloc(int n, int M, const void *L, const double *dt, double theta, void *P,
                                           int *s_used, int *status, hipStream_t stream) {
    LB_TRY(propagator_args("lindblad_propagator_noalloc", n, M, L, dt, theta, P));
    const size_t one = build_async_chunk_bytes(n, 1);
    if (one > kNoAllocScratchBytes)
        return fail(LB_ENOMEM, "lindblad_propagator_noalloc: one n x n build needs " + std::to_string(one) +
                                   " bytes of scratch at n = " + std::to_string(n) + ", the fixed scratch holds " +
                                   std::to_string(kNoAllocScratchBytes) + " bytes (n <= 809)");
    char *base = nullptr;
    LB_TRY(noalloc_scratch(&base));
    Workspace w;  // a view of the device's scratch: never grown, never freed
    w.base = base;
    w.size = w.cap = kNoAllocScratchBytes;
    w.fixed = true;
    (void)hipGetDevice(&w.device);
    ws_begin(&w, stream);
    return build_propagators_async(n, M, static_cast<const cd *>(L), dt, theta, static_cast<cd *>(P), s_used, status,
                                   &w, stream);
}
