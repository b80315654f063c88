// Internal declarations shared by the HIP sources of liblindblad.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>

#include "../../include/lindblad.h"

namespace lb {

// ------------------------------------------------------------ errors
void set_error(const std::string &msg);
int fail(int status, const std::string &msg);

#define LB_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::lb::fail(LB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define LB_TRY(expr)                \
    do {                                \
        int rc_ = (expr);               \
        if (rc_ != LB_OK) return rc_;   \
    } while (0)

// Launch status of the last kernel launch on this thread.
int check_launch(const char *what);

// Allow `kernel` up to `bytes` of dynamic LDS on the current device: one
// hipFuncSetAttribute per (device, kernel) and size increase, thread-safe.
int set_max_lds(const void *kernel, size_t bytes);

// --------------------------------------------------------- workspace
// Bump allocator over one device buffer; reset at the start of every call.
struct Workspace {
    size_t cap = 0;
    size_t size = 0;     // bytes allocated on the device
    size_t used = 0;     // bump offset within the current call
    char *base = nullptr;
    int device = -1;
    hipStream_t stream = nullptr;        // stream of the current call (growth is ordered on it)
    hipStream_t alloc_stream = nullptr;  // stream the buffer was allocated on
    bool fixed = false;            // a view of caller-provided memory: never grown or freed
};

// Bump allocation inside one device buffer.  A top-level entry point calls
// ws_begin(), which resets the bump offset and records the call's stream; a
// routine takes what it needs with ws_ensure() + ws_take() and gives it back
// by restoring ws->used.  ws_ensure grows the buffer only when nothing is
// taken yet, stream-ordered on the call's stream (the old buffer is released
// with hipFreeAsync after the work already enqueued there, the new one comes
// from hipMallocAsync), so growth never blocks the host; a nested request
// beyond the reservation fails with LB_ENOMEM, so callers that nest reserve
// the total first.  A fixed workspace (a view of caller-provided memory)
// never grows: requests beyond its size fail with LB_ENOMEM.
void ws_begin(Workspace *ws, hipStream_t s);
int ws_ensure(Workspace *ws, size_t bytes);
void *ws_take(Workspace *ws, size_t bytes);
Workspace *ws_resolve(lb_workspace *ws);

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Enqueues step(t, stream) for t in [0, nsteps) on `s`.  With `graph` (and
// more than 2 kGraphSteps steps), steps [0, kGraphSteps) are captured once
// into a HIP graph and replayed over all but the last step, which is always
// launched directly; `step` must depend on t only through t & 1 except on the
// last step (kGraphSteps is even) and must not record memset nodes.
constexpr long long kGraphSteps = 32;
int run_steps(long long nsteps, bool graph, const std::function<int(long long, hipStream_t)> &step, hipStream_t s);

// ------------------------------------------------------- complex FP64
struct cd {
    double re, im;
};

__host__ __device__ inline cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__host__ __device__ inline cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cd cconj(cd a) { return {a.re, -a.im}; }
__host__ __device__ inline cd cscale(cd a, double s) { return {a.re * s, a.im * s}; }
// a * conj(b) accumulate helpers
__host__ __device__ inline cd cfma(cd a, cd b, cd c) {  // c + a*b
    return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}

// ------------------------------------------------- batched complex GEMM
// D[b] = alpha * A[b] B[b] + beta * Cin[b] + sum_t coef[t] * X_t[b] + gamma * I
// All matrices complex128 row-major with the given leading dimensions and
// batch strides (elements).  D may alias Cin (in-place update) but must not
// overlap A or B.  If `active` is non-NULL, batch b is skipped unless
// active[b] > level (used by the squaring loop: active = s, level = k).
struct ZgemmBatch {
    int M = 0, N = 0, K = 0, batch = 1;
    const cd *A = nullptr; long long lda = 0, sA = 0;
    const cd *B = nullptr; long long ldb = 0, sB = 0;
    cd *D = nullptr; long long ldd = 0, sD = 0;
    double alpha = 1.0;
    double beta = 0.0;
    const cd *Cin = nullptr; long long ldc = 0, sC = 0;
    int nx = 0;
    const cd *X[3] = {nullptr, nullptr, nullptr};
    double coef[3] = {0, 0, 0};
    long long ldx = 0, sX = 0;  // shared by the X_t
    double gamma = 0.0;          // added on the diagonal (square D only)
    const int *active = nullptr;
    int level = 0;
    // optional: amask[b * sMask + tm * nkc + kc] == 0 marks an all-zero tile
    // of A (rows [64 tm, 64 tm + 64), columns [16 kc, 16 kc + 16)); such
    // k chunks are skipped (their products are exact zeros)
    const unsigned char *amask = nullptr;
    long long sMask = 0;
};
int zgemm_batched(const ZgemmBatch &g, hipStream_t s);
// Zero-tile mask of `batch` M x K matrices A (leading dimension lda, stride
// sA) in the layout ZgemmBatch::amask reads; mask_bytes(M, K) per matrix.
long long zgemm_mask_bytes(int M, int K);
int zgemm_tile_mask(int M, int K, int batch, const cd *A, long long lda, long long sA, unsigned char *mask,
                    hipStream_t s);

// Elementwise: D[b] = sum_t coef[t] X_t[b] + gamma I  (n x n, contiguous batches)
int zlincomb(int n, int batch, int nx, const cd *const *X, const double *coef, double gamma, cd *D,
             hipStream_t s);

// ------------------------------------------------------- propagator
// Stage clock of a build (measurement only): events recorded on the build's
// stream at the stage boundaries of every chunk, their intervals summed per
// stage after the chunk's synchronisation: ms = {LU solve, Pade products,
// squarings, other (scaling stage, V -/+ U, odd-s copy, host gaps)}.
struct StageClock {
    hipEvent_t ev[7] = {};
    double ms[4] = {0, 0, 0, 0};
};
// Build P[m] = exp(L[m] dt[m]) (Alg. 1) into P; s_host receives s per m.
// Uses the workspace; synchronises the stream.
int build_propagators(int n, int M, const cd *L, const double *dt_host, double theta, cd *P, int *s_host,
                      Workspace *ws, hipStream_t s, StageClock *clk = nullptr);
// Workspace bytes build_propagators needs for a batch of M (chunked inside).
size_t build_workspace_bytes(int n, int M);
// Alg. 1 after its scaling stage for M matrices with d_dt, d_s on the device
// and smax = max s known on the host; enqueue only (no host synchronisation),
// zero pivots flagged in d_info (which must start at 0).  Workspace: build_async_bytes.
int build_chunk_async(int n, int M, const cd *L, const double *d_dt, const int *d_s, int smax, cd *P, int *d_info,
                      Workspace *ws, hipStream_t s, StageClock *clk = nullptr);
size_t build_async_bytes(int n, int M);

// Alg. 1 for M generators without any host synchronisation: dt goes to the
// device through kernel arguments, s is computed on the device (d_s_out, M
// ints, or NULL), the squarings run as masked launches up to kMaxSquarings,
// and data-dependent failures are reported in the device status word
// d_status (or dropped if NULL): LB_ENONFINITE for a non-finite ||L dt||_1,
// LB_ESINGULAR for a zero pivot, LB_ENOTSUP for s > kMaxSquarings (the
// smallest code wins).  Chunks of the batch are enqueued one after another
// so that each fits what the workspace can give.
constexpr int kMaxSquarings = 24;
int build_propagators_async(int n, int M, const cd *L, const double *dt_host, double theta, cd *P, int *d_s_out,
                            int *d_status, Workspace *ws, hipStream_t s);
// Workspace bytes build_propagators_async needs for one chunk of M matrices.
size_t build_async_chunk_bytes(int n, int M);
// Argument checks of the propagator entry points (who names the caller).
int propagator_args(const char *who, int n, int M, const void *L, const double *dt, double theta, const void *P);

// Scaling stage of Alg. 1 for M generators: s[m] from ||L[m] dt[m]||_1
// (host sync), uploaded to d_s; d_dt receives dt.  Fails with LB_ENONFINITE.
int scaling_stage(int n, int M, const cd *L, const double *dt_host, double theta, double *d_dt,
                  unsigned long long *d_norm, int *d_s, int *s_host, hipStream_t s);
// A[m] = (L[m] dt[m]) 2^-s[m]
int scale_launch(int n, int M, const cd *L, const double *d_dt, const int *d_s, cd *A, hipStream_t s);
// p[0..count) = 0 with a kernel (no memset nodes in captured streams)
int fill_i32_launch(int *p, int count, hipStream_t s);
// dst[m] = src[m] for the m with odd s[m]
int odd_copy_launch(int n, int M, const int *d_s, const cd *src, cd *dst, hipStream_t s);

// Solve D X = N in place (X overwrites N) for `batch` systems of size n with
// nrhs right-hand sides (N is n x nrhs row-major) by LU with partial
// pivoting.  D is destroyed.  info[b] (device) is set non-zero on a zero pivot.
int lu_solve_batched(int n, int nrhs, int batch, cd *D, cd *N, int *ipiv, int *info, hipStream_t s);
// Solve D X = N again with the factorization lu_solve_batched left in D and
// ipiv (same batch size class), N overwritten by X.
int lu_resolve_batched(int n, int nrhs, int batch, const cd *D, cd *N, const int *ipiv, hipStream_t s);

// Pade [13/13] coefficients b_0..b_13 (b_13 = 1).
void pade13_coefficients(double b[14]);
int scaling_exponent(double norm, double theta);

}  // namespace lb
