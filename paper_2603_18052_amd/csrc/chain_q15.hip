// Fixed-point chain (Alg. 5): P and the states in Q1.15 (a value v is the
// 16-bit integer q = v 2^15), each complex value packed in one 32-bit word
// (real part in the low half, imaginary part in the high half).  One step
// forms acc_i = sum_j P_ij x_j exactly in 64-bit integers (products are
// Q2.30; n <= 4096 terms need at most 44 bits), then
// x_i = sat(floor(acc_i / 2^15)) -- an arithmetic shift -- for both parts.
// Quantisation of P and of the incoming states rounds to nearest (ties to
// even) and saturates, so 1.0 becomes 1 - 2^-15.  Integer sums do not depend
// on their order: every kernel here gives the same bits.
//
//  * q15_wave_kernel: one wavefront per state for n <= 16; lane i holds row i
//    of P and x_i in registers, x_k is broadcast with v_readlane (one 32-bit
//    word per complex value), no LDS and no barrier.
//  * q15_matvec_kernel: one wavefront per (state, row) for any n, lanes along
//    the row, 64-bit shuffle reduction; one launch per step.
#include "chain.hpp"

namespace lb {
namespace q15 {

__device__ __host__ inline int sat16(long long v) { return v < -32768 ? -32768 : (v > 32767 ? 32767 : (int)v); }

__device__ inline unsigned pack(int re, int im) { return (unsigned)(re & 0xffff) | ((unsigned)(im & 0xffff) << 16); }
__device__ inline int lo16(unsigned w) { return (int)(short)(w & 0xffffu); }
__device__ inline int hi16(unsigned w) { return (int)(short)(w >> 16); }

// round to nearest (ties to even), clamped in floating point before the
// conversion so that no value is out of the integer range
__device__ inline int q15_code(double v) { return (int)fmax(-32768.0, fmin(32767.0, rint(v * 32768.0))); }
__device__ inline unsigned quantize(cd v) { return pack(q15_code(v.re), q15_code(v.im)); }

__global__ void quantize_kernel(long long count, const cd *__restrict__ src, unsigned *__restrict__ dst) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (long long)gridDim.x * blockDim.x)
        dst[e] = quantize(src[e]);
}

__global__ void unpack_kernel(long long count, const unsigned *__restrict__ src, cd *__restrict__ dst) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (long long)gridDim.x * blockDim.x)
        dst[e] = {lo16(src[e]) / 32768.0, hi16(src[e]) / 32768.0};
}

template <int NP>
__global__ void __launch_bounds__(256) q15_wave_kernel(int n, const unsigned *__restrict__ Pq, int B,
                                                       cd *__restrict__ rho, long long nsteps) {
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (b >= B) return;  // uniform per wavefront
    const bool row = lane < n;
    int pr[NP], pi[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const unsigned w = (row && k < n) ? Pq[(size_t)lane * n + k] : 0u;
        pr[k] = lo16(w);
        pi[k] = hi16(w);
    }
    unsigned x = row ? quantize(rho[(size_t)b * n + lane]) : 0u;
    for (long long t = 0; t < nsteps; ++t) {
        long long ar = 0, ai = 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const unsigned w = (unsigned)__builtin_amdgcn_readlane((int)x, k);
            const int xr = lo16(w), xi = hi16(w);
            ar += (long long)pr[k] * xr - (long long)pi[k] * xi;
            ai += (long long)pr[k] * xi + (long long)pi[k] * xr;
        }
        x = row ? pack(sat16(ar >> 15), sat16(ai >> 15)) : 0u;
    }
    if (row) rho[(size_t)b * n + lane] = {lo16(x) / 32768.0, hi16(x) / 32768.0};
}

__global__ void __launch_bounds__(256) q15_matvec_kernel(int n, const unsigned *__restrict__ Pq,
                                                         const unsigned *__restrict__ X, unsigned *__restrict__ Y,
                                                         long long rows_total) {
    const int lane = threadIdx.x & 63;
    const long long nwaves = (long long)gridDim.x * (blockDim.x >> 6);
    for (long long w = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < rows_total; w += nwaves) {
        const long long b = w / n;
        const int i = (int)(w - b * n);
        const unsigned *Pi = Pq + (size_t)i * n;
        const unsigned *xb = X + (size_t)b * n;
        long long ar = 0, ai = 0;
        for (int j = lane; j < n; j += 64) {
            const unsigned p = Pi[j], v = xb[j];
            const int pr = lo16(p), pim = hi16(p), xr = lo16(v), xi = hi16(v);
            ar += (long long)pr * xr - (long long)pim * xi;
            ai += (long long)pr * xi + (long long)pim * xr;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            ar += __shfl_xor(ar, off);
            ai += __shfl_xor(ai, off);
        }
        if (lane == 0) Y[(size_t)b * n + i] = pack(sat16(ar >> 15), sat16(ai >> 15));
    }
}

static int grid1(long long work) {
    long long g = (work + 255) / 256;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace q15

size_t q15_ws_bytes(int n, int B, bool wave) {
    return align256((size_t)n * n * 4) + (wave ? 0 : 2 * align256((size_t)B * n * 4));
}

int chain_q15(int n, const cd *P, int B, cd *rho, long long nsteps, bool wave, bool graph, Workspace *ws,
              hipStream_t s) {
    using namespace q15;
    if (nsteps == 0 || B == 0) return LB_OK;
    if (wave && n > kWaveChainMaxN) return fail(LB_ESHAPE, "q15 wave chain: n <= 16");
    const size_t nn = (size_t)n * n;
    LB_TRY(ws_ensure(ws, q15_ws_bytes(n, B, wave)));
    unsigned *Pq = (unsigned *)ws_take(ws, nn * 4);
    quantize_kernel<<<grid1((long long)nn), 256, 0, s>>>((long long)nn, P, Pq);
    LB_TRY(check_launch("q15_quantize"));
    if (wave) {
        const int blocks = (B + 3) / 4;
        if (n <= 4)
            q15_wave_kernel<4><<<blocks, 256, 0, s>>>(n, Pq, B, rho, nsteps);
        else if (n <= 9)
            q15_wave_kernel<9><<<blocks, 256, 0, s>>>(n, Pq, B, rho, nsteps);
        else
            q15_wave_kernel<kWaveChainMaxN><<<blocks, 256, 0, s>>>(n, Pq, B, rho, nsteps);
        return check_launch("q15_wave");
    }
    unsigned *X0 = (unsigned *)ws_take(ws, (size_t)B * n * 4);
    unsigned *X1 = (unsigned *)ws_take(ws, (size_t)B * n * 4);
    quantize_kernel<<<grid1((long long)B * n), 256, 0, s>>>((long long)B * n, rho, X0);
    const long long rows = (long long)B * n;
    long long blocks = (rows + 3) / 4;
    if (blocks > 16384) blocks = 16384;
    LB_TRY(run_steps(nsteps, graph, [&](long long t, hipStream_t st) {
        q15_matvec_kernel<<<(int)blocks, 256, 0, st>>>(n, Pq, (t & 1) ? X1 : X0, (t & 1) ? X0 : X1, rows);
        return LB_OK;
    }, s));
    LB_TRY(check_launch("q15_matvec"));
    unpack_kernel<<<grid1(rows), 256, 0, s>>>(rows, (nsteps & 1) ? X1 : X0, rho);
    return check_launch("q15_unpack");
}

}  // namespace lb
