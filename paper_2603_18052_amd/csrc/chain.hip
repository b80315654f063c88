// The step chain x <- P x (Alg. 2), nsteps times, for B independent states
// (Alg. 3 parallelism: states never interact, steps of one state stay in order).
//
//  * chain_baseline: the plain FP64 per-state matvec, one launch per step;
//    each wavefront computes one output row of one state, lanes read that row
//    of P contiguously (coalesced) and reduce with cross-lane shuffles.
//  * fused_chain_kernel<T>: the whole chain in one launch for small n.  One
//    workgroup owns NS = 16 states for all steps; P sits in LDS (k-major,
//    planar re/im, converted once to T), the states ping-pong between two LDS
//    buffers, and each step is the complex GEMM Y = P X on the matrix cores
//    (FP64: v_mfma_f64_16x16x4f64, FP32: v_mfma_f32_16x16x4f32), four real
//    MFMAs per complex block, one barrier per step.  No HBM traffic between
//    the first load and the final store.
//  * large n (P does not fit in one CU's LDS): see chain_large.hip.
#include <cstring>

#include "chain.hpp"

namespace lb {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------- baseline
__global__ void __launch_bounds__(256) baseline_step_kernel(int n, const cd *__restrict__ P, const cd *__restrict__ x,
                                                            cd *__restrict__ y, long long rows_total) {
    const int lane = threadIdx.x & 63;
    const long long nwaves = (long long)gridDim.x * (blockDim.x >> 6);
    for (long long w = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < rows_total; w += nwaves) {
        const long long b = w / n;
        const int i = (int)(w - b * n);
        const cd *Pi = P + (size_t)i * n;
        const cd *xb = x + (size_t)b * n;
        double re = 0.0, im = 0.0;
        for (int j = lane; j < n; j += 64) {
            const cd p = Pi[j], v = xb[j];
            re = fma(p.re, v.re, fma(-p.im, v.im, re));
            im = fma(p.re, v.im, fma(p.im, v.re, im));
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            re += __shfl_xor(re, off);
            im += __shfl_xor(im, off);
        }
        if (lane == 0) y[(size_t)b * n + i] = {re, im};
    }
}

int chain_baseline(int n, const cd *P, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s, bool graph) {
    if (nsteps == 0 || B == 0) return LB_OK;
    const size_t bytes = (size_t)B * n * sizeof(cd);
    LB_TRY(ws_ensure(ws, bytes));
    cd *tmp = (cd *)ws_take(ws, bytes);
    const long long rows = (long long)B * n;
    long long blocks = (rows + 3) / 4;
    if (blocks > 16384) blocks = 16384;
    LB_TRY(run_steps(nsteps, graph, [&](long long t, hipStream_t st) {
        baseline_step_kernel<<<(int)blocks, 256, 0, st>>>(n, P, (t & 1) ? tmp : rho, (t & 1) ? rho : tmp, rows);
        return LB_OK;
    }, s));
    LB_TRY(check_launch("baseline_step"));
    if (nsteps & 1) LB_HIP(hipMemcpyAsync(rho, tmp, bytes, hipMemcpyDeviceToDevice, s));
    return LB_OK;
}

// ------------------------------------------------------- one state per wave
// Small n (d <= 4): one wavefront per state, no LDS and no barrier.  Lane i
// holds row i of P and element i of the state in registers; each step reads
// every x_k with v_readlane into scalar registers (a wavefront-wide broadcast)
// and lane i forms y_i = sum_k P_ik x_k with four independent FMA chains
// (Re/Im times Re/Im), so one step costs about 4n FMAs + 2n lane reads of
// latency.  This is the latency-bound single-state regime (B = 1, d = 3).
__device__ inline double lane_read(double v, int k) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, k);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), k);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ inline float lane_read(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

template <typename T, int NP>
__global__ void __launch_bounds__(256) wave_chain_kernel(int n, const cd *__restrict__ P, int B, cd *__restrict__ rho,
                                                         long long nsteps) {
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (b >= B) return;  // uniform per wavefront
    const bool row = lane < n;
    T pr[NP], pi[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        cd v = {0.0, 0.0};
        if (row && k < n) v = P[(size_t)lane * n + k];
        pr[k] = (T)v.re;
        pi[k] = (T)v.im;
    }
    cd v0 = {0.0, 0.0};
    if (row) v0 = rho[(size_t)b * n + lane];
    T xr = (T)v0.re, xi = (T)v0.im;
    for (long long t = 0; t < nsteps; ++t) {
        T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const T sr = lane_read(xr, k), si = lane_read(xi, k);
            a0 = fma(pr[k], sr, a0);
            a1 = fma(-pi[k], si, a1);
            a2 = fma(pr[k], si, a2);
            a3 = fma(pi[k], sr, a3);
        }
        xr = a0 + a1;
        xi = a2 + a3;
    }
    if (row) rho[(size_t)b * n + lane] = {(double)xr, (double)xi};
}

template <typename T>
static int launch_wave_chain(int n, const cd *P, int B, cd *rho, long long nsteps, hipStream_t s) {
    const int blocks = (B + 3) / 4;
    if (n <= 4)
        wave_chain_kernel<T, 4><<<blocks, 256, 0, s>>>(n, P, B, rho, nsteps);
    else if (n <= 9)
        wave_chain_kernel<T, 9><<<blocks, 256, 0, s>>>(n, P, B, rho, nsteps);
    else if (n <= kWaveChainMaxN)
        wave_chain_kernel<T, kWaveChainMaxN><<<blocks, 256, 0, s>>>(n, P, B, rho, nsteps);
    else
        return fail(LB_ESHAPE, "wave chain: n too large");
    return check_launch("wave_chain");
}

int chain_wave(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, hipStream_t s) {
    if (nsteps == 0 || B == 0) return LB_OK;
    if (n > kWaveChainMaxN) return fail(LB_ESHAPE, "wave chain: n too large");
    switch (prec) {
        case LB_C128: return launch_wave_chain<double>(n, P, B, rho, nsteps, s);
        case LB_C64: return launch_wave_chain<float>(n, P, B, rho, nsteps, s);
        default: return fail(LB_ENOTSUP, "wave chain: complex128 / complex64 only");
    }
}

// ------------------------------------------------------ fused small-n chain
// One workgroup of 8 wavefronts owns NS = 16 states for every step.  The
// product Y = P X (Mp x Kp times Kp x 16) is cut into units = (16-row tile of
// P, run of KPU consecutive 4-deep k steps).  Units are dealt round-robin to
// the wavefronts (at most UPW each); a unit's slice of P lives in registers as
// MFMA A fragments for the whole chain, so per step a wavefront only reads its
// X fragments from LDS, runs its MFMAs (all units interleaved for independent
// accumulator chains), and writes its partial tile to LDS.  After a barrier the
// partials of each tile are summed in a fixed order (deterministic) into the
// next X, and a second barrier ends the step.
constexpr int NS = 16;       // states per workgroup = one MFMA N tile
constexpr int CW = 8;        // wavefronts per workgroup
constexpr int MAXUPW = 4;    // units per wavefront, at most
constexpr int MAXU = CW * MAXUPW;

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef d4 acc;
    static __device__ inline acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
    // -a b + c through the instruction's negate-A modifier (the last operand
    // of the FP64 MFMA builtin selects neg:[a, b, c]); `na` (= -a) is unused
    static __device__ inline acc mma_neg_a(double a, double na, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 1);
    }
};
template <>
struct Mfma<float> {
    typedef f4 acc;
    static __device__ inline acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
    // -a b + c with the negated fragment `na` held in registers
    static __device__ inline acc mma_neg_a(float a, float na, float b, acc c) { return mma(na, b, c); }
};

struct FusedShape {
    int Kp, KS, mtiles, kparts, units, kpu;
};

// k steps per unit the fused kernel is instantiated for.
static const int kFusedKpu[] = {1, 2, 3, 4, 6, 8, 11};

static FusedShape fused_shape(int n, int kpu) {
    FusedShape f;
    f.Kp = (n + 3) & ~3;
    f.KS = f.Kp / 4;
    f.mtiles = (n + 15) / 16;
    f.kpu = kpu;
    f.kparts = (f.KS + kpu - 1) / kpu;
    f.units = f.mtiles * f.kparts;
    return f;
}

template <typename T>
static size_t fused_lds_bytes(const FusedShape &f) {
    return sizeof(T) * (2 * (size_t)f.Kp * NS + 2 * (size_t)f.units * 256);
}

template <typename T, int KPU, int UPW>
__global__ void __launch_bounds__(CW * 64) fused_chain_kernel(int n, int kparts, const cd *__restrict__ P, int B,
                                                              cd *__restrict__ rho, long long nsteps) {
    typedef typename Mfma<T>::acc acc_t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int Kp = (n + 3) & ~3, KS = Kp / 4, mtiles = (n + 15) >> 4, units = mtiles * kparts;
    T *X_re = reinterpret_cast<T *>(smem_raw);  // [Kp][NS]
    T *X_im = X_re + (size_t)Kp * NS;
    T *part_re = X_im + (size_t)Kp * NS;        // [units][256]
    T *part_im = part_re + (size_t)units * 256;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int b0 = blockIdx.x * NS;

    // This wavefront's A fragments (unit j = wave + CW j).  Missing work --
    // units past the last one, k steps past KS -- is a zero fragment, so the
    // step loop below runs without a single branch.
    T fr[UPW][KPU], fi[UPW][KPU];
    int xoff[UPW][KPU];  // LDS offset of the X fragment each MFMA reads
#pragma unroll
    for (int j = 0; j < UPW; ++j) {
        const int u = wave + CW * j;
        const int t = u / kparts, p = u - (u / kparts) * kparts;
        int row = t * 16 + (lane & 15);
        row = row < n ? row : n - 1;  // rows past n only feed discarded outputs
#pragma unroll
        for (int kk = 0; kk < KPU; ++kk) {
            const int ks = p * KPU + kk;
            int k = ks * 4 + (lane >> 4);
            cd v = {0.0, 0.0};
            if (u < units && ks < KS && k < n) v = P[(size_t)row * n + k];
            fr[j][kk] = (T)v.re;
            fi[j][kk] = (T)v.im;
            k = k < Kp ? k : Kp - 1;  // a finite X row times a zero fragment
            xoff[j][kk] = k * NS + (lane & 15);
        }
    }
    for (int e = tid; e < Kp * NS; e += CW * 64) {
        const int k = e / NS, sidx = e - k * NS;
        cd v = {0.0, 0.0};
        if (k < n && b0 + sidx < B) v = rho[(size_t)(b0 + sidx) * n + k];
        X_re[e] = (T)v.re;
        X_im[e] = (T)v.im;
    }
    __syncthreads();

    for (long long t = 0; t < nsteps; ++t) {
        acc_t ar[UPW], ai[UPW];
#pragma unroll
        for (int j = 0; j < UPW; ++j) {
            ar[j] = acc_t{0, 0, 0, 0};
            ai[j] = acc_t{0, 0, 0, 0};
        }
#pragma unroll
        for (int kk = 0; kk < KPU; ++kk) {
#pragma unroll
            for (int j = 0; j < UPW; ++j) {
                const T xr = X_re[xoff[j][kk]], xi = X_im[xoff[j][kk]];
                ar[j] = Mfma<T>::mma(fr[j][kk], xr, ar[j]);
                ai[j] = Mfma<T>::mma(fr[j][kk], xi, ai[j]);
                ar[j] = Mfma<T>::mma(fi[j][kk], -xi, ar[j]);
                ai[j] = Mfma<T>::mma(fi[j][kk], xr, ai[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < UPW; ++j) {
            const int u = wave + CW * j;
            if (u < units) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int o = Mfma<T>::row(lane, r) * 16 + (lane & 15);
                    part_re[u * 256 + o] = ar[j][r];
                    part_im[u * 256 + o] = ai[j][r];
                }
            }
        }
        __syncthreads();
        for (int o = tid; o < mtiles * 256; o += CW * 64) {
            const int tt = o >> 8, lo = o & 255;
            const int row = tt * 16 + (lo >> 4);
            if (row < n) {
                T sr = 0, si = 0;
                for (int p = 0; p < kparts; ++p) {
                    sr += part_re[(tt * kparts + p) * 256 + lo];
                    si += part_im[(tt * kparts + p) * 256 + lo];
                }
                X_re[row * NS + (lo & 15)] = sr;
                X_im[row * NS + (lo & 15)] = si;
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < n * NS; e += CW * 64) {
        const int sidx = e / n, k = e - sidx * n;
        if (b0 + sidx < B) rho[(size_t)(b0 + sidx) * n + k] = {(double)X_re[k * NS + sidx], (double)X_im[k * NS + sidx]};
    }
}

static const size_t kLdsLimit = 160 * 1024;

// ------------------------------------------------ SIMD-balanced fused chain
// Same on-chip chain for 81 <= n <= 96 (six 16-row tiles, KS = n/4 k steps),
// with the work laid out so that the two wavefronts sharing a SIMD (w and
// w + 4) issue the same number of MFMAs and no wavefront runs zero-padded k
// steps beyond a fraction of one: SIMD s owns tile s plus half of tile
// 4 + s/2.  Wavefront s takes k steps [0, LA) of tile s; wavefront s + 4 the
// rest of tile s, [LA, KS), and its half [H (s & 1), H (s & 1) + H) of the
// extra tile.  Every wavefront holds NF = LA fragments and runs one uniform,
// branch-free MFMA loop into two accumulator pairs (fragments [0, LB1) and
// [LB1, NF)); only the partial write differs.
//
// Each output tile t ends a step as two partials, slots 2t and 2t + 1, and
// the next step reads its MFMA B operands straight from them (x = sum of the
// two slots): no separate reduction pass, one barrier per step.  The slots
// are double-buffered so that a wavefront writing step t+1's partials never
// overwrites what a slower one still reads for step t+1.  Rows past n hold
// finite values that only ever meet zero fragments.
template <int KS>
struct Balanced {
    static constexpr int H = (KS + 1) / 2;         // k steps of a half extra tile
    static constexpr int LA = (KS + H + 1) / 2;    // wavefront s: tile s, [0, LA)
    static constexpr int LB1 = KS - LA;            // wavefront s + 4: tile s, [LA, KS)
    static constexpr int NF = LA;                  // fragments per wavefront
    static_assert(LB1 >= 1 && LB1 + H <= NF, "layout");
};

constexpr int kBalSlots = 12;                        // 6 tiles x 2 partials
constexpr int kBalBuf = kBalSlots * 2 * 256;         // one buffer: [slot][re, im][256]

template <typename T, int KS>
__global__ void __launch_bounds__(CW * 64) balanced_chain_kernel(int n, const cd *__restrict__ P, int B,
                                                                 cd *__restrict__ rho, long long nsteps) {
    typedef typename Mfma<T>::acc acc_t;
    typedef Balanced<KS> L;
    constexpr int Kp = 4 * KS;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *part = reinterpret_cast<T *>(smem_raw);  // [2][kBalSlots][2][256]
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int simd = wave & 3;
    const bool second = wave >= 4;
    const int b0 = blockIdx.x * NS;

    T fr[L::NF], fi[L::NF];
    int xoff[L::NF];  // offset of the slot-2t value of the X fragment in a buffer
#pragma unroll
    for (int kk = 0; kk < L::NF; ++kk) {
        int tile, ks, kend;
        if (!second) {
            tile = simd, ks = kk, kend = L::LA;
        } else if (kk < L::LB1) {
            tile = simd, ks = L::LA + kk, kend = KS;
        } else {
            tile = 4 + (simd >> 1), ks = (simd & 1) * L::H + (kk - L::LB1);
            kend = (simd & 1) * L::H + L::H < KS ? (simd & 1) * L::H + L::H : KS;
        }
        int row = tile * 16 + (lane & 15);
        row = row < n ? row : n - 1;  // rows past n only feed discarded outputs
        int k = ks * 4 + (lane >> 4);
        cd v = {0.0, 0.0};
        if (ks < kend && k < n) v = P[(size_t)row * n + k];
        fr[kk] = (T)v.re;
        fi[kk] = (T)v.im;
        k = k < Kp ? k : Kp - 1;  // a finite X row times a zero fragment
        xoff[kk] = (2 * (k >> 4)) * 512 + (k & 15) * 16 + (lane & 15);
    }
    // initial states: slot 2t holds x, slot 2t + 1 zero (buffer 0)
    for (int e = tid; e < kBalBuf; e += CW * 64) part[e] = (T)0;
    __syncthreads();
    for (int e = tid; e < Kp * NS; e += CW * 64) {
        const int k = e / NS, sidx = e - k * NS;
        cd v = {0.0, 0.0};
        if (k < n && b0 + sidx < B) v = rho[(size_t)(b0 + sidx) * n + k];
        const int o = (2 * (k >> 4)) * 512 + (k & 15) * 16 + sidx;
        part[o] = (T)v.re;
        part[o + 256] = (T)v.im;
    }
    __syncthreads();

    for (long long t = 0; t < nsteps; ++t) {
        const T *cur = part + (t & 1) * kBalBuf;
        T *nxt = part + ((t & 1) ^ 1) * kBalBuf;
        acc_t ar[2], ai[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) ar[j] = ai[j] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < L::NF; ++kk) {
            const int j = kk < L::LB1 ? 0 : 1;
            const T *c = cur + xoff[kk];
            const T xr = c[0] + c[512], xi = c[256] + c[768];
            ar[j] = Mfma<T>::mma(fr[kk], xr, ar[j]);
            ai[j] = Mfma<T>::mma(fr[kk], xi, ai[j]);
            ar[j] = Mfma<T>::mma(fi[kk], -xi, ar[j]);
            ai[j] = Mfma<T>::mma(fi[kk], xr, ai[j]);
        }
        if (!second) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = Mfma<T>::row(lane, r) * 16 + (lane & 15);
                nxt[(2 * simd) * 512 + o] = ar[0][r] + ar[1][r];
                nxt[(2 * simd) * 512 + 256 + o] = ai[0][r] + ai[1][r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = Mfma<T>::row(lane, r) * 16 + (lane & 15);
                nxt[(2 * simd + 1) * 512 + o] = ar[0][r];
                nxt[(2 * simd + 1) * 512 + 256 + o] = ai[0][r];
                nxt[(8 + simd) * 512 + o] = ar[1][r];
                nxt[(8 + simd) * 512 + 256 + o] = ai[1][r];
            }
        }
        __syncthreads();
    }
    const T *fin = part + (nsteps & 1) * kBalBuf;
    for (int e = tid; e < n * NS; e += CW * 64) {
        const int sidx = e / n, k = e - sidx * n;
        const int o = (2 * (k >> 4)) * 512 + (k & 15) * 16 + sidx;
        if (b0 + sidx < B) rho[(size_t)(b0 + sidx) * n + k] = {(double)(fin[o] + fin[o + 512]),
                                                               (double)(fin[o + 256] + fin[o + 768])};
    }
}

template <typename T, int KS>
static int launch_balanced_k(int n, const cd *P, int B, cd *rho, long long nsteps, hipStream_t s) {
    const size_t lds = sizeof(T) * 2 * (size_t)kBalBuf;
    LB_TRY(set_max_lds((const void *)balanced_chain_kernel<T, KS>, lds));
    balanced_chain_kernel<T, KS><<<(B + NS - 1) / NS, CW * 64, lds, s>>>(n, P, B, rho, nsteps);
    return check_launch("balanced_chain");
}

bool balanced_ok(int n, lb_precision prec) {
    if (prec == LB_C128) return n >= 81 && n <= 84;
    if (prec == LB_C64) return n >= 81 && n <= 96;
    return false;
}

int chain_balanced(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, hipStream_t s) {
    if (nsteps == 0 || B == 0) return LB_OK;
    if (!balanced_ok(n, prec)) return fail(LB_ESHAPE, "balanced chain: 81 <= n <= 84 (complex128) or 96 (complex64)");
    const int KS = (n + 3) / 4;
    if (prec == LB_C128) return launch_balanced_k<double, 21>(n, P, B, rho, nsteps, s);
    switch (KS) {
        case 21: return launch_balanced_k<float, 21>(n, P, B, rho, nsteps, s);
        case 22: return launch_balanced_k<float, 22>(n, P, B, rho, nsteps, s);
        case 23: return launch_balanced_k<float, 23>(n, P, B, rho, nsteps, s);
        default: return launch_balanced_k<float, 24>(n, P, B, rho, nsteps, s);
    }
}

// ------------------------------------------------ MFMA rows + VALU tail chain
// For n = 81 (d = 9) the sixth 16-row MFMA tile of the layouts above carries
// one useful row in sixteen.  This layout runs rows 0..79 on MFMA and the
// NV = n - 80 rows past them on the vector ALUs.  Tiles 0..4 are cut into
// three parts of 7 k steps (KS = 21): part p = 3 tile + q covers k steps
// [7q, 7q + 7) and writes partial slot p.  With WPB wavefronts a workgroup
// (8 or 16, wavefront w on SIMD w % 4), wavefront w owns the NPW = 16 / WPB
// parts NPW w .. NPW w + NPW - 1 below 15, so SIMDs 0..2 issue four parts a
// step (112 MFMAs against 128 in the balanced layout) and SIMD 3 three parts,
// one of each q: (6, 7, 14) with 8 wavefronts, (3, 7, 11) with 16.  The
// SIMD-3 wavefronts holding parts also multiply the x values they load for
// their MFMAs by the tail rows of P (registers), reduce over the four
// k lanes of each state and write partial slot 15 + q (q of their first part)
// of k-tile 5 (a slot no wavefront writes stays zero).  Every x operand is the
// sum of its k-tile's three slots, double-buffered, one barrier per step.
// Slots hold (re, im) pairs so one LDS instruction reads one complex value.
template <typename T>
struct alignas(2 * sizeof(T)) Pair {
    T re, im;
};

constexpr int kTailKS = 21;      // k steps (n <= 84)
constexpr int kTailPartKs = 7;   // k steps per part
constexpr int kTailParts = 15;   // 5 tiles x 3 parts
constexpr int kTailSlots = 18;   // 6 k-tiles x 3 partials
constexpr int kTailBuf = kTailSlots * 256;

template <typename T, int NV, bool TAIL>
__device__ inline void tail_part(const Pair<T> *__restrict__ cur, const T (&fr)[kTailPartKs],
                                 const T (&fi)[kTailPartKs], const T (&tr)[kTailPartKs][NV],
                                 const T (&ti)[kTailPartKs][NV], const int (&xoff)[kTailPartKs],
                                 typename Mfma<T>::acc &ar, typename Mfma<T>::acc &ai, T (&sr)[NV], T (&si)[NV]) {
#pragma unroll
    for (int f = 0; f < kTailPartKs; ++f) {
        const Pair<T> *c = cur + xoff[f];
        const Pair<T> x0 = c[0], x1 = c[256], x2 = c[512];
        const T xr = x0.re + x1.re + x2.re, xi = x0.im + x1.im + x2.im;
        ar = Mfma<T>::mma(fr[f], xr, ar);
        ai = Mfma<T>::mma(fr[f], xi, ai);
        ar = Mfma<T>::mma(fi[f], -xi, ar);
        ai = Mfma<T>::mma(fi[f], xr, ai);
        if (TAIL) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                sr[v] += tr[f][v] * xr - ti[f][v] * xi;
                si[v] += tr[f][v] * xi + ti[f][v] * xr;
            }
        }
    }
}

template <typename T, int NV, int WPB>
__global__ void __launch_bounds__(WPB * 64) tail_chain_kernel(int n, const cd *__restrict__ P, int B,
                                                              cd *__restrict__ rho, long long nsteps) {
    typedef typename Mfma<T>::acc acc_t;
    constexpr int NPW = 16 / WPB;
    constexpr int Kp = 4 * kTailKS;
    static_assert(WPB == 8 || WPB == 16, "8 or 16 wavefronts");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Pair<T> *slots = reinterpret_cast<Pair<T> *>(smem_raw);  // [2][kTailSlots][256]
    const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, j = lane & 15;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int p0 = NPW * wave;                            // first part of this wavefront
    const bool tail = (wave & 3) == 3 && p0 < kTailParts;  // SIMD 3, holding parts
    const int tail_slot = 15 + p0 % 3;
    const int b0 = blockIdx.x * NS;

    T fr[NPW][kTailPartKs], fi[NPW][kTailPartKs];
    T tr[NPW][kTailPartKs][NV], ti[NPW][kTailPartKs][NV];
    int xoff[NPW][kTailPartKs];  // entry of slot 0 of the lane's k-tile in a buffer
#pragma unroll
    for (int a = 0; a < NPW; ++a) {
        const int p = p0 + a;
        const bool live = p < kTailParts;
        const int tile = live ? p / 3 : 0, q = live ? p % 3 : 0;
#pragma unroll
        for (int f = 0; f < kTailPartKs; ++f) {
            const int k = 4 * (kTailPartKs * q + f) + g;  // < Kp
            cd v = {0.0, 0.0};
            if (live && k < n) v = P[(size_t)(tile * 16 + j) * n + k];
            fr[a][f] = (T)v.re;
            fi[a][f] = (T)v.im;
#pragma unroll
            for (int r = 0; r < NV; ++r) {
                cd u = {0.0, 0.0};
                if (live && tail && k < n) u = P[(size_t)(80 + r) * n + k];
                tr[a][f][r] = (T)u.re;
                ti[a][f][r] = (T)u.im;
            }
            xoff[a][f] = 3 * (k >> 4) * 256 + (k & 15) * 16 + j;
        }
    }
    // initial states: slot 3 (k >> 4) holds x, the other two zero (buffer 0)
    for (int e = tid; e < 2 * kTailBuf; e += WPB * 64) slots[e] = Pair<T>{(T)0, (T)0};
    __syncthreads();
    for (int e = tid; e < Kp * NS; e += WPB * 64) {
        const int k = e / NS, sidx = e - k * NS;
        cd v = {0.0, 0.0};
        if (k < n && b0 + sidx < B) v = rho[(size_t)(b0 + sidx) * n + k];
        slots[3 * (k >> 4) * 256 + (k & 15) * 16 + sidx] = Pair<T>{(T)v.re, (T)v.im};
    }
    __syncthreads();

    for (long long t = 0; t < nsteps; ++t) {
        const Pair<T> *cur = slots + (t & 1) * kTailBuf;
        Pair<T> *nxt = slots + ((t & 1) ^ 1) * kTailBuf;
        T sr[NV], si[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) sr[v] = si[v] = (T)0;
#pragma unroll
        for (int a = 0; a < NPW; ++a) {
            if (p0 + a >= kTailParts) break;  // uniform per wavefront
            acc_t ar = acc_t{0, 0, 0, 0}, ai = acc_t{0, 0, 0, 0};
            if (tail)
                tail_part<T, NV, true>(cur, fr[a], fi[a], tr[a], ti[a], xoff[a], ar, ai, sr, si);
            else
                tail_part<T, NV, false>(cur, fr[a], fi[a], tr[a], ti[a], xoff[a], ar, ai, sr, si);
            Pair<T> *dst = nxt + (p0 + a) * 256;
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[Mfma<T>::row(lane, r) * 16 + j] = Pair<T>{ar[r], ai[r]};
        }
        if (tail) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                sr[v] += __shfl_xor(sr[v], 16);
                si[v] += __shfl_xor(si[v], 16);
                sr[v] += __shfl_xor(sr[v], 32);
                si[v] += __shfl_xor(si[v], 32);
            }
            T wr = sr[0], wi = si[0];
#pragma unroll
            for (int v = 1; v < NV; ++v)
                if (g == v) wr = sr[v], wi = si[v];
            if (g < NV) nxt[tail_slot * 256 + g * 16 + j] = Pair<T>{wr, wi};
        }
        __syncthreads();
    }
    const Pair<T> *fin = slots + (nsteps & 1) * kTailBuf;
    for (int e = tid; e < n * NS; e += WPB * 64) {
        const int sidx = e / n, k = e - sidx * n;
        const Pair<T> *c = fin + 3 * (k >> 4) * 256 + (k & 15) * 16 + sidx;
        if (b0 + sidx < B)
            rho[(size_t)(b0 + sidx) * n + k] = {(double)(c[0].re + c[256].re + c[512].re),
                                                (double)(c[0].im + c[256].im + c[512].im)};
    }
}

template <typename T, int NV, int WPB>
static int launch_tail_k(int n, const cd *P, int B, cd *rho, long long nsteps, hipStream_t s) {
    const size_t lds = sizeof(Pair<T>) * 2 * (size_t)kTailBuf;
    LB_TRY(set_max_lds((const void *)tail_chain_kernel<T, NV, WPB>, lds));
    tail_chain_kernel<T, NV, WPB><<<(B + NS - 1) / NS, WPB * 64, lds, s>>>(n, P, B, rho, nsteps);
    return check_launch("tail_chain");
}

// Whole-tile layout for n = 81 (variant params 2 and 3).  The MFMAs cover
// rows 0..79 and columns 0..79 of P (20 k steps, no padding); row 80 and
// column 80 run on the VALU.  Wavefront s = 0..3 (SIMD s) owns output tile s
// over all 20 k steps, so rows 16 s .. 16 s + 15 end each step complete in its
// registers: slot s of the next buffer holds x of k-tile s.  Its two
// accumulators start the step at P[rows, 80] x_80 (column 80 as a rank-1
// term).  Wavefront 4 + s (SIMD s) owns k steps [5 s, 5 s + 5) of tile 4 and
// writes partial slot 4 + s (the last one starting from P[64..79, 80] x_80),
// and runs row 80 over the same columns (the last one also P[80, 80] x_80) on
// the VALU into partial slot 8 + s (entries of row 80 only).  These short
// wavefronts issue at a raised priority so that their MFMAs and VALU work
// interleave early with the long wavefront's.  x of k-tiles 0..3 is one LDS
// read per fragment that goes straight into the MFMA.  For k-tile 4 and x_80:
//  * PRESUM = false (param 2): every reader sums the four partial slots;
//  * PRESUM = true (param 3): each short wavefront bumps a workgroup counter
//    in LDS (release / acquire) after writing its partials and the last of
//    the four sums them in place into slots 4 and 8, so every read is one
//    LDS read.
// Each SIMD issues 80 + 20 = 100 MFMAs a step.  The product with -fi is the
// FP64 MFMA's negate modifier, or a negated copy in registers for FP32.
constexpr int kTilesKS = 20;     // MFMA k steps: columns 0..79
constexpr int kTilesSlots = 12;
constexpr int kTilesBuf = kTilesSlots * 256;
constexpr int kTilesShort = 5;   // k steps of a short wavefront

template <typename T>
__device__ inline void tiles_store(Pair<T> *__restrict__ dst, int lane, const typename Mfma<T>::acc &ar,
                                   const typename Mfma<T>::acc &ai) {
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[Mfma<T>::row(lane, r) * 16 + (lane & 15)] = Pair<T>{ar[r], ai[r]};
}

template <typename T>
__device__ inline Pair<T> sum4(const Pair<T> *__restrict__ c) {
    const Pair<T> a = c[0], b = c[256], d = c[512], f = c[768];
    return Pair<T>{(a.re + b.re) + (d.re + f.re), (a.im + b.im) + (d.im + f.im)};
}

// x of k step ks (< 20) for this lane: slot ks / 4, entry (4 (ks % 4) + g) 16 + j;
// SUM4: k-tile 4 as the sum of its four partial slots
template <typename T, bool SUM4>
__device__ inline Pair<T> tiles_x(const Pair<T> *__restrict__ cur, int ks, int lane) {
    const Pair<T> *c = cur + (ks >> 2) * 256 + lane + 64 * (ks & 3);
    if (SUM4) return sum4<T>(c);
    return c[0];
}

// x_80 of state j (entry j of slot 8, or the sum of slots 8..11)
template <typename T, bool SUM4>
__device__ inline Pair<T> tiles_x80(const Pair<T> *__restrict__ cur, int j) {
    if (SUM4) return sum4<T>(cur + 8 * 256 + j);
    return cur[8 * 256 + j];
}

// short wavefront s = 0..3: k steps [5 s, 5 s + 5) of tile 4 and of row 80;
// LAST (s = 3) also column 80 (P[64..79, 80] x_80 as the accumulators'
// starting value, P[80, 80] x_80)
template <typename T, bool PRESUM, bool LAST>
__device__ inline void tiles_short(int n, const cd *__restrict__ P, Pair<T> *__restrict__ slots, unsigned *ctr,
                                   int s, int lane, long long nsteps) {
    typedef typename Mfma<T>::acc acc_t;
    const int g = lane >> 4, j = lane & 15, kb = kTilesShort * s;
    __builtin_amdgcn_s_setprio(2);  // issue ahead of the long wavefront sharing the SIMD
    T fr[kTilesShort], fi[kTilesShort], fn[kTilesShort], tr[kTilesShort], ti[kTilesShort];
#pragma unroll
    for (int f = 0; f < kTilesShort; ++f) {
        const int k = 4 * (kb + f) + g;  // < 80 <= n
        const cd v = P[(size_t)(64 + j) * n + k], u = P[(size_t)80 * n + k];
        fr[f] = (T)v.re, fi[f] = (T)v.im, fn[f] = -(T)v.im;
        tr[f] = (T)u.re, ti[f] = (T)u.im;
    }
    T cr[4], ci[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        cd v = {0.0, 0.0};
        if (LAST) v = P[(size_t)(64 + Mfma<T>::row(lane, r)) * n + 80];
        cr[r] = (T)v.re, ci[r] = (T)v.im;
    }
    cd p80 = {0.0, 0.0};
    if (LAST && g == 0) p80 = P[(size_t)80 * n + 80];
    const T qr = (T)p80.re, qi = (T)p80.im;
    for (long long t = 0; t < nsteps; ++t) {
        const Pair<T> *cur = slots + (t & 1) * kTilesBuf;
        Pair<T> *nxt = slots + ((t & 1) ^ 1) * kTilesBuf;
        acc_t a0 = acc_t{0, 0, 0, 0}, a1 = a0;
        T sr = 0, si = 0;
        if (LAST) {
            const Pair<T> x80 = tiles_x80<T, !PRESUM>(cur, j);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a0[r] = cr[r] * x80.re - ci[r] * x80.im;
                a1[r] = cr[r] * x80.im + ci[r] * x80.re;
            }
            sr = qr * x80.re - qi * x80.im;
            si = qr * x80.im + qi * x80.re;
        }
#pragma unroll
        for (int f = 0; f < kTilesShort; ++f) {
            // only the last range reaches k-tile 4 (k steps 16..19)
            const Pair<T> x = (LAST && !PRESUM && f > 0) ? tiles_x<T, true>(cur, kb + f, lane)
                                                        : tiles_x<T, false>(cur, kb + f, lane);
            a0 = Mfma<T>::mma(fr[f], x.re, a0);
            a1 = Mfma<T>::mma(fr[f], x.im, a1);
            a0 = Mfma<T>::mma_neg_a(fi[f], fn[f], x.im, a0);
            a1 = Mfma<T>::mma(fi[f], x.re, a1);
            sr += tr[f] * x.re - ti[f] * x.im;
            si += tr[f] * x.im + ti[f] * x.re;
        }
        tiles_store<T>(nxt + (4 + s) * 256, lane, a0, a1);
        sr += __shfl_xor(sr, 16);
        si += __shfl_xor(si, 16);
        sr += __shfl_xor(sr, 32);
        si += __shfl_xor(si, 32);
        if (g == 0) nxt[(8 + s) * 256 + j] = Pair<T>{sr, si};
        if (PRESUM) {
            // the last short wavefront of the step to get here sums the partials
            unsigned prev = 0;
            if (lane == 0) prev = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            prev = __builtin_amdgcn_readfirstlane(prev);
            if ((prev & 3) == 3) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    nxt[4 * 256 + lane + 64 * q] = sum4<T>(nxt + 4 * 256 + lane + 64 * q);
                if (lane < 16) nxt[8 * 256 + lane] = sum4<T>(nxt + 8 * 256 + lane);
            }
        }
        __syncthreads();
    }
}

template <typename T, bool PRESUM>
__global__ void __launch_bounds__(CW * 64) tiles_chain_kernel(int n, const cd *__restrict__ P, int B,
                                                              cd *__restrict__ rho, long long nsteps) {
    typedef typename Mfma<T>::acc acc_t;
    constexpr int KS = kTilesKS, Kp = 4 * KS + 16;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ unsigned ctr;
    Pair<T> *slots = reinterpret_cast<Pair<T> *>(smem_raw);  // [2][kTilesSlots][256]
    const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, j = lane & 15;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int b0 = blockIdx.x * NS;

    if (tid == 0) ctr = 0;
    for (int e = tid; e < 2 * kTilesBuf; e += CW * 64) slots[e] = Pair<T>{(T)0, (T)0};
    __syncthreads();
    // x of k-tile kt < 5 in slot kt, x_80 in entry 0..15 of slot 8 (the other
    // partial slots zero)
    for (int e = tid; e < Kp * NS; e += CW * 64) {
        const int k = e / NS, sidx = e - k * NS, kt = k >> 4;
        cd v = {0.0, 0.0};
        if (k < n && b0 + sidx < B) v = rho[(size_t)(b0 + sidx) * n + k];
        slots[(kt < 5 ? kt : 8) * 256 + (k & 15) * 16 + sidx] = Pair<T>{(T)v.re, (T)v.im};
    }
    __syncthreads();

    if (wave < 4) {
        // long wavefront: tile `wave`, columns 0..79 on MFMA, column 80 as the
        // accumulators' starting value
        T fr[KS], fi[KS], fn[KS], cr[4], ci[4];
#pragma unroll
        for (int f = 0; f < KS; ++f) {
            const cd v = P[(size_t)(wave * 16 + j) * n + 4 * f + g];
            fr[f] = (T)v.re, fi[f] = (T)v.im, fn[f] = -(T)v.im;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const cd v = P[(size_t)(wave * 16 + Mfma<T>::row(lane, r)) * n + 80];
            cr[r] = (T)v.re, ci[r] = (T)v.im;
        }
        for (long long t = 0; t < nsteps; ++t) {
            const Pair<T> *cur = slots + (t & 1) * kTilesBuf;
            Pair<T> *nxt = slots + ((t & 1) ^ 1) * kTilesBuf;
            const Pair<T> x80 = tiles_x80<T, !PRESUM>(cur, j);
            acc_t a0, a1;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a0[r] = cr[r] * x80.re - ci[r] * x80.im;
                a1[r] = cr[r] * x80.im + ci[r] * x80.re;
            }
#pragma unroll
            for (int f = 0; f < KS; ++f) {
                const Pair<T> x = (!PRESUM && f >= 16) ? tiles_x<T, true>(cur, f, lane) : tiles_x<T, false>(cur, f, lane);
                a0 = Mfma<T>::mma(fr[f], x.re, a0);
                a1 = Mfma<T>::mma(fr[f], x.im, a1);
                a0 = Mfma<T>::mma_neg_a(fi[f], fn[f], x.im, a0);
                a1 = Mfma<T>::mma(fi[f], x.re, a1);
            }
            tiles_store<T>(nxt + wave * 256, lane, a0, a1);
            __syncthreads();
        }
    } else if (wave < 7) {
        tiles_short<T, PRESUM, false>(n, P, slots, &ctr, wave - 4, lane, nsteps);
    } else {
        tiles_short<T, PRESUM, true>(n, P, slots, &ctr, 3, lane, nsteps);
    }
    const Pair<T> *fin = slots + (nsteps & 1) * kTilesBuf;
    for (int e = tid; e < n * NS; e += CW * 64) {
        const int sidx = e / n, k = e - sidx * n, kt = k >> 4;
        const Pair<T> *c = fin + (kt < 5 ? kt : 8) * 256 + (k & 15) * 16 + sidx;
        const Pair<T> v = (!PRESUM && kt >= 4) ? sum4<T>(c) : c[0];
        if (b0 + sidx < B) rho[(size_t)(b0 + sidx) * n + k] = {(double)v.re, (double)v.im};
    }
}

template <typename T, bool PRESUM>
static int launch_tiles_k(int n, const cd *P, int B, cd *rho, long long nsteps, hipStream_t s) {
    const size_t lds = sizeof(Pair<T>) * 2 * (size_t)kTilesBuf;
    LB_TRY(set_max_lds((const void *)tiles_chain_kernel<T, PRESUM>, lds));
    tiles_chain_kernel<T, PRESUM><<<(B + NS - 1) / NS, CW * 64, lds, s>>>(n, P, B, rho, nsteps);
    return check_launch("tiles_chain");
}

bool tail_ok(int n, lb_precision prec) { return (prec == LB_C128 || prec == LB_C64) && n == 81; }

int chain_tail(int n, const cd *P, lb_precision prec, int layout, int B, cd *rho, long long nsteps, hipStream_t s) {
    if (nsteps == 0 || B == 0) return LB_OK;
    if (!tail_ok(n, prec)) return fail(LB_ESHAPE, "MFMA + tail chain: n = 81");
    if (prec == LB_C128) {
        switch (layout) {
            case 0: return launch_tail_k<double, 1, 8>(n, P, B, rho, nsteps, s);
            case 1: return launch_tail_k<double, 1, 16>(n, P, B, rho, nsteps, s);
            case 2: return launch_tiles_k<double, false>(n, P, B, rho, nsteps, s);
            default: return launch_tiles_k<double, true>(n, P, B, rho, nsteps, s);
        }
    }
    switch (layout) {
        case 0: return launch_tail_k<float, 1, 8>(n, P, B, rho, nsteps, s);
        case 1: return launch_tail_k<float, 1, 16>(n, P, B, rho, nsteps, s);
        case 2: return launch_tiles_k<float, false>(n, P, B, rho, nsteps, s);
        default: return launch_tiles_k<float, true>(n, P, B, rho, nsteps, s);
    }
}



int fused_max_n(lb_precision prec) {
    switch (prec) {
        case LB_C128: return 84;
        case LB_C64: return 124;
        default: return 0;
    }
}

template <typename T, int KPU, int UPW>
static int launch_fused_k(int n, int kparts, const cd *P, int B, cd *rho, long long nsteps, size_t lds,
                          hipStream_t s) {
    LB_TRY(set_max_lds((const void *)fused_chain_kernel<T, KPU, UPW>, kLdsLimit));
    const int blocks = (B + NS - 1) / NS;
    fused_chain_kernel<T, KPU, UPW><<<blocks, CW * 64, lds, s>>>(n, kparts, P, B, rho, nsteps);
    return check_launch("fused_chain");
}

template <typename T, int KPU>
static int launch_fused_u(int n, const FusedShape &f, const cd *P, int B, cd *rho, long long nsteps, size_t lds,
                          hipStream_t s) {
    switch ((f.units + CW - 1) / CW) {
        case 1: return launch_fused_k<T, KPU, 1>(n, f.kparts, P, B, rho, nsteps, lds, s);
        case 2: return launch_fused_k<T, KPU, 2>(n, f.kparts, P, B, rho, nsteps, lds, s);
        case 3: return launch_fused_k<T, KPU, 3>(n, f.kparts, P, B, rho, nsteps, lds, s);
        case 4: return launch_fused_k<T, KPU, 4>(n, f.kparts, P, B, rho, nsteps, lds, s);
        default: return fail(LB_ESHAPE, "fused chain: unsupported unit count");
    }
}

template <typename T>
static int launch_fused(int n, int kpu, const cd *P, int B, cd *rho, long long nsteps, hipStream_t s) {
    const FusedShape f = fused_shape(n, kpu);
    const size_t lds = fused_lds_bytes<T>(f);
    switch (kpu) {
        case 1: return launch_fused_u<T, 1>(n, f, P, B, rho, nsteps, lds, s);
        case 2: return launch_fused_u<T, 2>(n, f, P, B, rho, nsteps, lds, s);
        case 3: return launch_fused_u<T, 3>(n, f, P, B, rho, nsteps, lds, s);
        case 4: return launch_fused_u<T, 4>(n, f, P, B, rho, nsteps, lds, s);
        case 6: return launch_fused_u<T, 6>(n, f, P, B, rho, nsteps, lds, s);
        case 8: return launch_fused_u<T, 8>(n, f, P, B, rho, nsteps, lds, s);
        case 11: return launch_fused_u<T, 11>(n, f, P, B, rho, nsteps, lds, s);
        default: return fail(LB_ESHAPE, "fused chain: unsupported unit shape");
    }
}

// Valid k-steps-per-unit values for n, ascending; a larger value that gives
// the same number of k parts would only add zero fragments, so it is skipped.
int fused_kpus(int n, lb_precision prec, int *kpus, int max) {
    if (n < 1 || n > fused_max_n(prec) || (prec != LB_C128 && prec != LB_C64)) return 0;
    int c = 0, last_parts = 0;
    for (int k : kFusedKpu) {
        const FusedShape f = fused_shape(n, k);
        if (f.units > MAXU || f.kparts == last_parts) continue;
        const size_t lds = prec == LB_C128 ? fused_lds_bytes<double>(f) : fused_lds_bytes<float>(f);
        if (lds > kLdsLimit) continue;
        last_parts = f.kparts;
        if (c < max) kpus[c++] = k;
    }
    return c;
}

bool fused_kpu_ok(int n, lb_precision prec, int kpu) {
    int k[16];
    const int c = fused_kpus(n, prec, k, 16);
    for (int i = 0; i < c; ++i)
        if (k[i] == kpu) return true;
    return false;
}

int chain_fused(int n, const cd *P, lb_precision prec, int kpu, int B, cd *rho, long long nsteps, hipStream_t s) {
    if (nsteps == 0 || B == 0) return LB_OK;
    if (!fused_kpu_ok(n, prec, kpu)) return fail(LB_ESHAPE, "fused chain: shape not available for this n");
    switch (prec) {
        case LB_C128: return launch_fused<double>(n, kpu, P, B, rho, nsteps, s);
        case LB_C64: return launch_fused<float>(n, kpu, P, B, rho, nsteps, s);
        default: return fail(LB_ENOTSUP, "fused chain: complex128 / complex64 only");
    }
}

}  // namespace lb

using namespace lb;

int lb::validate_chain(const char *who, int n, const void *P, int B, const void *rho, long long nsteps) {
    if (n < 1 || n > 4096) return fail(LB_ESHAPE, std::string(who) + ": n must be in [1, 4096]");
    if (B < 1) return fail(LB_ESHAPE, std::string(who) + ": B must be >= 1");
    if (nsteps < 0) return fail(LB_EINVAL, std::string(who) + ": nsteps must be >= 0");
    if (!P || !rho) return fail(LB_EINVAL, std::string(who) + ": NULL pointer");
    return LB_OK;
}

extern "C" int lindblad_propagate_baseline(int n, const void *P, int B, void *rho, long long nsteps, lb_workspace *ws,
                                           hipStream_t stream) {
    LB_TRY(validate_chain("lindblad_propagate_baseline", n, P, B, rho, nsteps));
    Workspace *w = ws_resolve(ws);
    ws_begin(w, stream);
    return chain_baseline(n, static_cast<const cd *>(P), B, static_cast<cd *>(rho), nsteps, w, stream);
}
