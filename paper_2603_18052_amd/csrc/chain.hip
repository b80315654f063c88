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
//  * large n (P does not fit in one CU's LDS): one GEMM launch per step,
//    Y = X P^T with P^T prepared once.
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

int chain_baseline(int n, const cd *P, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s) {
    if (nsteps == 0 || B == 0) return LB_OK;
    const size_t bytes = (size_t)B * n * sizeof(cd);
    LB_TRY(ws_reserve_total(ws, align256(bytes)));
    cd *tmp = (cd *)ws_take(ws, bytes);
    const long long rows = (long long)B * n;
    long long blocks = (rows + 3) / 4;
    if (blocks > 16384) blocks = 16384;
    cd *x = rho, *y = tmp;
    for (long long t = 0; t < nsteps; ++t) {
        baseline_step_kernel<<<(int)blocks, 256, 0, s>>>(n, P, x, y, rows);
        cd *z = x;
        x = y;
        y = z;
    }
    LB_TRY(check_launch("baseline_step"));
    if (x != rho) LB_HIP(hipMemcpyAsync(rho, x, bytes, hipMemcpyDeviceToDevice, s));
    return LB_OK;
}

// ------------------------------------------------------ fused small-n chain
constexpr int NS = 16;  // states per workgroup = one MFMA N tile

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef d4 acc;
    static __device__ inline acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
    typedef f4 acc;
    static __device__ inline acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T>
static size_t fused_lds_bytes(int n) {
    const int Kp = (n + 3) & ~3;
    return sizeof(T) * (2 * (size_t)Kp * n + 4 * (size_t)Kp * NS);
}

template <typename T>
__global__ void __launch_bounds__(256) fused_chain_kernel(int n, const cd *__restrict__ P, int B, cd *__restrict__ rho,
                                                          long long nsteps) {
    typedef typename Mfma<T>::acc acc_t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *smem = reinterpret_cast<T *>(smem_raw);
    const int Kp = (n + 3) & ~3;
    T *PT_re = smem;                 // [Kp][n]: PT[k][i] = P[i][k]
    T *PT_im = PT_re + (size_t)Kp * n;
    T *X_re = PT_im + (size_t)Kp * n;  // [2][Kp][NS]
    T *X_im = X_re + 2 * (size_t)Kp * NS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int b0 = blockIdx.x * NS;

    for (int e = tid; e < Kp * n; e += 256) {
        const int k = e / n, i = e - (e / n) * n;
        const cd v = k < n ? P[(size_t)i * n + k] : cd{0.0, 0.0};
        PT_re[e] = (T)v.re;
        PT_im[e] = (T)v.im;
    }
    for (int e = tid; e < 2 * Kp * NS; e += 256) {
        const int buf = e / (Kp * NS), r = e - buf * (Kp * NS);
        const int k = r / NS, sidx = r - k * NS;
        cd v = {0.0, 0.0};
        if (buf == 0 && k < n && b0 + sidx < B) v = rho[(size_t)(b0 + sidx) * n + k];
        X_re[e] = (T)v.re;
        X_im[e] = (T)v.im;
    }
    __syncthreads();

    const int mtiles = (n + 15) >> 4;
    int cur = 0;
    for (long long t = 0; t < nsteps; ++t) {
        const T *xr = X_re + (size_t)cur * Kp * NS, *xi = X_im + (size_t)cur * Kp * NS;
        T *yr = X_re + (size_t)(cur ^ 1) * Kp * NS, *yi = X_im + (size_t)(cur ^ 1) * Kp * NS;
        for (int mt0 = wave; mt0 < mtiles; mt0 += 8) {
            const int mt1 = mt0 + 4;
            const bool two = mt1 < mtiles;
            acc_t a0[4], a1[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a0[q] = acc_t{0, 0, 0, 0};
                a1[q] = acc_t{0, 0, 0, 0};
            }
            const int r0 = mt0 * 16 + (lane & 15), r1 = mt1 * 16 + (lane & 15);
            const bool v0 = r0 < n, v1 = two && r1 < n;
            for (int k0 = 0; k0 < Kp; k0 += 4) {
                const int k = k0 + (lane >> 4);
                const T xbr = xr[k * NS + (lane & 15)], xbi = xi[k * NS + (lane & 15)];
                const T p0r = v0 ? PT_re[(size_t)k * n + r0] : T(0), p0i = v0 ? PT_im[(size_t)k * n + r0] : T(0);
                a0[0] = Mfma<T>::mma(p0r, xbr, a0[0]);
                a0[1] = Mfma<T>::mma(-p0i, xbi, a0[1]);
                a0[2] = Mfma<T>::mma(p0r, xbi, a0[2]);
                a0[3] = Mfma<T>::mma(p0i, xbr, a0[3]);
                if (two) {
                    const T p1r = v1 ? PT_re[(size_t)k * n + r1] : T(0), p1i = v1 ? PT_im[(size_t)k * n + r1] : T(0);
                    a1[0] = Mfma<T>::mma(p1r, xbr, a1[0]);
                    a1[1] = Mfma<T>::mma(-p1i, xbi, a1[1]);
                    a1[2] = Mfma<T>::mma(p1r, xbi, a1[2]);
                    a1[3] = Mfma<T>::mma(p1i, xbr, a1[3]);
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i0 = mt0 * 16 + Mfma<T>::row(lane, r);
                if (i0 < n) {
                    yr[i0 * NS + (lane & 15)] = a0[0][r] + a0[1][r];
                    yi[i0 * NS + (lane & 15)] = a0[2][r] + a0[3][r];
                }
                const int i1 = mt1 * 16 + Mfma<T>::row(lane, r);
                if (two && i1 < n) {
                    yr[i1 * NS + (lane & 15)] = a1[0][r] + a1[1][r];
                    yi[i1 * NS + (lane & 15)] = a1[2][r] + a1[3][r];
                }
            }
        }
        cur ^= 1;
        __syncthreads();
    }
    const T *xr = X_re + (size_t)cur * Kp * NS, *xi = X_im + (size_t)cur * Kp * NS;
    for (int e = tid; e < n * NS; e += 256) {
        const int sidx = e / n, k = e - sidx * n;
        if (b0 + sidx < B) rho[(size_t)(b0 + sidx) * n + k] = {(double)xr[k * NS + sidx], (double)xi[k * NS + sidx]};
    }
}

static const size_t kLdsLimit = 160 * 1024;

int fused_max_n(lb_precision prec) {
    switch (prec) {
        case LB_C128: return 84;
        case LB_C64: return 124;
        default: return 0;
    }
}

template <typename T>
static int launch_fused(int n, const cd *P, int B, cd *rho, long long nsteps, hipStream_t s) {
    const size_t lds = fused_lds_bytes<T>(n);
    if (lds > kLdsLimit) return fail(LB_ESHAPE, "fused chain: n too large for LDS");
    static bool attr_set = false;
    if (!attr_set) {
        LB_HIP(hipFuncSetAttribute((const void *)fused_chain_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)kLdsLimit));
        attr_set = true;
    }
    const int blocks = (B + NS - 1) / NS;
    fused_chain_kernel<T><<<blocks, 256, lds, s>>>(n, P, B, rho, nsteps);
    return check_launch("fused_chain");
}

// ------------------------------------------------------------- large n
__global__ void __launch_bounds__(256) transpose_kernel(int n, const cd *__restrict__ P, cd *__restrict__ PT) {
    __shared__ cd tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int j = ty; j < 32; j += 8) {
        const int r = by + j, c = bx + tx;
        if (r < n && c < n) tile[j][tx] = P[(size_t)r * n + c];
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int r = bx + j, c = by + tx;
        if (r < n && c < n) PT[(size_t)r * n + c] = tile[tx][j];
    }
}

static int chain_large_c128(int n, const cd *P, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s) {
    const size_t pbytes = (size_t)n * n * sizeof(cd), xbytes = (size_t)B * n * sizeof(cd);
    LB_TRY(ws_reserve_total(ws, align256(pbytes) + align256(xbytes)));
    cd *PT = (cd *)ws_take(ws, pbytes);
    cd *tmp = (cd *)ws_take(ws, xbytes);
    dim3 tg((n + 31) / 32, (n + 31) / 32);
    transpose_kernel<<<tg, 256, 0, s>>>(n, P, PT);
    LB_TRY(check_launch("transpose"));
    ZgemmBatch g;
    g.M = B;
    g.N = n;
    g.K = n;
    g.lda = n;
    g.B = PT;
    g.ldb = n;
    g.ldd = n;
    cd *x = rho, *y = tmp;
    for (long long t = 0; t < nsteps; ++t) {
        g.A = x;
        g.D = y;
        LB_TRY(zgemm_batched(g, s));
        cd *z = x;
        x = y;
        y = z;
    }
    if (x != rho) LB_HIP(hipMemcpyAsync(rho, x, xbytes, hipMemcpyDeviceToDevice, s));
    return LB_OK;
}

int chain_run(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s) {
    if (nsteps == 0 || B == 0) return LB_OK;
    switch (prec) {
        case LB_C128:
            if (n <= fused_max_n(LB_C128)) return launch_fused<double>(n, P, B, rho, nsteps, s);
            return chain_large_c128(n, P, B, rho, nsteps, ws, s);
        case LB_C64:
            if (n <= fused_max_n(LB_C64)) return launch_fused<float>(n, P, B, rho, nsteps, s);
            return fail(LB_ENOTSUP, "lindblad_propagate: LB_C64 for n > 124 is not built yet");
        default:
            return fail(LB_ENOTSUP, "lindblad_propagate: precision not built yet");
    }
}

}  // namespace lb

using namespace lb;

static int validate_chain(const char *who, int n, const void *P, int B, const void *rho, long long nsteps) {
    if (n < 1 || n > 4096) return fail(LB_ESHAPE, std::string(who) + ": n must be in [1, 4096]");
    if (B < 1) return fail(LB_ESHAPE, std::string(who) + ": B must be >= 1");
    if (nsteps < 0) return fail(LB_EINVAL, std::string(who) + ": nsteps must be >= 0");
    if (!P || !rho) return fail(LB_EINVAL, std::string(who) + ": NULL pointer");
    return LB_OK;
}

extern "C" int lindblad_propagate(int n, const void *P, lb_precision prec, int B, void *rho, long long nsteps,
                                  lb_workspace *ws, hipStream_t stream) {
    LB_TRY(validate_chain("lindblad_propagate", n, P, B, rho, nsteps));
    if ((int)prec < LB_C128 || (int)prec > LB_BF16_SLICED) return fail(LB_EINVAL, "lindblad_propagate: bad precision");
    return chain_run(n, static_cast<const cd *>(P), prec, B, static_cast<cd *>(rho), nsteps, ws_resolve(ws), stream);
}

extern "C" int lindblad_propagate_baseline(int n, const void *P, int B, void *rho, long long nsteps, lb_workspace *ws,
                                           hipStream_t stream) {
    LB_TRY(validate_chain("lindblad_propagate_baseline", n, P, B, rho, nsteps));
    return chain_baseline(n, static_cast<const cd *>(P), B, static_cast<cd *>(rho), nsteps, ws_resolve(ws), stream);
}
