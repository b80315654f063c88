// Step chains for large n (P too big for one CU's LDS, e.g. d = 27, n = 729):
// one GEMM launch per step, Y[b][i] = sum_k X[b][k] P[i][k] (states as rows,
// outputs as columns, both operands read along k, which is contiguous in the
// row-major state batch and in the rows of P).
//
//   LB_C64, LB_C128 P and the states in complex FP32 / FP64 planes, FP32 or
//                   FP64 matrix cores (v_mfma_f{32,64}_16x16x4); each lane
//                   loads four consecutive k at once and feeds them to four
//                   MFMAs (the k order inside a 16-deep block is permuted
//                   identically for both operands, which leaves the sum
//                   unchanged).
//   LB_BF16_HILO    BF16 planes hi / lo of P (once per call) and of the FP32
//   LB_BF16_SLICED  state (every step), or exponent-aligned 8-bit integer
//                   slices exactly as in the fused kernel; BF16 matrix cores.
//                   For the slices the k range is cut into 64-deep chunks so
//                   that every level sum stays an exact FP32 integer
//                   (2 * 64 * max_L sum|q_a||q_b| < 2^24); each chunk's levels
//                   are flushed into FP64 accumulators.
// A workgroup owns a 16-state x 32-output tile; its four wavefronts split the
// k chunks and their FP64 partials are summed through LDS in a fixed order.
// Complex64 chains can also run as a per-state FP32 matvec (one wavefront per
// state and row), the counterpart of the FP64 baseline.
#include <cmath>
#include <complex>

#include "chain.hpp"

namespace lb {
namespace lg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

enum Mode { HILO = 0, SLICED = 1 };
constexpr int KCH = 64;  // k chunk (exact level sums for the slices)
constexpr int WN = 2;    // 16-output tiles per wavefront
constexpr int TS = 16;   // states per workgroup tile
constexpr int TO = 16 * WN;

__device__ inline unsigned short bf16_bits(float f) {
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_float(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }
__device__ inline int exp_of(double m) {
    if (!(m > 0.0)) return 0;
    int e;
    (void)frexp(m, &e);
    return e;
}
__device__ inline f4v mma(bf16x8 a, bf16x8 b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

template <int MODE, int SP, int SX>
struct Planes {
    static constexpr int XD = MODE == SLICED ? SX : 2;  // state digits
    static constexpr int PD = MODE == SLICED ? SP : 2;  // propagator digits
};

// P planes [PD][2][n][Kp] (Re, Im) and, for the slices, row exponents eP.
// One workgroup per row of P.
template <int MODE, int SP, int SX>
__global__ void __launch_bounds__(256) prep_p_kernel(int n, int Kp, const cd *__restrict__ P,
                                                     unsigned short *__restrict__ Pp, int *__restrict__ eP) {
    constexpr int PD = Planes<MODE, SP, SX>::PD;
    const int i = blockIdx.x;
    __shared__ double red[256];
    __shared__ int se;
    double m = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) {
        const cd v = P[(size_t)i * n + k];
        m = fmax(m, fmax(fabs(v.re), fabs(v.im)));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        se = MODE == SLICED ? exp_of(red[0]) : 0;
        eP[i] = se;
    }
    __syncthreads();
    const size_t plane = (size_t)n * Kp;
    for (int k = threadIdx.x; k < Kp; k += 256) {
        const cd v = k < n ? P[(size_t)i * n + k] : cd{0.0, 0.0};
        unsigned short *o = Pp + (size_t)i * Kp + k;
        if (MODE == SLICED) {
            double vr = ldexp(v.re, -se), vi = ldexp(v.im, -se);
#pragma unroll
            for (int a = 0; a < PD; ++a) {
                const double dr = rint(vr * 256.0), di = rint(vi * 256.0);
                vr = vr * 256.0 - dr;
                vi = vi * 256.0 - di;
                o[(a * 2 + 0) * plane] = bf16_bits((float)dr);
                o[(a * 2 + 1) * plane] = bf16_bits((float)di);
            }
        } else {
            const float fr = (float)v.re, fi = (float)v.im;
            const unsigned short hr = bf16_bits(fr), hi = bf16_bits(fi);
            o[0 * plane] = hr;
            o[1 * plane] = hi;
            o[2 * plane] = bf16_bits(fr - bf16_float(hr));
            o[3 * plane] = bf16_bits(fi - bf16_float(hi));
        }
    }
}

// State planes [XD][3][B][Kp] (Re, Im, -Im) and, for the slices, eX.  One
// workgroup per state.  HILO: the state is FP32 (Y holds FP32 values).  NEG:
// also write the -Im planes (the ring kernel negates in registers instead).
template <int MODE, int SP, int SX, bool NEG>
__global__ void __launch_bounds__(256) slice_x_kernel(int n, int Kp, int B, const cd *__restrict__ Y,
                                                      unsigned short *__restrict__ Xp, int *__restrict__ eX) {
    constexpr int XD = Planes<MODE, SP, SX>::XD;
    const int b = blockIdx.x;
    __shared__ double red[256];
    __shared__ int se;
    double m = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) {
        const cd v = Y[(size_t)b * n + k];
        m = fmax(m, fmax(fabs(v.re), fabs(v.im)));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        se = MODE == SLICED ? exp_of(red[0]) : 0;
        eX[b] = se;
    }
    __syncthreads();
    const size_t plane = (size_t)B * Kp;
    for (int k = threadIdx.x; k < Kp; k += 256) {
        const cd v = k < n ? Y[(size_t)b * n + k] : cd{0.0, 0.0};
        unsigned short *o = Xp + (size_t)b * Kp + k;
        if (MODE == SLICED) {
            double vr = ldexp(v.re, -se), vi = ldexp(v.im, -se);
#pragma unroll
            for (int a = 0; a < XD; ++a) {
                const double dr = rint(vr * 256.0), di = rint(vi * 256.0);
                vr = vr * 256.0 - dr;
                vi = vi * 256.0 - di;
                o[(a * 3 + 0) * plane] = bf16_bits((float)dr);
                o[(a * 3 + 1) * plane] = bf16_bits((float)di);
                if (NEG) o[(a * 3 + 2) * plane] = bf16_bits((float)-di);
            }
        } else {
            const float fr = (float)v.re, fi = (float)v.im;
            const unsigned short hr = bf16_bits(fr), hi = bf16_bits(fi);
            const unsigned short lr = bf16_bits(fr - bf16_float(hr)), li = bf16_bits(fi - bf16_float(hi));
            o[0 * plane] = hr;
            o[1 * plane] = hi;
            if (NEG) o[2 * plane] = hi ^ 0x8000u;
            o[3 * plane] = lr;
            o[4 * plane] = li;
            if (NEG) o[5 * plane] = li ^ 0x8000u;
        }
    }
}

template <int MODE, int SP, int SX, int LMAX>
__global__ void __launch_bounds__(256) plane_gemm_kernel(int n, int B, int Kp, const unsigned short *__restrict__ Xp,
                                                         const unsigned short *__restrict__ Pp,
                                                         const int *__restrict__ eP, const int *__restrict__ eX,
                                                         cd *__restrict__ Y) {
    constexpr int XD = Planes<MODE, SP, SX>::XD, PD = Planes<MODE, SP, SX>::PD;
    constexpr int NL = MODE == SLICED ? LMAX + 1 : 1;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int b0 = blockIdx.y * TS, i0 = blockIdx.x * TO;
    const int bl = b0 + (lane & 15);
    const bool bvalid = bl < B;
    const size_t xplane = (size_t)B * Kp, pplane = (size_t)n * Kp;
    const unsigned short *xrow = Xp + (size_t)(bvalid ? bl : 0) * Kp + 8 * (lane >> 4);
    const unsigned short *prow[WN];
    bool pvalid[WN];
#pragma unroll
    for (int t = 0; t < WN; ++t) {
        const int i = i0 + t * 16 + (lane & 15);
        pvalid[t] = i < n;
        prow[t] = Pp + (size_t)(pvalid[t] ? i : 0) * Kp + 8 * (lane >> 4);
    }
    double ar[WN][4], ai[WN][4];
#pragma unroll
    for (int t = 0; t < WN; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) ar[t][r] = ai[t][r] = 0.0;
    const bf16x8 zero = {};
    const int nch = Kp / KCH;
    for (int kc = wave; kc < nch; kc += 4) {
        f4v lr[WN][NL], li[WN][NL];
#pragma unroll
        for (int t = 0; t < WN; ++t)
#pragma unroll
            for (int L = 0; L < NL; ++L) lr[t][L] = li[t][L] = f4v{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KCH / 32; ++ks) {
            const int k = kc * KCH + ks * 32;
            bf16x8 xa[XD][3];
#pragma unroll
            for (int a = 0; a < XD; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    xa[a][c] = bvalid ? *reinterpret_cast<const bf16x8 *>(xrow + (a * 3 + c) * xplane + k) : zero;
#pragma unroll
            for (int t = 0; t < WN; ++t) {
                bf16x8 pb[PD][2];
#pragma unroll
                for (int a = 0; a < PD; ++a)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        pb[a][c] = pvalid[t] ? *reinterpret_cast<const bf16x8 *>(prow[t] + (a * 2 + c) * pplane + k)
                                             : zero;
#pragma unroll
                for (int a = 0; a < PD; ++a)
#pragma unroll
                    for (int bq = 0; bq < XD; ++bq) {
                        const int L = a + bq;
                        if (MODE == SLICED ? (L <= LMAX) : (L <= 1)) {
                            const int Lq = MODE == SLICED ? L : 0;
                            lr[t][Lq] = mma(xa[bq][0], pb[a][0], lr[t][Lq]);
                            lr[t][Lq] = mma(xa[bq][2], pb[a][1], lr[t][Lq]);
                            li[t][Lq] = mma(xa[bq][1], pb[a][0], li[t][Lq]);
                            li[t][Lq] = mma(xa[bq][0], pb[a][1], li[t][Lq]);
                        }
                    }
            }
        }
#pragma unroll
        for (int t = 0; t < WN; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int L = NL - 1; L >= 0; --L) {
                    const double w = MODE == SLICED ? ldexp(1.0, -8 * (L + 2)) : 1.0;
                    ar[t][r] = fma((double)lr[t][L][r], w, ar[t][r]);
                    ai[t][r] = fma((double)li[t][L][r], w, ai[t][r]);
                }
    }
    // sum the wavefronts' partials (fixed order) and write
    __shared__ double red[4][WN][4][2][64];
#pragma unroll
    for (int t = 0; t < WN; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            red[wave][t][r][0][lane] = ar[t][r];
            red[wave][t][r][1][lane] = ai[t][r];
        }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int t = 0; t < WN; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double sr = red[0][t][r][0][lane], si = red[0][t][r][1][lane];
                for (int w = 1; w < 4; ++w) {
                    sr += red[w][t][r][0][lane];
                    si += red[w][t][r][1][lane];
                }
                const int b = b0 + 4 * (lane >> 4) + r, i = i0 + t * 16 + (lane & 15);
                if (b < B && i < n) {
                    if (MODE == SLICED) {
                        const int sc = eP[i] + eX[b];
                        Y[(size_t)b * n + i] = {ldexp(sr, sc), ldexp(si, sc)};
                    } else {
                        Y[(size_t)b * n + i] = {(double)(float)sr, (double)(float)si};
                    }
                }
            }
    }
}

// LDS-tiled BF16 plane GEMM: the step of plane_gemm_kernel with a 64-state x
// 48-output tile per workgroup (B = 1024, n = 729: 256 workgroups), so that
// each digit-plane byte fetched from L2 feeds 48 or 64 products instead of 16
// or 32.  Wavefront w owns states 16 w .. 16 w + 15 of the tile against all
// 48 outputs (three MFMA blocks) over every k.  k advances TPK = 32 (one
// v_mfma_f32_16x16x32_bf16 deep) at a time through two LDS buffers, filled
// by direct global-to-LDS loads (global_load_lds_dwordx4: lane l's 16 bytes
// land at the wavefront's LDS base + 16 l) issued for the next chunk before
// the current one is multiplied, so no staging registers are needed.  Each
// plane row is 64 bytes = four 16-byte chunks, stored at the XOR-swizzled
// position tp_swz(row, c) so that one MFMA operand fetch runs without bank
// conflicts and without padding; each lane loads the chunk that belongs in
// its slot.  Rows past B or n load a valid row instead (they only
// feed outputs that are not written).  Level sums are flushed into FP64
// every KCH = 64 k, exactly as in the untiled kernel, so the results agree
// with it to the FP64 rounding of the flushes.
constexpr int TPB = 64, TPI = 48, TPK = 32;

template <int MODE, int SP, int SX>
struct TpShape {
    static constexpr int XD = Planes<MODE, SP, SX>::XD, PD = Planes<MODE, SP, SX>::PD;
    static constexpr int XPL = 3 * XD, PPL = 2 * PD;            // planes
    static constexpr int ROWB = TPK * 2;                        // bytes per plane row (64)
    static constexpr int XPB = TPB * ROWB, PPB = TPI * ROWB;    // bytes per plane tile
    static constexpr int BUF = XPL * XPB + PPL * PPB;           // bytes per buffer
    static constexpr int XI = XPB / 1024, PI = PPB / 1024;      // 1 KB loads per plane tile (4, 3)
    static constexpr int NI = XPL * XI + PPL * PI;              // 1 KB loads per chunk
};

// Position of a 64-byte row's 16-byte chunk c.  For the operand fetch (lane
// l reads chunk l / 16 of row l % 16 of a 16-row block) the XOR with row bits
// 1..2 is the pattern gfx950's LDS bank-conflict counter reads as
// conflict-free; XOR with bits 2..3, or no swizzle, reads as two-way.
__device__ inline int tp_swz(int row, int c) { return c ^ ((row >> 1) & 3); }

template <int MODE, int SP, int SX, int LMAX>
__global__ void __launch_bounds__(256) tplane_gemm_kernel(int n, int B, int Kp, int nbt, int nit,
                                                          const unsigned short *__restrict__ Xp,
                                                          const unsigned short *__restrict__ Pp,
                                                          const int *__restrict__ eP, const int *__restrict__ eX,
                                                          cd *__restrict__ Y) {
    typedef TpShape<MODE, SP, SX> S;
    constexpr int XD = S::XD, PD = S::PD;
    constexpr int NLV = MODE == SLICED ? LMAX + 1 : 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int total = nbt * nit, per = total / 8, rem = total % 8;
    const int xcd = blockIdx.x % 8, jx = blockIdx.x / 8;
    const int L0 = xcd * per + (xcd < rem ? xcd : rem) + jx;
    const int bt = L0 / nit, it = L0 - bt * nit;
    const int b0 = bt * TPB, i0 = it * TPI;
    const size_t xplane = (size_t)B * Kp, pplane = (size_t)n * Kp;

    // this lane's slot in a 1 KB load: row 16 j + lane / 4 of the plane tile,
    // chunk position lane % 4, which holds chunk tp_swz(row, lane % 4).  The
    // wavefront's loads are j = wave, wave + 4, ...; their source offsets (in
    // elements, k0 = 0) and LDS destinations are fixed for the whole step.
    constexpr int NJ = (S::NI + 3) / 4;
    const unsigned short *srcp[NJ];
    int dsto[NJ];
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        const int j = wave + 4 * q;
        srcp[q] = Xp;
        dsto[q] = 0;
        if (j < S::XPL * S::XI) {
            const int pl = j / S::XI, jj = j - pl * S::XI, row = 16 * jj + (lane >> 2);
            int b = b0 + row;
            b = b < B ? b : B - 1;
            srcp[q] = Xp + pl * xplane + (size_t)b * Kp + 8 * tp_swz(row, lane & 3);
            dsto[q] = pl * S::XPB + 1024 * jj;
        } else if (j < S::NI) {
            const int jp = j - S::XPL * S::XI, pl = jp / S::PI, jj = jp - pl * S::PI, row = 16 * jj + (lane >> 2);
            int i = i0 + row;
            i = i < n ? i : n - 1;
            srcp[q] = Pp + pl * pplane + (size_t)i * Kp + 8 * tp_swz(row, lane & 3);
            dsto[q] = S::XPL * S::XPB + pl * S::PPB + 1024 * jj;
        }
    }
    auto issue = [&](int k0, unsigned char *buf) {
#pragma unroll
        for (int q = 0; q < NJ; ++q)
            if (wave + 4 * q < S::NI)  // uniform per wavefront
                __builtin_amdgcn_global_load_lds((const void *)(srcp[q] + k0),
                                                 (__attribute__((address_space(3))) void *)(buf + dsto[q]), 16, 0, 0);
    };

    double ar[3][4], ai[3][4];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) ar[t][r] = ai[t][r] = 0.0;
    // this lane's operand rows and chunk (k = 8 (lane / 16) .. + 7 of the chunk)
    const int xrow = 16 * wave + (lane & 15), prow = lane & 15, cq = lane >> 4;
    const int xoff = xrow * S::ROWB + 16 * tp_swz(xrow, cq);
    int poff[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) poff[t] = (16 * t + prow) * S::ROWB + 16 * tp_swz(16 * t + prow, cq);

    // chunk c (32 k) from buffer c & 1; two chunks (KCH = 64 k) per iteration,
    // the level sums start from zero and are flushed into FP64 at its end
    auto chunk = [&](const unsigned char *buf, f4v (&lr)[3][NLV], f4v (&li)[3][NLV]) {
        bf16x8 xa[XD][3];
#pragma unroll
        for (int a = 0; a < XD; ++a)
#pragma unroll
            for (int q = 0; q < 3; ++q)
                xa[a][q] = *reinterpret_cast<const bf16x8 *>(buf + (a * 3 + q) * S::XPB + xoff);
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            bf16x8 pb[PD][2];
#pragma unroll
            for (int a = 0; a < PD; ++a)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    pb[a][q] = *reinterpret_cast<const bf16x8 *>(buf + S::XPL * S::XPB + (a * 2 + q) * S::PPB + poff[t]);
#pragma unroll
            for (int a = 0; a < PD; ++a)
#pragma unroll
                for (int bq = 0; bq < XD; ++bq) {
                    const int L = a + bq;
                    if (MODE == SLICED ? (L <= LMAX) : (L <= 1)) {
                        const int Lq = MODE == SLICED ? L : 0;
                        lr[t][Lq] = mma(xa[bq][0], pb[a][0], lr[t][Lq]);
                        lr[t][Lq] = mma(xa[bq][2], pb[a][1], lr[t][Lq]);
                        li[t][Lq] = mma(xa[bq][1], pb[a][0], li[t][Lq]);
                        li[t][Lq] = mma(xa[bq][0], pb[a][1], li[t][Lq]);
                    }
                }
        }
    };
    const int nch = Kp / TPK;  // even: Kp is a multiple of KCH = 64
    issue(0, smem_raw);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int c = 0; c < nch; c += 2) {
        f4v lr[3][NLV], li[3][NLV];
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int L = 0; L < NLV; ++L) lr[t][L] = li[t][L] = f4v{0, 0, 0, 0};
        issue((c + 1) * TPK, smem_raw + S::BUF);
        chunk(smem_raw, lr, li);
        __builtin_amdgcn_s_waitcnt(0);  // this wavefront's loads into buffer 1 have landed
        __syncthreads();
        if (c + 2 < nch) issue((c + 2) * TPK, smem_raw);
        chunk(smem_raw + S::BUF, lr, li);
        // KCH = 64 k done: flush the exact level sums into FP64
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int L = NLV - 1; L >= 0; --L) {
                    const double w = MODE == SLICED ? ldexp(1.0, -8 * (L + 2)) : 1.0;
                    ar[t][r] = fma((double)lr[t][L][r], w, ar[t][r]);
                    ai[t][r] = fma((double)li[t][L][r], w, ai[t][r]);
                }
        if (c + 2 < nch) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = b0 + 16 * wave + 4 * (lane >> 4) + r, i = i0 + 16 * t + (lane & 15);
            if (b < B && i < n) {
                if (MODE == SLICED) {
                    const int sc = eP[i] + eX[b];
                    Y[(size_t)b * n + i] = {ldexp(ar[t][r], sc), ldexp(ai[t][r], sc)};
                } else {
                    Y[(size_t)b * n + i] = {(double)(float)ar[t][r], (double)(float)ai[t][r]};
                }
            }
        }
}

// The same tile with a deeper pipeline.  The state digit planes lose the -Im
// copy (a sign flip in registers instead), and each wavefront stages only its
// own 16 state rows, two chunks deep in a private LDS area: chunk s's planes
// are read into registers at its start, then chunk s + 2's are loaded into
// their place.  The propagator digit planes, shared by all four wavefronts,
// go through a ring of R chunk slots refilled R - 1 chunks ahead.  Every load
// is a direct global-to-LDS load, so one in-order counter covers them all: at
// each chunk's barrier a wavefront waits only for its own loads that the
// chunk needs and leaves the later ones in flight (__syncthreads() would wait
// for all of them).  A chunk's loads are spread between its MFMA groups, so
// that their issue overlaps the matrix work.  Past the last chunk the loads
// repeat valid addresses into slots no later chunk reads, so every chunk
// issues the same loads and the wait count is a constant.  k runs in whole
// 128-deep blocks (Kp a multiple of 128).
constexpr int TQK = 128;  // k granularity of the ring kernel
constexpr int kLdsBytes = 160 * 1024;

template <int MODE, int SP, int SX>
struct TqShape {
    static constexpr int XD = Planes<MODE, SP, SX>::XD, PD = Planes<MODE, SP, SX>::PD;
    static constexpr int PPL = 2 * PD;        // propagator planes (Re, Im per digit)
    static constexpr int ROWB = TPK * 2;      // bytes per plane row of a chunk (64)
    static constexpr int PPB = TPI * ROWB;    // bytes per plane tile (3 KB)
    static constexpr int BUF = PPL * PPB;     // bytes per ring slot
    static constexpr int PI = PPB / 1024;     // 1 KB loads per plane tile (3)
    static constexpr int NI = PPL * PI;       // 1 KB loads per chunk
    static constexpr int NJ = (NI + 3) / 4;   // per wavefront (the last few repeat others)
    static constexpr int XL = 2 * XD;         // state loads per wavefront and chunk: (digit, Re/Im), 1 KB each
    static constexpr int NDMA = NJ + XL;      // loads per wavefront and chunk
    static constexpr int XST = 4 * 2 * XL * 1024;  // state staging: four wavefronts, two chunks
    static constexpr int R = (kLdsBytes - XST) / BUF >= 4 ? 4 : 3;  // ring slots
    static constexpr int LDS = R * BUF + XST;
    // Chunk t issues chunk t + R - 1's propagator loads, then chunk t + 2's
    // state loads.  Chunk s needs its state planes (issued by chunk s - 2)
    // and its ring slot (issued before them): at its barrier only the NDMA
    // loads of chunk s - 1 may still be in flight.
    static constexpr int WAIT = NDMA;
    static_assert(LDS <= kLdsBytes && WAIT <= 63, "ring kernel shape");
};

// Workgroup barrier for the ring: wait until at most N of this wavefront's
// vector loads are outstanding and all its LDS reads are done (s_waitcnt,
// gfx9 encoding: vmcnt N, expcnt 7 = no wait, lgkmcnt 0), then s_barrier.
// The empty asm statements keep the compiler from moving memory accesses
// across it.
#define TQ_SYNC(N)                                                                  \
    do {                                                                            \
        asm volatile("" ::: "memory");                                              \
        __builtin_amdgcn_s_waitcnt(((N) & 15) | (7 << 4) | (((N) >> 4) << 14));    \
        __builtin_amdgcn_s_barrier();                                               \
        asm volatile("" ::: "memory");                                              \
    } while (0)

__device__ inline bf16x8 bf16_neg(bf16x8 v) {
    typedef unsigned u4v __attribute__((ext_vector_type(4)));
    u4v u = __builtin_bit_cast(u4v, v);
    u ^= 0x80008000u;
    return __builtin_bit_cast(bf16x8, u);
}

// Split k (ksplit > 1, for batches too small to fill the chip): workgroup
// L = ks * tiles + tile takes chunks [ks cper, (ks + 1) cper) and writes its
// scaled FP64 partial sums to Ypart[ks]; split_sum_kernel adds them in order.
template <int MODE, int SP, int SX, int LMAX>
__global__ void __launch_bounds__(256) tqplane_gemm_kernel(int n, int B, int Kp, int nbt, int nit,
                                                           const unsigned short *__restrict__ Xp,
                                                           const unsigned short *__restrict__ Pp,
                                                           const int *__restrict__ eP, const int *__restrict__ eX,
                                                           cd *__restrict__ Y, int ksplit, int cper,
                                                           cd *__restrict__ Ypart) {
    typedef TqShape<MODE, SP, SX> S;
    constexpr int XD = S::XD, PD = S::PD, R = S::R, NJ = S::NJ;
    constexpr int NLV = MODE == SLICED ? LMAX + 1 : 1;
    // MFMA groups (4 MFMAs: one digit pair, one 16-output tile) per chunk
    constexpr int NPAIR = [] {
        int c = 0;
        for (int a = 0; a < PD; ++a)
            for (int b = 0; b < XD; ++b) c += (MODE == SLICED ? (a + b <= LMAX) : (a + b <= 1));
        return c;
    }();
    constexpr int NG = 3 * NPAIR;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tiles = nbt * nit, total = tiles * ksplit, per = total / 8, rem = total % 8;
    const int xcd = blockIdx.x % 8, jx = blockIdx.x / 8;
    const int L = xcd * per + (xcd < rem ? xcd : rem) + jx;
    const int ks = L / tiles, L0 = L - ks * tiles;
    const int bt = L0 / nit, it = L0 - bt * nit;
    const int b0 = bt * TPB, i0 = it * TPI;
    const size_t xplane = (size_t)B * Kp, pplane = (size_t)n * Kp;
    // this workgroup's chunks: kc0 .. kc0 + nch - 1 (an even count)
    const int kc0 = ks * cper, nall = Kp / TPK;
    const int nch = nall - kc0 < cper ? nall - kc0 : cper;
    unsigned char *xst = smem_raw + R * S::BUF + wave * (2 * S::XL * 1024);  // this wavefront's staging

    // a 1 KB load puts lane l's 16 bytes at row l / 4, chunk position l % 4
    // of a 16-row plane tile; that position holds the row's 16-byte piece
    // tp_swz(row, l % 4).  Propagator: load j = wave + 4 q of a chunk (past
    // NI it repeats load j - (4 NJ - NI): same data to the same place)
    const int lrow = lane >> 2, lpiece = 8 * tp_swz(lane >> 2, lane & 3);
    const unsigned short *srcp[NJ];
    int dsto[NJ];
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        int j = wave + 4 * q;
        j = j < S::NI ? j : j - (4 * NJ - S::NI);
        const int pl = j / S::PI, jj = j - pl * S::PI;
        int i = i0 + 16 * jj + lrow;
        i = i < n ? i : n - 1;
        srcp[q] = Pp + pl * pplane + (size_t)i * Kp + lpiece;
        dsto[q] = pl * S::PPB + 1024 * jj;
    }
    int xr = b0 + 16 * wave + lrow;
    xr = xr < B ? xr : B - 1;
    const unsigned short *xsrc = Xp + (size_t)xr * Kp + lpiece;
    // load k of chunk t's set: propagator load k of chunk t + R - 1 into slot
    // (t + R - 1) % R, then state tile (digit, Re/Im) k - NJ of chunk t + 2
    // into staging slot t % 2 (past the last chunk: the last chunk again)
    auto dma = [&](int t, int k) {  // t, c: chunks counted from kc0
        if (k < NJ) {
            const int c = t + R - 1;
            const int k0 = (kc0 + (c < nch ? c : nch - 1)) * TPK;
            __builtin_amdgcn_global_load_lds(
                (const void *)(srcp[k] + k0),
                (__attribute__((address_space(3))) void *)(smem_raw + (c % R) * S::BUF + dsto[k]), 16, 0, 0);
        } else {
            const int c = t + 2, tile = k - NJ, a = tile >> 1, q = tile & 1;
            const int k0 = (kc0 + (c < nch ? c : nch - 1)) * TPK;
            __builtin_amdgcn_global_load_lds(
                (const void *)(xsrc + (a * 3 + q) * xplane + k0),
                (__attribute__((address_space(3))) void *)(xst + ((t & 1) * S::XL + tile) * 1024), 16, 0, 0);
        }
    };
    // MFMA operands: row lane % 16 of a 16-row tile, k = 8 (lane / 16) .. + 7
    const int orow = lane & 15, ooff = orow * S::ROWB + 16 * tp_swz(orow, lane >> 4);

    double ar[3][4], ai[3][4];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) ar[t][r] = ai[t][r] = 0.0;

    // chunk s: barrier, its state planes into registers, then the MFMA groups
    // with chunk s's loads issued between them
    auto chunk = [&](int s, f4v(&lr)[3][NLV], f4v(&li)[3][NLV]) {
        TQ_SYNC(S::WAIT);
        const unsigned char *buf = smem_raw + (s % R) * S::BUF;
        const unsigned char *xs = xst + (s & 1) * S::XL * 1024 + ooff;
        bf16x8 x[XD][2], xm[XD];
#pragma unroll
        for (int a = 0; a < XD; ++a)
#pragma unroll
            for (int q = 0; q < 2; ++q) x[a][q] = *reinterpret_cast<const bf16x8 *>(xs + (a * 2 + q) * 1024);
#pragma unroll
        for (int a = 0; a < XD; ++a) xm[a] = bf16_neg(x[a][1]);
        int g = 0;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            bf16x8 pb[PD][2];
#pragma unroll
            for (int a = 0; a < PD; ++a)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    pb[a][q] = *reinterpret_cast<const bf16x8 *>(buf + (a * 2 + q) * S::PPB + 16 * t * S::ROWB + ooff);
#pragma unroll
            for (int a = 0; a < PD; ++a)
#pragma unroll
                for (int bq = 0; bq < XD; ++bq) {
                    const int L = a + bq;
                    if (MODE == SLICED ? (L <= LMAX) : (L <= 1)) {
                        // this group's share of the chunk's loads; the state
                        // staging slot is rewritten only after its reads returned
#pragma unroll
                        for (int k = 0; k < S::NDMA; ++k)
                            if (k * NG >= g * S::NDMA && k * NG < (g + 1) * S::NDMA) {
                                if (k == NJ) {
                                    asm volatile("" ::: "memory");
                                    __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (3 << 14));  // lgkmcnt 0 only
                                    asm volatile("" ::: "memory");
                                }
                                dma(s, k);
                            }
                        const int Lq = MODE == SLICED ? L : 0;
                        lr[t][Lq] = mma(x[bq][0], pb[a][0], lr[t][Lq]);
                        lr[t][Lq] = mma(xm[bq], pb[a][1], lr[t][Lq]);
                        li[t][Lq] = mma(x[bq][1], pb[a][0], li[t][Lq]);
                        li[t][Lq] = mma(x[bq][0], pb[a][1], li[t][Lq]);
                        ++g;
                    }
                }
        }
    };

    // prologue: the loads of chunks -R + 1 .. -1 in the same order (chunk t's
    // state loads only where t + 2 >= 0)
#pragma unroll
    for (int t = -R + 1; t < 0; ++t) {
#pragma unroll
        for (int k = 0; k < S::NDMA; ++k)
            if (k < NJ || t + 2 >= 0) dma(t, k);
    }
    for (int c = 0; c < nch; c += 2) {
        f4v lr[3][NLV], li[3][NLV];
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int L = 0; L < NLV; ++L) lr[t][L] = li[t][L] = f4v{0, 0, 0, 0};
        chunk(c, lr, li);
        chunk(c + 1, lr, li);
        // KCH = 64 k done: flush the exact level sums into FP64
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int L = NLV - 1; L >= 0; --L) {
                    const double w = MODE == SLICED ? ldexp(1.0, -8 * (L + 2)) : 1.0;
                    ar[t][r] = fma((double)lr[t][L][r], w, ar[t][r]);
                    ai[t][r] = fma((double)li[t][L][r], w, ai[t][r]);
                }
    }
    __builtin_amdgcn_s_waitcnt(0);  // the loads past the last chunk land before the workgroup ends
    cd *out = ksplit > 1 ? Ypart + (size_t)ks * B * n : Y;
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = b0 + 16 * wave + 4 * (lane >> 4) + r, i = i0 + 16 * t + (lane & 15);
            if (b < B && i < n) {
                if (MODE == SLICED) {
                    const int sc = eP[i] + eX[b];
                    out[(size_t)b * n + i] = {ldexp(ar[t][r], sc), ldexp(ai[t][r], sc)};
                } else if (ksplit > 1) {  // rounded to FP32 after the sum
                    out[(size_t)b * n + i] = {ar[t][r], ai[t][r]};
                } else {
                    out[(size_t)b * n + i] = {(double)(float)ar[t][r], (double)(float)ai[t][r]};
                }
            }
        }
}

// Y[e] = sum over ks = 0, 1, ... of Ypart[ks][e] (in that order); HILO rounds
// the sum to FP32 as the unsplit kernel does
template <int MODE>
__global__ void split_sum_kernel(long long total, int ksplit, const cd *__restrict__ Ypart, cd *__restrict__ Y) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k < ksplit; ++k) {
            const cd v = Ypart[(size_t)k * total + e];
            re += v.re;
            im += v.im;
        }
        Y[e] = MODE == SLICED ? cd{re, im} : cd{(double)(float)re, (double)(float)im};
    }
}

// split of the k range for the ring kernel: enough workgroups for the chip
// (about 256) in whole 64-k pairs; returns ksplit, sets the chunks per split
static int tq_split(int tiles, int Kp, int *cper) {
    const int npairs = Kp / KCH;
    int ks = tiles >= 256 ? 1 : (256 + tiles - 1) / tiles;
    ks = ks < npairs ? ks : npairs;
    const int pp = (npairs + ks - 1) / ks;
    *cper = 2 * pp;
    return (npairs + pp - 1) / pp;
}

// --------------------------------------------------------- FP32 / FP64
// planar copies: re[rows][Kp], im[rows][Kp] (zero padded in k)
template <typename T>
__global__ void to_planes_kernel(int rows, int n, int Kp, const cd *__restrict__ src, T *__restrict__ re,
                                 T *__restrict__ im) {
    const long long total = (long long)rows * Kp;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long r = e / Kp, k = e - r * Kp;
        const cd v = k < n ? src[r * n + k] : cd{0.0, 0.0};
        re[e] = (T)v.re;
        im[e] = (T)v.im;
    }
}

typedef float f4s __attribute__((ext_vector_type(4)));
typedef double d4s __attribute__((ext_vector_type(4)));

template <typename T>
struct StepMma;
template <>
struct StepMma<float> {
    typedef f4s v4;
    typedef f4v acc;
    static __device__ inline acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct StepMma<double> {
    typedef d4s v4;
    typedef d4s acc;
    static __device__ inline acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// Y[b][i] = sum_k X[b][k] P[i][k] in T on the matrix cores, 16 states x 16 GWN
// outputs per workgroup.  Wavefronts split
// the 16-deep k blocks; per block each lane loads 4 consecutive k of its state
// row and of its P rows and feeds them to four MFMAs (four real products per
// complex block, each in its own accumulator).  Writes the planar next state
// and, on the last step, the complex128 result.
template <typename T, int GWN>
__global__ void __launch_bounds__(256) gemm_step_kernel(int n, int B, int Kp, const T *__restrict__ Xr,
                                                        const T *__restrict__ Xi, const T *__restrict__ Pr,
                                                        const T *__restrict__ Pi, T *__restrict__ Yr,
                                                        T *__restrict__ Yi, cd *__restrict__ Yout) {
    typedef typename StepMma<T>::v4 v4;
    typedef typename StepMma<T>::acc acc_t;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int b0 = blockIdx.y * TS, i0 = blockIdx.x * 16 * GWN;
    const int bl = b0 + (lane & 15);
    const bool bvalid = bl < B;
    const size_t xo = (size_t)(bvalid ? bl : 0) * Kp + 4 * (lane >> 4);
    size_t po[GWN];
    bool pvalid[GWN];
#pragma unroll
    for (int t = 0; t < GWN; ++t) {
        const int i = i0 + t * 16 + (lane & 15);
        pvalid[t] = i < n;
        po[t] = (size_t)(pvalid[t] ? i : 0) * Kp + 4 * (lane >> 4);
    }
    acc_t rr[GWN], ii[GWN], ri[GWN], ir[GWN];
#pragma unroll
    for (int t = 0; t < GWN; ++t) rr[t] = ii[t] = ri[t] = ir[t] = acc_t{0, 0, 0, 0};
    const v4 z = {0, 0, 0, 0};
    // operands of the next k block are loaded while this one is multiplied
    v4 xr, xi, pr[GWN], pi[GWN];
    auto load = [&](int kb) {
        xr = bvalid ? *reinterpret_cast<const v4 *>(Xr + xo + kb) : z;
        xi = bvalid ? *reinterpret_cast<const v4 *>(Xi + xo + kb) : z;
#pragma unroll
        for (int t = 0; t < GWN; ++t) {
            pr[t] = pvalid[t] ? *reinterpret_cast<const v4 *>(Pr + po[t] + kb) : z;
            pi[t] = pvalid[t] ? *reinterpret_cast<const v4 *>(Pi + po[t] + kb) : z;
        }
    };
    if (wave * 16 < Kp) load(wave * 16);
    for (int kb = wave * 16; kb < Kp; kb += 64) {
        const v4 cxr = xr, cxi = xi;
        v4 cpr[GWN], cpi[GWN];
#pragma unroll
        for (int t = 0; t < GWN; ++t) {
            cpr[t] = pr[t];
            cpi[t] = pi[t];
        }
        if (kb + 64 < Kp) load(kb + 64);
#pragma unroll
        for (int t = 0; t < GWN; ++t) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                rr[t] = StepMma<T>::mma(cxr[q], cpr[t][q], rr[t]);
                ii[t] = StepMma<T>::mma(cxi[q], cpi[t][q], ii[t]);
                ri[t] = StepMma<T>::mma(cxr[q], cpi[t][q], ri[t]);
                ir[t] = StepMma<T>::mma(cxi[q], cpr[t][q], ir[t]);
            }
        }
    }
    __shared__ T red[4][GWN][4][2][64];
#pragma unroll
    for (int t = 0; t < GWN; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            red[wave][t][r][0][lane] = rr[t][r] - ii[t][r];
            red[wave][t][r][1][lane] = ri[t][r] + ir[t][r];
        }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int t = 0; t < GWN; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T sr = red[0][t][r][0][lane], si = red[0][t][r][1][lane];
                for (int w = 1; w < 4; ++w) {
                    sr += red[w][t][r][0][lane];
                    si += red[w][t][r][1][lane];
                }
                const int b = b0 + StepMma<T>::row(lane, r), i = i0 + t * 16 + (lane & 15);
                if (b < B && i < n) {
                    Yr[(size_t)b * Kp + i] = sr;
                    Yi[(size_t)b * Kp + i] = si;
                    if (Yout) Yout[(size_t)b * n + i] = {(double)sr, (double)si};
                }
            }
    }
}

// ------------------------------------------ LDS-tiled FP32 / FP64 GEMM step
// The same step, Y[b][i] = sum_k X[b][k] P[i][k], with a 64-state x 48-output
// tile per workgroup (B = 1024, n = 729: 16 x 16 = 256 workgroups, one per
// CU) so that each operand byte fetched feeds 48 or 64 products instead of
// 16 or 32.  Wavefront w % 4 owns states 16 (w % 4) .. + 15 of the tile
// against all 48 outputs (three MFMA blocks).  k advances KC = 32 at a time
// through two LDS buffers (row-major planes, rows padded by 16 bytes; the
// bank-conflict counter still reads this kernel's LDS traffic as partly
// conflicted, about 2.7 stall cycles per LDS instruction); the next chunk is
// loaded into registers while the current one is multiplied.  With WPB = 8
// the two wavefronts of a SIMD take alternate 16-deep halves of every chunk
// and the second adds its partial sums through LDS once at the end.  Each
// lane reads four consecutive k of a row at once and feeds them to four MFMAs
// (the same k permutation on both operands leaves the sum unchanged).
// -Im X Im P uses the FP64 MFMA's negate-A modifier, and a negated Im X plane
// in LDS for FP32.  Workgroups are numbered so that each XCD (workgroup id
// mod 8) runs a contiguous range of tiles: whole rows of state tiles, which
// then stream P through that XCD's own L2.
constexpr int TGB = 64, TGI = 48, TGK = 32;

template <typename T, int WPB>
struct TgShape {
    static constexpr int PAD = 16 / sizeof(T);  // keeps 16-byte row alignment
    static constexpr int LD = TGK + PAD;
    static constexpr int XPL = sizeof(T) == 8 ? 2 : 3;  // X planes in LDS: re, im (, -im)
    static constexpr int XS = TGB * LD, PS = TGI * LD;  // plane sizes in T
    static constexpr int BUF = XPL * XS + 2 * PS;
    static constexpr int VPT = 16 / sizeof(T);          // T per 16-byte load
    static constexpr int NT = 64 * WPB;                 // threads
    // 16-byte loads per chunk (X: 2 planes, P: 2 planes) and per thread
    static constexpr int XN = 2 * TGB * TGK / VPT, PN = 2 * TGI * TGK / VPT;
    static constexpr int XL = (XN + NT - 1) / NT, PL = (PN + NT - 1) / NT;
};

template <typename T>
struct TgMma;
template <>
struct TgMma<double> {
    typedef d4s acc;
    static __device__ inline acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    // -a b + c (negate-A modifier)
    static __device__ inline acc mma_na(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 1);
    }
    static __device__ inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct TgMma<float> {
    typedef f4v acc;
    static __device__ inline acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T, int WPB>
__global__ void __launch_bounds__(64 * WPB) tgemm_step_kernel(int n, int B, int Kp, int nbt, int nit,
                                                              const T *__restrict__ Xr, const T *__restrict__ Xi,
                                                              const T *__restrict__ Pr, const T *__restrict__ Pi,
                                                              T *__restrict__ Yr, T *__restrict__ Yi,
                                                              cd *__restrict__ Yout) {
    typedef TgShape<T, WPB> S;
    typedef typename TgMma<T>::acc acc_t;
    typedef T v4 __attribute__((ext_vector_type(4)));
    typedef T vl __attribute__((ext_vector_type(S::VPT)));  // one 16-byte load
    constexpr int KSPLIT = WPB / 4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);  // [2][BUF]
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wq = wave & 3, kh = wave >> 2;  // state rows; k half (WPB = 8)
    // XCD-contiguous tile numbering (bijective on [0, nbt * nit))
    const int total = nbt * nit, per = total / 8, rem = total % 8;
    const int xcd = blockIdx.x % 8, jx = blockIdx.x / 8;
    const int L = xcd * per + (xcd < rem ? xcd : rem) + jx;
    const int bt = L / nit, it = L - bt * nit;
    const int b0 = bt * TGB, i0 = it * TGI;

    // global -> register staging: load e covers 16 bytes of one row of one plane
    constexpr int RX = TGK / S::VPT;  // loads per row
    vl rx[S::XL], rp[S::PL];
    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < S::XL; ++q) {
            const int e = tid + S::NT * q;
            const int pl = e / (TGB * RX), rem2 = e - pl * TGB * RX, r = rem2 / RX, c = rem2 - r * RX;
            const int b = b0 + r;
            const bool ok = (S::XN % S::NT == 0 || e < S::XN) && b < B;
            const T *src = (pl == 0 ? Xr : Xi) + (size_t)(ok ? b : 0) * Kp + k0 + c * S::VPT;
            rx[q] = ok ? *reinterpret_cast<const vl *>(src) : vl{};
        }
#pragma unroll
        for (int q = 0; q < S::PL; ++q) {
            const int e = tid + S::NT * q;
            const int pl = e / (TGI * RX), rem2 = e - pl * TGI * RX, r = rem2 / RX, c = rem2 - r * RX;
            const int i = i0 + r;
            const bool ok = (S::PN % S::NT == 0 || e < S::PN) && i < n;
            const T *src = (pl == 0 ? Pr : Pi) + (size_t)(ok ? i : 0) * Kp + k0 + c * S::VPT;
            rp[q] = ok ? *reinterpret_cast<const vl *>(src) : vl{};
        }
    };
    auto lstore = [&](T *buf) {
#pragma unroll
        for (int q = 0; q < S::XL; ++q) {
            const int e = tid + S::NT * q;
            if (S::XN % S::NT != 0 && e >= S::XN) break;
            const int pl = e / (TGB * RX), rem2 = e - pl * TGB * RX, r = rem2 / RX, c = rem2 - r * RX;
            *reinterpret_cast<vl *>(buf + pl * S::XS + r * S::LD + c * S::VPT) = rx[q];
            if (S::XPL == 3 && pl == 1) *reinterpret_cast<vl *>(buf + 2 * S::XS + r * S::LD + c * S::VPT) = -rx[q];
        }
#pragma unroll
        for (int q = 0; q < S::PL; ++q) {
            const int e = tid + S::NT * q;
            if (S::PN % S::NT != 0 && e >= S::PN) break;
            const int pl = e / (TGI * RX), rem2 = e - pl * TGI * RX, r = rem2 / RX, c = rem2 - r * RX;
            *reinterpret_cast<vl *>(buf + S::XPL * S::XS + pl * S::PS + r * S::LD + c * S::VPT) = rp[q];
        }
    };

    acc_t re[3], im[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) re[t] = im[t] = acc_t{0, 0, 0, 0};
    const int nch = Kp / TGK;
    gload(0);
    lstore(lds);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const T *buf = lds + (c & 1) * S::BUF;
        if (c + 1 < nch) gload((c + 1) * TGK);
        const T *xr = buf + (16 * wq + (lane & 15)) * S::LD + 4 * (lane >> 4);
        const T *xi = xr + S::XS;
        const T *xn = xr + 2 * S::XS;  // FP32 only
        const T *pr = buf + S::XPL * S::XS + (lane & 15) * S::LD + 4 * (lane >> 4);
        const T *pi = pr + S::PS;
#pragma unroll
        for (int kq = 0; kq < TGK / 16 / KSPLIT; ++kq) {
            const int kb = 16 * (kq * KSPLIT + kh);
            const v4 ar = *reinterpret_cast<const v4 *>(xr + kb), ai = *reinterpret_cast<const v4 *>(xi + kb);
            v4 an;
            if (S::XPL == 3) an = *reinterpret_cast<const v4 *>(xn + kb);
            v4 br[3], bi[3];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                br[t] = *reinterpret_cast<const v4 *>(pr + 16 * t * S::LD + kb);
                bi[t] = *reinterpret_cast<const v4 *>(pi + 16 * t * S::LD + kb);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    re[t] = TgMma<T>::mma(ar[q], br[t][q], re[t]);
                    im[t] = TgMma<T>::mma(ar[q], bi[t][q], im[t]);
                }
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    if constexpr (sizeof(T) == 8)
                        re[t] = TgMma<T>::mma_na(ai[q], bi[t][q], re[t]);
                    else
                        re[t] = TgMma<T>::mma(an[q], bi[t][q], re[t]);
                    im[t] = TgMma<T>::mma(ai[q], br[t][q], im[t]);
                }
            }
        }
        if (c + 1 < nch) {
            lstore(lds + ((c + 1) & 1) * S::BUF);
            __syncthreads();
        }
    }
    if (KSPLIT == 2) {
        // the second k half adds its partial sums (fixed order: first + second)
        __syncthreads();  // every wavefront is done with the LDS operands
        T *red = lds;     // [4 wq][3 t][4 r][2][64]
        if (kh == 1) {
#pragma unroll
            for (int t = 0; t < 3; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    red[(((wq * 3 + t) * 4 + r) * 2 + 0) * 64 + lane] = re[t][r];
                    red[(((wq * 3 + t) * 4 + r) * 2 + 1) * 64 + lane] = im[t][r];
                }
        }
        __syncthreads();
        if (kh == 1) return;  // uniform per wavefront; no barrier follows
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                re[t][r] += red[(((wq * 3 + t) * 4 + r) * 2 + 0) * 64 + lane];
                im[t][r] += red[(((wq * 3 + t) * 4 + r) * 2 + 1) * 64 + lane];
            }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = b0 + 16 * wq + TgMma<T>::row(lane, r), i = i0 + 16 * t + (lane & 15);
            if (b < B && i < n) {
                Yr[(size_t)b * Kp + i] = re[t][r];
                Yi[(size_t)b * Kp + i] = im[t][r];
                if (Yout) Yout[(size_t)b * n + i] = {(double)re[t][r], (double)im[t][r]};
            }
        }
}

// ------------------------------------------------- per-state matvec in T
template <typename T>
struct Cx {
    T re, im;
};

// One wavefront per (state, row): lanes read the row of P (in T) and the
// state contiguously and reduce with cross-lane shuffles.
template <typename T>
__global__ void __launch_bounds__(256) matvec_step_kernel(int n, const Cx<T> *__restrict__ P,
                                                          const Cx<T> *__restrict__ X, Cx<T> *__restrict__ Y,
                                                          long long rows_total) {
    const int lane = threadIdx.x & 63;
    const long long nwaves = (long long)gridDim.x * (blockDim.x >> 6);
    for (long long w = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < rows_total; w += nwaves) {
        const long long b = w / n;
        const int i = (int)(w - b * n);
        const Cx<T> *Pi = P + (size_t)i * n;
        const Cx<T> *xb = X + (size_t)b * n;
        T re = 0, im = 0;
        for (int j = lane; j < n; j += 64) {
            const Cx<T> p = Pi[j], v = xb[j];
            re = fma(p.re, v.re, fma(-p.im, v.im, re));
            im = fma(p.re, v.im, fma(p.im, v.re, im));
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            re += __shfl_xor(re, off);
            im += __shfl_xor(im, off);
        }
        if (lane == 0) Y[(size_t)b * n + i] = {re, im};
    }
}

template <typename T>
__global__ void convert_kernel(long long count, const cd *__restrict__ src, Cx<T> *__restrict__ dst) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (long long)gridDim.x * blockDim.x)
        dst[e] = {(T)src[e].re, (T)src[e].im};
}

template <typename T>
__global__ void back_kernel(long long count, const Cx<T> *__restrict__ src, cd *__restrict__ dst) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (long long)gridDim.x * blockDim.x)
        dst[e] = {(double)src[e].re, (double)src[e].im};
}

static int grid1(long long work) {
    long long g = (work + 255) / 256;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace lg

using namespace lg;

template <typename T>
static int matvec_run(int n, const cd *P, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s,
                      bool graph) {
    const size_t nn = (size_t)n * n;
    LB_TRY(ws_ensure(ws, align256(nn * sizeof(Cx<T>)) + 2 * align256((size_t)B * n * sizeof(Cx<T>))));
    Cx<T> *Pc = (Cx<T> *)ws_take(ws, nn * sizeof(Cx<T>));
    Cx<T> *X0 = (Cx<T> *)ws_take(ws, (size_t)B * n * sizeof(Cx<T>));
    Cx<T> *X1 = (Cx<T> *)ws_take(ws, (size_t)B * n * sizeof(Cx<T>));
    convert_kernel<T><<<grid1(nn), 256, 0, s>>>((long long)nn, P, Pc);
    convert_kernel<T><<<grid1((long long)B * n), 256, 0, s>>>((long long)B * n, rho, X0);
    const long long rows = (long long)B * n;
    long long blocks = (rows + 3) / 4;
    if (blocks > 16384) blocks = 16384;
    LB_TRY(run_steps(nsteps, graph, [&](long long t, hipStream_t st) {
        matvec_step_kernel<T><<<(int)blocks, 256, 0, st>>>(n, Pc, (t & 1) ? X1 : X0, (t & 1) ? X0 : X1, rows);
        return LB_OK;
    }, s));
    LB_TRY(check_launch("matvec_step"));
    back_kernel<T><<<grid1((long long)B * n), 256, 0, s>>>((long long)B * n, (nsteps & 1) ? X1 : X0, rho);
    return check_launch("matvec_back");
}

template <typename T, int GWN>
static int gemm_run(int n, const cd *P, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s,
                    bool graph) {
    const int Kp = (n + 63) / 64 * 64;
    const size_t pp = (size_t)n * Kp * sizeof(T), xp = (size_t)B * Kp * sizeof(T);
    LB_TRY(ws_ensure(ws, 2 * align256(pp) + 4 * align256(xp)));
    T *Pr = (T *)ws_take(ws, pp), *Pi = (T *)ws_take(ws, pp);
    T *X[2][2];
    for (int q = 0; q < 2; ++q)
        for (int c = 0; c < 2; ++c) X[q][c] = (T *)ws_take(ws, xp);
    to_planes_kernel<T><<<grid1((long long)n * Kp), 256, 0, s>>>(n, n, Kp, P, Pr, Pi);
    for (int q = 0; q < 2; ++q)  // zero k padding of both buffers
        to_planes_kernel<T><<<grid1((long long)B * Kp), 256, 0, s>>>(B, n, Kp, rho, X[q][0], X[q][1]);
    LB_TRY(check_launch("to_planes"));
    dim3 grid((n + 16 * GWN - 1) / (16 * GWN), (B + TS - 1) / TS);
    LB_TRY(run_steps(nsteps, graph, [&](long long t, hipStream_t st) {
        const int c = (int)(t & 1);
        gemm_step_kernel<T, GWN><<<grid, 256, 0, st>>>(n, B, Kp, X[c][0], X[c][1], Pr, Pi, X[c ^ 1][0], X[c ^ 1][1],
                                                       t + 1 == nsteps ? rho : nullptr);
        return LB_OK;
    }, s));
    return check_launch("gemm_step");
}

// Ring-pipelined FP32 / FP64 GEMM step: the tile of tgemm_step_kernel (64
// states x 48 outputs; wavefront w owns states 16 w .. + 15 against all 48
// outputs over every k) with k in 16-deep chunks that reach LDS by direct
// global-to-LDS loads into a ring of R slots, R - 1 chunks ahead, instead of
// through registers: no staging registers, no store phase, and at each
// chunk's barrier a wavefront waits only for its own loads of that chunk
// (the count of later loads is a constant: every chunk issues the same loads,
// past the last one repeating valid addresses into slots no later chunk
// reads).  Plane rows (16 k = 64 or 128 bytes) keep their 16-byte pieces at
// XOR-swizzled positions (tr_swz) so that an MFMA operand fetch runs without
// bank conflicts and without padding.  -Im X Im P uses the FP64 negate-A
// modifier, a sign flip in registers for FP32.
constexpr int TRK = 16;  // k per ring chunk

template <typename T>
struct TrShape {
    static constexpr int RB = TRK * (int)sizeof(T);  // bytes per plane row of a chunk
    static constexpr int NPC = RB / 16;              // 16-byte pieces per row
    static constexpr int RPL = 1024 / RB;            // rows per 1 KB load
    static constexpr int XPB = TGB * RB, PPB = TGI * RB;
    static constexpr int BUF = 2 * XPB + 2 * PPB;    // slot: Re X, Im X, Re P, Im P
    static constexpr int XI = XPB / 1024, PI = PPB / 1024;
    static constexpr int NI = BUF / 1024;            // 1 KB loads per chunk
    static constexpr int NJ = (NI + 3) / 4;          // per wavefront (the last few repeat others)
    static constexpr int R = kLdsBytes / BUF > 6 ? 6 : kLdsBytes / BUF;
    static constexpr int LDS = R * BUF;
    // at the wait for chunk c + 1 the loads of chunks c + 2 .. c + R - 1 stay
    // in flight (chunk c + R is issued after it); before the first chunk
    // those of chunks 1 .. R - 1
    static constexpr int WAIT = (R - 2) * NJ, WAIT0 = (R - 1) * NJ;
    static_assert(BUF % 1024 == 0 && R >= 3 && WAIT0 <= 63, "ring GEMM shape");
};
// position of a row's 16-byte piece: piece ^ f(row).  FP32 rows are 64
// bytes with the operand fetch of tp_swz, and take its conflict-free f.  FP64
// rows are 128 bytes and a lane fetches pieces 2 g and 2 g + 1 (g = lane /
// 16) of row lane % 16 in two reads; f = row bit 1 into piece bit 0 and row
// bit 2 into piece bit 2 is one of the maps gfx950's bank-conflict counter
// reads as conflict-free for both reads (XOR with (row >> 1) & 7 reads as
// two-way).
template <typename T>
__device__ inline int tr_swz(int row, int piece) {
    return sizeof(T) == 8 ? piece ^ (((row >> 1) & 1) | (row & 4)) : piece ^ ((row >> 1) & 3);
}

// Split k (ksplit > 1): workgroup L = ks * tiles + tile takes chunks
// [ks cper, (ks + 1) cper) and writes its partial sums (FP64) to Ypart[ks];
// tr_split_sum_kernel adds them in order and writes the next state.
template <typename T>
__global__ void __launch_bounds__(256) trgemm_step_kernel(int n, int B, int Kp, int nbt, int nit,
                                                          const T *__restrict__ Xr, const T *__restrict__ Xi,
                                                          const T *__restrict__ Pr, const T *__restrict__ Pi,
                                                          T *__restrict__ Yr, T *__restrict__ Yi,
                                                          cd *__restrict__ Yout, int ksplit, int cper,
                                                          cd *__restrict__ Ypart) {
    typedef TrShape<T> S;
    typedef typename TgMma<T>::acc acc_t;
    typedef T v4 __attribute__((ext_vector_type(4)));
    typedef T vh __attribute__((ext_vector_type(16 / sizeof(T))));  // one 16-byte piece
    constexpr int R = S::R, NJ = S::NJ, VP = 16 / (int)sizeof(T);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tiles = nbt * nit, total = tiles * ksplit, per = total / 8, rem = total % 8;
    const int xcd = blockIdx.x % 8, jx = blockIdx.x / 8;
    const int L = xcd * per + (xcd < rem ? xcd : rem) + jx;
    const int ks = L / tiles, L0 = L - ks * tiles;
    const int bt = L0 / nit, it = L0 - bt * nit;
    const int b0 = bt * TGB, i0 = it * TGI;
    // this workgroup's chunks: kc0 .. kc0 + nch - 1
    const int kc0 = ks * cper, nall = Kp / TRK;
    const int nch = nall - kc0 < cper ? nall - kc0 : cper;

    // load j = wave + 4 q of a chunk: plane tile (Re X, Im X, Re P, Im P),
    // its 1 KB part jj; lane l fills row RPL jj + l / NPC, position l % NPC,
    // which holds the row's piece tr_swz(row, position)
    const T *srcp[NJ];
    int dsto[NJ];
#pragma unroll
    for (int q = 0; q < NJ; ++q) {
        int j = wave + 4 * q;
        j = j < S::NI ? j : j - (4 * NJ - S::NI);
        int pl, jj;
        if (j < 2 * S::XI) pl = j / S::XI, jj = j - pl * S::XI;
        else pl = 2 + (j - 2 * S::XI) / S::PI, jj = (j - 2 * S::XI) - (pl - 2) * S::PI;
        const int row = S::RPL * jj + lane / S::NPC, pos = lane % S::NPC;
        const int piece = tr_swz<T>(row, pos);
        if (pl < 2) {
            int b = b0 + row;
            b = b < B ? b : B - 1;
            srcp[q] = (pl == 0 ? Xr : Xi) + (size_t)b * Kp + piece * VP;
            dsto[q] = pl * S::XPB + 1024 * jj;
        } else {
            int i = i0 + row;
            i = i < n ? i : n - 1;
            srcp[q] = (pl == 2 ? Pr : Pi) + (size_t)i * Kp + piece * VP;
            dsto[q] = 2 * S::XPB + (pl - 2) * S::PPB + 1024 * jj;
        }
    }
    auto dma = [&](int c, int q) {  // load q of chunk c (from kc0) into slot c % R (past the end: the last chunk)
        const int k0 = (kc0 + (c < nch ? c : nch - 1)) * TRK;
        __builtin_amdgcn_global_load_lds((const void *)(srcp[q] + k0),
                                         (__attribute__((address_space(3))) void *)(smem_raw + (c % R) * S::BUF +
                                                                                    dsto[q]),
                                         16, 0, 0);
    };
    // MFMA operands: row lane % 16 of a 16-row block, k = 4 (lane / 16) .. + 3
    const int orow = lane & 15, g = lane >> 4;
    auto opnd = [&](const unsigned char *plane, int row) -> v4 {
        const unsigned char *rp = plane + row * S::RB;
        if constexpr (sizeof(T) == 8) {
            const vh lo = *reinterpret_cast<const vh *>(rp + 16 * tr_swz<T>(row, 2 * g));
            const vh hi = *reinterpret_cast<const vh *>(rp + 16 * tr_swz<T>(row, 2 * g + 1));
            return v4{lo[0], lo[1], hi[0], hi[1]};
        } else {
            return *reinterpret_cast<const v4 *>(rp + 16 * tr_swz<T>(row, g));
        }
    };

    acc_t re[3], im[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) re[t] = im[t] = acc_t{0, 0, 0, 0};
    // The operands of chunk c + 1 are read into registers before chunk c's
    // MFMAs are issued, so the LDS latency hides behind them; the barrier
    // before those reads also tells every wavefront that chunk c's slot,
    // already in registers everywhere, may take chunk c + R.
    struct Ops {
        v4 ar, ai, br[3], bi[3];
    };
    auto readops = [&](int c, Ops &o) {
        const unsigned char *buf = smem_raw + (c % R) * S::BUF;
        o.ar = opnd(buf, 16 * wave + orow);
        o.ai = opnd(buf + S::XPB, 16 * wave + orow);
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            o.br[t] = opnd(buf + 2 * S::XPB, 16 * t + orow);
            o.bi[t] = opnd(buf + 2 * S::XPB + S::PPB, 16 * t + orow);
        }
    };
    // the chunk's MFMAs, with chunk cd's loads spread between them (cd < 0: none)
    auto mmas = [&](const Ops &o, int cd) {
        v4 an;
        if constexpr (sizeof(T) == 4) an = -o.ai;
        int grp = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int t = 0; t < 3; ++t, ++grp) {
#pragma unroll
                for (int k = 0; k < NJ; ++k)
                    if (cd >= 0 && k * 12 >= grp * NJ && k * 12 < (grp + 1) * NJ) dma(cd, k);
                re[t] = TgMma<T>::mma(o.ar[q], o.br[t][q], re[t]);
                im[t] = TgMma<T>::mma(o.ar[q], o.bi[t][q], im[t]);
                if constexpr (sizeof(T) == 8)
                    re[t] = TgMma<T>::mma_na(o.ai[q], o.bi[t][q], re[t]);
                else
                    re[t] = TgMma<T>::mma(an[q], o.bi[t][q], re[t]);
                im[t] = TgMma<T>::mma(o.ai[q], o.br[t][q], im[t]);
            }
    };
    // prologue: chunks 0 .. R - 1, one per slot
#pragma unroll
    for (int c = 0; c < R; ++c)
#pragma unroll
        for (int q = 0; q < NJ; ++q) dma(c, q);
    TQ_SYNC(S::WAIT0);
    Ops oa, ob;
    readops(0, oa);
    // step(c, cur, nxt): chunk c + 1 has landed and chunk c is in every
    // wavefront's registers: read chunk c + 1, then chunk c's MFMAs with
    // chunk c + R's loads into chunk c's slot.  Two steps per iteration so
    // that the operand sets alternate without copies.
    auto step = [&](int c, const Ops &cur, Ops &nxt) {
        TQ_SYNC(S::WAIT);
        readops(c + 1, nxt);
        mmas(cur, c + R);
    };
    int c = 0;
    for (; c + 2 < nch; c += 2) {
        step(c, oa, ob);
        step(c + 1, ob, oa);
    }
    if (c + 1 < nch) {  // two chunks left: c in oa
        step(c, oa, ob);
        mmas(ob, -1);
    } else {  // one chunk left
        mmas(oa, -1);
    }
    __builtin_amdgcn_s_waitcnt(0);  // the loads past the last chunk land before the workgroup ends
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = b0 + 16 * wave + TgMma<T>::row(lane, r), i = i0 + 16 * t + (lane & 15);
            if (b < B && i < n) {
                if (ksplit > 1) {
                    Ypart[((size_t)ks * B + b) * n + i] = {(double)re[t][r], (double)im[t][r]};
                } else {
                    Yr[(size_t)b * Kp + i] = re[t][r];
                    Yi[(size_t)b * Kp + i] = im[t][r];
                    if (Yout) Yout[(size_t)b * n + i] = {(double)re[t][r], (double)im[t][r]};
                }
            }
        }
}

// the next state from the split-k partials: sum over ks in order (FP64),
// rounded to T into the planes, and on the last step the complex128 result
template <typename T>
__global__ void tr_split_sum_kernel(int n, int B, int Kp, int ksplit, const cd *__restrict__ Ypart,
                                    T *__restrict__ Yr, T *__restrict__ Yi, cd *__restrict__ Yout) {
    const long long total = (long long)B * n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k < ksplit; ++k) {
            const cd v = Ypart[(size_t)k * total + e];
            re += v.re;
            im += v.im;
        }
        const long long b = e / n, i = e - b * n;
        const T tr = (T)re, ti = (T)im;
        Yr[b * Kp + i] = tr;
        Yi[b * Kp + i] = ti;
        if (Yout) Yout[e] = {(double)tr, (double)ti};
    }
}

// split of the k range (16-deep chunks) for the ring GEMM: about 256
// workgroups; returns ksplit, sets the chunks per split
static int tr_split(int tiles, int Kp, int *cper) {
    const int nch = Kp / TRK;
    int ks = tiles >= 256 ? 1 : (256 + tiles - 1) / tiles;
    ks = ks < nch ? ks : nch;
    const int cp = (nch + ks - 1) / ks;
    *cper = cp;
    return (nch + cp - 1) / cp;
}

template <typename T>
static int trgemm_run(int n, const cd *P, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s,
                      bool graph, bool split) {
    typedef TrShape<T> S;
    const int Kp = (n + 63) / 64 * 64;
    const int nbt = (B + TGB - 1) / TGB, nit = (n + TGI - 1) / TGI;
    int cper = Kp / TRK;
    const int ksplit = split ? tr_split(nbt * nit, Kp, &cper) : 1;
    const size_t pp = (size_t)n * Kp * sizeof(T), xp = (size_t)B * Kp * sizeof(T);
    const size_t partb = ksplit > 1 ? (size_t)ksplit * B * n * sizeof(cd) : 0;
    LB_TRY(ws_ensure(ws, 2 * align256(pp) + 4 * align256(xp) + align256(partb)));
    T *Pr = (T *)ws_take(ws, pp), *Pi = (T *)ws_take(ws, pp);
    T *X[2][2];
    for (int q = 0; q < 2; ++q)
        for (int c = 0; c < 2; ++c) X[q][c] = (T *)ws_take(ws, xp);
    cd *Ypart = ksplit > 1 ? (cd *)ws_take(ws, partb) : nullptr;
    to_planes_kernel<T><<<grid1((long long)n * Kp), 256, 0, s>>>(n, n, Kp, P, Pr, Pi);
    for (int q = 0; q < 2; ++q)  // zero k padding of both buffers
        to_planes_kernel<T><<<grid1((long long)B * Kp), 256, 0, s>>>(B, n, Kp, rho, X[q][0], X[q][1]);
    LB_TRY(check_launch("to_planes"));
    LB_TRY(set_max_lds((const void *)trgemm_step_kernel<T>, S::LDS));
    LB_TRY(run_steps(nsteps, graph, [&](long long t, hipStream_t st) {
        const int c = (int)(t & 1);
        cd *out = t + 1 == nsteps ? rho : nullptr;
        trgemm_step_kernel<T><<<nbt * nit * ksplit, 256, S::LDS, st>>>(n, B, Kp, nbt, nit, X[c][0], X[c][1], Pr, Pi,
                                                                       X[c ^ 1][0], X[c ^ 1][1], out, ksplit, cper,
                                                                       Ypart);
        if (ksplit > 1)
            tr_split_sum_kernel<T><<<grid1((long long)B * n), 256, 0, st>>>(n, B, Kp, ksplit, Ypart, X[c ^ 1][0],
                                                                            X[c ^ 1][1], out);
        return LB_OK;
    }, s));
    return check_launch("trgemm_step");
}

template <typename T, int WPB>
static int tgemm_run(int n, const cd *P, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s,
                     bool graph) {
    typedef TgShape<T, WPB> S;
    const int Kp = (n + 63) / 64 * 64;
    const size_t pp = (size_t)n * Kp * sizeof(T), xp = (size_t)B * Kp * sizeof(T);
    LB_TRY(ws_ensure(ws, 2 * align256(pp) + 4 * align256(xp)));
    T *Pr = (T *)ws_take(ws, pp), *Pi = (T *)ws_take(ws, pp);
    T *X[2][2];
    for (int q = 0; q < 2; ++q)
        for (int c = 0; c < 2; ++c) X[q][c] = (T *)ws_take(ws, xp);
    to_planes_kernel<T><<<grid1((long long)n * Kp), 256, 0, s>>>(n, n, Kp, P, Pr, Pi);
    for (int q = 0; q < 2; ++q)  // zero k padding of both buffers
        to_planes_kernel<T><<<grid1((long long)B * Kp), 256, 0, s>>>(B, n, Kp, rho, X[q][0], X[q][1]);
    LB_TRY(check_launch("to_planes"));
    const size_t lds = 2 * (size_t)S::BUF * sizeof(T);
    LB_TRY(set_max_lds((const void *)tgemm_step_kernel<T, WPB>, lds));
    const int nbt = (B + TGB - 1) / TGB, nit = (n + TGI - 1) / TGI;
    LB_TRY(run_steps(nsteps, graph, [&](long long t, hipStream_t st) {
        const int c = (int)(t & 1);
        tgemm_step_kernel<T, WPB><<<nbt * nit, 64 * WPB, lds, st>>>(n, B, Kp, nbt, nit, X[c][0], X[c][1], Pr, Pi,
                                                                    X[c ^ 1][0], X[c ^ 1][1],
                                                                    t + 1 == nsteps ? rho : nullptr);
        return LB_OK;
    }, s));
    return check_launch("tgemm_step");
}

template <int MODE, int SP, int SX, int LMAX>
// tiled: 0 = untiled plane GEMM, 1 = LDS-tiled (state and propagator planes in
// LDS), 2 = ring-pipelined (per-wavefront state staging, propagator ring),
// 3 = ring-pipelined with the k range split over workgroups (small batches)
static int planes_run(int n, const cd *P, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s,
                      bool graph, int tiled) {
    constexpr int XD = Planes<MODE, SP, SX>::XD, PD = Planes<MODE, SP, SX>::PD;
    const int kq = tiled >= 2 ? TQK : KCH;
    const int Kp = (n + kq - 1) / kq * kq;
    const size_t pbytes = (size_t)PD * 2 * n * Kp * 2, xbytes = (size_t)XD * 3 * B * Kp * 2;
    const size_t ybytes = (size_t)B * n * sizeof(cd);
    const int nbt = (B + TPB - 1) / TPB, nit = (n + TPI - 1) / TPI;
    int cper = Kp / TPK;
    const int ksplit = tiled == 3 ? tq_split(nbt * nit, Kp, &cper) : 1;
    const size_t pbytes_part = ksplit > 1 ? (size_t)ksplit * ybytes : 0;
    LB_TRY(ws_ensure(ws, align256(pbytes) + align256(xbytes) + align256(ybytes) + align256(n * 4) + align256(B * 4) +
                             align256(pbytes_part)));
    unsigned short *Pp = (unsigned short *)ws_take(ws, pbytes);
    unsigned short *Xp = (unsigned short *)ws_take(ws, xbytes);
    cd *Yt = (cd *)ws_take(ws, ybytes);
    int *eP = (int *)ws_take(ws, n * 4);
    int *eX = (int *)ws_take(ws, B * 4);
    cd *Ypart = ksplit > 1 ? (cd *)ws_take(ws, pbytes_part) : nullptr;
    prep_p_kernel<MODE, SP, SX><<<n, 256, 0, s>>>(n, Kp, P, Pp, eP);
    LB_TRY(check_launch("prep_p"));
    dim3 grid((n + TO - 1) / TO, (B + TS - 1) / TS);
    const size_t lds = tiled >= 2 ? (size_t)TqShape<MODE, SP, SX>::LDS : 2 * (size_t)TpShape<MODE, SP, SX>::BUF;
    if (tiled == 1) {
        LB_TRY(set_max_lds((const void *)tplane_gemm_kernel<MODE, SP, SX, LMAX>, lds));
    } else if (tiled >= 2) {
        LB_TRY(set_max_lds((const void *)tqplane_gemm_kernel<MODE, SP, SX, LMAX>, lds));
    }
    // the state ping-pongs between rho and Yt
    LB_TRY(run_steps(nsteps, graph, [&](long long t, hipStream_t st) {
        cd *cur = (t & 1) ? Yt : rho, *nxt = (t & 1) ? rho : Yt;
        if (tiled >= 2)
            slice_x_kernel<MODE, SP, SX, false><<<B, 256, 0, st>>>(n, Kp, B, cur, Xp, eX);
        else
            slice_x_kernel<MODE, SP, SX, true><<<B, 256, 0, st>>>(n, Kp, B, cur, Xp, eX);
        if (tiled == 1)
            tplane_gemm_kernel<MODE, SP, SX, LMAX><<<nbt * nit, 256, lds, st>>>(n, B, Kp, nbt, nit, Xp, Pp, eP, eX,
                                                                                nxt);
        else if (tiled >= 2) {
            // with the k range split, the partial sums are added in order into nxt
            tqplane_gemm_kernel<MODE, SP, SX, LMAX><<<nbt * nit * ksplit, 256, lds, st>>>(
                n, B, Kp, nbt, nit, Xp, Pp, eP, eX, nxt, ksplit, cper, Ypart);
            if (ksplit > 1)
                split_sum_kernel<MODE><<<grid1((long long)B * n), 256, 0, st>>>((long long)B * n, ksplit, Ypart, nxt);
        } else
            plane_gemm_kernel<MODE, SP, SX, LMAX><<<grid, 256, 0, st>>>(n, B, Kp, Xp, Pp, eP, eX, nxt);
        return LB_OK;
    }, s));
    LB_TRY(check_launch("plane_gemm"));
    if (nsteps & 1) LB_HIP(hipMemcpyAsync(rho, Yt, ybytes, hipMemcpyDeviceToDevice, s));
    return LB_OK;
}

// ------------------------------------------------ action of the exponential
// One Taylor term of e^{tL} v with shift mu: V <- alpha (Y - mu V) (Y = L V
// from the step GEMM), F <- F + V.  Planes [B][Kp]; padding columns stay zero.
__global__ void __launch_bounds__(256) expmv_term_kernel(int n, int B, int Kp, const double *__restrict__ Yr,
                                                         const double *__restrict__ Yi, double *__restrict__ Vr,
                                                         double *__restrict__ Vi, double *__restrict__ Fr,
                                                         double *__restrict__ Fi, double alpha, double mur,
                                                         double mui) {
    const long long total = (long long)B * n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long b = e / n, i = e - b * n, o = b * Kp + i;
        const double vr = Vr[o], vi = Vi[o];
        const double tr = alpha * (Yr[o] - (mur * vr - mui * vi));
        const double ti = alpha * (Yi[o] - (mur * vi + mui * vr));
        Vr[o] = tr;
        Vi[o] = ti;
        Fr[o] += tr;
        Fi[o] += ti;
    }
}

// End of a sub-step: F <- eta F; V <- F (the next sub-step starts from it);
// on the last sub-step of the last step F goes to rho (complex128).
__global__ void __launch_bounds__(256) expmv_rescale_kernel(int n, int B, int Kp, double *__restrict__ Fr,
                                                            double *__restrict__ Fi, double *__restrict__ Vr,
                                                            double *__restrict__ Vi, double er, double ei,
                                                            cd *__restrict__ out) {
    const long long total = (long long)B * n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long b = e / n, i = e - b * n, o = b * Kp + i;
        const double fr = Fr[o], fi = Fi[o];
        const double gr = er * fr - ei * fi, gi = er * fi + ei * fr;
        Fr[o] = gr;
        Fi[o] = gi;
        Vr[o] = gr;
        Vi[o] = gi;
        if (out) out[e] = {gr, gi};
    }
}

// Small batches: one wavefront per (state, row) forms (L v)_i with lanes
// along the row (coalesced reads of L, fixed-order shuffle reduction) and
// applies the term update in its epilogue: one launch per product.
__global__ void __launch_bounds__(256) expmv_matvec_kernel(int n, const cd *__restrict__ L, const cd *__restrict__ V,
                                                           cd *__restrict__ Vn, cd *__restrict__ F,
                                                           long long rows_total, double alpha, double mur,
                                                           double mui) {
    const int lane = threadIdx.x & 63;
    const long long nwaves = (long long)gridDim.x * (blockDim.x >> 6);
    for (long long w = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < rows_total; w += nwaves) {
        const long long b = w / n;
        const int i = (int)(w - b * n);
        const cd *Li = L + (size_t)i * n;
        const cd *vb = V + (size_t)b * n;
        double re = 0.0, im = 0.0;
        for (int k = lane; k < n; k += 64) {
            const cd a = Li[k], v = vb[k];
            re = fma(a.re, v.re, fma(-a.im, v.im, re));
            im = fma(a.re, v.im, fma(a.im, v.re, im));
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            re += __shfl_xor(re, off);
            im += __shfl_xor(im, off);
        }
        if (lane == 0) {
            const size_t o = (size_t)b * n + i;
            const cd v = vb[i];
            const double tr = alpha * (re - (mur * v.re - mui * v.im));
            const double ti = alpha * (im - (mur * v.im + mui * v.re));
            Vn[o] = {tr, ti};
            F[o] = {F[o].re + tr, F[o].im + ti};
        }
    }
}

__global__ void __launch_bounds__(256) expmv_rescale_c_kernel(long long count, cd *__restrict__ F, cd *__restrict__ V,
                                                              double er, double ei, cd *__restrict__ out) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (long long)gridDim.x * blockDim.x) {
        const cd f = F[e];
        const cd g = {er * f.re - ei * f.im, er * f.im + ei * f.re};
        F[e] = g;
        V[e] = g;
        if (out) out[e] = g;
    }
}

constexpr int kExpmvSmallB = 8;  // up to this many states: the per-row matvec path

// rho_b <- (e^{tL})^nsteps rho_b by s sub-steps of the m-term Taylor series
// of t (L - mu I) / s, each sub-step scaled by eta = e^{t mu / s}.  The
// products L V are the FP64 step GEMMs of the chain (the LDS-tiled one when
// its tiles fill the chip).
int expmv_run(int n, const cd *L, double t, double mur, double mui, int s, int m, int B, cd *rho, long long nsteps,
              Workspace *ws, hipStream_t st) {
    if (nsteps == 0 || B == 0) return LB_OK;
    const std::complex<double> eta = std::exp(std::complex<double>(t * mur / s, t * mui / s));
    if (B <= kExpmvSmallB) {
        const size_t xb = (size_t)B * n * sizeof(cd);
        LB_TRY(ws_ensure(ws, 3 * align256(xb)));
        cd *F = (cd *)ws_take(ws, xb), *V[2] = {(cd *)ws_take(ws, xb), (cd *)ws_take(ws, xb)};
        LB_HIP(hipMemcpyAsync(F, rho, xb, hipMemcpyDeviceToDevice, st));
        LB_HIP(hipMemcpyAsync(V[0], rho, xb, hipMemcpyDeviceToDevice, st));
        const long long rows = (long long)B * n;
        const int blocks = (int)((rows + 3) / 4);
        for (long long step = 0; step < nsteps; ++step) {
            for (int q = 0; q < s; ++q) {
                for (int j = 1; j <= m; ++j)
                    expmv_matvec_kernel<<<blocks, 256, 0, st>>>(n, L, V[(j - 1) & 1], V[j & 1], F, rows,
                                                                t / ((double)s * j), mur, mui);
                const bool last = step + 1 == nsteps && q + 1 == s;
                expmv_rescale_c_kernel<<<grid1(rows), 256, 0, st>>>(rows, F, V[0], eta.real(), eta.imag(),
                                                                    last ? rho : nullptr);
            }
            LB_TRY(check_launch("expmv_step"));
        }
        return LB_OK;
    }
    const int Kp = (n + 63) / 64 * 64;
    const size_t pp = (size_t)n * Kp * sizeof(double), xp = (size_t)B * Kp * sizeof(double);
    LB_TRY(ws_ensure(ws, 2 * align256(pp) + 6 * align256(xp)));
    double *Lr = (double *)ws_take(ws, pp), *Li = (double *)ws_take(ws, pp);
    double *Vr = (double *)ws_take(ws, xp), *Vi = (double *)ws_take(ws, xp);
    double *Yr = (double *)ws_take(ws, xp), *Yi = (double *)ws_take(ws, xp);
    double *Fr = (double *)ws_take(ws, xp), *Fi = (double *)ws_take(ws, xp);
    to_planes_kernel<double><<<grid1((long long)n * Kp), 256, 0, st>>>(n, n, Kp, L, Lr, Li);
    to_planes_kernel<double><<<grid1((long long)B * Kp), 256, 0, st>>>(B, n, Kp, rho, Vr, Vi);
    to_planes_kernel<double><<<grid1((long long)B * Kp), 256, 0, st>>>(B, n, Kp, rho, Fr, Fi);
    // Y: zero padding columns (its other entries are written by every product)
    to_planes_kernel<double><<<grid1((long long)B * Kp), 256, 0, st>>>(B, n, Kp, rho, Yr, Yi);
    LB_TRY(check_launch("expmv_planes"));
    typedef TgShape<double, 8> S;
    const bool tiled = (long long)((B + TGB - 1) / TGB) * ((n + TGI - 1) / TGI) >= 240;
    const size_t lds = 2 * (size_t)S::BUF * sizeof(double);
    if (tiled) {
        LB_TRY(set_max_lds((const void *)tgemm_step_kernel<double, 8>, lds));
    }
    const int nbt = (B + TGB - 1) / TGB, nit = (n + TGI - 1) / TGI;
    dim3 grid((n + 15) / 16, (B + TS - 1) / TS);
    const int eg = grid1((long long)B * n);
    for (long long step = 0; step < nsteps; ++step) {
        for (int q = 0; q < s; ++q) {
            for (int j = 1; j <= m; ++j) {
                if (tiled)
                    tgemm_step_kernel<double, 8><<<nbt * nit, 512, lds, st>>>(n, B, Kp, nbt, nit, Vr, Vi, Lr, Li, Yr,
                                                                            Yi, nullptr);
                else
                    gemm_step_kernel<double, 1><<<grid, 256, 0, st>>>(n, B, Kp, Vr, Vi, Lr, Li, Yr, Yi, nullptr);
                expmv_term_kernel<<<eg, 256, 0, st>>>(n, B, Kp, Yr, Yi, Vr, Vi, Fr, Fi, t / ((double)s * j), mur, mui);
            }
            const bool last = step + 1 == nsteps && q + 1 == s;
            expmv_rescale_kernel<<<eg, 256, 0, st>>>(n, B, Kp, Fr, Fi, Vr, Vi, eta.real(), eta.imag(),
                                                     last ? rho : nullptr);
        }
        LB_TRY(check_launch("expmv_step"));
    }
    return LB_OK;
}

size_t expmv_ws_bytes(int n, int B) {
    const size_t Kp = (size_t)(n + 63) / 64 * 64;
    return 2 * align256(n * Kp * sizeof(double)) + 6 * align256((size_t)B * Kp * sizeof(double));
}

int chain_matvec(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, Workspace *ws,
                 hipStream_t s, bool graph) {
    if (nsteps == 0 || B == 0) return LB_OK;
    if (prec != LB_C64) return fail(LB_ENOTSUP, "matvec chain: complex64 only (complex128 is the baseline)");
    return matvec_run<float>(n, P, B, rho, nsteps, ws, s, graph);
}

int chain_gemm(int n, const cd *P, lb_precision prec, int wn, int B, cd *rho, long long nsteps, Workspace *ws,
               hipStream_t s, bool graph) {
    if (nsteps == 0 || B == 0) return LB_OK;
    if (wn != 1 && wn != 2) return fail(LB_ESHAPE, "gemm chain: 1 or 2 output tiles per wavefront");
    switch (prec) {
        case LB_C128:
            return wn == 1 ? gemm_run<double, 1>(n, P, B, rho, nsteps, ws, s, graph)
                           : gemm_run<double, 2>(n, P, B, rho, nsteps, ws, s, graph);
        case LB_C64:
            return wn == 1 ? gemm_run<float, 1>(n, P, B, rho, nsteps, ws, s, graph)
                           : gemm_run<float, 2>(n, P, B, rho, nsteps, ws, s, graph);
        default: return fail(LB_ENOTSUP, "gemm chain: complex128 / complex64 only");
    }
}

int chain_tgemm(int n, const cd *P, lb_precision prec, int waves, int B, cd *rho, long long nsteps, Workspace *ws,
                hipStream_t s, bool graph) {
    if (nsteps == 0 || B == 0) return LB_OK;
    if (waves < 1 || (waves > 2 && waves != 4 && waves != 8))
        return fail(LB_ESHAPE, "tiled gemm chain: 4 or 8 wavefronts, 1 (ring) or 2 (ring, split k)");
    switch (prec) {
        case LB_C128:
            if (waves <= 2) return trgemm_run<double>(n, P, B, rho, nsteps, ws, s, graph, waves == 2);
            return waves == 4 ? tgemm_run<double, 4>(n, P, B, rho, nsteps, ws, s, graph)
                              : tgemm_run<double, 8>(n, P, B, rho, nsteps, ws, s, graph);
        case LB_C64:
            if (waves <= 2) return trgemm_run<float>(n, P, B, rho, nsteps, ws, s, graph, waves == 2);
            return waves == 4 ? tgemm_run<float, 4>(n, P, B, rho, nsteps, ws, s, graph)
                              : tgemm_run<float, 8>(n, P, B, rho, nsteps, ws, s, graph);
        default: return fail(LB_ENOTSUP, "tiled gemm chain: complex128 / complex64 only");
    }
}

int chain_planes(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, Workspace *ws,
                 hipStream_t s, bool graph, int tiled) {
    if (nsteps == 0 || B == 0) return LB_OK;
    switch (prec) {
        case LB_BF16_HILO: return planes_run<HILO, 2, 2, 1>(n, P, B, rho, nsteps, ws, s, graph, tiled);
        case LB_BF16_SLICED:
            return planes_run<SLICED, 5, 4, 4>(n, P, B, rho, nsteps, ws, s, graph, tiled);
        default: return fail(LB_ENOTSUP, "plane chain: BF16 precisions only");
    }
}

size_t large_ws_bytes(int family, int n, lb_precision prec, int B) {
    const size_t tsz = prec == LB_C128 ? 8 : 4;
    if (family == VF_MATVEC) return align256((size_t)n * n * 2 * tsz) + 2 * align256((size_t)B * n * 2 * tsz);
    if (family == VF_GEMM || family == VF_TGEMM) {
        const size_t Kp = (size_t)(n + 63) / 64 * 64;
        int cper = 0;
        const size_t ks = family == VF_TGEMM ? (size_t)tr_split(((B + TGB - 1) / TGB) * ((n + TGI - 1) / TGI), (int)Kp, &cper) : 1;
        return 2 * align256(n * Kp * tsz) + 4 * align256(B * Kp * tsz) +
               (ks > 1 ? align256(ks * (size_t)B * n * sizeof(cd)) : 0);  // split-k partials (param 2)
    }
    if (family == VF_PLANES || family == VF_TPLANES) {
        const size_t kq = family == VF_TPLANES ? TQK : KCH;  // the ring kernel's k granularity bounds both
        const size_t Kp = (size_t)(n + kq - 1) / kq * kq;
        const size_t PD = prec == LB_BF16_HILO ? 2 : 5, XD = prec == LB_BF16_HILO ? 2 : 4;
        int cper = 0;
        const size_t ks = family == VF_TPLANES ? (size_t)tq_split(((B + TPB - 1) / TPB) * ((n + TPI - 1) / TPI), (int)Kp, &cper) : 1;
        return align256(PD * 2 * n * Kp * 2) + align256(XD * 3 * B * Kp * 2) + align256((size_t)B * n * sizeof(cd)) +
               align256((size_t)n * 4) + align256((size_t)B * 4) +
               (ks > 1 ? align256(ks * (size_t)B * n * sizeof(cd)) : 0);  // split-k partials (param 2)
    }
    return 0;
}

}  // namespace lb
