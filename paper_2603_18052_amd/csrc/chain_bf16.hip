// Fused BF16 step chains on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16),
// one launch for all steps, P resident in registers as MFMA A fragments.
//
// Two representations of P and of the in-flight state:
//
//  HILO    P = Phi + Plo and x = xhi + xlo, each part the nearest BF16 of what
//          is left; Y = Phi xhi + Phi xlo + Plo xhi accumulated in FP32; the
//          state is kept in FP32 between steps.
//
//  SLICED  exponent-aligned integer slices.  Row i of P is scaled by 2^-eP[i]
//          (eP[i] the exponent of the row's largest |Re|, |Im|) and each
//          scaled entry is written as SP base-256 digits q_a (|q_0| <= 256,
//          |q_a| <= 128 for a >= 1, nearest-integer digits), every one exact
//          in BF16.  Each state is scaled by its own 2^-eX (largest |Re|, |Im|
//          of that state) and written as SX digits.  All slice pairs (a, b)
//          of one level L = a + b <= LMAX are summed in ONE FP32 accumulator:
//          each product is an integer and the worst-case level sum,
//          2 n max_L sum_{a+b=L} |q_a||q_b|, stays below 2^24 for n <= 85, so
//          the matrix cores add them exactly.  The levels are combined in FP64
//          (y = 2^(eP+eX) sum_L 2^(-8(L+2)) S_L), the state stays FP64 between
//          steps and is re-sliced every step.
//
// Work split: units = (16-row tile of P, 32-deep k step), dealt to the four
// wavefronts in contiguous runs.  A unit owns its P fragments (all digits,
// Re and Im) in registers; per step it reads the state digits of its k step
// from LDS (planes Re, Im and -Im, so no negation in the loop), runs its
// MFMAs and writes its tile's partial (levels already combined, FP64) to its
// own LDS slot.  Then the slots of each tile are summed in a fixed order
// (deterministic), each state's new exponent is found with an LDS max, and
// the state is re-sliced.  Three barriers per step.
#include "chain.hpp"

namespace lb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

namespace bfc {

constexpr int NS = 16;       // states per workgroup (MFMA N)
constexpr int WAVES = 4;     // wavefronts per workgroup (one per SIMD)
constexpr int UMAX = 5;      // units per wavefront, at most
constexpr int KSTEP = 32;    // MFMA k depth
constexpr int MAXN_SLICED = 85;
constexpr int MAXN_HILO = 96;

enum Mode { HILO = 0, SLICED = 1 };

__device__ inline f4v mma(bf16x8 a, bf16x8 b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

// nearest-even BF16 of a float, as the raw 16 bits
__device__ inline unsigned short bf16_bits(float f) {
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_float(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

// exponent e with max|v| <= 2^e (0 for a zero vector)
__device__ inline int exp_of(double m) {
    if (!(m > 0.0)) return 0;
    int e;
    const double fr = frexp(m, &e);  // m = fr 2^e, fr in [0.5, 1)
    (void)fr;
    return e;
}

struct Shape {
    int Kp, KS, mtiles, units, stride;  // stride: padded k length of a state digit row
};

__host__ __device__ inline Shape shape(int n) {
    Shape s;
    s.Kp = (n + KSTEP - 1) / KSTEP * KSTEP;
    s.KS = s.Kp / KSTEP;
    s.mtiles = (n + 15) / 16;
    s.units = s.mtiles * s.KS;
    // 32-byte pad: rows 32 bytes off a multiple of 64 bytes, the stride at
    // which gfx950's bank-conflict counter reads the operand fetch (16 B of
    // row l % 16 at piece l / 16) as conflict-free; a 16-byte pad reads as
    // two-way
    s.stride = s.Kp + 16;
    return s;
}

template <int MODE, int SP, int SX>
__host__ __device__ constexpr int nplanes() { return MODE == SLICED ? SX : 2; }

template <int MODE, int SP, int SX>
static size_t lds_bytes(int n) {
    const Shape s = shape(n);
    const int xd = nplanes<MODE, SP, SX>();
    size_t b = (size_t)xd * 3 * NS * s.stride * 2;        // state digits (Re, Im, -Im)
    b += (size_t)s.units * 256 * 2 * sizeof(double);       // per-unit partial tiles
    b += 2 * NS * sizeof(unsigned long long) + 256;        // state max / exponents
    b += (size_t)((n + 15) / 16 * 16) * sizeof(int);       // row exponents of P
    return b;
}

template <int MODE, int SP, int SX, int LMAX>
__global__ void __launch_bounds__(WAVES * 64) bf16_chain_kernel(int n, const cd *__restrict__ P, int B,
                                                                cd *__restrict__ rho, long long nsteps) {
    constexpr int XD = nplanes<MODE, SP, SX>();
    constexpr int PD = MODE == SLICED ? SP : 2;
    constexpr int NL = MODE == SLICED ? LMAX + 1 : 1;  // accumulators per component
    extern __shared__ __align__(16) unsigned char smem[];
    const Shape sh = shape(n);
    unsigned short *xdig = reinterpret_cast<unsigned short *>(smem);  // [XD][3][NS][stride]
    double *slots = reinterpret_cast<double *>(smem + (size_t)XD * 3 * NS * sh.stride * 2);  // [units][4][64] x {Re, Im}
    unsigned long long *smax = reinterpret_cast<unsigned long long *>(slots + (size_t)sh.units * 512);  // [NS]
    int *sexp = reinterpret_cast<int *>(smax + NS);        // [NS]
    int *pexp = sexp + NS + 48;                            // [mtiles*16]
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int b0 = blockIdx.x * NS;
    const int plane = NS * sh.stride;  // elements per (digit, component) plane

    // ---- row exponents of P
    for (int r = tid; r < sh.mtiles * 16; r += WAVES * 64) {
        int e = 0;
        if (MODE == SLICED && r < n) {
            double m = 0.0;
            for (int k = 0; k < n; ++k) {
                const cd v = P[(size_t)r * n + k];
                m = fmax(m, fmax(fabs(v.re), fabs(v.im)));
            }
            e = exp_of(m);
        }
        pexp[r] = e;
    }
    __syncthreads();

    // ---- this wavefront's units and their P fragments
    const int u0 = (sh.units * wave) / WAVES, u1 = (sh.units * (wave + 1)) / WAVES;
    const int nu = u1 - u0;
    bf16x8 pf[UMAX][PD][2];
#pragma unroll
    for (int j = 0; j < UMAX; ++j) {
        const int u = u0 + j;
        const int t = u / sh.KS, ks = u - (u / sh.KS) * sh.KS;
        const int row = t * 16 + (lane & 15);
        const int e = (j < nu && row < n) ? pexp[row] : 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = ks * KSTEP + 8 * (lane >> 4) + q;
            cd v = {0.0, 0.0};
            if (j < nu && row < n && k < n) v = P[(size_t)row * n + k];
            if (MODE == SLICED) {
                double vr = ldexp(v.re, -e), vi = ldexp(v.im, -e);
#pragma unroll
                for (int a = 0; a < PD; ++a) {
                    const double dr = rint(vr * 256.0), di = rint(vi * 256.0);
                    vr = vr * 256.0 - dr;
                    vi = vi * 256.0 - di;
                    pf[j][a][0][q] = (__bf16)(float)dr;
                    pf[j][a][1][q] = (__bf16)(float)di;
                }
            } else {
                const float fr = (float)v.re, fi = (float)v.im;
                const unsigned short hr = bf16_bits(fr), hi = bf16_bits(fi);
                const float lr = fr - bf16_float(hr), li = fi - bf16_float(hi);
                pf[j][0][0][q] = (__bf16)bf16_float(hr);
                pf[j][0][1][q] = (__bf16)bf16_float(hi);
                pf[j][1][0][q] = (__bf16)lr;
                pf[j][1][1][q] = (__bf16)li;
            }
        }
    }

    // ---- elements owned by this thread in the combine / slice phases: pairs
    // of consecutive k of one state, so that the slicing phase writes each
    // digit plane as one 4-byte word (two BF16) per lane.  Register i holds
    // pair q = tid + (i / 2) * 256 (state q % 16, k = 2 (q / 16) + i % 2);
    // every pair of a thread belongs to the same state tid % 16.
    constexpr int EPT = 2 * ((MAXN_HILO / 2 * NS + WAVES * 64 - 1) / (WAVES * 64));  // 6
    double yr[EPT], yi[EPT];
    const int npair = (n + 1) / 2 * NS;
    const int es = tid % NS;  // this thread's state
    auto elem_k = [&](int i) { return 2 * ((tid + (i >> 1) * WAVES * 64) / NS) + (i & 1); };
    auto elem_ok = [&](int i) { return tid + (i >> 1) * WAVES * 64 < npair && elem_k(i) < n; };

    // slice y (registers) into the state digit planes, given exponents
    auto slice_out = [&]() {
#pragma unroll
        for (int i = 0; i < EPT; i += 2) {
            if (tid + (i >> 1) * WAVES * 64 < npair) {
                const int k = elem_k(i);  // even
                const bool hi_ok = k + 1 < n;
                unsigned *base = reinterpret_cast<unsigned *>(xdig + (size_t)es * sh.stride + k);
                // the two BF16 of a word: element k in the low half, k + 1 in the high half
                auto put = [&](int pl, unsigned short lo, unsigned short hi) {
                    base[(size_t)pl * plane / 2] = (unsigned)lo | ((unsigned)(hi_ok ? hi : 0) << 16);
                };
                if (MODE == SLICED) {
                    const int ex = sexp[es];
                    double vr0 = ldexp(yr[i], -ex), vi0 = ldexp(yi[i], -ex);
                    double vr1 = ldexp(yr[i + 1], -ex), vi1 = ldexp(yi[i + 1], -ex);
#pragma unroll
                    for (int b = 0; b < XD; ++b) {
                        const double dr0 = rint(vr0 * 256.0), di0 = rint(vi0 * 256.0);
                        const double dr1 = rint(vr1 * 256.0), di1 = rint(vi1 * 256.0);
                        vr0 = vr0 * 256.0 - dr0;
                        vi0 = vi0 * 256.0 - di0;
                        vr1 = vr1 * 256.0 - dr1;
                        vi1 = vi1 * 256.0 - di1;
                        put(b * 3 + 0, bf16_bits((float)dr0), bf16_bits((float)dr1));
                        put(b * 3 + 1, bf16_bits((float)di0), bf16_bits((float)di1));
                        put(b * 3 + 2, bf16_bits((float)-di0), bf16_bits((float)-di1));
                    }
                } else {
                    unsigned short h[2][6];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const float fr = (float)yr[i + q], fi = (float)yi[i + q];
                        const unsigned short hr = bf16_bits(fr), hi = bf16_bits(fi);
                        const float lr = fr - bf16_float(hr), li = fi - bf16_float(hi);
                        const unsigned short blr = bf16_bits(lr), bli = bf16_bits(li);
                        h[q][0] = hr, h[q][1] = hi, h[q][2] = hi ^ 0x8000u;
                        h[q][3] = blr, h[q][4] = bli, h[q][5] = bli ^ 0x8000u;
                    }
#pragma unroll
                    for (int pl = 0; pl < 6; ++pl) put(pl, h[0][pl], h[1][pl]);
                }
            }
        }
    };
    // per-state max of |Re|, |Im| over this thread's elements -> LDS max
    auto state_max = [&]() {
        if (MODE == SLICED) {
            double m = 0.0;
#pragma unroll
            for (int i = 0; i < EPT; ++i)
                if (elem_ok(i)) m = fmax(m, fmax(fabs(yr[i]), fabs(yi[i])));
            if (tid < npair) atomicMax(smax + es, (unsigned long long)__double_as_longlong(m));
        }
    };

    // ---- initial state
    if (tid < NS) smax[tid] = 0ull;
    for (int e = tid; e < 3 * XD * plane; e += WAVES * 64) xdig[e] = 0;  // zero padding rows
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        yr[i] = yi[i] = 0.0;
        if (elem_ok(i)) {
            const int k = elem_k(i), s = es;
            if (b0 + s < B) {
                const cd v = rho[(size_t)(b0 + s) * n + k];
                yr[i] = MODE == SLICED ? v.re : (double)(float)v.re;
                yi[i] = MODE == SLICED ? v.im : (double)(float)v.im;
            }
        }
    }
    state_max();
    __syncthreads();
    if (MODE == SLICED && tid < NS) sexp[tid] = exp_of(__longlong_as_double((long long)smax[tid]));
    __syncthreads();
    slice_out();
    __syncthreads();

    for (long long t = 0; t < nsteps; ++t) {
        if (tid < NS) smax[tid] = 0ull;
        // ---- MFMA phase
#pragma unroll
        for (int j = 0; j < UMAX; ++j) {
            if (j < nu) {  // uniform
                const int u = u0 + j;
                const int ks = u - (u / sh.KS) * sh.KS;
                const int koff = ks * KSTEP + 8 * (lane >> 4);
                bf16x8 xf[XD][3];
#pragma unroll
                for (int b = 0; b < XD; ++b)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        xf[b][c] = *reinterpret_cast<const bf16x8 *>(xdig + (size_t)(b * 3 + c) * plane +
                                                                     (lane & 15) * sh.stride + koff);
                f4v ar[NL], ai[NL];
#pragma unroll
                for (int L = 0; L < NL; ++L) {
                    ar[L] = f4v{0, 0, 0, 0};
                    ai[L] = f4v{0, 0, 0, 0};
                }
#pragma unroll
                for (int a = 0; a < PD; ++a)
#pragma unroll
                    for (int b = 0; b < XD; ++b) {
                        const int L = a + b;
                        if (MODE == SLICED ? (L <= LMAX) : (L <= 1)) {
                            const int Lq = MODE == SLICED ? L : 0;
                            ar[Lq] = mma(pf[j][a][0], xf[b][0], ar[Lq]);
                            ar[Lq] = mma(pf[j][a][1], xf[b][2], ar[Lq]);
                            ai[Lq] = mma(pf[j][a][0], xf[b][1], ai[Lq]);
                            ai[Lq] = mma(pf[j][a][1], xf[b][0], ai[Lq]);
                        }
                    }
                // the unit's partial tile, lane-major: register r of lane l (row
                // 4 (l / 16) + r, state l % 16) at pair r * 64 + l, {Re, Im}
                // together, so that each register is one contiguous 1 KB write
                d2v *slot = reinterpret_cast<d2v *>(slots) + (size_t)u * 256;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double vr = 0.0, vi = 0.0;
#pragma unroll
                    for (int L = NL - 1; L >= 0; --L) {  // smallest terms first
                        const double w = MODE == SLICED ? ldexp(1.0, -8 * (L + 2)) : 1.0;
                        vr = fma((double)ar[L][r], w, vr);
                        vi = fma((double)ai[L][r], w, vi);
                    }
                    slot[r * 64 + lane] = d2v{vr, vi};
                }
            }
        }
        __syncthreads();
        // ---- combine the k-step slots of every tile (fixed order)
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            if (elem_ok(i)) {
                const int k = elem_k(i), s = es;
                // row k % 16 of the tile = register (k % 16) % 4 of lane 16 ((k % 16) / 4) + s
                const int tt = k >> 4, o = ((k & 15) & 3) * 64 + 16 * ((k & 15) >> 2) + s;
                double vr = 0.0, vi = 0.0;
                for (int q = 0; q < sh.KS; ++q) {
                    const d2v v = reinterpret_cast<const d2v *>(slots)[(size_t)(tt * sh.KS + q) * 256 + o];
                    vr += v[0];
                    vi += v[1];
                }
                if (MODE == SLICED) {
                    const int sc = pexp[k] + sexp[s];
                    yr[i] = ldexp(vr, sc);
                    yi[i] = ldexp(vi, sc);
                } else {
                    yr[i] = (double)(float)vr;  // FP32 state
                    yi[i] = (double)(float)vi;
                }
            }
        }
        if (t + 1 == nsteps) break;  // uniform
        state_max();
        __syncthreads();
        if (MODE == SLICED && tid < NS) sexp[tid] = exp_of(__longlong_as_double((long long)smax[tid]));
        __syncthreads();
        slice_out();
        __syncthreads();
    }
    if (nsteps == 0) return;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        if (elem_ok(i)) {
            const int k = elem_k(i), s = es;
            if (b0 + s < B) rho[(size_t)(b0 + s) * n + k] = {yr[i], yi[i]};
        }
    }
}

static const size_t kLds = 160 * 1024;

template <int MODE, int SP, int SX, int LMAX>
static int launch(int n, const cd *P, int B, cd *rho, long long nsteps, hipStream_t s) {
    const size_t lds = lds_bytes<MODE, SP, SX>(n);
    const Shape sh = shape(n);
    if (lds > kLds || (sh.units + WAVES - 1) / WAVES > UMAX)
        return fail(LB_ESHAPE, "bf16 chain: n too large for the fused kernel");
    LB_TRY(set_max_lds((const void *)bf16_chain_kernel<MODE, SP, SX, LMAX>, kLds));
    bf16_chain_kernel<MODE, SP, SX, LMAX><<<(B + NS - 1) / NS, WAVES * 64, lds, s>>>(n, P, B, rho, nsteps);
    return check_launch("bf16_chain");
}

}  // namespace bfc

int bf16_fused_max_n(lb_precision prec) {
    return prec == LB_BF16_SLICED ? bfc::MAXN_SLICED : prec == LB_BF16_HILO ? bfc::MAXN_HILO : 0;
}

int chain_bf16_fused(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, hipStream_t s) {
    if (prec == LB_BF16_HILO) return bfc::launch<bfc::HILO, 2, 2, 1>(n, P, B, rho, nsteps, s);
    // 5 x 4 digits, levels <= 4 (14 slice pairs) for every step count
    return bfc::launch<bfc::SLICED, 5, 4, 4>(n, P, B, rho, nsteps, s);
}

}  // namespace lb
