// INT8-digit chain (LB_I8_SLICED) past the fused limit (n > 96): one
// LDS-tiled INT8 GEMM launch per step on v_mfma_i32_16x16x64_i8.
//
// The representation is the fused kernel's (chain_i8.hip): the real
// embedding Q = [[PR, -PI], [PI, PR]] (2n x 2n), each row scaled by its own
// power of two and rounded to 38 fraction bits in five balanced base-256
// digits; each state rounded to 30 fraction bits below its own power of two
// in four digits; the 14 digit pairs of levels <= 4 summed exactly in int32
// over the whole k range (a level sum is at most 5 * 2n * 2^14 < 2^31 for
// n <= 4096), levels combined in FP64.
//
// One difference: a step cannot agree on the new state's exponent before
// slicing it (that would need a grid-wide barrier), so state x_{t+1} is sliced
// below 2^(M_t + g), where M_t is the exponent of max |x_t| (the previous
// step's, complete when the step starts) and 2^g bounds the growth of one
// step: 2^g >= max_r sum_k |Q_rk| >= max |x_{t+1}| / max |x_t|.  Each step
// records M_{t+1} with atomic maxima for the step after it; four slots of
// exponents rotate so that a step reads two, writes one and clears one.
// The FP64 state exists only in the epilogue: the step's output is sliced
// straight into the next step's digit planes (four consecutive k of one
// state per lane: one 4-byte write per digit plane).
//
// Tile: 96 rows of Q x 64 states per workgroup (256 workgroups at n = 729,
// B = 1024: one per CU, one wavefront per SIMD), four wavefronts in a 2 x 2
// grid of 48 rows x 32 states each; k in 64-deep chunks through a ring of
// three LDS slots (47 KB each) filled by direct global-to-LDS loads.  With
// one wavefront per SIMD nothing hides an LDS fetch behind another
// wavefront's MFMAs, so each wavefront hides its own: the operands of chunk
// c + 1 come from LDS into a second register set while chunk c's MFMAs run
// from the first, and chunks c + 2, c + 3 are in flight into the ring.
// 64-byte digit rows sit at XOR-swizzled 16-byte positions so that the
// operand fetches run without bank conflicts.  Each XCD takes a 4 x 8 block
// of tiles, so that 4 row blocks of Q's digits and 8 state blocks pass
// through its L2.  Smaller batches use smaller tiles with deeper rings: 96 x
// 32 (four 38 KB slots) and 64 x 16 (one MFMA tile per wavefront, six 24 KB
// slots): more workgroups (92 at n = 729, B <= 64 against 16) and more
// chunks in flight for the load latency that fewer MFMAs per chunk cannot
// cover.  The digit planes are chunk-major, [digit][k / 64][row][64], so one
// chunk of a tile is contiguous: a 1 KB load reads eight whole 128-byte lines.
#include "chain.hpp"

namespace lb {
namespace i8g {

typedef int i4v __attribute__((ext_vector_type(4)));

constexpr int NPD = 5, NXD = 4, LMAX = 4;
constexpr int FRAC_P = 38, FRAC_X = 30;
constexpr int YSHIFT = FRAC_P + FRAC_X - 8 * (NPD - 1) - 8 * (NXD - 1);  // 12
constexpr int EMPTY = -100000;
constexpr int KC = 64;    // k per chunk (one MFMA deep)
constexpr int TRMAX = 96;  // the tallest tile: row exponents are padded by less than this

// A workgroup tile: TR rows of Q x TS states, four wavefronts in a WR x WS
// grid of RT x ST MFMA tiles each, a ring of RING LDS slots of STAGE bytes
// (one chunk: five Q digit planes and four state digit planes), each chunk
// NLT loads of 1 KB (NLW per wavefront), then TS ints of exponent maxima.
template <int TR_, int TS_, int RT_, int ST_, int RING_>
struct GShape {
    static constexpr int TR = TR_, TS = TS_, RT = RT_, ST = ST_, RING = RING_;
    static constexpr int WR = TR / (16 * RT), WS = TS / (16 * ST);
    static constexpr int APL = TR * KC, BPL = TS * KC;
    static constexpr int STAGE = NPD * APL + NXD * BPL;
    static constexpr int NLA = NPD * TR / 16, NLB = NXD * TS / 16, NLT = NLA + NLB;
    static constexpr int NLW = (NLT + 3) / 4;
    static constexpr int LDS = RING * STAGE + TS * 4;
    static_assert(WR * WS == 4 && TR <= TRMAX && LDS <= 160 * 1024, "tile shape");
    static_assert((RING - 1) * NLW < 64, "vmcnt range");
};
// 96 x 64 (256 workgroups at n = 729, B = 1024): 47 KB slots, two chunks in
// flight behind the one being fetched
using BigTile = GShape<96, 64, 3, 2, 3>;
// 96 x 32 for middle batches (256 workgroups at n = 729, B = 512): 38 KB
// slots, three chunks in flight
using MidTile = GShape<96, 32, 3, 1, 4>;
// 64 x 16 for small batches (92 workgroups at n = 729, B = 64): 24 KB slots,
// five chunks in flight
using SmallTile = GShape<64, 16, 1, 1, 6>;
// 96 x 32 with two slots (76 KB): two workgroups share a CU, so one
// workgroup's MFMAs cover the other's loads
using PairTile = GShape<96, 32, 3, 1, 2>;

// Workgroup barrier of the ring: wait until at most N of this wavefront's
// vector loads are outstanding and its LDS accesses are done (s_waitcnt,
// gfx9 fields: vmcnt N, expcnt 7 = no wait, lgkmcnt 0), then s_barrier; the
// empty asm statements keep memory accesses from moving across it.
#define I8_SYNC(N)                                                                 \
    do {                                                                           \
        asm volatile("" ::: "memory");                                             \
        __builtin_amdgcn_s_waitcnt(((N) & 15) | (7 << 4) | (((N) >> 4) << 14));   \
        __builtin_amdgcn_s_barrier();                                              \
        asm volatile("" ::: "memory");                                             \
    } while (0)
constexpr int XLIM = (1 << FRAC_X) - 1;

__device__ inline i4v mma(i4v a, i4v b, i4v c) { return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0); }
__device__ inline int swz(int row, int piece) { return piece ^ ((row >> 1) & 3); }

__device__ inline int exp_of(double m) {
    if (!(m > 0.0)) return EMPTY;
    int e;
    (void)frexp(m, &e);
    return e;
}

// Q[R][k] of the real embedding
__device__ inline double qval(const cd *__restrict__ P, int n, int R, int k) {
    if (R >= 2 * n || k >= 2 * n) return 0.0;
    const bool rim = R >= n, kim = k >= n;
    const cd v = P[(size_t)(rim ? R - n : R) * n + (kim ? k - n : k)];
    if (!rim) return kim ? -v.im : v.re;
    return kim ? v.re : v.im;
}

// Hermitian coordinates (n = d^2): the real step R on h_(i,j) = Re rho_ij
// (i <= j), Im rho_ij (i > j).  With u = P[r, (a, b)], v = P[r, (b, a)]:
// z = u (a = b), u + v (a < b), i (u - v) (a > b); R[r, q] = Re z for a
// row r = (i, j) with i <= j, else Im z.
__device__ inline double hval(const cd *__restrict__ P, int n, int d, int r, int q) {
    if (r >= n || q >= n) return 0.0;
    const int a = q / d, b = q - a * d, i = r / d, j = r - i * d;
    const cd u = P[(size_t)r * n + q], v = P[(size_t)r * n + b * d + a];
    double re = u.re, im = u.im;
    if (a < b) {
        re += v.re;
        im += v.im;
    } else if (a > b) {
        re = v.im - u.im;
        im = u.re - v.re;
    }
    return i <= j ? re : im;
}

__device__ inline int dim_of(int n) {
    int d = 1;
    while ((d + 1) * (d + 1) <= n) ++d;
    return d;
}

// digits of a row of the step matrix (Q, or R of the Hermitian form; one
// workgroup per row): exponent, five planes, and the row's absolute sum
// into gbits (atomic max of the non-negative bits)
template <bool HERM>
__global__ void __launch_bounds__(256) prep_q_kernel(int n, int Kp, int npad, const cd *__restrict__ P,
                                                     signed char *__restrict__ Qd, int *__restrict__ eP,
                                                     unsigned long long *__restrict__ gbits) {
    const int R = blockIdx.x, tid = threadIdx.x;
    const int r = R < n ? R : R - n;
    const int m2 = HERM ? n : 2 * n, dd = HERM ? dim_of(n) : 1;
    double m = 0.0, sum = 0.0;
    for (int k = tid; k < n; k += 256) {
        if (HERM) {
            const double h = fabs(hval(P, n, dd, R, k));
            m = fmax(m, h);
            sum += h;
        } else {
            const cd v = P[(size_t)r * n + k];
            m = fmax(m, fmax(fabs(v.re), fabs(v.im)));
            sum += fabs(v.re) + fabs(v.im);
        }
    }
    __shared__ double rm[256], rs[256];
    rm[tid] = m;
    rs[tid] = sum;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            rm[tid] = fmax(rm[tid], rm[tid + w]);
            rs[tid] += rs[tid + w];
        }
        __syncthreads();
    }
    const int e = rm[0] > 0.0 ? exp_of(rm[0]) : 0;
    if (tid == 0) {
        eP[R] = e;
        atomicMax(gbits, (unsigned long long)__double_as_longlong(rs[0]));
    }
    // rows past 2n (up to whole row blocks) repeat the last row: the step
    // kernel loads them from the last row too, so their outputs copy its
    // output and need no masking before the exponent maximum
    if (R == m2 - 1)
        for (int q = m2 + tid; q < npad; q += 256) eP[q] = e;
    const size_t plane = (size_t)m2 * Kp;
    for (int k0 = 4 * tid; k0 < Kp; k0 += 4 * 256) {
        unsigned w[NPD] = {0u, 0u, 0u, 0u, 0u};
        for (int q = 0; q < 4; ++q) {
            const double qv = HERM ? hval(P, n, dd, R, k0 + q) : qval(P, n, R, k0 + q);
            const long long V = (long long)rint(ldexp(qv, FRAC_P - e));
            const unsigned long long U = (unsigned long long)(V + 0x80808080LL);
            for (int j = 0; j < NPD; ++j) {
                const unsigned byte = j < NPD - 1 ? (unsigned)((U >> (8 * j)) & 0xFFu) ^ 0x80u
                                                  : (unsigned)((unsigned long long)((long long)U >> 32) & 0xFFu);
                w[NPD - 1 - j] |= byte << (8 * q);
            }
        }
        for (int a = 0; a < NPD; ++a)
            *reinterpret_cast<unsigned *>(Qd + a * plane + (size_t)(k0 / KC) * (m2 * KC) + (size_t)R * KC + k0 % KC) =
                w[a];
    }
}

// growth bound g (2^g >= max row sum, 0 for contractions) from gbits
__device__ inline int growth_bits(const unsigned long long *gbits) {
    const double s = __longlong_as_double((long long)*gbits) * (1.0 + 0x1p-20);
    return s > 1.0 ? exp_of(s) : 0;
}

// initial state of each state (one workgroup per state): exact exponent
// M_0, digits of x_0 into buffer 0 (zeros past 2n), zero padding of buffer
// 1, and the exponent slots: slot 3 = M_0 - g (so that S_0 = M_0), slot 0 =
// M_0, slots 1 and 2 empty
template <bool HERM>
__global__ void __launch_bounds__(256) init_x_kernel(int n, int Kp, int B, const cd *__restrict__ rho,
                                                     signed char *__restrict__ X0, signed char *__restrict__ X1,
                                                     int *__restrict__ Mx, const unsigned long long *__restrict__ gbits) {
    const int b = blockIdx.x, tid = threadIdx.x, n2 = HERM ? n : 2 * n, dd = HERM ? dim_of(n) : 1;
    const cd *x = rho + (size_t)b * n;
    // coordinate k of the state: Re / Im of the embedding, or h_k
    auto coord = [&](int k) {
        if (HERM) return k < n ? ((k / dd <= k % dd) ? x[k].re : x[k].im) : 0.0;
        return k < n ? x[k].re : (k < n2 ? x[k - n].im : 0.0);
    };
    int m = EMPTY;
    for (int k = tid; k < n2; k += 256) m = max(m, exp_of(fabs(coord(k))));
    __shared__ int red[256];
    red[tid] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] = max(red[tid], red[tid + w]);
        __syncthreads();
    }
    const int M0 = red[0];
    const int S = M0 == EMPTY ? 0 : M0;
    const size_t plane = (size_t)B * Kp;
    for (int k0 = 4 * tid; k0 < Kp; k0 += 4 * 256) {
        unsigned W[4];
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + q;
            const double v = coord(k);
            int V = (int)rint(ldexp(v, FRAC_X - S));
            V = V > XLIM ? XLIM : (V < -XLIM ? -XLIM : V);
            W[q] = (unsigned)(V + 0x00808080) ^ 0x00808080u;
        }
        for (int bd = 0; bd < NXD; ++bd) {
            const int sh = 8 * (NXD - 1 - bd);
            const unsigned D = ((W[0] >> sh) & 0xFFu) | (((W[1] >> sh) & 0xFFu) << 8) | (((W[2] >> sh) & 0xFFu) << 16) |
                               (((W[3] >> sh) & 0xFFu) << 24);
            const size_t at = bd * plane + (size_t)(k0 / KC) * ((size_t)B * KC) + (size_t)b * KC + k0 % KC;
            *reinterpret_cast<unsigned *>(X0 + at) = D;
            if (k0 + 4 > n2) *reinterpret_cast<unsigned *>(X1 + at) = 0u;
        }
    }
    if (tid == 0) {
        const int g = growth_bits(gbits);
        Mx[3 * B + b] = M0 == EMPTY ? EMPTY : M0 - g;
        Mx[0 * B + b] = M0;
        Mx[1 * B + b] = EMPTY;
        Mx[2 * B + b] = EMPTY;
    }
}

// Tile T -> (row block, state block): super-tiles of GR row blocks x GS
// state blocks in row-major order, row-block major inside one (the last
// super-row and super-column may be narrower).  32 consecutive tiles (one
// XCD's share at n = 729, B = 1024) form one 4 x 8 super-tile: 4 row blocks
// of Q's digits and 8 state blocks pass through that XCD's L2, 5.8 MB
// against 7.4 MB for 2 x 16.
constexpr int GR = 4, GS = 8;
__device__ inline void tile_of(int T, int nrb, int nsb, int &rb, int &sb) {
    const int rbase = T / (GR * nsb) * GR;
    const int gr = min(GR, nrb - rbase);
    const int Tp = T - rbase * nsb;
    const int sg = Tp / (gr * GS);
    const int gs = min(GS, nsb - sg * GS);
    const int w = Tp - sg * gr * GS;
    rb = rbase + w / gs;
    sb = sg * GS + w % gs;
}

// one step: x_{t+1} = Q x_t for all states (t4 = t mod 4); the last step
// (LAST) writes FP64 into rho instead of digits.  Dynamic LDS (smem): the
// ring, then TS ints for the workgroup's exponent maxima.
template <class S, bool LAST>
__device__ __forceinline__ void i8_gemm_body(unsigned char *smem, int n, int m2, int Kp, int B, int nrb, int nsb,
                                             const signed char *__restrict__ Qd, const int *__restrict__ eP,
                                             const signed char *__restrict__ Xc, signed char *__restrict__ Xn,
                                             int *__restrict__ Mx, const unsigned long long *__restrict__ gbits,
                                             int t4, cd *__restrict__ rho) {
    constexpr int TR = S::TR, TS = S::TS, RT = S::RT, ST = S::ST, RING = S::RING;
    constexpr int APL = S::APL, BPL = S::BPL, STAGE = S::STAGE, NLA = S::NLA, NLT = S::NLT, NLW = S::NLW;
    int *emx = reinterpret_cast<int *>(smem + RING * STAGE);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n2 = m2;  // rows and k of the step: 2n, or n for the Hermitian coordinates
    // tile order: each XCD takes consecutive tiles
    const int total = nrb * nsb, per = total / 8, rem = total % 8;
    const int xcd = blockIdx.x % 8, jx = blockIdx.x / 8;
    int rb, sb;
    tile_of(xcd * per + (xcd < rem ? xcd : rem) + jx, nrb, nsb, rb, sb);
    const int r0 = rb * TR, s0 = sb * TS;
    const size_t qplane = (size_t)n2 * Kp, xplane = (size_t)B * Kp;
    const int nch = Kp / KC;
    const int wr = (wave % S::WR) * (RT * 16), ws = (wave / S::WR) * (ST * 16);  // this wavefront's rows / states
    const int fr = lane & 15, fp = lane >> 4;

    // The epilogue's operands, loaded first so that they land under the k
    // loop: the exponents of this lane's 4 x RT rows (eP is padded to whole
    // row blocks) and the exponent slots of its ST states (clamped to the
    // last state: the copies past B are neither stored nor reduced).
    const int *Mcur = Mx + ((t4 + 3) & 3) * B;  // x_t was sliced below 2^(Mcur + g)
    const int *Mnow = Mx + t4 * B;              // exponent of max |x_t|
    i4v er[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) er[i] = *reinterpret_cast<const i4v *>(eP + r0 + wr + 16 * i + 4 * fp);
    int mc[ST], mn[ST];
#pragma unroll
    for (int j = 0; j < ST; ++j) {
        const int b = min(s0 + ws + 16 * j + fr, B - 1);
        mc[j] = Mcur[b];
        mn[j] = Mnow[b];
    }
    if (!LAST && tid < TS) emx[tid] = EMPTY;  // ordered before its use by the ring's barriers

    // A chunk is NLT loads of 1 KB (16 rows x 64 bytes of one digit plane),
    // straight from global memory into LDS; lane l's 16 bytes land at row
    // l / 4, position l % 4 of the tile, which holds the row's piece
    // swz(row, l % 4).  Wavefront w issues loads w, w + 4, ... (past NLT they
    // repeat earlier ones: same data to the same place).
    const signed char *src[NLW];
    int dst[NLW];
    bool isq[NLW];  // a load of Q's digits (else of the states'): wave-uniform
#pragma unroll
    for (int q = 0; q < NLW; ++q) {
        int j = wave + 4 * q;
        j = j < NLT ? j : j - (4 * NLW - NLT);
        const int row = lane >> 2, pc = swz(row, lane & 3);
        if (j < NLA) {
            const int a = j / (TR / 16), tq = j - a * (TR / 16);
            int R = r0 + 16 * tq + row;
            R = R < n2 ? R : n2 - 1;
            src[q] = Qd + a * qplane + (size_t)R * KC + pc * 16;
            isq[q] = true;
            dst[q] = a * APL + tq * 1024;
        } else {
            const int jj = j - NLA, bd = jj / (TS / 16), tq = jj - bd * (TS / 16);
            int b = s0 + 16 * tq + row;
            b = b < B ? b : B - 1;
            src[q] = Xc + bd * xplane + (size_t)b * KC + pc * 16;
            isq[q] = false;
            dst[q] = NPD * APL + bd * BPL + tq * 1024;
        }
    }
    // loads of chunk c into ring slot `slot` (chunk-major planes: chunk c of
    // Q's digits starts c 2n 64 bytes in, of the states' c B 64)
    auto dma = [&](int c, int slot) {
        const size_t qo = (size_t)c * (n2 * KC), xo = (size_t)c * (B * KC);
#pragma unroll
        for (int q = 0; q < NLW; ++q)
            __builtin_amdgcn_global_load_lds((const void *)(src[q] + (isq[q] ? qo : xo)),
                                             (__attribute__((address_space(3))) void *)(smem + slot * STAGE + dst[q]),
                                             16, 0, 0);
    };

    i4v acc[RT][ST][LMAX + 1];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < ST; ++j)
#pragma unroll
            for (int L = 0; L <= LMAX; ++L) acc[i][j][L] = i4v{0, 0, 0, 0};

    // The operands of one chunk (this wavefront's state and row digits)
    // from LDS into registers, and the chunk's 14 x RT x ST MFMAs.
    auto fetch = [&](int c, i4v (&xb)[ST][NXD], i4v (&pa)[RT][NPD]) {
        const unsigned char *st = smem + (c % RING) * STAGE;
#pragma unroll
        for (int j = 0; j < ST; ++j) {
            const int s = ws + 16 * j + fr;
#pragma unroll
            for (int bd = 0; bd < NXD; ++bd)
                xb[j][bd] = *reinterpret_cast<const i4v *>(st + NPD * APL + bd * BPL + s * 64 + swz(s, fp) * 16);
        }
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            const int row = wr + 16 * i + fr;
#pragma unroll
            for (int a = 0; a < NPD; ++a)
                pa[i][a] = *reinterpret_cast<const i4v *>(st + a * APL + row * 64 + swz(row, fp) * 16);
        }
    };
    auto mfmas = [&](const i4v (&xb)[ST][NXD], const i4v (&pa)[RT][NPD]) {
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int a = 0; a < NPD; ++a)
#pragma unroll
                for (int bd = 0; bd < NXD; ++bd)
                    if (a + bd <= LMAX)
#pragma unroll
                        for (int j = 0; j < ST; ++j) acc[i][j][a + bd] = mma(pa[i][a], xb[j][bd], acc[i][j][a + bd]);
    };
    // Chunk c is computed from registers while chunk c + 1's operands come
    // from LDS into the other register set and chunks c + 2 .. c + RING load
    // into the ring: the barrier before chunk c + 1's fetch (its loads landed
    // in every wavefront; every wavefront's fetch of chunk c is complete)
    // frees chunk c's slot for chunk c + RING.  The last chunk fetches itself
    // again (its slot is no longer written) so that the fetch and the MFMAs
    // form one branch-free block.
    auto step = [&](int c, const i4v (&xc)[ST][NXD], const i4v (&pc)[RT][NPD], i4v (&xn)[ST][NXD],
                    i4v (&pn)[RT][NPD]) {
        // (one barrier on every path: the compiler's wait analysis then sees
        // every earlier fetch complete before the MFMAs)
        // (near the end fewer than RING - 2 chunks follow c + 1: wait for all)
        if (c + RING - 1 >= nch) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt 0
        I8_SYNC((RING - 2) * NLW);
        if (c + RING < nch) dma(c + RING, c % RING);
        fetch(c + 1 < nch ? c + 1 : c, xn, pn);
        mfmas(xc, pc);
    };

    i4v x0[ST][NXD], p0[RT][NPD], x1[ST][NXD], p1[RT][NPD];
#pragma unroll
    for (int c = 0; c < RING; ++c)
        if (c < nch) dma(c, c);
    if (nch >= RING)
        I8_SYNC((RING - 1) * NLW);  // chunk 0 landed, 1 .. RING - 1 may be in flight
    else
        I8_SYNC(0);
    fetch(0, x0, p0);
    // chunks in pairs, both steps unconditional (a conditional second step
    // lets the compiler sink the first step's fetch into it, after the MFMAs
    // it should overlap); an odd count computes chunk 0 first
    int c0 = 0;
    if (nch & 1) {
        step(0, x0, p0, x1, p1);
#pragma unroll
        for (int j = 0; j < ST; ++j)
#pragma unroll
            for (int bd = 0; bd < NXD; ++bd) x0[j][bd] = x1[j][bd];
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int a = 0; a < NPD; ++a) p0[i][a] = p1[i][a];
        c0 = 1;
    }
    for (int c = c0; c < nch; c += 2) {
        step(c, x0, p0, x1, p1);
        step(c + 1, x1, p1, x0, p0);
    }

    // ---- epilogue: y = 2^(eP + Sc - YSHIFT) sum_L 2^(-8L) acc_L for the
    // lane's four consecutive rows R0 .. R0 + 3 of each (i, j)
    const int g = growth_bits(gbits);
    if (!LAST && rb == 0 && tid < TS && s0 + tid < B) Mx[((t4 + 2) & 3) * B + s0 + tid] = EMPTY;
#pragma unroll
    for (int j = 0; j < ST; ++j) {
        const int b = s0 + ws + 16 * j + fr;
        const bool bok = b < B;
        const int Sc = mc[j] == EMPTY ? 0 : mc[j] + g;
        const int Sn = mn[j] == EMPTY ? 0 : mn[j] + g;
        int emax = EMPTY;
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            const int R0 = r0 + wr + 16 * i + 4 * fp;
            double v[4];
            int ey[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                v[r] = (double)acc[i][j][LMAX][r];
#pragma unroll
                for (int L = LMAX - 1; L >= 0; --L) v[r] = fma(v[r], 1.0 / 256.0, (double)acc[i][j][L][r]);
                ey[r] = er[i][r] + Sc - YSHIFT;  // y = v 2^ey, exactly
            }
            if (LAST) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int R = R0 + r;
                    if (bok && R < n2) {
                        const double y = __builtin_amdgcn_ldexp(v[r], ey[r]);
                        if (n2 == 2 * n) {
                            double *o = reinterpret_cast<double *>(rho + (size_t)b * n + (R < n ? R : R - n));
                            o[R < n ? 0 : 1] = y;
                        } else {
                            // h_(i,j): Re rho_ij = Re rho_ji (i <= j), or Im rho_ij = -Im rho_ji (i > j)
                            const int d = dim_of(n), i = R / d, jj = R - i * d, c = i <= jj ? 0 : 1;
                            double *o = reinterpret_cast<double *>(rho + (size_t)b * n);
                            o[2 * R + c] = y;
                            if (i == jj)
                                o[2 * R + 1] = 0.0;
                            else
                                o[2 * (jj * d + i) + c] = c ? -y : y;
                        }
                    }
                }
            } else {
                unsigned W[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // frexp exponent of y (zero outputs do not count)
                    emax = max(emax, v[r] != 0.0 ? __builtin_amdgcn_frexp_exp(v[r]) + ey[r] : EMPTY);
                    int V = (int)rint(__builtin_amdgcn_ldexp(v[r], ey[r] + FRAC_X - Sn));
                    V = V > XLIM ? XLIM : (V < -XLIM ? -XLIM : V);
                    W[r] = (unsigned)(V + 0x00808080) ^ 0x00808080u;
                }
                if (bok && R0 < Kp) {
#pragma unroll
                    for (int bd = 0; bd < NXD; ++bd) {
                        const int sh = 8 * (NXD - 1 - bd);
                        const unsigned D = ((W[0] >> sh) & 0xFFu) | (((W[1] >> sh) & 0xFFu) << 8) |
                                           (((W[2] >> sh) & 0xFFu) << 16) | (((W[3] >> sh) & 0xFFu) << 24);
                        *reinterpret_cast<unsigned *>(Xn + bd * xplane + (size_t)(R0 / KC) * ((size_t)B * KC) +
                                                      (size_t)b * KC + R0 % KC) = D;
                    }
                }
            }
        }
        if (!LAST) {
            emax = max(emax, __shfl_xor(emax, 16));
            emax = max(emax, __shfl_xor(emax, 32));
            if (fp == 0) atomicMax(emx + ws + 16 * j + fr, emax);
        }
    }
    if (!LAST) {
        // one global maximum per state and workgroup
        __syncthreads();
        if (tid < TS && s0 + tid < B && emx[tid] != EMPTY) atomicMax(Mx + ((t4 + 1) & 3) * B + s0 + tid, emx[tid]);
    }
}

template <bool LAST>
__global__ void __launch_bounds__(256) i8_gemm_step_kernel(int n, int m2, int Kp, int B, int nrb, int nsb,
                                                           const signed char *__restrict__ Qd,
                                                           const int *__restrict__ eP,
                                                           const signed char *__restrict__ Xc,
                                                           signed char *__restrict__ Xn, int *__restrict__ Mx,
                                                           const unsigned long long *__restrict__ gbits, int t4,
                                                           cd *__restrict__ rho) {
    extern __shared__ __align__(16) unsigned char smem[];
    i8_gemm_body<BigTile, LAST>(smem, n, m2, Kp, B, nrb, nsb, Qd, eP, Xc, Xn, Mx, gbits, t4, rho);
}

template <bool LAST>
__global__ void __launch_bounds__(256) i8_gemm_mid_kernel(int n, int m2, int Kp, int B, int nrb, int nsb,
                                                          const signed char *__restrict__ Qd,
                                                          const int *__restrict__ eP,
                                                          const signed char *__restrict__ Xc,
                                                          signed char *__restrict__ Xn, int *__restrict__ Mx,
                                                          const unsigned long long *__restrict__ gbits, int t4,
                                                          cd *__restrict__ rho) {
    extern __shared__ __align__(16) unsigned char smem[];
    i8_gemm_body<MidTile, LAST>(smem, n, m2, Kp, B, nrb, nsb, Qd, eP, Xc, Xn, Mx, gbits, t4, rho);
}

template <bool LAST>
__global__ void __launch_bounds__(256) i8_gemm_small_kernel(int n, int m2, int Kp, int B, int nrb, int nsb,
                                                            const signed char *__restrict__ Qd,
                                                            const int *__restrict__ eP,
                                                            const signed char *__restrict__ Xc,
                                                            signed char *__restrict__ Xn, int *__restrict__ Mx,
                                                            const unsigned long long *__restrict__ gbits, int t4,
                                                            cd *__restrict__ rho) {
    extern __shared__ __align__(16) unsigned char smem[];
    i8_gemm_body<SmallTile, LAST>(smem, n, m2, Kp, B, nrb, nsb, Qd, eP, Xc, Xn, Mx, gbits, t4, rho);
}

template <bool LAST>
__global__ void __launch_bounds__(256, 2) i8_gemm_pair_kernel(int n, int m2, int Kp, int B, int nrb, int nsb,
                                                              const signed char *__restrict__ Qd,
                                                              const int *__restrict__ eP,
                                                              const signed char *__restrict__ Xc,
                                                              signed char *__restrict__ Xn, int *__restrict__ Mx,
                                                              const unsigned long long *__restrict__ gbits, int t4,
                                                              cd *__restrict__ rho) {
    extern __shared__ __align__(16) unsigned char smem[];
    i8_gemm_body<PairTile, LAST>(smem, n, m2, Kp, B, nrb, nsb, Qd, eP, Xc, Xn, Mx, gbits, t4, rho);
}

static int grid1(long long work) {
    long long g = (work + 255) / 256;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace i8g

size_t i8_gemm_ws_bytes(int n, int B, bool herm) {
    const size_t m2 = herm ? n : 2 * (size_t)n;
    const size_t Kp = (m2 + 63) / 64 * 64;
    const size_t npad = m2 + i8g::TRMAX;  // row exponents padded to whole row blocks of any tile
    return align256((size_t)i8g::NPD * m2 * Kp) + align256(npad * 4) +
           2 * align256((size_t)i8g::NXD * B * Kp) + align256((size_t)4 * B * 4) + 256;
}

namespace i8g {
// the step launches of one tile shape (K<LAST> = its two kernels)
template <class S, class Launch>
static int run_tiles(int n, int m2, int Kp, int B, const signed char *Qd, const int *eP, signed char *X0, signed char *X1,
                     int *Mx, const unsigned long long *gbits, cd *rho, long long nsteps, bool graph, hipStream_t s,
                     const void *k_step, const void *k_last, Launch launch) {
    const int nrb = (m2 + S::TR - 1) / S::TR, nsb = (B + S::TS - 1) / S::TS;
    LB_TRY(set_max_lds(k_step, S::LDS));
    LB_TRY(set_max_lds(k_last, S::LDS));
    LB_TRY(run_steps(nsteps, graph, [&](long long t, hipStream_t st) {
        launch(t + 1 == nsteps, nrb * nsb, S::LDS, st, n, m2, Kp, B, nrb, nsb, Qd, eP, (t & 1) ? X1 : X0,
               (t & 1) ? X0 : X1, Mx, gbits, (int)(t & 3), rho);
        return LB_OK;
    }, s));
    return check_launch("i8 gemm step");
}
}  // namespace i8g

int chain_i8_gemm(int n, const cd *P, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s, bool graph,
                  int shape, bool herm) {
    using namespace i8g;
    if (herm && !i8_herm_shape_ok(n)) return fail(LB_ESHAPE, "i8 Hermitian chain: n must be d^2");
    if (nsteps == 0 || B == 0) return LB_OK;
    const int n2 = herm ? n : 2 * n, Kp = (n2 + 63) / 64 * 64;
    LB_TRY(ws_ensure(ws, i8_gemm_ws_bytes(n, B, herm)));
    const size_t mark = ws->used;
    signed char *Qd = (signed char *)ws_take(ws, (size_t)NPD * n2 * Kp);
    int *eP = (int *)ws_take(ws, (size_t)(n2 + TRMAX) * 4);
    signed char *X0 = (signed char *)ws_take(ws, (size_t)NXD * B * Kp);
    signed char *X1 = (signed char *)ws_take(ws, (size_t)NXD * B * Kp);
    int *Mx = (int *)ws_take(ws, (size_t)4 * B * 4);
    unsigned long long *gbits = (unsigned long long *)ws_take(ws, 256);
    struct Release {
        Workspace *w;
        size_t m;
        ~Release() { w->used = m; }
    } release{ws, mark};
    const int tr = shape == 2 ? SmallTile::TR : shape == 1 ? MidTile::TR : shape == 3 ? PairTile::TR : BigTile::TR;
    LB_TRY(fill_i32_launch(reinterpret_cast<int *>(gbits), 2, s));
    if (herm) {
        prep_q_kernel<true><<<n2, 256, 0, s>>>(n, Kp, (n2 + tr - 1) / tr * tr, P, Qd, eP, gbits);
        LB_TRY(check_launch("i8 prep_q"));
        init_x_kernel<true><<<B, 256, 0, s>>>(n, Kp, B, rho, X0, X1, Mx, gbits);
    } else {
        prep_q_kernel<false><<<n2, 256, 0, s>>>(n, Kp, (n2 + tr - 1) / tr * tr, P, Qd, eP, gbits);
        LB_TRY(check_launch("i8 prep_q"));
        init_x_kernel<false><<<B, 256, 0, s>>>(n, Kp, B, rho, X0, X1, Mx, gbits);
    }
    LB_TRY(check_launch("i8 init_x"));
    if (shape == 1)
        return run_tiles<MidTile>(
            n, n2, Kp, B, Qd, eP, X0, X1, Mx, gbits, rho, nsteps, graph, s, (const void *)i8_gemm_mid_kernel<false>,
            (const void *)i8_gemm_mid_kernel<true>, [](bool last, int grid, int lds, hipStream_t st, auto... a) {
                if (last)
                    i8_gemm_mid_kernel<true><<<grid, 256, lds, st>>>(a...);
                else
                    i8_gemm_mid_kernel<false><<<grid, 256, lds, st>>>(a...);
            });
    if (shape == 3)
        return run_tiles<PairTile>(
            n, n2, Kp, B, Qd, eP, X0, X1, Mx, gbits, rho, nsteps, graph, s, (const void *)i8_gemm_pair_kernel<false>,
            (const void *)i8_gemm_pair_kernel<true>, [](bool last, int grid, int lds, hipStream_t st, auto... a) {
                if (last)
                    i8_gemm_pair_kernel<true><<<grid, 256, lds, st>>>(a...);
                else
                    i8_gemm_pair_kernel<false><<<grid, 256, lds, st>>>(a...);
            });
    if (shape == 2)
        return run_tiles<SmallTile>(
            n, n2, Kp, B, Qd, eP, X0, X1, Mx, gbits, rho, nsteps, graph, s, (const void *)i8_gemm_small_kernel<false>,
            (const void *)i8_gemm_small_kernel<true>, [](bool last, int grid, int lds, hipStream_t st, auto... a) {
                if (last)
                    i8_gemm_small_kernel<true><<<grid, 256, lds, st>>>(a...);
                else
                    i8_gemm_small_kernel<false><<<grid, 256, lds, st>>>(a...);
            });
    return run_tiles<BigTile>(
        n, n2, Kp, B, Qd, eP, X0, X1, Mx, gbits, rho, nsteps, graph, s, (const void *)i8_gemm_step_kernel<false>,
        (const void *)i8_gemm_step_kernel<true>, [](bool last, int grid, int lds, hipStream_t st, auto... a) {
            if (last)
                i8_gemm_step_kernel<true><<<grid, 256, lds, st>>>(a...);
            else
                i8_gemm_step_kernel<false><<<grid, 256, lds, st>>>(a...);
        });
}

}  // namespace lb
