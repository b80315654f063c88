// Fused INT8-digit step chain (LB_I8_SLICED) on the INT8 matrix cores
// (v_mfma_i32_16x16x64_i8), the whole chain in one launch with P resident in
// registers as MFMA A fragments.
//
// Representation.  The complex step y = P x is run as its real embedding
//     [yR; yI] = Q [xR; xI],   Q = [[PR, -PI], [PI, PR]]   (2n x 2n),
// so every product is one real GEMM over k < 2n.
//   P:  row r of Q is scaled by 2^-e_r (|Q[r, k]| < 2^e_r) and rounded to the
//       integer V = rint(Q 2^(38 - e_r)), |V| <= 2^38, written as five
//       balanced base-256 digits p_a in [-128, 127] (a = 0 most significant).
//   x:  each state is scaled by 2^-S, S the exponent of its largest |Re|,
//       |Im| (exact for the initial state, the previous state's after
//       that), rounded to the integer V = rint(x 2^(30 - S)) and written as
//       four balanced digits q_b.
// All digit pairs of one level L = a + b <= 4 (14 pairs) accumulate in ONE
// int32 MFMA accumulator: each product is an integer and a level sum is at
// most 5 * 2n * 128^2 < 2^31 for n <= 96 (and for any n <= 1600), so the
// matrix cores add them exactly, over the whole k range.  The levels are
// combined in FP64, y = 2^(e_r + S - 12) sum_L 2^-8L acc_L; y is the state
// of the next step, sliced below the previous state's exponent (the top
// digit has a bit of headroom) and re-sliced below its own exponent only
// when it grew out of that headroom.
//
// Balanced digits come from the two's-complement integer in two operations:
// U = V + 0x80..80 (128 added at every digit below the top one) holds d + 128
// in each low byte and the top digit in the top byte, so U ^ 0x80..80 is the
// digits packed as int8, least significant first.
//
// Work split: 16 states per workgroup (the MFMA N), NW = 8 wavefronts (two
// per SIMD) or 4 (one per SIMD, up to three tiles each); wavefront w owns
// 16-row tiles w, w + NW, ... of Q over all of k, so its outputs end each
// step complete (no partial sums).  Per step and tile: MFMAs (state digits
// read from LDS as B fragments, chunk 0's right after the previous barrier),
// combine in registers, slicing of the tile's rows below the previous
// state's exponent (four consecutive k of one state per lane: each digit
// plane one 4-byte LDS write); then the per-state exponent by LDS maxima and
// one barrier (and a second one in a step where some state outgrew the top
// digit's headroom).  The pipelined form replaces the barrier by per-tile
// progress words in LDS (see the body).
//
// Hermitian states.  The generator of Eq. (1) maps rho^dagger to
// (L rho)^dagger, and so do P = exp(L dt) and its Pade-13 approximant (real
// coefficients), so a density matrix stays Hermitian and is fixed by n = d^2
// real coordinates, h_p = Re rho_p for p = (i, j) with i <= j and
// h_p = Im rho_p for i > j.  On them the step is one real n x n matrix
// (the HERM form, half the rows and half the k of the real embedding):
//     with z = P[r, q]                     for q = (a, a),
//          z = P[r, q] + P[r, q']          for q = (a, b), a < b,
//          z = i (P[r, q] - P[r, q'])      for q = (a, b), a > b,
// (q' = (b, a)), R[r, q] = Re z if row r = (i, j) has i <= j, else Im z.
// The final state is written back as the Hermitian matrix of its
// coordinates: rho_ij = h_(i,j) - i h_(j,i) for i < j, conjugate below.
#include <algorithm>

#include "chain.hpp"

namespace lb {

typedef int i4v __attribute__((ext_vector_type(4)));

namespace i8c {

constexpr int NS = 16;      // states per workgroup (MFMA N)
constexpr int WAVES = 8;    // wavefronts per workgroup (two per SIMD)
constexpr int KCMAX = 3;    // 64-deep k chunks, at most (2n <= 192)
constexpr int MAXN = 96;
constexpr int NPD = 5;      // digits of Q
constexpr int NXD = 4;      // digits of the state
constexpr int LMAX = 4;     // highest level kept: a + b <= 4, 14 pairs
constexpr int FRAC_P = 38;  // fraction bits of Q's row-scaled integer
constexpr int FRAC_X = 30;  // fraction bits of the state's integer
constexpr int EMPTY = -100000;  // exponent of an all-zero state
constexpr double VFIT = 2147483648.0 - 16777216.0;  // |V| below this fits four balanced digits
constexpr int SPIN_LIMIT = 1 << 16;  // polls of a pipelined wait before it gives up (a backstop)
constexpr long long PIPE_MAX_STEPS = 1LL << 28;  // steps per pipelined launch (the counters stay in int)
// y = 2^(e_r + S - YSHIFT) sum_L 2^-8L acc_L: the digits carry weights
// 256^(NPD-1-a) 2^(e_r - FRAC_P) and 256^(NXD-1-b) 2^(S - FRAC_X)
constexpr int YSHIFT = FRAC_P + FRAC_X - 8 * (NPD - 1) - 8 * (NXD - 1);

__device__ inline i4v mma(i4v a, i4v b, i4v c) { return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0); }

// n2: the real dimension of the step (2n for the embedding, n for the
// Hermitian coordinates)
struct Shape {
    int n2, mt, kc, stride, plane;
};

__host__ __device__ inline Shape shape(int n, bool herm = false) {
    Shape s;
    s.n2 = herm ? n : 2 * n;
    s.mt = (s.n2 + 15) / 16;
    s.kc = (s.n2 + 63) / 64;
    s.stride = s.kc * 64 + 32;  // 32 bytes off a multiple of 64: conflict-free 16-byte fragment reads
    s.plane = NS * s.stride;
    return s;
}

// LDS: the state digit buffers ([NBUF][NXD][NS][stride]: two with a
// barrier per step, three when the step is pipelined), the exponent slots
// ([4][NS]), the pipelined step's progress words (per 16-row tile: the
// number of steps whose slicing of that tile is complete; the four tiles of
// a k chunk are one 16-byte word) and re-slice round counter, and the row
// exponents of Q ([mt * 16]).
struct Lds {
    signed char *xdig;
    int *mexp, *prog, *rcnt, *pexp;
};
constexpr int NCNT = 4 * KCMAX + 1;

__host__ __device__ inline size_t lds_ints_offset(const Shape &s, bool pipe) {
    return (size_t)(pipe ? 3 : 2) * NXD * s.plane;
}

__device__ inline Lds lds_layout(unsigned char *smem, const Shape &s, bool pipe) {
    Lds L;
    L.xdig = reinterpret_cast<signed char *>(smem);
    L.mexp = reinterpret_cast<int *>(smem + lds_ints_offset(s, pipe));
    L.prog = L.mexp + 4 * NS;
    L.rcnt = L.prog + 4 * KCMAX;
    L.pexp = L.prog + NCNT;
    return L;
}

inline size_t lds_bytes(int n, bool pipe, bool herm) {
    const Shape s = shape(n, herm);
    return lds_ints_offset(s, pipe) + (4 * NS + NCNT) * sizeof(int) + (size_t)s.mt * 16 * sizeof(int);
}

// exponent e with |v| < 2^e (frexp's), EMPTY for 0
__device__ inline int exp_of(double m) {
    if (!(m > 0.0)) return EMPTY;
    int e;
    (void)frexp(m, &e);
    return e;
}

// Q[R][k] of the real embedding, from P (n x n complex, row-major)
__device__ inline double qval(const cd *__restrict__ P, int n, int R, int k) {
    if (R >= 2 * n || k >= 2 * n) return 0.0;
    const bool rim = R >= n, kim = k >= n;
    const cd v = P[(size_t)(rim ? R - n : R) * n + (kim ? k - n : k)];
    if (!rim) return kim ? -v.im : v.re;
    return kim ? v.re : v.im;
}

// R[r][q] of the Hermitian-coordinate step (n = d^2), from P.  Row r =
// (i, j) takes the real parts of z for i <= j and the imaginary parts
// otherwise, so one component of u = P[r, q] and v = P[r, q'] serves:
// z = u (a = b), u + v (a < b), i (u - v) (a > b); the imaginary parts
// for an upper row with a > b or a lower row with a <= b, else the real.
// Index pairs by multiplying with dm = ceil(2^16 / d): (x dm) >> 16 is
// x / d for every x < 2^16 / d (here x < 192, d <= 13).
__device__ inline double hval(const cd *__restrict__ P, int n, int d, int dm, int r, int q) {
    // branch-free: indices clamped into the matrix, padding selected to 0
    const int rc = min(r, n - 1), qc = min(q, n - 1);
    const int a = (qc * dm) >> 16, b = qc - a * d, i = (rc * dm) >> 16, j = rc - i * d;
    const bool upper = i <= j, below = a > b;
    const double *Pr = reinterpret_cast<const double *>(P + (size_t)rc * n);
    const int c = upper == below ? 1 : 0;
    const double x = Pr[2 * qc + c], y = Pr[2 * (b * d + a) + c];  // y = x on the diagonal
    const double z = a == b ? x : !below ? x + y : upper ? y - x : x - y;
    return r < n && q < n ? z : 0.0;
}

// isqrt of a perfect square n = d^2 (d <= 13 here)
__device__ inline int dim_of(int n) {
    int d = 1;
    while ((d + 1) * (d + 1) <= n) ++d;
    return d;
}

// The chain as run by one wavefront of NW that owns NT row tiles (w, w + NW,
// ...) over KC k chunks (all fixed at compile time, so the step loop has no
// branches).  Every wavefront of the workgroup runs the same number of
// barriers.  A step runs tile by tile: a tile's combine and slicing have no
// dependence on the next tile's MFMAs, so the VALU work of one overlaps the
// matrix-core work of the next within the wavefront.
template <int NT, int KC, int NW, bool PIPE, bool HERM>
__device__ __forceinline__ void i8_body(int n, const cd *__restrict__ P, int B, cd *__restrict__ rho, long long nsteps,
                        unsigned char *smem, int wave, int lane) {
    constexpr int NTA = NT > 0 ? NT : 1;
    const Shape sh = shape(n, HERM);
    const int dd = HERM ? dim_of(n) : 1, dm = (65536 + dd - 1) / dd;
    const Lds lay = lds_layout(smem, sh, PIPE);
    signed char *xdig = lay.xdig;
    int *mexp = lay.mexp;
    int *pexp = lay.pexp;
    const int tid = threadIdx.x;
    const int b0 = blockIdx.x * NS;
    const int s = lane & 15, grp = lane >> 4;
    // the digit layout's strides as constants (the shape's, for 2n in this
    // k chunk count): LDS offsets become instruction immediates
    constexpr int STRIDE = KC * 64 + 32, PLANE = NS * STRIDE, BUF = NXD * PLANE;

    // ---- Q digit fragments of this wavefront's tiles
    i4v pf[NTA][KC][NPD];
#pragma unroll
    for (int tl = 0; tl < NT; ++tl) {
        const int R = (wave + tl * NW) * 16 + (lane & 15);
        const int e = pexp[R];
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            unsigned w[NPD][4];
#pragma unroll
            for (int a = 0; a < NPD; ++a)
#pragma unroll
                for (int i = 0; i < 4; ++i) w[a][i] = 0u;
            if constexpr (HERM) {
                // the Hermitian form gathers two entries per value: one value
                // at a time (a rolled loop), else the hoisted gathers of all
                // sixteen outgrow the registers the step loop leaves
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4) {
                    unsigned wq[NPD] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll 1
                    for (int q = 0; q < 4; ++q) {
                        const int k = c * 64 + grp * 16 + 4 * q4 + q;
                        const long long V = (long long)rint(ldexp(hval(P, n, dd, dm, R, k), FRAC_P - e));
                        const unsigned long long U = (unsigned long long)(V + 0x80808080LL);
#pragma unroll
                        for (int j = 0; j < NPD; ++j) {  // j = 0 least significant
                            const unsigned byte = j < NPD - 1
                                                      ? (unsigned)((U >> (8 * j)) & 0xFFu) ^ 0x80u
                                                      : (unsigned)((unsigned long long)((long long)U >> 32) & 0xFFu);
                            wq[NPD - 1 - j] |= byte << (8 * q);
                        }
                    }
#pragma unroll
                    for (int a = 0; a < NPD; ++a) w[a][q4] = wq[a];
                }
            } else {
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int k = c * 64 + grp * 16 + q;
                    const long long V = (long long)rint(ldexp(qval(P, n, R, k), FRAC_P - e));
                    const unsigned long long U = (unsigned long long)(V + 0x80808080LL);
#pragma unroll
                    for (int j = 0; j < NPD; ++j) {  // j = 0 least significant
                        const unsigned byte = j < NPD - 1
                                                  ? (unsigned)((U >> (8 * j)) & 0xFFu) ^ 0x80u
                                                  : (unsigned)((unsigned long long)((long long)U >> 32) & 0xFFu);
                        w[NPD - 1 - j][q >> 2] |= byte << (8 * (q & 3));
                    }
                }
            }
#pragma unroll
            for (int a = 0; a < NPD; ++a) pf[tl][c][a] = i4v{(int)w[a][0], (int)w[a][1], (int)w[a][2], (int)w[a][3]};
        }
    }

    // ---- output rows of this lane: tile (wave + 8 tl), register r -> row 16 (wave + 8 tl) + 4 grp + r
    int pe[NTA][4];  // their row exponents
#pragma unroll
    for (int tl = 0; tl < NT; ++tl)
#pragma unroll
        for (int r = 0; r < 4; ++r) pe[tl][r] = pexp[(wave + tl * NW) * 16 + grp * 4 + r];
    // y: the initial state, then each step's combined levels v (the step's
    // output is v 2^(pe + Sx - YSHIFT), formed only after the last step)
    double y[NTA][4];
    // The digits of V = rint(y 2^(off + shift)) (off = the row exponent for a
    // step's v, 0 for the initial state) into buffer `to`, four consecutive k
    // of one state per lane: one word per plane.  Rounding to nearest even by
    // adding 1.5 2^52 (exact for |V| < 2^51: the sum's low 32 bits are V in
    // two's complement; a V past the 31-bit range only occurs in a state that
    // is re-sliced after the barrier).  Returns max |y 2^(off + shift)| over the
    // lane's values, unrounded: its exponent is the state's exponent plus the
    // same shift, exactly.
    auto slice = [&](int tl, bool rows, int shift, int to) {
        double vmax = 0.0;
        {
            unsigned W[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double u = ldexp(y[tl][r], (rows ? pe[tl][r] : 0) + shift);
                vmax = fmax(vmax, fabs(u));
                const unsigned V = (unsigned)__double_as_longlong(u + 0x1.8p52);
                W[r] = (V + 0x00808080u) ^ 0x00808080u;  // digits, least significant first
            }
            // byte transpose: E[j] holds digit j of the four values, value r in byte r
            const unsigned A0 = __builtin_amdgcn_perm(W[1], W[0], 0x06020400u);  // bytes 0, 2 of W0, W1
            const unsigned A1 = __builtin_amdgcn_perm(W[1], W[0], 0x07030501u);  // bytes 1, 3
            const unsigned C0 = __builtin_amdgcn_perm(W[3], W[2], 0x06020400u);
            const unsigned C1 = __builtin_amdgcn_perm(W[3], W[2], 0x07030501u);
            const unsigned E[4] = {__builtin_amdgcn_perm(C0, A0, 0x05040100u), __builtin_amdgcn_perm(C1, A1, 0x05040100u),
                                   __builtin_amdgcn_perm(C0, A0, 0x07060302u), __builtin_amdgcn_perm(C1, A1, 0x07060302u)};
            const int k0 = (wave + tl * NW) * 16 + grp * 4;
#pragma unroll
            for (int b = 0; b < NXD; ++b)  // b = 0 most significant
                *reinterpret_cast<unsigned *>(xdig + to * BUF + b * PLANE + s * STRIDE + k0) = E[NXD - 1 - b];
        }
        return vmax;
    };
    // The exponent slot's entry for the lane's rows from slice's maximum
    // |V| (taken below exponent S; EMPTY for zeros); the lane groups meet in
    // the LDS maximum.  It is the frexp exponent of the largest |y|, except
    // that a |V| of VFIT = 2^31 - 2^24 or more (four balanced base-256
    // digits reach 127 (256^4 - 1) / 255, about 0.996 2^31) counts one
    // higher.  So the digits just written are good while the slot is at most
    // S + 1 (a state may grow to nearly twice 2^S: the top digit's
    // headroom), and a slot of S + 2 or more calls for re-slicing below it.
    auto exp_slot = [&](double vmax, int S) {
        if (!(vmax > 0.0)) return EMPTY;
        return __builtin_amdgcn_frexp_exp(vmax) - FRAC_X + S + (vmax >= VFIT && vmax < 0x1p31 ? 1 : 0);
    };
    // chunk c's state digits (one B fragment per digit plane) from buffer
    // `from`; the volatile form is for the reads issued early on purpose
    // (the compiler would otherwise sink them to their first use)
    auto fetch_x = [&](int from, int c, i4v (&xf)[NXD], bool early) {
#pragma unroll
        for (int b = 0; b < NXD; ++b) {
            const i4v *q = reinterpret_cast<const i4v *>(xdig + from * BUF + b * PLANE + s * STRIDE +
                                                         c * 64 + grp * 16);
            xf[b] = early ? *(const volatile __attribute__((address_space(3))) i4v *)(q) : *q;
        }
    };

    // ---- initial state: its exact exponent, digits into buffer 0
    int m0 = EMPTY;
#pragma unroll
    for (int tl = 0; tl < NT; ++tl)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            y[tl][r] = 0.0;
            const int k = (wave + tl * NW) * 16 + grp * 4 + r;
            if (k < sh.n2 && b0 + s < B) {
                if constexpr (HERM) {
                    const cd v = rho[(size_t)(b0 + s) * n + k];
                    const int i = (k * dm) >> 16, j = k - i * dd;
                    y[tl][r] = i <= j ? v.re : v.im;
                } else {
                    const cd v = rho[(size_t)(b0 + s) * n + (k < n ? k : k - n)];
                    y[tl][r] = k < n ? v.re : v.im;
                }
            }
            m0 = max(m0, exp_of(fabs(y[tl][r])));
        }
    if (NT > 0) atomicMax(mexp + s, m0);
    __syncthreads();
    int Sx = mexp[s] == EMPTY ? 0 : mexp[s];  // the exponent the current state's digits were sliced with
#pragma unroll
    for (int tl = 0; tl < NT; ++tl) (void)slice(tl, false, FRAC_X - Sx, 0);
    __syncthreads();
    if constexpr (PIPE) {
        // ---- pipelined steps, no barrier: a wavefront starts the MFMAs of
        // step t on k chunk c as soon as the tiles of step t - 1 covering
        // chunk c are sliced (each tile's progress word, written after the
        // tile's digit and exponent writes), so one wavefront's combine and
        // slicing overlap the others' MFMAs across the step boundary.  Wavefronts
        // are at most one step apart (a step waits for every tile of the
        // previous one), so three digit buffers suffice: step t reads buffer
        // t mod 3 and writes t + 1 mod 3, whose readers (step t - 2) have
        // all finished.  M_t is complete once all of step t - 1's tiles are;
        // a state that outgrew the exponent it was sliced below (slot M_t
        // two or more above it) is re-sliced by every wavefront from the kept levels, the
        // wavefronts meet on a round counter, and the first tile's MFMAs are
        // redone.  Waves without tiles leave after the prologue.  Eight
        // wavefronts only (the four-wavefront body would spill).
        if (NT == 0) return;
        const int na = sh.mt < NW ? sh.mt : NW;  // wavefronts with tiles
        // Ordering: one wavefront's LDS instructions execute in issue order,
        // so a progress word written after a tile's digit and exponent
        // writes is seen only after them, and a read issued after a progress
        // read sees everything that value stands for.  The words are plain
        // LDS stores (every lane stores the same value: no branch in the
        // instruction stream) and volatile reads, behind compiler-only
        // fences: no hardware wait in the release, none in the acquire
        // beyond the read's own latency.
        auto ld = [&](const int *p) { return *(const volatile __attribute__((address_space(3))) int *)(p); };
        auto publish = [&](int *p, int v) {
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            *(volatile __attribute__((address_space(3))) int *)(p) = v;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
        };
        // the least progress of chunk c's four tiles
        auto chunk_prog = [&](int c) {
            const i4v v = *(const volatile __attribute__((address_space(3))) i4v *)(lay.prog + 4 * c);
            return min(min(v[0], v[1]), min(v[2], v[3]));
        };
        // bounded wait: every wait ends once the wavefronts it waits for
        // finish their part of the previous step, which waits on nothing
        // later; the bound (a few ms) is a backstop, after which this
        // wavefront stops waiting altogether so that the launch still ends
        bool stalled = false;
        auto wait_chunk = [&](int c, int need) {
            if (stalled) return;
            for (int it = 0;; ++it) {
                if (__builtin_amdgcn_readfirstlane(chunk_prog(c)) >= need) return;
                if (it == SPIN_LIMIT) break;
                __builtin_amdgcn_s_sleep(1);
            }
            stalled = true;
        };
        auto wait_rounds = [&](int need) {
            if (stalled) return;
            for (int it = 0;; ++it) {
                if (__builtin_amdgcn_readfirstlane(ld(lay.rcnt)) >= need) return;
                if (it == SPIN_LIMIT) break;
                __builtin_amdgcn_s_sleep(1);
            }
            stalled = true;
        };
        int Sspec = mexp[s] == EMPTY ? 0 : mexp[s];  // the exponent x_t+1 is sliced below (M_t)
        int shs = 0;
        int nredo = 0;
        int bc = 0;  // buffer of the current state
        i4v xa[KC][NXD];
        i4v acc[LMAX + 1];
        auto mfma_chunk = [&](int tl, int c) {
#pragma unroll
            for (int a = 0; a < NPD; ++a)
#pragma unroll
                for (int b = 0; b < NXD; ++b)
                    if (a + b <= LMAX) acc[a + b] = mma(pf[tl][c][a], xa[c][b], acc[a + b]);
        };
        auto zero_acc = [&]() {
#pragma unroll
            for (int L = 0; L <= LMAX; ++L) acc[L] = i4v{0, 0, 0, 0};
        };
        // One step; `last` (a constant at both call sites) drops the
        // slicing, so the tile loop has no branch between the MFMAs.
        auto step = [&](long long t, bool last) {
            const int ti = (int)t;
            const int bn = bc == 2 ? 0 : bc + 1;
            // slot t + 2 (read last in step t - 2, written from step t + 1
            // on, after every wavefront has passed this point): cleared
            // by every wavefront, four lanes per state, without a branch
            *(volatile __attribute__((address_space(3))) int *)(mexp + ((t + 2) & 3) * NS + s) = EMPTY;
            // ---- first tile.  Every chunk's counter and digits are read in
            // one go (the digits are good if the counter read before them
            // was); the chunks but the last hold tiles that each wavefront
            // slices first, so they are in; the last chunk's counter is read
            // again under chunk 0's MFMAs, with M_t behind it.
            int have[KC];
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                have[c] = chunk_prog(c);
                fetch_x(bc, c, xa[c], true);
            }
            bool early_in = true;
#pragma unroll
            for (int c = 0; c + 1 < KC; ++c) early_in = early_in && have[c] >= ti;
            if (!__builtin_amdgcn_readfirstlane(early_in)) {
#pragma unroll
                for (int c = 0; c + 1 < KC; ++c) {
                    wait_chunk(c, ti);
                    fetch_x(bc, c, xa[c], true);
                }
            }
            zero_acc();
            int last_have = have[KC - 1];
            int Mt = 0;
            if (KC > 1) {
                mfma_chunk(0, 0);
                last_have = chunk_prog(KC - 1);
                fetch_x(bc, KC - 1, xa[KC - 1], true);
                Mt = ld(mexp + (t & 3) * NS + s);
#pragma unroll
                for (int c = 1; c + 1 < KC; ++c) mfma_chunk(0, c);
            } else {
                Mt = ld(mexp + (t & 3) * NS + s);
            }
            if (__builtin_amdgcn_readfirstlane(last_have) < ti) {
                wait_chunk(KC - 1, ti);
                fetch_x(bc, KC - 1, xa[KC - 1], true);
                Mt = ld(mexp + (t & 3) * NS + s);
            }
            if (KC == 1) zero_acc();
            mfma_chunk(0, KC - 1);
            if (t > 0) {
                // every tile of step t - 1 is in: M_t is complete
                const bool over = Mt > Sspec + 1;  // false for a zero state (EMPTY)
                if (__builtin_amdgcn_ballot_w64(over) != 0) {  // the same vote in every wavefront
                    if (over) {
#pragma unroll
                        for (int tl = 0; tl < NT; ++tl) (void)slice(tl, true, shs + Sspec - Mt, bc);
                    }
                    ++nredo;
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    if (lane == 0)
                        __hip_atomic_fetch_add((__attribute__((address_space(3))) int *)(lay.rcnt), 1, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    wait_rounds(na * nredo);
#pragma unroll
                    for (int c = 0; c < KC; ++c) fetch_x(bc, c, xa[c], true);
                    zero_acc();
#pragma unroll
                    for (int c = 0; c < KC; ++c) mfma_chunk(0, c);
                }
                Sx = over ? Mt : Sspec;
                Sspec = Mt == EMPTY ? 0 : Mt;
            }
            shs = Sx - YSHIFT + FRAC_X - Sspec;  // V = v 2^(pe + shs)
#pragma unroll
            for (int tl = 0; tl < NT; ++tl) {
                if (tl > 0) {
                    zero_acc();
#pragma unroll
                    for (int c = 0; c < KC; ++c) mfma_chunk(tl, c);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double v = (double)acc[LMAX][r];
#pragma unroll
                    for (int L = LMAX - 1; L >= 0; --L) v = fma(v, 1.0 / 256.0, (double)acc[L][r]);
                    y[tl][r] = v;
                }
                if (!last) {
                    const double vmax = slice(tl, true, shs, bn);
                    atomicMax(mexp + ((t + 1) & 3) * NS + s, exp_slot(vmax, Sspec));
                    publish(lay.prog + wave + tl * NW, ti + 1);
                }
            }
            bc = bn;
        };
        for (long long t = 0; t + 1 < nsteps; ++t) step(t, false);
        step(nsteps - 1, true);
    } else {
        i4v x0[NXD];  // chunk 0 of the current state, fetched right after the barrier that completes it
        fetch_x(0, 0, x0, true);
        // M_t: frexp exponent of the current state's largest entry (EMPTY for a
        // zero state), read together with chunk 0 after the barrier
        int Mt = mexp[s];

        for (long long t = 0; t < nsteps; ++t) {
            const int cur = (int)(t & 1);
            // the other chunks of the current state, for every tile
            i4v xa[KC][NXD];
#pragma unroll
            for (int b = 0; b < NXD; ++b) xa[0][b] = x0[b];
#pragma unroll
            for (int c = 1; c < KC; ++c) fetch_x(cur, c, xa[c], false);
            // ---- per tile: MFMAs, combine (Horner, smallest level first), and
            // the slicing of the tile's rows below the previous state's exponent
            // M_t (speculative: a state that grows past the top digit's
            // headroom in one step, slot M_t+1 > M_t + 1, is re-sliced below
            // the slot after the barrier).  The last step's slicing is not read.
            const int Sspec = Mt == EMPTY ? 0 : Mt;
            const int shs = Sx - YSHIFT + FRAC_X - Sspec;  // V = v 2^(pe + shs)
            double vmax = 0.0;
#pragma unroll
            for (int tl = 0; tl < NT; ++tl) {
                i4v acc[LMAX + 1];
#pragma unroll
                for (int L = 0; L <= LMAX; ++L) acc[L] = i4v{0, 0, 0, 0};
#pragma unroll
                for (int c = 0; c < KC; ++c)
#pragma unroll
                    for (int a = 0; a < NPD; ++a)
#pragma unroll
                        for (int b = 0; b < NXD; ++b)
                            if (a + b <= LMAX) acc[a + b] = mma(pf[tl][c][a], xa[c][b], acc[a + b]);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double v = (double)acc[LMAX][r];
#pragma unroll
                    for (int L = LMAX - 1; L >= 0; --L) v = fma(v, 1.0 / 256.0, (double)acc[L][r]);
                    y[tl][r] = v;
                }
                vmax = fmax(vmax, slice(tl, true, shs, cur ^ 1));
            }
            if (t + 1 == nsteps) break;  // uniform
            if (NT > 0) atomicMax(mexp + ((t + 1) & 3) * NS + s, exp_slot(vmax, Sspec));
            if (tid < NS) *(volatile __attribute__((address_space(3))) int *)(mexp + ((t + 2) & 3) * NS + tid) = EMPTY;  // read last in step t - 2
            __syncthreads();
            fetch_x(cur ^ 1, 0, x0, true);  // with M_t+1: one LDS round trip
            const int Mn = *(const volatile __attribute__((address_space(3))) int *)(mexp + ((t + 1) & 3) * NS + s);
            Sx = Sspec;
            Mt = Mn;
            // every wavefront holds all 16 states (lane & 15), so the vote is
            // the same in all of them: uniform over the workgroup
            const bool over = Mn > Sspec + 1;  // false for a zero state (EMPTY)
            if (__builtin_amdgcn_ballot_w64(over) != 0) {
                if (over) {
#pragma unroll
                    for (int tl = 0; tl < NT; ++tl) (void)slice(tl, true, shs + Sspec - Mn, cur ^ 1);
                    Sx = Mn;
                }
                __syncthreads();
                fetch_x(cur ^ 1, 0, x0, true);
            }
        }
    }
    // the output, y = v 2^(pe + Sx - YSHIFT)
#pragma unroll
    for (int tl = 0; tl < NT; ++tl)
#pragma unroll
        for (int r = 0; r < 4; ++r) y[tl][r] = ldexp(y[tl][r], pe[tl][r] + Sx - YSHIFT);
    // ---- write the final state
#pragma unroll
    for (int tl = 0; tl < NT; ++tl)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = (wave + tl * NW) * 16 + grp * 4 + r;
            if (k < sh.n2 && b0 + s < B) {
                if constexpr (HERM) {
                    // h_(i,j) is Re rho_ij = Re rho_ji (i <= j), or Im rho_ij = -Im rho_ji (i > j)
                    const int i = (k * dm) >> 16, j = k - i * dd;
                    double *o = reinterpret_cast<double *>(rho + (size_t)(b0 + s) * n);
                    if (i == j) {
                        o[2 * k] = y[tl][r];
                        o[2 * k + 1] = 0.0;
                    } else {
                        const int kt = j * dd + i, c = i < j ? 0 : 1;
                        o[2 * k + c] = y[tl][r];
                        o[2 * kt + c] = c ? -y[tl][r] : y[tl][r];
                    }
                } else {
                    double *o = reinterpret_cast<double *>(rho + (size_t)(b0 + s) * n + (k < n ? k : k - n));
                    o[k < n ? 0 : 1] = y[tl][r];
                }
            }
        }
}

template <int NW, bool PIPE, bool HERM>
__global__ void __launch_bounds__(NW * 64) i8_chain_kernel(int n, const cd *__restrict__ P, int B,
                                                           cd *__restrict__ rho, long long nsteps) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Shape sh = shape(n, HERM);
    const Lds lay = lds_layout(smem, sh, PIPE);
    int *mexp = lay.mexp;
    int *pexp = lay.pexp;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // ---- row exponents of Q (rows r and r + n share one; the Hermitian
    // form's rows each their own), cleared buffers and slots
    const int dd = HERM ? dim_of(n) : 1, dm = (65536 + dd - 1) / dd;
    for (int R = tid; R < sh.mt * 16; R += NW * 64) {
        int e = 0;
        if (R < sh.n2) {
            double m = 0.0;
            if constexpr (HERM) {
                for (int k = 0; k < n; ++k) m = fmax(m, fabs(hval(P, n, dd, dm, R, k)));
            } else {
                const int r = R < n ? R : R - n;
                for (int k = 0; k < n; ++k) {
                    const cd v = P[(size_t)r * n + k];
                    m = fmax(m, fmax(fabs(v.re), fabs(v.im)));
                }
            }
            e = m > 0.0 ? exp_of(m) : 0;
        }
        pexp[R] = e;
    }
    for (int i = tid; i < (int)(lds_ints_offset(sh, PIPE) / 4); i += NW * 64) reinterpret_cast<int *>(smem)[i] = 0;
    if (tid < 4 * NS) mexp[tid] = EMPTY;
    // progress: 0 for every tile that exists, never waited on past the last
    if (tid < NCNT) lay.prog[tid] = tid < 4 * KCMAX && tid >= sh.mt ? 0x7fffffff : 0;
    if (nsteps == 0) return;  // uniform
    __syncthreads();
    const int ntile = wave < sh.mt ? (sh.mt - wave + NW - 1) / NW : 0;
    // wave-uniform dispatch to the compile-time shape (only the pairs that
    // occur for 2n <= 192: the kernel's registers are the largest body's)
    if constexpr (NW == 8) {
        switch (ntile * 4 + sh.kc) {
            case 0 * 4 + 1: i8_body<0, 1, NW, PIPE, HERM>(n, P, B, rho, nsteps, smem, wave, lane); break;
            case 1 * 4 + 1: i8_body<1, 1, NW, PIPE, HERM>(n, P, B, rho, nsteps, smem, wave, lane); break;
            case 0 * 4 + 2: i8_body<0, 2, NW, PIPE, HERM>(n, P, B, rho, nsteps, smem, wave, lane); break;
            case 1 * 4 + 2: i8_body<1, 2, NW, PIPE, HERM>(n, P, B, rho, nsteps, smem, wave, lane); break;
            case 1 * 4 + 3: i8_body<1, 3, NW, PIPE, HERM>(n, P, B, rho, nsteps, smem, wave, lane); break;
            default: i8_body<2, 3, NW, PIPE, HERM>(n, P, B, rho, nsteps, smem, wave, lane); break;
        }
    } else {
        static_assert(NW == 4, "four or eight wavefronts");
        switch (ntile * 4 + sh.kc) {
            case 0 * 4 + 1: i8_body<0, 1, NW, PIPE, HERM>(n, P, B, rho, nsteps, smem, wave, lane); break;
            case 1 * 4 + 1: i8_body<1, 1, NW, PIPE, HERM>(n, P, B, rho, nsteps, smem, wave, lane); break;
            case 1 * 4 + 2: i8_body<1, 2, NW, PIPE, HERM>(n, P, B, rho, nsteps, smem, wave, lane); break;
            case 2 * 4 + 2: i8_body<2, 2, NW, PIPE, HERM>(n, P, B, rho, nsteps, smem, wave, lane); break;
            case 2 * 4 + 3: i8_body<2, 3, NW, PIPE, HERM>(n, P, B, rho, nsteps, smem, wave, lane); break;
            default: i8_body<3, 3, NW, PIPE, HERM>(n, P, B, rho, nsteps, smem, wave, lane); break;
        }
    }
}

// ------------------------------------------------------------------
// Fixed-point chain (Alg. 5) on the INT8 matrix cores: P and the state in
// Q1.F (F = 15 or 31: a value v is the integer code c = v 2^F; P and the
// incoming states quantised by round-to-nearest (ties to even) with
// saturation to [-2^F, 2^F - 1]).  The real embedding's codes (the -Im P
// block negated after quantisation, so its codes reach 2^F) and the state
// codes are written as ND balanced base-256 digits (ND = 3 for F = 15, 5 for
// F = 31: enough that every code, negated or not, is in range), ALL ND^2
// digit pairs are summed in 2 ND - 1 level accumulators (each exact in
// int32), and the levels are combined exactly in 128-bit integers:
//     acc_r = sum_k Q_rk x_k = sum_L acc_L 256^(2 ND - 2 - L),
// then x_r = sat(floor(acc_r / 2^F)) -- the oracle's integer step bit for
// bit, whatever the summation order.  Same tiling as the sliced chain, one
// barrier per step (no exponent to agree on).
template <int ND, int FRAC, int TPWF>
__global__ void __launch_bounds__(WAVES * 64) fx_chain_kernel(int n, const cd *__restrict__ P, int B,
                                                              cd *__restrict__ rho, long long nsteps) {
    constexpr int NL = 2 * ND - 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const Shape sh = shape(n);
    signed char *xdig = reinterpret_cast<signed char *>(smem);  // [ND][NS][stride]
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int b0 = blockIdx.x * NS;
    const int s = lane & 15, grp = lane >> 4;
    const long long cmax = (1LL << FRAC) - 1, cmin = -(1LL << FRAC);
    auto quant = [&](double v) {  // round to nearest (ties to even), saturate
        return (long long)fmax((double)cmin, fmin((double)cmax, rint(ldexp(v, FRAC))));
    };
    // code of Q[R][k]: quantised parts of P, the -Im block negated afterwards
    auto qcode = [&](int R, int k) -> long long {
        if (R >= sh.n2 || k >= sh.n2) return 0;
        const bool rim = R >= n, kim = k >= n;
        const cd v = P[(size_t)(rim ? R - n : R) * n + (kim ? k - n : k)];
        if (!rim) return kim ? -quant(v.im) : quant(v.re);
        return kim ? quant(v.re) : quant(v.im);
    };
    // ND balanced digits of |c| <= 2^(8 ND - 1) - 2^(8 ND - 9): byte j of
    // c + 0x80..80 (ND - 1 offsets) xor 0x80 for j < ND - 1, the top digit by
    // an arithmetic shift; returned packed per digit, least significant first
    auto digit = [&](long long c, int j) -> unsigned {
        long long off = 0;
#pragma unroll
        for (int i = 0; i < ND - 1; ++i) off |= 0x80LL << (8 * i);
        const long long U = c + off;
        if (j < ND - 1) return (unsigned)((U >> (8 * j)) & 0xFF) ^ 0x80u;
        return (unsigned)((U >> (8 * (ND - 1))) & 0xFF);
    };

    for (int i = tid; i < ND * sh.plane / 4; i += WAVES * 64) reinterpret_cast<int *>(xdig)[i] = 0;
    __syncthreads();

    const int ntile = (wave < sh.mt ? 1 : 0) + (TPWF > 1 && wave + WAVES < sh.mt ? 1 : 0);
    i4v pf[TPWF][KCMAX][ND];
#pragma unroll
    for (int tl = 0; tl < TPWF; ++tl)
#pragma unroll
        for (int c = 0; c < KCMAX; ++c)
#pragma unroll
            for (int a = 0; a < ND; ++a) pf[tl][c][a] = i4v{0, 0, 0, 0};
#pragma unroll
    for (int tl = 0; tl < TPWF; ++tl) {
        if (tl < ntile) {
            const int R = (wave + tl * WAVES) * 16 + (lane & 15);
#pragma unroll
            for (int c = 0; c < KCMAX; ++c) {
                if (c < sh.kc) {
                    unsigned w[ND][4];
#pragma unroll
                    for (int a = 0; a < ND; ++a)
#pragma unroll
                        for (int i = 0; i < 4; ++i) w[a][i] = 0u;
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const long long code = qcode(R, c * 64 + grp * 16 + q);
#pragma unroll
                        for (int j = 0; j < ND; ++j) w[ND - 1 - j][q >> 2] |= digit(code, j) << (8 * (q & 3));
                    }
#pragma unroll
                    for (int a = 0; a < ND; ++a)
                        pf[tl][c][a] = i4v{(int)w[a][0], (int)w[a][1], (int)w[a][2], (int)w[a][3]};
                }
            }
        }
    }

    long long x[TPWF][4];  // state codes of this lane's rows
    auto publish = [&]() {
#pragma unroll
        for (int tl = 0; tl < TPWF; ++tl) {
            if (tl < ntile) {
                const int k0 = (wave + tl * WAVES) * 16 + grp * 4;
#pragma unroll
                for (int b = 0; b < ND; ++b) {  // b = 0 most significant
                    unsigned D = 0u;
#pragma unroll
                    for (int r = 0; r < 4; ++r) D |= digit(x[tl][r], ND - 1 - b) << (8 * r);
                    *reinterpret_cast<unsigned *>(xdig + (size_t)b * sh.plane + s * sh.stride + k0) = D;
                }
            }
        }
        __syncthreads();
    };

#pragma unroll
    for (int tl = 0; tl < TPWF; ++tl)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            x[tl][r] = 0;
            const int k = (wave + tl * WAVES) * 16 + grp * 4 + r;
            if (tl < ntile && k < sh.n2 && b0 + s < B) {
                const cd v = rho[(size_t)(b0 + s) * n + (k < n ? k : k - n)];
                x[tl][r] = quant(k < n ? v.re : v.im);
            }
        }
    if (nsteps == 0) return;
    publish();

    for (long long t = 0; t < nsteps; ++t) {
        i4v acc[TPWF][NL];
#pragma unroll
        for (int tl = 0; tl < TPWF; ++tl)
#pragma unroll
            for (int L = 0; L < NL; ++L) acc[tl][L] = i4v{0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < KCMAX; ++c) {
            if (c < sh.kc) {
                i4v xf[ND];
#pragma unroll
                for (int b = 0; b < ND; ++b)
                    xf[b] = *reinterpret_cast<const i4v *>(xdig + (size_t)b * sh.plane + s * sh.stride + c * 64 +
                                                           grp * 16);
#pragma unroll
                for (int a = 0; a < ND; ++a)
#pragma unroll
                    for (int b = 0; b < ND; ++b)
#pragma unroll
                        for (int tl = 0; tl < TPWF; ++tl)
                            if (tl < ntile) acc[tl][a + b] = mma(pf[tl][c][a], xf[b], acc[tl][a + b]);
            }
        }
        __syncthreads();  // every wavefront's fragment reads are done before the digits are rewritten
#pragma unroll
        for (int tl = 0; tl < TPWF; ++tl) {
            if (tl < ntile) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    __int128 Y = 0;
#pragma unroll
                    for (int L = 0; L < NL; ++L) Y += (__int128)acc[tl][L][r] << (8 * (NL - 1 - L));
                    const __int128 q = Y >> FRAC;  // floor division by 2^F
                    x[tl][r] = q < (__int128)cmin ? cmin : (q > (__int128)cmax ? cmax : (long long)q);
                }
            }
        }
        if (t + 1 == nsteps) break;  // uniform
        publish();
    }
#pragma unroll
    for (int tl = 0; tl < TPWF; ++tl)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = (wave + tl * WAVES) * 16 + grp * 4 + r;
            if (tl < ntile && k < sh.n2 && b0 + s < B) {
                double *o = reinterpret_cast<double *>(rho + (size_t)(b0 + s) * n + (k < n ? k : k - n));
                o[k < n ? 0 : 1] = ldexp((double)x[tl][r], -FRAC);
            }
        }
}

static const size_t kLds = 160 * 1024;

}  // namespace i8c

int i8_fused_max_n() { return i8c::MAXN; }
int fx_i8_max_n() { return i8c::MAXN; }

// Alg. 5 on the INT8 matrix cores (LB_Q15: 3 digits, LB_Q31: 5 digits);
// one 16-row tile per wavefront up to n = 64, two up to 96.
int chain_fx_i8(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, hipStream_t s) {
    using namespace i8c;
    if (n > MAXN) return fail(LB_ESHAPE, "fixed-point INT8 chain: n <= 96");
    if (prec != LB_Q15 && prec != LB_Q31) return fail(LB_EINVAL, "fixed-point INT8 chain: LB_Q15 or LB_Q31");
    if (nsteps == 0 || B == 0) return LB_OK;
    const int nd = prec == LB_Q15 ? 3 : 5;
    const size_t lds = (size_t)nd * shape(n).plane;
    const dim3 grid((B + NS - 1) / NS), block(WAVES * 64);
    const bool two = shape(n).mt > WAVES;
    if (prec == LB_Q15) {
        if (two)
            fx_chain_kernel<3, 15, 2><<<grid, block, lds, s>>>(n, P, B, rho, nsteps);
        else
            fx_chain_kernel<3, 15, 1><<<grid, block, lds, s>>>(n, P, B, rho, nsteps);
    } else {
        if (two)
            fx_chain_kernel<5, 31, 2><<<grid, block, lds, s>>>(n, P, B, rho, nsteps);
        else
            fx_chain_kernel<5, 31, 1><<<grid, block, lds, s>>>(n, P, B, rho, nsteps);
    }
    return check_launch("fx_i8_chain");
}

int i8_herm_fused_max_n() { return 2 * i8c::MAXN; }

bool i8_herm_shape_ok(int n) {
    int d = 1;
    while ((d + 1) * (d + 1) <= n) ++d;
    return n >= 1 && d * d == n;
}

int chain_i8_fused(int n, const cd *P, int B, cd *rho, long long nsteps, hipStream_t s, int waves, bool pipe,
                   bool herm) {
    using namespace i8c;
    if (herm && !i8_herm_shape_ok(n)) return fail(LB_ESHAPE, "i8 Hermitian chain: n must be d^2");
    if (n > (herm ? 2 * MAXN : MAXN)) return fail(LB_ESHAPE, "i8 chain: n too large for the fused kernel");
    if (waves != 4 && waves != 8) return fail(LB_EINVAL, "i8 chain: 4 or 8 wavefronts per workgroup");
    if (pipe && waves != 8) return fail(LB_EINVAL, "i8 chain: the pipelined step runs eight wavefronts");
    if (nsteps == 0 || B == 0) return LB_OK;
    const size_t lds = lds_bytes(n, pipe, herm);
    const int grid = (B + NS - 1) / NS;
    // a pipelined launch counts tiles in int: longer chains run as several
    // launches (each starts from its state's exact exponent)
    for (long long done = 0; done < nsteps;) {
        const long long k = pipe ? std::min(nsteps - done, PIPE_MAX_STEPS) : nsteps - done;
        if (herm) {
            if (pipe)
                i8_chain_kernel<8, true, true><<<grid, 8 * 64, lds, s>>>(n, P, B, rho, k);
            else if (waves == 8)
                i8_chain_kernel<8, false, true><<<grid, 8 * 64, lds, s>>>(n, P, B, rho, k);
            else
                i8_chain_kernel<4, false, true><<<grid, 4 * 64, lds, s>>>(n, P, B, rho, k);
        } else if (pipe)
            i8_chain_kernel<8, true, false><<<grid, 8 * 64, lds, s>>>(n, P, B, rho, k);
        else if (waves == 8)
            i8_chain_kernel<8, false, false><<<grid, 8 * 64, lds, s>>>(n, P, B, rho, k);
        else
            i8_chain_kernel<4, false, false><<<grid, 4 * 64, lds, s>>>(n, P, B, rho, k);
        done += k;
    }
    return check_launch("i8_chain");
}

}  // namespace lb
