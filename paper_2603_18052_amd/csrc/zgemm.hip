// Batched complex FP64 GEMM on the FP64 matrix cores (v_mfma_f64_16x16x4f64)
// with a fused linear-combination epilogue.
//
// Tile: 64 x 64 outputs per workgroup of 256 threads (4 wavefronts as 2 x 2),
// each wavefront owns 32 x 32 outputs = 2 x 2 MFMA blocks, each with a real
// and an imaginary FP64 accumulator.  A complex product takes four real MFMAs:
//   C.re += A.re B.re,  C.re += (-A.im) B.im,  C.im += A.re B.im,  C.im += A.im B.re.
// K advances 16 at a time through LDS, stored planar (re / im) and k-major so
// that each MFMA operand fetch is 16 consecutive doubles per k row; the next
// tile is prefetched into registers while the current one is multiplied.
//
// MFMA f64 16x16x4 lane layout (gfx950): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l is D[l / 16 + 4 r][l % 16].
#include "lb_internal.hpp"

namespace lb {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64, TK = 16;
constexpr int APAD = TM + 1;  // padded k-major row of the A tile (LDS bank spread)

__device__ inline d4 mfma64(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

__global__ void __launch_bounds__(256) zgemm_kernel(ZgemmBatch g, int tiles_n) {
    const int b = blockIdx.y;
    if (g.active && g.active[b] <= g.level) return;  // uniform per workgroup
    const int tm = blockIdx.x / tiles_n, tn = blockIdx.x - tm * tiles_n;
    const int row0 = tm * TM, col0 = tn * TN;
    const cd *__restrict__ A = g.A + (size_t)b * g.sA;
    const cd *__restrict__ B = g.B + (size_t)b * g.sB;

    __shared__ double As_re[TK][APAD], As_im[TK][APAD];
    __shared__ double Bs_re[TK][TN], Bs_im[TK][TN];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    d4 acc_re[2][2], acc_im[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            acc_re[i][j] = d4{0.0, 0.0, 0.0, 0.0};
            acc_im[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        }

    cd ra[4], rb[4];
    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q;
            const int ar = e >> 4, ak = e & 15;
            const int gr = row0 + ar, gk = k0 + ak;
            ra[q] = (gr < g.M && gk < g.K) ? A[(size_t)gr * g.lda + gk] : cd{0.0, 0.0};
            const int bk = e >> 6, bc = e & 63;
            const int gk2 = k0 + bk, gc = col0 + bc;
            rb[q] = (gk2 < g.K && gc < g.N) ? B[(size_t)gk2 * g.ldb + gc] : cd{0.0, 0.0};
        }
    };
    // k chunks in order, skipping all-zero tiles of A when a mask is given
    // (uniform per workgroup: scalar reads of the mask)
    const int nkc = (g.K + TK - 1) / TK;
    const unsigned char *mrow = g.amask ? g.amask + (size_t)b * g.sMask + (size_t)tm * nkc : nullptr;
    auto next_chunk = [&](int kc) {
        if (mrow)
            while (kc < nkc && !mrow[kc]) ++kc;
        return kc;
    };
    int kc = next_chunk(0);
    if (kc < nkc) load_tiles(kc * TK);
    while (kc < nkc) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q;
            const int ar = e >> 4, ak = e & 15;
            As_re[ak][ar] = ra[q].re;
            As_im[ak][ar] = ra[q].im;
            const int bk = e >> 6, bc = e & 63;
            Bs_re[bk][bc] = rb[q].re;
            Bs_im[bk][bc] = rb[q].im;
        }
        __syncthreads();
        const int kn = next_chunk(kc + 1);
        if (kn < nkc) load_tiles(kn * TK);
        kc = kn;
#pragma unroll
        for (int ks = 0; ks < TK / 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            double are[2], aim[2], bre[2], bim[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int r = wm * 32 + i * 16 + (lane & 15);
                are[i] = As_re[kk][r];
                aim[i] = As_im[kk][r];
                const int c = wn * 32 + i * 16 + (lane & 15);
                bre[i] = Bs_re[kk][c];
                bim[i] = Bs_im[kk][c];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc_re[i][j] = mfma64(are[i], bre[j], acc_re[i][j]);
                    acc_re[i][j] = mfma64(-aim[i], bim[j], acc_re[i][j]);
                    acc_im[i][j] = mfma64(are[i], bim[j], acc_im[i][j]);
                    acc_im[i][j] = mfma64(aim[i], bre[j], acc_im[i][j]);
                }
        }
    }

    cd *__restrict__ D = g.D + (size_t)b * g.sD;
    const cd *__restrict__ Cin = g.Cin ? g.Cin + (size_t)b * g.sC : nullptr;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = row0 + wm * 32 + i * 16 + (lane >> 4) + 4 * r;
                const int gj = col0 + wn * 32 + j * 16 + (lane & 15);
                if (gi < g.M && gj < g.N) {
                    cd v = {g.alpha * acc_re[i][j][r], g.alpha * acc_im[i][j][r]};
                    if (Cin) {
                        const cd c = Cin[(size_t)gi * g.ldc + gj];
                        v.re = fma(g.beta, c.re, v.re);
                        v.im = fma(g.beta, c.im, v.im);
                    }
                    for (int t = 0; t < g.nx; ++t) {
                        const cd x = g.X[t][(size_t)b * g.sX + (size_t)gi * g.ldx + gj];
                        v.re = fma(g.coef[t], x.re, v.re);
                        v.im = fma(g.coef[t], x.im, v.im);
                    }
                    if (gi == gj) v.re += g.gamma;
                    D[(size_t)gi * g.ldd + gj] = v;
                }
            }
}

// One wavefront per 64 x 16 tile: any nonzero entry sets its mask byte.
__global__ void __launch_bounds__(256) tile_mask_kernel(int M, int K, int batch, const cd *__restrict__ A,
                                                        long long lda, long long sA, unsigned char *__restrict__ mask,
                                                        long long tiles_per) {
    const int lane = threadIdx.x & 63;
    const long long total = tiles_per * batch;
    const int nkc = (K + TK - 1) / TK;
    for (long long w = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < total;
         w += (long long)gridDim.x * (blockDim.x >> 6)) {
        const long long b = w / tiles_per, t = w - b * tiles_per;
        const int tm = (int)(t / nkc), kc = (int)(t - (long long)tm * nkc);
        const cd *Ab = A + (size_t)b * sA;
        bool nz = false;
        for (int e = lane; e < TM * TK; e += 64) {
            const int r = tm * TM + e / TK, k = kc * TK + e % TK;
            if (r < M && k < K) {
                const cd v = Ab[(size_t)r * lda + k];
                nz = nz || v.re != 0.0 || v.im != 0.0;
            }
        }
        const bool any = __any(nz);
        if (lane == 0) mask[w] = any ? 1 : 0;
    }
}

long long zgemm_mask_bytes(int M, int K) { return (long long)((M + TM - 1) / TM) * ((K + TK - 1) / TK); }

int zgemm_tile_mask(int M, int K, int batch, const cd *A, long long lda, long long sA, unsigned char *mask,
                    hipStream_t s) {
    const long long per = zgemm_mask_bytes(M, K), total = per * batch;
    long long blocks = (total + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    tile_mask_kernel<<<(int)blocks, 256, 0, s>>>(M, K, batch, A, lda, sA, mask, per);
    return check_launch("tile_mask");
}

int zgemm_batched(const ZgemmBatch &g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return LB_OK;
    const int tiles_m = (g.M + TM - 1) / TM, tiles_n = (g.N + TN - 1) / TN;
    if (g.batch > 65535) return fail(LB_ESHAPE, "zgemm: batch > 65535");
    dim3 grid(tiles_m * tiles_n, g.batch);
    if (g.K <= 0) {
        // pure epilogue (K = 0): still handled by the kernel, whose k loop is empty
    }
    zgemm_kernel<<<grid, 256, 0, s>>>(g, tiles_n);
    return check_launch("zgemm");
}

// ------------------------------------------------------------ elementwise
struct Lincomb {
    const cd *X[4];
    double coef[4];
};

__global__ void __launch_bounds__(256) zlincomb_kernel(long long nn, int n, long long total, int nx, Lincomb lc,
                                                      double gamma, cd *__restrict__ D) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        cd v = {0.0, 0.0};
        for (int t = 0; t < nx; ++t) {
            const cd x = lc.X[t][e];
            v.re = fma(lc.coef[t], x.re, v.re);
            v.im = fma(lc.coef[t], x.im, v.im);
        }
        const long long w = e % nn;
        if (w / n == w % n) v.re += gamma;
        D[e] = v;
    }
}

int zlincomb(int n, int batch, int nx, const cd *const *X, const double *coef, double gamma, cd *D, hipStream_t s) {
    if (nx > 4) return fail(LB_EINVAL, "zlincomb: at most 4 terms");
    Lincomb lc{};
    for (int t = 0; t < nx; ++t) {
        lc.X[t] = X[t];
        lc.coef[t] = coef[t];
    }
    const long long nn = (long long)n * n, total = nn * batch;
    long long grid = (total + 255) / 256;
    if (grid > 65536) grid = 65536;
    zlincomb_kernel<<<(int)grid, 256, 0, s>>>(nn, n, total, nx, lc, gamma, D);
    return check_launch("zlincomb");
}

}  // namespace lb
