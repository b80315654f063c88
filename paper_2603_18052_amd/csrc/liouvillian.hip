// Superoperator assembly (Eq. (1) in the row-major vectorisation) and the
// control-affine slice generators (Eq. (5)).  Both are HBM-write-bound: every
// output element is written once with consecutive threads on consecutive
// columns; the operators they read are a few KB and stay in L1/L2.
#include "lb_internal.hpp"

namespace lb {

// Element (r, c) of L with r = i d + j and c = k d + l:
//   -i (H[i,k] delta_jl - delta_ik H[l,j])
//   + sum_q Lq[i,k] conj(Lq[j,l])
//   - 1/2 delta_jl M[i,k] - 1/2 delta_ik M[l,j],   M = sum_q Lq^dag Lq.
// M is formed on the fly where a delta fires (a fraction 2/d of the elements).
__device__ inline cd mdag(const cd *__restrict__ Lk, int K, int d, int a, int b) {
    cd acc = {0.0, 0.0};
    for (int q = 0; q < K; ++q) {
        const cd *L = Lk + (size_t)q * d * d;
        for (int m = 0; m < d; ++m) acc = cfma(cconj(L[m * d + a]), L[m * d + b], acc);
    }
    return acc;
}

__global__ void __launch_bounds__(256) liouvillian_kernel(int d, const cd *__restrict__ H, int K,
                                                          const cd *__restrict__ Lk, cd *__restrict__ Lout) {
    const long long n = (long long)d * d;
    const long long total = n * n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(e / n), c = (int)(e - (long long)r * n);
        const int i = r / d, j = r - i * d, k = c / d, l = c - k * d;
        cd comm = {0.0, 0.0};
        if (j == l) comm = H[i * d + k];
        if (i == k) comm = csub(comm, H[l * d + j]);
        cd v = {comm.im, -comm.re};  // -i * comm
        for (int q = 0; q < K; ++q) {
            const cd *L = Lk + (size_t)q * d * d;
            v = cfma(L[i * d + k], cconj(L[j * d + l]), v);
        }
        if (K > 0) {
            if (j == l) v = csub(v, cscale(mdag(Lk, K, d, i, k), 0.5));
            if (i == k) v = csub(v, cscale(mdag(Lk, K, d, l, j), 0.5));
        }
        Lout[e] = v;
    }
}

// Lout[m][e] = L0[e] + sum_c u[m C + c] Lc[c][e]; each thread keeps its
// element of L0 and of the C control generators in registers and writes it
// for every slice, so the inputs are read once and the M n^2 outputs stream.
template <int CMAX>
__global__ void __launch_bounds__(256) generators_kernel(long long nn, int M, int C, const cd *__restrict__ L0,
                                                         const cd *__restrict__ Lc, const double *__restrict__ u,
                                                         cd *__restrict__ Lout) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
         e += (long long)gridDim.x * blockDim.x) {
        cd base = L0[e];
        cd lc[CMAX];
#pragma unroll
        for (int c = 0; c < CMAX; ++c) lc[c] = c < C ? Lc[(size_t)c * nn + e] : cd{0.0, 0.0};
        for (int m = 0; m < M; ++m) {
            cd g = base;
#pragma unroll
            for (int c = 0; c < CMAX; ++c)
                if (c < C) {
                    const double a = u[(size_t)m * C + c];
                    g.re = fma(a, lc[c].re, g.re);
                    g.im = fma(a, lc[c].im, g.im);
                }
            Lout[(size_t)m * nn + e] = g;
        }
    }
}

// Generic fallback for C > 16: the controls are re-read per slice.
__global__ void __launch_bounds__(256) generators_kernel_any(long long nn, int M, int C, const cd *__restrict__ L0,
                                                             const cd *__restrict__ Lc, const double *__restrict__ u,
                                                             cd *__restrict__ Lout) {
    const long long total = nn * M;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const long long m = t / nn, e = t - m * nn;
        cd g = L0[e];
        for (int c = 0; c < C; ++c) {
            const double a = u[m * C + c];
            const cd x = Lc[(size_t)c * nn + e];
            g.re = fma(a, x.re, g.re);
            g.im = fma(a, x.im, g.im);
        }
        Lout[t] = g;
    }
}

static int grid_for(long long work, int block) {
    long long g = (work + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

int generators_launch(int n, int M, int C, const cd *L0, const cd *Lc, const double *u, cd *Lout, hipStream_t s) {
    const long long nn = (long long)n * n;
    if (M == 0 || nn == 0) return LB_OK;
    const int g = grid_for(nn, 256);
    if (C <= 4)
        generators_kernel<4><<<g, 256, 0, s>>>(nn, M, C, L0, Lc, u, Lout);
    else if (C <= 8)
        generators_kernel<8><<<g, 256, 0, s>>>(nn, M, C, L0, Lc, u, Lout);
    else if (C <= 16)
        generators_kernel<16><<<g, 256, 0, s>>>(nn, M, C, L0, Lc, u, Lout);
    else
        generators_kernel_any<<<grid_for(nn * M, 256), 256, 0, s>>>(nn, M, C, L0, Lc, u, Lout);
    return check_launch("generators");
}

int liouvillian_launch(int d, const cd *H, int K, const cd *Lk, cd *Lout, hipStream_t s) {
    const long long n = (long long)d * d;
    liouvillian_kernel<<<grid_for(n * n, 256), 256, 0, s>>>(d, H, K, Lk, Lout);
    return check_launch("liouvillian");
}

}  // namespace lb

using namespace lb;

extern "C" int lindblad_liouvillian(int d, const void *H, int K, const void *Lk, void *Lout, hipStream_t stream) {
    if (d < 1 || d > 64) return fail(LB_ESHAPE, "lindblad_liouvillian: d must be in [1, 64]");
    if (K < 0 || K > 64) return fail(LB_ESHAPE, "lindblad_liouvillian: K must be in [0, 64]");
    if (!H || !Lout || (K > 0 && !Lk)) return fail(LB_EINVAL, "lindblad_liouvillian: NULL pointer");
    return liouvillian_launch(d, static_cast<const cd *>(H), K, static_cast<const cd *>(Lk),
                              static_cast<cd *>(Lout), stream);
}

extern "C" int lindblad_generators(int n, int M, int C, const void *L0, const void *Lc, const double *u, void *Lout,
                                   hipStream_t stream) {
    if (n < 1 || n > 4096) return fail(LB_ESHAPE, "lindblad_generators: n must be in [1, 4096]");
    if (M < 0 || C < 0 || C > 64) return fail(LB_ESHAPE, "lindblad_generators: need M >= 0, 0 <= C <= 64");
    if (M == 0) return LB_OK;
    if (!L0 || !Lout || (C > 0 && (!Lc || !u))) return fail(LB_EINVAL, "lindblad_generators: NULL pointer");
    return generators_launch(n, M, C, static_cast<const cd *>(L0), static_cast<const cd *>(Lc), u,
                             static_cast<cd *>(Lout), stream);
}
