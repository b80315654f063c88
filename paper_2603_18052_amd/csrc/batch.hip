// Mixed serving batch: many independent problems, each with its own
// generator, step, step count and single state.
//
//  1. Problems are grouped by n.  Each group's generators are gathered into
//     one contiguous batch and its propagators are built together (Alg. 1,
//     batched FP64 build), then converted once to the chain precision.
//  2. n <= 128: one workgroup per problem runs all of that problem's steps
//     with its P resident in LDS; each row of P x is split over G lanes that
//     reduce with cross-lane shuffles, one barrier per step.
//  3. larger n: problems are sorted by step count; step t launches one grid
//     over the prefix of problems still running, 16 rows of one problem per
//     workgroup, lanes reading P rows contiguously (coalesced).  P streams
//     from HBM/MALL every step: this group is bandwidth-bound.
// Every problem's result is independent of the others in the batch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "lb_internal.hpp"

namespace lb {
namespace mb {

template <typename T>
struct Cx {
    T re, im;
};

__global__ void gather_kernel(long long nn, const cd *const *__restrict__ srcs, cd *__restrict__ dst, int M) {
    const long long total = nn * M;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long m = e / nn, r = e - m * nn;
        dst[e] = srcs[m][r];
    }
}

template <typename T>
__global__ void convert_kernel(long long count, const cd *__restrict__ src, Cx<T> *__restrict__ dst) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (long long)gridDim.x * blockDim.x)
        dst[e] = {(T)src[e].re, (T)src[e].im};
}

constexpr int G = 4;  // lanes per row in the small-n kernel

template <typename T>
__global__ void __launch_bounds__(512) small_chain_kernel(int n, const Cx<T> *__restrict__ Pall, cd *const *__restrict__ rhos,
                                                          const long long *__restrict__ nsteps) {
    extern __shared__ __align__(16) unsigned char smem[];
    Cx<T> *Ps = reinterpret_cast<Cx<T> *>(smem);  // n x n
    Cx<T> *xs = Ps + (size_t)n * n;                // 2 x n
    const int m = blockIdx.x;
    const Cx<T> *P = Pall + (size_t)m * n * n;
    cd *rho = rhos[m];
    const long long N = nsteps[m];
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) Ps[e] = P[e];
    for (int e = threadIdx.x; e < n; e += blockDim.x) xs[e] = {(T)rho[e].re, (T)rho[e].im};
    __syncthreads();
    const int row = threadIdx.x / G, sub = threadIdx.x % G;
    int cur = 0;
    for (long long t = 0; t < N; ++t) {
        const Cx<T> *x = xs + cur * n;
        T re = 0, im = 0;
        if (row < n) {
            const Cx<T> *Pr = Ps + (size_t)row * n;
            for (int j = sub; j < n; j += G) {
                const Cx<T> p = Pr[j], v = x[j];
                re = fma(p.re, v.re, fma(-p.im, v.im, re));
                im = fma(p.re, v.im, fma(p.im, v.re, im));
            }
        }
#pragma unroll
        for (int off = G / 2; off >= 1; off >>= 1) {
            re += __shfl_xor(re, off);
            im += __shfl_xor(im, off);
        }
        if (row < n && sub == 0) xs[(cur ^ 1) * n + row] = {re, im};
        cur ^= 1;
        __syncthreads();
    }
    for (int e = threadIdx.x; e < n; e += blockDim.x) rho[e] = {(double)xs[cur * n + e].re, (double)xs[cur * n + e].im};
}

// one step for the problems [0, active) of a sorted group: y = P x
template <typename T>
__global__ void __launch_bounds__(256) large_step_kernel(int n, const Cx<T> *__restrict__ Pall,
                                                         const Cx<T> *__restrict__ X, Cx<T> *__restrict__ Y) {
    const int m = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const Cx<T> *P = Pall + (size_t)m * n * n;
    const Cx<T> *x = X + (size_t)m * n;
    for (int r = 0; r < 4; ++r) {
        const int row = blockIdx.x * 16 + wave * 4 + r;
        if (row >= n) break;
        const Cx<T> *Pr = P + (size_t)row * n;
        T re = 0, im = 0;
        for (int j = lane; j < n; j += 64) {
            const Cx<T> p = Pr[j], v = x[j];
            re = fma(p.re, v.re, fma(-p.im, v.im, re));
            im = fma(p.re, v.im, fma(p.im, v.re, im));
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            re += __shfl_xor(re, off);
            im += __shfl_xor(im, off);
        }
        if (lane == 0) Y[(size_t)m * n + row] = {re, im};
    }
}

template <typename T>
__global__ void load_states_kernel(int n, int M, cd *const *__restrict__ rhos, Cx<T> *__restrict__ X) {
    const long long total = (long long)n * M;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long m = e / n, i = e - m * n;
        const cd v = rhos[m][i];
        X[e] = {(T)v.re, (T)v.im};
    }
}

template <typename T>
__global__ void store_states_kernel(int n, int M, const Cx<T> *__restrict__ X0, const Cx<T> *__restrict__ X1,
                                    const long long *__restrict__ nsteps, cd *const *__restrict__ rhos) {
    const long long total = (long long)n * M;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long m = e / n, i = e - m * n;
        const Cx<T> v = (nsteps[m] & 1) ? X1[e] : X0[e];
        rhos[m][i] = {(double)v.re, (double)v.im};
    }
}

static int grid1(long long work) {
    long long g = (work + 255) / 256;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

template <typename T>
static int run_group(int n, const std::vector<const lb_problem *> &probs, double theta, Workspace *ws, hipStream_t s) {
    const int M = (int)probs.size();
    const size_t nn = (size_t)n * n;
    // largest step count first: the running problems are always a prefix
    std::vector<int> order(M);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return probs[a]->nsteps > probs[b]->nsteps; });
    std::vector<const cd *> srcs(M);
    std::vector<cd *> rhos(M);
    std::vector<long long> steps(M);
    std::vector<double> dts(M);
    for (int i = 0; i < M; ++i) {
        const lb_problem *p = probs[order[i]];
        srcs[i] = static_cast<const cd *>(p->L);
        rhos[i] = static_cast<cd *>(p->rho);
        steps[i] = p->nsteps;
        dts[i] = p->dt;
    }
    const size_t mats = align256(nn * sizeof(cd) * M);
    const size_t need = 2 * mats + align256(nn * sizeof(Cx<T>) * M) + 3 * align256(M * sizeof(void *)) +
                        2 * align256((size_t)n * M * sizeof(Cx<T>)) + build_workspace_bytes(n, M);
    LB_TRY(ws_ensure(ws, need));
    const size_t mark = ws->used;
    cd *Lg = (cd *)ws_take(ws, nn * sizeof(cd) * M);
    cd *P = (cd *)ws_take(ws, nn * sizeof(cd) * M);
    Cx<T> *PT = (Cx<T> *)ws_take(ws, nn * sizeof(Cx<T>) * M);
    const cd **d_srcs = (const cd **)ws_take(ws, M * sizeof(void *));
    cd **d_rhos = (cd **)ws_take(ws, M * sizeof(void *));
    long long *d_steps = (long long *)ws_take(ws, M * sizeof(long long));
    Cx<T> *X0 = (Cx<T> *)ws_take(ws, (size_t)n * M * sizeof(Cx<T>));
    Cx<T> *X1 = (Cx<T> *)ws_take(ws, (size_t)n * M * sizeof(Cx<T>));
    LB_HIP(hipMemcpyAsync(d_srcs, srcs.data(), M * sizeof(void *), hipMemcpyHostToDevice, s));
    LB_HIP(hipMemcpyAsync(d_rhos, rhos.data(), M * sizeof(void *), hipMemcpyHostToDevice, s));
    LB_HIP(hipMemcpyAsync(d_steps, steps.data(), M * sizeof(long long), hipMemcpyHostToDevice, s));
    gather_kernel<<<grid1((long long)nn * M), 256, 0, s>>>((long long)nn, d_srcs, Lg, M);
    LB_TRY(check_launch("gather"));
    LB_TRY(build_propagators(n, M, Lg, dts.data(), theta, P, nullptr, ws, s));
    convert_kernel<T><<<grid1((long long)nn * M), 256, 0, s>>>((long long)nn * M, P, PT);
    LB_TRY(check_launch("convert"));
    const size_t lds = (nn + 2 * (size_t)n) * sizeof(Cx<T>);
    if (n <= 128 && lds <= 160 * 1024) {
        static bool attr = false;
        if (!attr) {
            LB_HIP(hipFuncSetAttribute((const void *)small_chain_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024));
            attr = true;
        }
        int threads = ((n * G + 63) / 64) * 64;
        if (threads > 512) threads = 512;
        small_chain_kernel<T><<<M, threads, lds, s>>>(n, PT, d_rhos, d_steps);
        LB_TRY(check_launch("small_chain"));
    } else {
        load_states_kernel<T><<<grid1((long long)n * M), 256, 0, s>>>(n, M, d_rhos, X0);
        LB_TRY(check_launch("load_states"));
        const int rowblocks = (n + 15) / 16;
        int active = M;
        for (long long t = 0; t < steps[0]; ++t) {
            while (active > 0 && steps[active - 1] <= t) --active;
            dim3 grid(rowblocks, active);
            const Cx<T> *x = (t & 1) ? X1 : X0;
            Cx<T> *y = (t & 1) ? X0 : X1;
            large_step_kernel<T><<<grid, 256, 0, s>>>(n, PT, x, y);
        }
        LB_TRY(check_launch("large_step"));
        store_states_kernel<T><<<grid1((long long)n * M), 256, 0, s>>>(n, M, X0, X1, d_steps, d_rhos);
        LB_TRY(check_launch("store_states"));
    }
    LB_HIP(hipStreamSynchronize(s));  // host arrays above go out of scope
    ws->used = mark;
    return LB_OK;
}

}  // namespace mb
}  // namespace lb

using namespace lb;

extern "C" int lindblad_batch_run(const lb_problem *probs, int nprob, lb_precision prec, double theta,
                                  lb_workspace *ws, hipStream_t stream) {
    if (nprob < 0) return fail(LB_EINVAL, "lindblad_batch_run: nprob < 0");
    if (nprob == 0) return LB_OK;
    if (!probs) return fail(LB_EINVAL, "lindblad_batch_run: probs is NULL");
    if (prec != LB_C128 && prec != LB_C64)
        return fail(LB_ENOTSUP, "lindblad_batch_run: single-state problems run in LB_C128 or LB_C64");
    if (!(theta > 0.0)) return fail(LB_EINVAL, "lindblad_batch_run: theta must be > 0");
    std::vector<int> sizes;
    for (int i = 0; i < nprob; ++i) {
        const lb_problem &p = probs[i];
        if (p.d < 1 || p.d > 64) return fail(LB_ESHAPE, "lindblad_batch_run: d must be in [1, 64]");
        if (p.nsteps < 0) return fail(LB_EINVAL, "lindblad_batch_run: nsteps < 0");
        if (!p.L || !p.rho) return fail(LB_EINVAL, "lindblad_batch_run: NULL pointer in a problem");
        if (!std::isfinite(p.dt)) return fail(LB_EINVAL, "lindblad_batch_run: dt must be finite");
        if (std::find(sizes.begin(), sizes.end(), p.d) == sizes.end()) sizes.push_back(p.d);
    }
    Workspace *w = ws_resolve(ws);
    ws_begin(w);
    std::sort(sizes.begin(), sizes.end());
    for (int d : sizes) {
        std::vector<const lb_problem *> group;
        for (int i = 0; i < nprob; ++i)
            if (probs[i].d == d) group.push_back(&probs[i]);
        const int n = d * d;
        // keep a group's workspace bounded: at most 512 problems per build
        for (size_t g0 = 0; g0 < group.size(); g0 += 512) {
            std::vector<const lb_problem *> part(group.begin() + g0,
                                                 group.begin() + std::min(group.size(), g0 + 512));
            LB_TRY(prec == LB_C64 ? mb::run_group<float>(n, part, theta, w, stream)
                                  : mb::run_group<double>(n, part, theta, w, stream));
        }
    }
    return LB_OK;
}
