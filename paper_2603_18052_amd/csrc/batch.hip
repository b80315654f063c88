// Mixed serving batch: many independent problems, each with its own
// generator, step, step count and single state.
//
//  1. Problems are grouped by n.  Each group's generators are gathered into
//     one contiguous batch and its propagators are built together (Alg. 1,
//     batched FP64 build), then converted once to the chain precision.
//  2. n <= 128: one workgroup per problem runs all of that problem's steps
//     with its P resident in LDS; each row of P x is split over G lanes that
//     reduce with cross-lane shuffles, one barrier per step.
//  3. larger n: every step reads each running problem's whole P, so this
//     group streams P at the device's read bandwidth (measured ~7 TB/s, the
//     same whether the working set fits the 256 MB Infinity Cache or not).
//     Problems run in a sliding window: at most W at a time, longest first,
//     each started as soon as a slot frees (W from a byte budget of the
//     window's P's; 192 MiB measured ~5 % faster than all at once and 9 %
//     faster than 64 MiB).  Step t launches one grid over the window, 16 rows
//     of one problem per workgroup; rows of P are padded so every lane reads
//     16 bytes at a time, the state sits in registers, and each wavefront
//     interleaves 4 rows.
// Every problem's result is independent of the others in the batch.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
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
    if (N == 0) return;  // untouched (no round trip through T)
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

// 16-byte vectors of complex values: 2 complex FP32 or 1 complex FP64
template <typename T>
struct Vec;
template <>
struct Vec<float> {
    typedef float v __attribute__((ext_vector_type(4)));
    static constexpr int C = 2;
};
template <>
struct Vec<double> {
    typedef double v __attribute__((ext_vector_type(2)));
    static constexpr int C = 1;
};

// P rows converted to T and zero padded to Kp columns: PT[m][i][Kp]
template <typename T>
__global__ void convert_pad_kernel(int n, int Kp, int M, const cd *__restrict__ src, Cx<T> *__restrict__ dst) {
    const long long total = (long long)M * n * Kp;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long r = e / Kp;  // m * n + i
        const int k = (int)(e - r * Kp);
        const cd v = k < n ? src[r * n + k] : cd{0.0, 0.0};
        dst[e] = {(T)v.re, (T)v.im};
    }
}

// y = P x for the window's problems at global step t.  Problem m started at
// step start[m]; its local step parity picks the ping-pong buffer.  Lane l
// holds x[(l + 64 i) VEC .. + VEC - 1] for i < NJ (Kp = 64 VEC NJ, padding
// zero), each wavefront 4 rows.
template <typename T, int NJ>
__global__ void __launch_bounds__(256) window_step_kernel(int n, int Kp, const Cx<T> *__restrict__ PT,
                                                          const int *__restrict__ list,
                                                          const long long *__restrict__ start, long long t,
                                                          Cx<T> *__restrict__ X0, Cx<T> *__restrict__ X1) {
    typedef typename Vec<T>::v V;
    constexpr int VC = Vec<T>::C;
    const int m = list[blockIdx.y];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool odd = ((t - start[m]) & 1) != 0;
    const Cx<T> *x = (odd ? X1 : X0) + (size_t)m * Kp;
    Cx<T> *y = (odd ? X0 : X1) + (size_t)m * Kp;
    const Cx<T> *P = PT + (size_t)m * n * Kp;
    constexpr int NR = NJ > 0 ? NJ : 1;
    V xv[NR];
    if (NJ > 0) {
#pragma unroll
        for (int i = 0; i < NR; ++i) xv[i] = *reinterpret_cast<const V *>(x + (size_t)(lane + 64 * i) * VC);
    }
    const int rb = blockIdx.x * 16 + wave * 4;
    const Cx<T> *prow[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) prow[q] = P + (size_t)(rb + q < n ? rb + q : n - 1) * Kp + (size_t)lane * VC;
    T re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
    auto mac = [&](const V &xq, int i) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const V p = *reinterpret_cast<const V *>(prow[q] + (size_t)64 * VC * i);
#pragma unroll
            for (int c = 0; c < VC; ++c) {
                const T pr = p[2 * c], pi = p[2 * c + 1], xr = xq[2 * c], xi = xq[2 * c + 1];
                re[q] = fma(pr, xr, fma(-pi, xi, re[q]));
                im[q] = fma(pr, xi, fma(pi, xr, im[q]));
            }
        }
    };
    if (NJ > 0) {
#pragma unroll
        for (int i = 0; i < NR; ++i) mac(xv[i], i);
    } else {  // wide rows: the state is re-read from cache
        const int nj = Kp / (64 * VC);
        for (int i = 0; i < nj; ++i) mac(*reinterpret_cast<const V *>(x + (size_t)(lane + 64 * i) * VC), i);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            re[q] += __shfl_xor(re[q], off);
            im[q] += __shfl_xor(im[q], off);
        }
    }
    if (lane < 4) {
        T r = re[0], i = im[0];
#pragma unroll
        for (int q = 1; q < 4; ++q)
            if (lane == q) {
                r = re[q];
                i = im[q];
            }
        if (rb + lane < n) y[rb + lane] = {r, i};
    }
}

template <typename T>
__global__ void load_states_kernel(int n, int Kp, int M, cd *const *__restrict__ rhos, Cx<T> *__restrict__ X0,
                                   Cx<T> *__restrict__ X1) {
    const long long total = (long long)Kp * M;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long m = e / Kp, i = e - m * Kp;
        const cd v = i < n ? rhos[m][i] : cd{0.0, 0.0};
        X0[e] = {(T)v.re, (T)v.im};
        X1[e] = {(T)0, (T)0};
    }
}

template <typename T>
__global__ void store_states_kernel(int n, int Kp, int M, const Cx<T> *__restrict__ X0, const Cx<T> *__restrict__ X1,
                                    const long long *__restrict__ nsteps, cd *const *__restrict__ rhos) {
    const long long total = (long long)n * M;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long m = e / n, i = e - m * n;
        if (nsteps[m] == 0) continue;  // untouched (no round trip through T)
        const Cx<T> v = (nsteps[m] & 1) ? X1[m * Kp + i] : X0[m * Kp + i];
        rhos[m][i] = {(double)v.re, (double)v.im};
    }
}

static int grid1(long long work) {
    long long g = (work + 255) / 256;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

// Default byte budget of the window's propagators (the fastest of the
// measured budgets on the d = 27 mixed batch).
constexpr size_t kWindowBytes = 192ull << 20;
static std::atomic<size_t> g_window_bytes{kWindowBytes};

// Supported register tiles of the step kernel (x values per lane, in 16-byte
// vectors); wider rows use the kernel's cache-read path (NJ = 0).
static int window_nj(int n, int vc) {
    const int need = (n + 64 * vc - 1) / (64 * vc);
    for (int c : {1, 2, 3, 4, 6, 8, 12, 16})
        if (need <= c) return c;
    return 0;
}

template <typename T>
static int window_launch(int nj, dim3 grid, int n, int Kp, const Cx<T> *PT, const int *list, const long long *start,
                         long long t, Cx<T> *X0, Cx<T> *X1, hipStream_t s) {
    switch (nj) {
        case 1: window_step_kernel<T, 1><<<grid, 256, 0, s>>>(n, Kp, PT, list, start, t, X0, X1); break;
        case 2: window_step_kernel<T, 2><<<grid, 256, 0, s>>>(n, Kp, PT, list, start, t, X0, X1); break;
        case 3: window_step_kernel<T, 3><<<grid, 256, 0, s>>>(n, Kp, PT, list, start, t, X0, X1); break;
        case 4: window_step_kernel<T, 4><<<grid, 256, 0, s>>>(n, Kp, PT, list, start, t, X0, X1); break;
        case 6: window_step_kernel<T, 6><<<grid, 256, 0, s>>>(n, Kp, PT, list, start, t, X0, X1); break;
        case 8: window_step_kernel<T, 8><<<grid, 256, 0, s>>>(n, Kp, PT, list, start, t, X0, X1); break;
        case 12: window_step_kernel<T, 12><<<grid, 256, 0, s>>>(n, Kp, PT, list, start, t, X0, X1); break;
        case 16: window_step_kernel<T, 16><<<grid, 256, 0, s>>>(n, Kp, PT, list, start, t, X0, X1); break;
        default: window_step_kernel<T, 0><<<grid, 256, 0, s>>>(n, Kp, PT, list, start, t, X0, X1); break;
    }
    return LB_OK;
}

// Sliding-window schedule: problems (sorted by step count, longest first)
// take the slot that frees earliest among W.  Returns the start step of each
// problem and the segments [t_k, t_{k+1}) of constant running set.
struct Window {
    std::vector<long long> start, seg_t;   // seg_t: segment boundaries (size segs + 1)
    std::vector<int> seg_off, list;        // running problems of segment k: list[seg_off[k] .. seg_off[k+1])
};

static Window window_schedule(const std::vector<long long> &steps, int W) {
    const int M = (int)steps.size();
    Window w;
    w.start.assign(M, 0);
    std::vector<long long> slot(W, 0);
    std::vector<long long> ev;
    for (int i = 0; i < M; ++i) {
        if (steps[i] == 0) continue;
        const int k = (int)(std::min_element(slot.begin(), slot.end()) - slot.begin());
        w.start[i] = slot[k];
        slot[k] += steps[i];
        ev.push_back(w.start[i]);
        ev.push_back(w.start[i] + steps[i]);
    }
    std::sort(ev.begin(), ev.end());
    ev.erase(std::unique(ev.begin(), ev.end()), ev.end());
    for (size_t k = 0; k + 1 < ev.size(); ++k) {
        w.seg_t.push_back(ev[k]);
        w.seg_off.push_back((int)w.list.size());
        for (int i = 0; i < M; ++i)
            if (steps[i] > 0 && w.start[i] <= ev[k] && ev[k] < w.start[i] + steps[i]) w.list.push_back(i);
    }
    if (!ev.empty()) w.seg_t.push_back(ev.back());
    w.seg_off.push_back((int)w.list.size());
    return w;
}

// Small host arrays reach the device as kernel arguments (2 KB per launch),
// so nothing the call enqueues reads host memory after it returns: the whole
// batch can be captured into a HIP graph and replayed.
constexpr int kArgWords = 256;
struct WordArgs {
    unsigned long long v[kArgWords];
};
__global__ void put_words_kernel(WordArgs a, int count, unsigned long long *__restrict__ dst) {
    const int i = threadIdx.x;
    if (i < count) dst[i] = a.v[i];
}
// dst must hold nbytes rounded up to 8
static int upload(const void *src, size_t nbytes, void *dst, hipStream_t s) {
    const unsigned char *p = static_cast<const unsigned char *>(src);
    unsigned long long *d = static_cast<unsigned long long *>(dst);
    for (size_t off = 0; off < nbytes; off += 8 * kArgWords) {
        WordArgs a;
        const size_t b = std::min(nbytes - off, (size_t)8 * kArgWords);
        std::memset(a.v, 0, sizeof a.v);
        std::memcpy(a.v, p + off, b);
        const int words = (int)((b + 7) / 8);
        put_words_kernel<<<1, kArgWords, 0, s>>>(a, words, d + off / 8);
        LB_TRY(check_launch("batch upload"));
    }
    return LB_OK;
}

// Everything one size group needs, laid out in the workspace by plan_group
// and enqueued by run_group; the group's build scratch follows its buffers,
// so groups on different streams never share memory.
struct Group {
    int n = 0, M = 0, Kp = 0, nj = 0;
    bool small = false;
    std::vector<const cd *> srcs;
    std::vector<cd *> rhos;
    std::vector<long long> steps;
    std::vector<double> dts;
    Window win;
    size_t prow = 0, bytes = 0;
};

template <typename T>
static Group plan_group(int n, const std::vector<const lb_problem *> &probs) {
    Group g;
    g.n = n;
    g.M = (int)probs.size();
    const size_t nn = (size_t)n * n;
    // longest first (the window schedule takes them in this order)
    std::vector<int> order(g.M);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return probs[a]->nsteps > probs[b]->nsteps; });
    for (int i = 0; i < g.M; ++i) {
        const lb_problem *p = probs[order[i]];
        g.srcs.push_back(static_cast<const cd *>(p->L));
        g.rhos.push_back(static_cast<cd *>(p->rho));
        g.steps.push_back(p->nsteps);
        g.dts.push_back(p->dt);
    }
    const size_t lds = (nn + 2 * (size_t)n) * sizeof(Cx<T>);
    g.small = n <= 128 && lds <= 160 * 1024;
    const int VC = Vec<T>::C;
    g.nj = window_nj(n, VC);
    g.Kp = g.small ? n : (g.nj > 0 ? g.nj : (n + 64 * VC - 1) / (64 * VC)) * 64 * VC;
    g.prow = (size_t)g.Kp * sizeof(Cx<T>);
    if (!g.small) {
        long long W = (long long)(g_window_bytes.load() / ((size_t)n * g.prow));
        W = std::max(1LL, std::min<long long>(W, g.M));
        g.win = window_schedule(g.steps, (int)W);
    }
    const size_t M = (size_t)g.M;
    g.bytes = 2 * align256(nn * sizeof(cd) * M) + align256((size_t)n * g.prow * M) + 3 * align256(M * sizeof(void *)) +
              align256(M * sizeof(long long)) + align256(g.win.list.size() * sizeof(int) + 8) +
              2 * align256((size_t)g.Kp * M * sizeof(Cx<T>)) + build_async_chunk_bytes(n, g.M);
    return g;
}

// Enqueue one group on `s` (no host synchronisation); its buffers are taken
// from the workspace and kept (the caller ensured plan_group's bytes).
template <typename T>
static int run_group(const Group &g, double theta, int *d_status, Workspace *ws, hipStream_t s) {
    const int n = g.n, M = g.M, Kp = g.Kp;
    const size_t nn = (size_t)n * n;
    cd *Lg = (cd *)ws_take(ws, nn * sizeof(cd) * M);
    cd *P = (cd *)ws_take(ws, nn * sizeof(cd) * M);
    Cx<T> *PT = (Cx<T> *)ws_take(ws, (size_t)n * g.prow * M);
    const cd **d_srcs = (const cd **)ws_take(ws, M * sizeof(void *));
    cd **d_rhos = (cd **)ws_take(ws, M * sizeof(void *));
    long long *d_steps = (long long *)ws_take(ws, M * sizeof(long long));
    long long *d_start = (long long *)ws_take(ws, M * sizeof(long long));
    int *d_list = (int *)ws_take(ws, g.win.list.size() * sizeof(int) + 8);
    Cx<T> *X0 = (Cx<T> *)ws_take(ws, (size_t)Kp * M * sizeof(Cx<T>));
    Cx<T> *X1 = (Cx<T> *)ws_take(ws, (size_t)Kp * M * sizeof(Cx<T>));
    LB_TRY(upload(g.srcs.data(), M * sizeof(void *), d_srcs, s));
    LB_TRY(upload(g.rhos.data(), M * sizeof(void *), d_rhos, s));
    LB_TRY(upload(g.steps.data(), M * sizeof(long long), d_steps, s));
    gather_kernel<<<grid1((long long)nn * M), 256, 0, s>>>((long long)nn, d_srcs, Lg, M);
    LB_TRY(check_launch("gather"));
    // the build's scratch: right here, and kept (another group may run beside it)
    const size_t build_at = ws->used;
    LB_TRY(build_propagators_async(n, M, Lg, g.dts.data(), theta, P, nullptr, d_status, ws, s));
    ws->used = build_at + build_async_chunk_bytes(n, M);
    if (g.small) {
        convert_kernel<T><<<grid1((long long)nn * M), 256, 0, s>>>((long long)nn * M, P, PT);
        LB_TRY(check_launch("convert"));
        int threads = ((n * G + 63) / 64) * 64;
        if (threads > 512) threads = 512;
        const size_t lds = (nn + 2 * (size_t)n) * sizeof(Cx<T>);
        small_chain_kernel<T><<<M, threads, lds, s>>>(n, PT, d_rhos, d_steps);
        return check_launch("small_chain");
    }
    convert_pad_kernel<T><<<grid1((long long)M * n * Kp), 256, 0, s>>>(n, Kp, M, P, PT);
    LB_TRY(check_launch("convert_pad"));
    LB_TRY(upload(g.win.start.data(), M * sizeof(long long), d_start, s));
    if (!g.win.list.empty()) LB_TRY(upload(g.win.list.data(), g.win.list.size() * sizeof(int), d_list, s));
    load_states_kernel<T><<<grid1((long long)Kp * M), 256, 0, s>>>(n, Kp, M, d_rhos, X0, X1);
    LB_TRY(check_launch("load_states"));
    const int rowblocks = (n + 15) / 16;
    for (size_t k = 0; k + 1 < g.win.seg_t.size(); ++k) {
        const int cnt = g.win.seg_off[k + 1] - g.win.seg_off[k];
        const dim3 grid(rowblocks, cnt);
        for (long long t = g.win.seg_t[k]; t < g.win.seg_t[k + 1]; ++t)
            window_launch<T>(g.nj, grid, n, Kp, PT, d_list + g.win.seg_off[k], d_start, t, X0, X1, s);
    }
    LB_TRY(check_launch("window_step"));
    store_states_kernel<T><<<grid1((long long)n * M), 256, 0, s>>>(n, Kp, M, X0, X1, d_steps, d_rhos);
    return check_launch("store_states");
}

// A second stream per device for the groups that run beside the largest one
// (default priority; created on first use, kept for the process).
static std::mutex g_side_mu;
static std::map<int, hipStream_t> g_side;

template <typename T>
static int enqueue_all(const std::vector<std::vector<const lb_problem *>> &parts, double theta, int *d_status,
                       Workspace *w, hipStream_t s) {
    std::vector<Group> groups;
    size_t total = 0;
    for (const auto &part : parts) {
        groups.push_back(plan_group<T>(part[0]->d * part[0]->d, part));
        total += groups.back().bytes;
    }
    LB_TRY(ws_ensure(w, total));
    // the kernel's LDS limit (a host-side attribute, set once per device; not
    // a stream operation, so also allowed while the caller captures a graph)
    LB_TRY(set_max_lds((const void *)small_chain_kernel<T>, 160 * 1024));
    bool any_small = false, any_large = false;
    for (const Group &g : groups) (g.small ? any_small : any_large) = true;
    if (!(any_small && any_large)) {  // one stream
        for (const Group &g : groups) LB_TRY(run_group<T>(g, theta, d_status, w, s));
        return LB_OK;
    }
    // fork: the small-n groups on the side stream, the rest on the caller's
    std::lock_guard<std::mutex> lock(g_side_mu);
    int dev = 0;
    LB_HIP(hipGetDevice(&dev));
    hipStream_t &side = g_side[dev];
    if (!side) LB_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    hipEvent_t fork = nullptr, join = nullptr;
    LB_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    if (hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
        (void)hipEventDestroy(fork);
        return fail(LB_EHIP, "batch: hipEventCreate failed");
    }
    int rc = LB_OK;
    if (hipEventRecord(fork, s) != hipSuccess || hipStreamWaitEvent(side, fork, 0) != hipSuccess)
        rc = fail(LB_EHIP, "batch: fork failed");
    for (size_t i = 0; i < groups.size() && rc == LB_OK; ++i)
        rc = run_group<T>(groups[i], theta, d_status, w, groups[i].small ? side : s);
    // the join is enqueued whatever happened, so the caller's stream never
    // runs ahead of work on the side stream
    if (hipEventRecord(join, side) != hipSuccess || hipStreamWaitEvent(s, join, 0) != hipSuccess)
        if (rc == LB_OK) rc = fail(LB_EHIP, "batch: join failed");
    (void)hipEventDestroy(fork);
    (void)hipEventDestroy(join);
    return rc;
}

}  // namespace mb
}  // namespace lb

using namespace lb;

static int batch_args(const char *who, const lb_problem *probs, int nprob, lb_precision prec, double theta) {
    const std::string w(who);
    if (nprob < 0) return fail(LB_EINVAL, w + ": nprob < 0");
    if (nprob > 0 && !probs) return fail(LB_EINVAL, w + ": probs is NULL");
    if (prec != LB_C128 && prec != LB_C64)
        return fail(LB_ENOTSUP, w + ": single-state problems run in LB_C128 or LB_C64");
    if (!(theta > 0.0)) return fail(LB_EINVAL, w + ": theta must be > 0");
    for (int i = 0; i < nprob; ++i) {
        const lb_problem &p = probs[i];
        if (p.d < 1 || p.d > 64) return fail(LB_ESHAPE, w + ": d must be in [1, 64]");
        if (p.nsteps < 0) return fail(LB_EINVAL, w + ": nsteps < 0");
        if (!p.L || !p.rho) return fail(LB_EINVAL, w + ": NULL pointer in a problem");
        if (!std::isfinite(p.dt)) return fail(LB_EINVAL, w + ": dt must be finite");
    }
    return LB_OK;
}

// size groups (ascending d), at most 512 problems each
static std::vector<std::vector<const lb_problem *>> batch_parts(const lb_problem *probs, int nprob) {
    std::vector<int> sizes;
    for (int i = 0; i < nprob; ++i)
        if (std::find(sizes.begin(), sizes.end(), probs[i].d) == sizes.end()) sizes.push_back(probs[i].d);
    std::sort(sizes.begin(), sizes.end());
    std::vector<std::vector<const lb_problem *>> parts;
    for (int d : sizes) {
        std::vector<const lb_problem *> group;
        for (int i = 0; i < nprob; ++i)
            if (probs[i].d == d) group.push_back(&probs[i]);
        for (size_t g0 = 0; g0 < group.size(); g0 += 512)
            parts.emplace_back(group.begin() + g0, group.begin() + std::min(group.size(), g0 + 512));
    }
    return parts;
}

extern "C" int lindblad_batch_enqueue(const lb_problem *probs, int nprob, lb_precision prec, double theta,
                                      int *status, lb_workspace *ws, hipStream_t stream) {
    LB_TRY(batch_args("lindblad_batch_enqueue", probs, nprob, prec, theta));
    if (nprob == 0) return LB_OK;
    Workspace *w = ws_resolve(ws);
    ws_begin(w, stream);
    const auto parts = batch_parts(probs, nprob);
    return prec == LB_C64 ? mb::enqueue_all<float>(parts, theta, status, w, stream)
                          : mb::enqueue_all<double>(parts, theta, status, w, stream);
}

extern "C" int lindblad_batch_run(const lb_problem *probs, int nprob, lb_precision prec, double theta,
                                  lb_workspace *ws, hipStream_t stream) {
    LB_TRY(batch_args("lindblad_batch_run", probs, nprob, prec, theta));
    if (nprob == 0) return LB_OK;
    Workspace *w = ws_resolve(ws);
    ws_begin(w, stream);
    const auto parts = batch_parts(probs, nprob);
    // the status word sits past the groups' buffers
    size_t total = 256;
    for (const auto &part : parts) {
        const int n = part[0]->d * part[0]->d;
        total += prec == LB_C64 ? mb::plan_group<float>(n, part).bytes : mb::plan_group<double>(n, part).bytes;
    }
    LB_TRY(ws_ensure(w, total));
    int *d_status = (int *)ws_take(w, 256);
    LB_TRY(fill_i32_launch(d_status, 1, stream));
    LB_TRY(prec == LB_C64 ? mb::enqueue_all<float>(parts, theta, d_status, w, stream)
                          : mb::enqueue_all<double>(parts, theta, d_status, w, stream));
    int st = 0;
    LB_HIP(hipMemcpyAsync(&st, d_status, sizeof(int), hipMemcpyDeviceToHost, stream));
    LB_HIP(hipStreamSynchronize(stream));
    if (st == LB_ENONFINITE) return fail(st, "lindblad_batch_run: ||L dt||_1 of some problem is not finite");
    if (st == LB_ESINGULAR) return fail(st, "lindblad_batch_run: zero pivot in some problem's Pade denominator");
    if (st == LB_ENOTSUP) return fail(st, "lindblad_batch_run: some problem's scaling exponent exceeds the cap");
    return st == LB_OK ? LB_OK : fail(st, "lindblad_batch_run: device status " + std::to_string(st));
}

extern "C" int lindblad_batch_set_window(size_t bytes) {
    mb::g_window_bytes.store(bytes ? bytes : mb::kWindowBytes);
    return LB_OK;
}
