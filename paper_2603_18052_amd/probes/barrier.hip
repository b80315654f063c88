// Device probe: latency of a barrier among G workgroups through a
// device-scope counter (release add, acquire polls), the cost a persistent
// chain would pay per step if P were spread over G compute units.  256
// workgroups, cooperative launch (all co-resident), 256 / G groups of G each
// run 2000 barriers.  Every poll loop is bounded: after spin_limit polls the
// waiting wave raises a shared abort flag and every wave leaves.  Prints one
// JSON line per G.
#include <hip/hip_runtime.h>

#include <cstdio>

#define CHECK(x)                                                                               \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) {                                                                \
            std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));                \
            return 1;                                                                          \
        }                                                                                      \
    } while (0)

__global__ void __launch_bounds__(256) barrier_kernel(unsigned *counters, int G, int rounds, int *abort_flag,
                                                      long long spin_limit, float *sink) {
    const int g = blockIdx.x / G;
    unsigned *cnt = counters + 64 * g;  // one counter per 256-byte line
    float acc = 0.f;
    for (int r = 0; r < rounds; ++r) {
        acc += (float)threadIdx.x * 1e-9f;
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned target = (unsigned)G * (unsigned)(r + 1);
            long long spins = 0;
            while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (++spins > spin_limit || __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = acc;
}

int main() {
    const int NWG = 256;
    unsigned *cnt = nullptr;
    int *ab = nullptr;
    float *sink = nullptr;
    CHECK(hipMalloc(&cnt, NWG * 64 * sizeof(unsigned)));
    CHECK(hipMalloc(&ab, sizeof(int)));
    CHECK(hipMalloc(&sink, NWG * sizeof(float)));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    for (int G : {1, 4, 8, 16, 32, 64, 256}) {
        int rounds = 2000;
        long long spin_limit = 2000000;
        float best = 0.f;
        int aborted = 0;
        for (int rep = 0; rep < 2; ++rep) {
            CHECK(hipMemset(cnt, 0, NWG * 64 * sizeof(unsigned)));
            CHECK(hipMemset(ab, 0, sizeof(int)));
            void *args[] = {&cnt, &G, &rounds, &ab, &spin_limit, &sink};
            CHECK(hipEventRecord(e0));
            CHECK(hipLaunchCooperativeKernel((const void *)barrier_kernel, dim3(NWG), dim3(256), args, 0, 0));
            CHECK(hipEventRecord(e1));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            int ah = 0;
            CHECK(hipMemcpy(&ah, ab, sizeof(int), hipMemcpyDeviceToHost));
            aborted |= ah;
            const float us = ms * 1e3f / rounds;
            if (rep == 0 || us < best) best = us;
        }
        std::printf("{\"probe\": \"group_barrier\", \"G\": %d, \"groups\": %d, \"us_per_barrier\": %.3f, \"aborted\": %d}\n",
                    G, NWG / G, best, aborted);
        std::fflush(stdout);
    }
    return 0;
}
