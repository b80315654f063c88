// Device probe: streaming-read bandwidth against buffer size, the measured
// ceilings of the bandwidth-bound kernels (the paper's coalesced-stream
// probe, Table of GPU device probes, redone on this device).  Sizes from
// L2-resident (a few MB) through the 256 MB Infinity Cache to HBM; each
// size is read 20 times by a grid-stride kernel of 16-byte loads after one
// warm-up pass, timed with HIP events.  Prints one JSON line per size.
#include <hip/hip_runtime.h>

#include <cstdio>

typedef float f4 __attribute__((ext_vector_type(4)));

#define CHECK(x)                                                                               \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) {                                                                \
            std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));                \
            return 1;                                                                          \
        }                                                                                      \
    } while (0)

__global__ void __launch_bounds__(256) read_kernel(const f4 *__restrict__ a, long long n4, float *__restrict__ out) {
    f4 acc = {0, 0, 0, 0};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (long long)gridDim.x * blockDim.x)
        acc += a[i];
    __shared__ float red[256];
    red[threadIdx.x] = acc[0] + acc[1] + acc[2] + acc[3];
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0;
        for (int k = 0; k < 256; ++k) s += red[k];
        out[blockIdx.x] = s;  // keeps the loads live
    }
}

int main() {
    const size_t maxb = 1024ull << 20;
    const int grids[] = {2048, 8192, 32768};
    const size_t sizes_mb[] = {2, 16, 32, 64, 128, 192, 256, 320, 512, 1024};
    f4 *a = nullptr;
    float *o = nullptr;
    CHECK(hipMalloc(&a, maxb));
    CHECK(hipMalloc(&o, 32768 * sizeof(float)));
    CHECK(hipMemset(a, 0, maxb));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    for (size_t mb : sizes_mb) {
        const long long n4 = (long long)(mb << 20) / 16;
        double best = 0.0;
        int best_grid = 0;
        for (int grid : grids) {
            read_kernel<<<grid, 256>>>(a, n4, o);
            CHECK(hipEventRecord(e0));
            const int reps = 20;
            for (int r = 0; r < reps; ++r) read_kernel<<<grid, 256>>>(a, n4, o);
            CHECK(hipEventRecord(e1));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            const double tbps = (double)(mb << 20) * reps / (ms * 1e-3) / 1e12;
            if (tbps > best) best = tbps, best_grid = grid;
        }
        std::printf("{\"probe\": \"stream_read\", \"MB\": %zu, \"TBps\": %.3f, \"grid\": %d}\n", mb, best, best_grid);
        std::fflush(stdout);
    }
    CHECK(hipFree(a));
    CHECK(hipFree(o));
    return 0;
}
