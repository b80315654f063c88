// Device probe: LDS bank conflicts of 16-byte-per-lane fetch patterns, the
// shapes the MFMA operand fetches of the chain kernels use.  Each pattern is
// a table of 64 byte offsets (lane l reads 16 bytes at offset tab[l] of an
// 8 KB LDS array, 64 times, in all four wavefronts of 256 workgroups); one
// launch per pattern, in the order printed.  The probe itself only runs the
// launches: the conflict counts come from running it under rocprofv3 with
// SQ_LDS_BANK_CONFLICT, one dispatch per pattern.  Prints one JSON line per
// pattern (its launch index and name).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <string>
#include <vector>

#define CHECK(x)                                                                               \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) {                                                                \
            std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));                \
            return 1;                                                                          \
        }                                                                                      \
    } while (0)

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kLdsBytes = 8192;

__global__ void __launch_bounds__(256) lds_fetch_kernel(const int *__restrict__ tab, float *out, int iters) {
    __shared__ __align__(16) unsigned char lds[kLdsBytes];
    for (int i = threadIdx.x; i < kLdsBytes / 4; i += 256) reinterpret_cast<float *>(lds)[i] = (float)i;
    __syncthreads();
    const int a = tab[threadIdx.x & 63];
    f4 s = f4{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it) {
        s += *reinterpret_cast<const f4 *>(lds + a);
        asm volatile("" ::: "memory");
    }
    out[blockIdx.x * 256 + threadIdx.x] = s[0] + s[1] + s[2] + s[3];
}

struct Pattern {
    std::string name;
    std::vector<int> tab;
};

// lane l: row l % 16 of a 16-row block with row stride `stride` bytes, 16-byte
// piece f(l / 16, row)
template <typename F>
static Pattern make(const std::string &name, int stride, F piece) {
    Pattern p{name, std::vector<int>(64)};
    for (int l = 0; l < 64; ++l) p.tab[l] = (l & 15) * stride + 16 * piece(l >> 4, l & 15);
    return p;
}

int main() {
    std::vector<Pattern> pats;
    Pattern lin{"contiguous 1 KB", std::vector<int>(64)};
    for (int l = 0; l < 64; ++l) lin.tab[l] = 16 * l;
    pats.push_back(lin);
    // 64-byte rows (BF16 planes, FP32 ring operands): piece g of row r
    pats.push_back(make("64B rows, no swizzle", 64, [](int g, int r) { return g; }));
    pats.push_back(make("64B rows, g ^ ((r >> 2) & 3)", 64, [](int g, int r) { return g ^ ((r >> 2) & 3); }));
    pats.push_back(make("64B rows, g ^ ((r >> 1) & 3)", 64, [](int g, int r) { return g ^ ((r >> 1) & 3); }));
    // 128-byte rows (FP64 ring operands): pieces 2 g and 2 g + 1 in two reads
    for (int h = 0; h < 2; ++h) {
        const std::string hs = h ? " (high piece)" : " (low piece)";
        pats.push_back(make("128B rows, (2g+h) ^ ((r >> 1) & 7)" + hs, 128,
                            [h](int g, int r) { return (2 * g + h) ^ ((r >> 1) & 7); }));
        pats.push_back(make("128B rows, (2g+h) ^ (r bit 1 | r bit 2 << 2)" + hs, 128,
                            [h](int g, int r) { return (2 * g + h) ^ (((r >> 1) & 1) | (r & 4)); }));
    }
    // the fused BF16 chain's state digit rows: 16 bytes at piece g of a row of `stride` bytes
    for (int stride = 192; stride <= 352; stride += 16)
        pats.push_back(make("row stride " + std::to_string(stride) + "B, no swizzle", stride,
                            [](int g, int r) { return g; }));

    int *dtab;
    float *out;
    CHECK(hipMalloc(&dtab, 64 * sizeof(int) * pats.size()));
    CHECK(hipMalloc(&out, 256 * 256 * sizeof(float)));
    for (size_t i = 0; i < pats.size(); ++i) {
        for (int a : pats[i].tab)
            if (a < 0 || a > kLdsBytes - 16 || a % 16) {
                std::fprintf(stderr, "pattern %zu out of range\n", i);
                return 1;
            }
        CHECK(hipMemcpy(dtab + 64 * i, pats[i].tab.data(), 64 * sizeof(int), hipMemcpyHostToDevice));
    }
    for (size_t i = 0; i < pats.size(); ++i) {
        lds_fetch_kernel<<<256, 256>>>(dtab + 64 * i, out, 64);
        CHECK(hipGetLastError());
    }
    CHECK(hipDeviceSynchronize());
    for (size_t i = 0; i < pats.size(); ++i)
        std::printf("{\"probe\": \"lds_fetch\", \"launch\": %zu, \"pattern\": \"%s\"}\n", i, pats[i].name.c_str());
    CHECK(hipFree(dtab));
    CHECK(hipFree(out));
    return 0;
}
