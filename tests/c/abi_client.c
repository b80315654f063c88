/* A plain C client of liblindblad.so: reads H, the collapse operators and a
 * batch of states from raw files, runs the Liouvillian, the propagator and
 * two chains (built-in choice and an explicit variant) through the C ABI on
 * device memory from the HIP runtime, and writes L, P and the final states.
 * Used by tests/test_gpu_c_client.py; no Python or torch involved.
 *
 *   abi_client DIR d K B nsteps dt variant
 * DIR holds H.bin (d*d complex128), Lk.bin (K*d*d), rho.bin (B*d*d);
 * it receives L.bin, P.bin, rho_out.bin, rho_variant.bin and s.txt. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lindblad.h"

static void *load(const char *dir, const char *name, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) return NULL;
    void *buf = malloc(bytes);
    if (buf && fread(buf, 1, bytes, f) != bytes) {
        free(buf);
        buf = NULL;
    }
    fclose(f);
    return buf;
}

static int save(const char *dir, const char *name, const void *buf, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "wb");
    if (!f) return 1;
    const size_t w = fwrite(buf, 1, bytes, f);
    fclose(f);
    return w != bytes;
}

#define HIP(x)                                                       \
    do {                                                             \
        if ((x) != hipSuccess) {                                     \
            fprintf(stderr, "HIP call failed: %s\n", #x);            \
            return 2;                                                \
        }                                                            \
    } while (0)
#define LB(x)                                                                  \
    do {                                                                       \
        int st_ = (x);                                                         \
        if (st_ != LB_OK) {                                                    \
            fprintf(stderr, "%s -> %d: %s\n", #x, st_, lindblad_last_error()); \
            return 3;                                                          \
        }                                                                      \
    } while (0)

int main(int argc, char **argv) {
    if (argc != 8) {
        fprintf(stderr, "usage: abi_client DIR d K B nsteps dt variant\n");
        return 1;
    }
    const char *dir = argv[1];
    const int d = atoi(argv[2]), K = atoi(argv[3]), B = atoi(argv[4]);
    const long long nsteps = atoll(argv[5]);
    const double dt = atof(argv[6]);
    const int variant = atoi(argv[7]);
    const int n = d * d;
    const size_t cz = 16;  /* complex128 */
    void *H = load(dir, "H.bin", (size_t)d * d * cz), *Lk = load(dir, "Lk.bin", (size_t)K * d * d * cz);
    void *rho = load(dir, "rho.bin", (size_t)B * n * cz);
    if (!H || !rho || (K > 0 && !Lk)) {
        fprintf(stderr, "missing input files\n");
        return 1;
    }
    void *dH, *dLk = NULL, *dL, *dP, *dX, *dY;
    HIP(hipMalloc(&dH, (size_t)d * d * cz));
    if (K > 0) HIP(hipMalloc(&dLk, (size_t)K * d * d * cz));
    HIP(hipMalloc(&dL, (size_t)n * n * cz));
    HIP(hipMalloc(&dP, (size_t)n * n * cz));
    HIP(hipMalloc(&dX, (size_t)B * n * cz));
    HIP(hipMalloc(&dY, (size_t)B * n * cz));
    HIP(hipMemcpy(dH, H, (size_t)d * d * cz, hipMemcpyHostToDevice));
    if (K > 0) HIP(hipMemcpy(dLk, Lk, (size_t)K * d * d * cz, hipMemcpyHostToDevice));
    HIP(hipMemcpy(dX, rho, (size_t)B * n * cz, hipMemcpyHostToDevice));
    HIP(hipMemcpy(dY, rho, (size_t)B * n * cz, hipMemcpyHostToDevice));

    lb_workspace *ws = NULL;
    LB(lb_workspace_create((size_t)1 << 30, &ws));
    hipStream_t stream;
    HIP(hipStreamCreate(&stream));
    LB(lindblad_liouvillian(d, dH, K, dLk, dL, stream));
    int s_used = -1, status = -100;
    int *dS = NULL, *dStatus = NULL;
    HIP(hipMalloc((void **)&dS, sizeof(int)));
    HIP(hipMalloc((void **)&dStatus, sizeof(int)));
    HIP(hipMemsetAsync(dStatus, 0, sizeof(int), stream));
    LB(lindblad_propagator(n, 1, dL, &dt, 0.25, dP, dS, dStatus, ws, stream));
    int chosen = 0;
    LB(lindblad_chain_variant(n, LB_C128, B, &chosen));
    LB(lindblad_propagate(n, dP, LB_C128, B, dX, nsteps, ws, stream));
    LB(lindblad_propagate_variant(n, dP, LB_C128, B, dY, nsteps, variant, ws, stream));
    HIP(hipStreamSynchronize(stream));
    HIP(hipMemcpy(&s_used, dS, sizeof(int), hipMemcpyDeviceToHost));
    HIP(hipMemcpy(&status, dStatus, sizeof(int), hipMemcpyDeviceToHost));
    if (status != LB_OK) return 6;

    void *out = malloc((size_t)n * n * cz);
    if (!out) return 1;
    HIP(hipMemcpy(out, dL, (size_t)n * n * cz, hipMemcpyDeviceToHost));
    if (save(dir, "L.bin", out, (size_t)n * n * cz)) return 4;
    HIP(hipMemcpy(out, dP, (size_t)n * n * cz, hipMemcpyDeviceToHost));
    if (save(dir, "P.bin", out, (size_t)n * n * cz)) return 4;
    HIP(hipMemcpy(rho, dX, (size_t)B * n * cz, hipMemcpyDeviceToHost));
    if (save(dir, "rho_out.bin", rho, (size_t)B * n * cz)) return 4;
    HIP(hipMemcpy(rho, dY, (size_t)B * n * cz, hipMemcpyDeviceToHost));
    if (save(dir, "rho_variant.bin", rho, (size_t)B * n * cz)) return 4;
    char txt[64];
    snprintf(txt, sizeof txt, "%d %d\n", s_used, chosen);
    if (save(dir, "s.txt", txt, strlen(txt))) return 4;

    /* an invalid call is rejected with a status and a message, nothing crashes */
    if (lindblad_propagate(0, dP, LB_C128, B, dX, 1, ws, stream) != LB_ESHAPE) return 5;
    if (strlen(lindblad_last_error()) == 0) return 5;

    LB(lb_workspace_destroy(ws));
    HIP(hipStreamDestroy(stream));
    hipFree(dH);
    if (dLk) hipFree(dLk);
    hipFree(dL);
    hipFree(dP);
    hipFree(dX);
    hipFree(dY);
    hipFree(dS);
    hipFree(dStatus);
    free(out);
    free(H);
    free(Lk);
    free(rho);
    return 0;
}
