// Internal launchers of the propagation chain (lindblad_propagate) and its
// variants.  Every variant runs the same N steps x <- P x on each state; they
// differ in kernel, tiling and summation order only.
#pragma once
#include "lb_internal.hpp"

namespace lb {

// Variant ids: family * 100 + tile parameter; + kGraphVariant for the
// per-step families (baseline, GEMM, matvec, planes) replays the steps from a
// captured HIP graph.
constexpr int kGraphVariant = 50;
enum ChainFamily : int {
    VF_BASELINE = 1,    // plain FP64 per-state matvec, one launch per step
    VF_WAVE = 2,        // one wavefront per state, P rows in registers (n <= kWaveChainMaxN)
    VF_FUSED = 3,       // whole chain in one launch, P on chip; param = k steps per unit
    VF_BF16_FUSED = 4,  // whole BF16 chain in one launch (n <= bf16_fused_max_n)
    VF_GEMM = 5,        // one MFMA GEMM launch per step; param = 16-output tiles per wavefront
    VF_MATVEC = 6,      // per-state FP32 matvec, one launch per step (LB_C64)
    VF_PLANES = 7,      // one BF16 plane-GEMM launch per step
    VF_BALANCED = 8,    // fused chain with the SIMD-balanced layout (81 <= n <= 84 / 96)
    VF_Q15 = 9,         // fixed-point chain (LB_Q15); param 0 one wavefront per state, 1 per-row matvec
    VF_TAIL = 10,       // fused chain, rows 0..79 on MFMA, the rest on the VALU (n = 81); param = layout 0..3
    VF_TGEMM = 11,      // one LDS-tiled MFMA GEMM launch per step (64 states x 48 outputs); param = wavefronts 4 / 8, 1 = ring, 2 = ring + split k
    VF_TPLANES = 12,    // one LDS-tiled BF16 plane-GEMM launch per step (64 states x 48 outputs); param 1: ring-pipelined, 2: ring + split k
    VF_I8_FUSED = 13,   // whole INT8-digit chain in one launch (LB_I8_SLICED, n <= i8_fused_max_n; LB_I8_HERM)
    VF_FX_I8 = 14,      // fixed-point chain (LB_Q15, LB_Q31) on the INT8 matrix cores, one launch (n <= 96)
    VF_I8_GEMM = 15,    // one LDS-tiled INT8-digit GEMM launch per step (LB_I8_SLICED, any n)
};
inline int variant_family(int v) { return v / 100; }
inline int variant_param(int v) { return v % 100; }

int validate_chain(const char *who, int n, const void *P, int B, const void *rho, long long nsteps);

// Largest n whose fused, LDS-resident chain exists for each precision.
int fused_max_n(lb_precision prec);
bool fused_kpu_ok(int n, lb_precision prec, int kpu);
int fused_kpus(int n, lb_precision prec, int *kpus, int max);  // valid k-steps-per-unit values, ascending

int chain_baseline(int n, const cd *P, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s,
                   bool graph = false);
constexpr int kWaveChainMaxN = 16;
int chain_wave(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, hipStream_t s);
int chain_fused(int n, const cd *P, lb_precision prec, int kpu, int B, cd *rho, long long nsteps, hipStream_t s);
bool balanced_ok(int n, lb_precision prec);
int chain_balanced(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, hipStream_t s);
bool tail_ok(int n, lb_precision prec);
int chain_tail(int n, const cd *P, lb_precision prec, int layout, int B, cd *rho, long long nsteps, hipStream_t s);

// LB_BF16_SLICED always runs 5 x 4 digits with levels <= 4 (14 slice pairs),
// whatever the call's step count: a long run issued as many short calls
// keeps the bound of one long call, and the tuner's short probes time the
// kernels that the real call runs.
int bf16_fused_max_n(lb_precision prec);
int i8_fused_max_n();
// waves: 8 (two wavefronts per SIMD) or 4 (one); pipe: steps synchronised
// by per-tile progress words instead of a barrier (eight wavefronts only).
// Variants 1300 / 1301 (8 / 4, barrier), 1302 (8, pipelined).  herm: the
// Hermitian-coordinate form (LB_I8_HERM: n = d^2, the n x n real step on
// the d^2 real coordinates of a Hermitian state), n <= i8_herm_fused_max_n
int chain_i8_fused(int n, const cd *P, int B, cd *rho, long long nsteps, hipStream_t s, int waves, bool pipe,
                   bool herm);
int i8_herm_fused_max_n();
bool i8_herm_shape_ok(int n);  // n = d^2
int fx_i8_max_n();
size_t i8_gemm_ws_bytes(int n, int B, bool herm);
// shape: 0 = 96 x 64 tiles, 1 = 96 x 32, 2 = 64 x 16 (rows of Q x states), 3 = 96 x 32
// with two LDS slots, two workgroups per CU; herm: the Hermitian-coordinate
// form (LB_I8_HERM, n = d^2: the n x n real step)
int chain_i8_gemm(int n, const cd *P, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s, bool graph,
                  int shape, bool herm);
int chain_fx_i8(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, hipStream_t s);
int chain_bf16_fused(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, hipStream_t s);

int chain_gemm(int n, const cd *P, lb_precision prec, int wn, int B, cd *rho, long long nsteps, Workspace *ws,
               hipStream_t s, bool graph = false);
int chain_matvec(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, Workspace *ws,
                 hipStream_t s, bool graph = false);
int chain_planes(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, Workspace *ws,
                 hipStream_t s, bool graph = false, int tiled = 0);
int chain_tgemm(int n, const cd *P, lb_precision prec, int waves, int B, cd *rho, long long nsteps, Workspace *ws,
                hipStream_t s, bool graph = false);
size_t large_ws_bytes(int family, int n, lb_precision prec, int B);
// e^{tL} applied by s sub-steps of an m-term Taylor series of t (L - mu I) / s
int expmv_run(int n, const cd *L, double t, double mur, double mui, int s, int m, int B, cd *rho, long long nsteps,
              Workspace *ws, hipStream_t st);
int expmv_params(double a, int *s, int *m);
int chain_q15(int n, const cd *P, int B, cd *rho, long long nsteps, bool wave, bool graph, Workspace *ws,
              hipStream_t s);
size_t q15_ws_bytes(int n, int B, bool wave);

// Variant selection (tune.hip): the list of variants that exist for a shape,
// the built-in choice, the tuned choice if any, and the dispatcher.
int chain_variants(int n, lb_precision prec, int B, int *ids, int max);
int chain_heuristic(int n, lb_precision prec, int B);
size_t chain_ws_bytes(int n, lb_precision prec, int B, int variant);
int chain_run_variant(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, int variant,
                      Workspace *ws, hipStream_t s);
int chain_run(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s);

}  // namespace lb
