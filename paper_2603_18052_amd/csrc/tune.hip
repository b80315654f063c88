// Variant selection for the step chain and its autotuner.
//
// Several kernels can run the chain of one shape (n, precision, B); which is
// fastest depends on the shape and the device, so the library lists the
// variants that exist for a shape, picks one by a built-in rule, and lets a
// caller time them all once (lindblad_tune) and keep the winner for the rest
// of the process.  Every variant computes the same N steps; results differ by
// summation order only (within each precision's documented error).
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "chain.hpp"

namespace lb {

namespace {

typedef std::tuple<int, int, int, int> TuneKey;  // device, n, precision, B

std::mutex g_tune_mu;
std::map<TuneKey, int> g_tuned;

int current_device() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    return dev;
}

int tuned_variant(int n, lb_precision prec, int B) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tuned.find(TuneKey(current_device(), n, (int)prec, B));
    return it == g_tuned.end() ? 0 : it->second;
}

void set_tuned(int n, lb_precision prec, int B, int variant) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const TuneKey k(current_device(), n, (int)prec, B);
    if (variant == 0)
        g_tuned.erase(k);
    else
        g_tuned[k] = variant;
}

bool is_c(lb_precision p) { return p == LB_C128 || p == LB_C64; }

}  // namespace

int chain_variants(int n, lb_precision prec, int B, int *ids, int max) {
    int c = 0;
    auto add = [&](int v) {
        if (c < max) ids[c] = v;
        ++c;
    };
    auto add2 = [&](int v) {  // a per-step family: eager and graph-replayed
        add(v);
        add(v + kGraphVariant);
    };
    if (is_c(prec)) {
        if (prec == LB_C128) add2(VF_BASELINE * 100);
        if (n <= kWaveChainMaxN) add(VF_WAVE * 100);
        int kpus[8];
        const int nk = fused_kpus(n, prec, kpus, 8);
        for (int i = 0; i < nk; ++i) add(VF_FUSED * 100 + kpus[i]);
        if (balanced_ok(n, prec)) add(VF_BALANCED * 100);
        if (tail_ok(n, prec)) {
            add(VF_TAIL * 100);
            add(VF_TAIL * 100 + 1);
            add(VF_TAIL * 100 + 2);
            add(VF_TAIL * 100 + 3);
        }
        add2(VF_GEMM * 100 + 1);
        add2(VF_GEMM * 100 + 2);
        add2(VF_TGEMM * 100 + 4);
        add2(VF_TGEMM * 100 + 8);
        add2(VF_TGEMM * 100 + 1);
        add2(VF_TGEMM * 100 + 2);
        if (prec == LB_C64) add2(VF_MATVEC * 100);
    } else if (prec == LB_BF16_HILO || prec == LB_BF16_SLICED) {
        if (n <= bf16_fused_max_n(prec)) add(VF_BF16_FUSED * 100);
        add2(VF_PLANES * 100);
        add2(VF_TPLANES * 100);
        add2(VF_TPLANES * 100 + 1);
        add2(VF_TPLANES * 100 + 2);
    } else if (prec == LB_Q15) {
        if (n <= kWaveChainMaxN) add(VF_Q15 * 100);
        add2(VF_Q15 * 100 + 1);
        if (n <= fx_i8_max_n()) add(VF_FX_I8 * 100);
    } else if (prec == LB_Q31) {
        if (n <= fx_i8_max_n()) add(VF_FX_I8 * 100);
    } else if (prec == LB_I8_SLICED) {
        if (n <= i8_fused_max_n()) {
            add(VF_I8_FUSED * 100);
            add(VF_I8_FUSED * 100 + 1);
            add(VF_I8_FUSED * 100 + 2);
        }
        add2(VF_I8_GEMM * 100);
        add2(VF_I8_GEMM * 100 + 1);
        add2(VF_I8_GEMM * 100 + 2);
        add2(VF_I8_GEMM * 100 + 3);
    } else if (prec == LB_I8_HERM && i8_herm_shape_ok(n)) {
        if (n <= i8_herm_fused_max_n()) {
            add(VF_I8_FUSED * 100);
            add(VF_I8_FUSED * 100 + 1);
            add(VF_I8_FUSED * 100 + 2);
        }
        add2(VF_I8_GEMM * 100);
        add2(VF_I8_GEMM * 100 + 1);
        add2(VF_I8_GEMM * 100 + 2);
        add2(VF_I8_GEMM * 100 + 3);
    }
    return c;
}

// Built-in rule, from measurements on MI355X (d = 3 / 9 / 27 transmon
// chains): the register-resident wave chain for n <= 16 at every batch size;
// for FP64 with little work per step (B n^2 up to ~1e6) the plain per-state
// matvec, whose step is shorter than the fused kernel's 8-wavefront MFMA
// step; for n = 81 the fused chain with rows and columns 0..79 on MFMA, one
// whole 16-row tile per long wavefront, and row / column 80 on the VALU
// (21-26 % faster than the SIMD-balanced layout), else the SIMD-balanced
// fused chain where its layout exists (81 <= n <= 84 / 96, 17-20 % faster
// than the round-robin units there), the round-robin
// fused chain elsewhere while P fits in one CU's LDS; otherwise a
// GEMM per step: the LDS-tiled one (64 states x 48 outputs per workgroup,
// ring-pipelined) once its tiles fill the chip (>= 240), else one output
// tile per wavefront up to 256 states (more workgroups) and two beyond, or a
// matvec for few states.  BF16: the fused chain while P fits on chip, else
// the BF16 plane GEMM per step, LDS-tiled once its tiles fill the chip.
// INT8 digits: the fused chain while Q's digits fit in registers, else the
// per-step INT8 GEMM with the tile shape that fills the chip.
int chain_heuristic(int n, lb_precision prec, int B) {
    switch (prec) {
        case LB_C128:
        case LB_C64: {
            if (n <= kWaveChainMaxN) return VF_WAVE * 100;
            if (prec == LB_C128 && (double)B * n * n <= 1.1e6) return VF_BASELINE * 100;
            if (tail_ok(n, prec)) return VF_TAIL * 100 + (prec == LB_C128 ? 2 : 3);
            if (balanced_ok(n, prec)) return VF_BALANCED * 100;
            int kpu;
            if (fused_kpus(n, prec, &kpu, 1) == 1) return VF_FUSED * 100 + kpu;
            if (B >= 16) {
                const long long tiles = (long long)((B + 63) / 64) * ((n + 47) / 48);
                if (tiles >= 240)  // about one tile per CU or more: the ring-pipelined form
                    return VF_TGEMM * 100 + 1;
                return VF_GEMM * 100 + (B <= 256 ? 1 : 2);
            }
            return prec == LB_C128 ? VF_BASELINE * 100 : VF_MATVEC * 100;
        }
        case LB_BF16_HILO:
        case LB_BF16_SLICED: {
            if (n <= bf16_fused_max_n(prec)) return VF_BF16_FUSED * 100;
            return VF_TPLANES * 100 + 2;  // the ring kernel, k split over workgroups below 256 tiles
        }
        case LB_Q15:
            if (n <= kWaveChainMaxN) return VF_Q15 * 100;
            return n <= fx_i8_max_n() ? VF_FX_I8 * 100 : VF_Q15 * 100 + 1;
        case LB_Q31:
            return n <= fx_i8_max_n() ? VF_FX_I8 * 100 : 0;
        case LB_I8_SLICED: {
            if (n <= i8_fused_max_n()) return VF_I8_FUSED * 100;
            // 96 x 32 tiles with two LDS slots and two workgroups per CU
            // (variant 1503) while they give 240 or more workgroups, else
            // 64 x 16 with six slots (1502).  n = 729, us per step for 1500
            // (96 x 64) / 1501 (96 x 32, four slots) / 1502 / 1503, one box:
            // B = 1024 33.2 / 39.2 / 54.5 / 31.4, B = 768 30.4 / 38.7 / 45.7
            // / 29.1, B = 512 29.9 / 21.2 / 28.5 / 20.3, B = 256 30.4 / 21.1
            // / 19.9 / 20.6, B = 128 29.8 / 20.4 / 11.4 / 19.8
            const long long rb96 = (2 * n + 95) / 96;
            if (rb96 * ((B + 31) / 32) >= 240) return VF_I8_GEMM * 100 + 3;
            return VF_I8_GEMM * 100 + 2;
        }
        case LB_I8_HERM: {
            if (!i8_herm_shape_ok(n)) return 0;
            if (n <= i8_herm_fused_max_n()) return VF_I8_FUSED * 100;
            // the embedding's rule on the n rows of the Hermitian step
            const long long rb96 = (n + 95) / 96;
            if (rb96 * ((B + 31) / 32) >= 240) return VF_I8_GEMM * 100 + 3;
            return VF_I8_GEMM * 100 + 2;
        }
        default:
            return 0;
    }
}

static bool variant_listed(int n, lb_precision prec, int B, int variant) {
    int ids[32];
    const int c = chain_variants(n, prec, B, ids, 32);
    for (int i = 0; i < c && i < 32; ++i)
        if (ids[i] == variant) return true;
    return false;
}

size_t chain_ws_bytes(int n, lb_precision prec, int B, int variant) {
    const int fam = variant_family(variant);
    if (fam == VF_BASELINE) return align256((size_t)B * n * sizeof(cd));  // same for the graph twin
    if (fam == VF_Q15) return q15_ws_bytes(n, B, variant_param(variant) == 0);
    if (fam == VF_I8_GEMM) return i8_gemm_ws_bytes(n, B, prec == LB_I8_HERM);
    return large_ws_bytes(fam, n, prec, B);
}

int chain_run_variant(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, int variant,
                      Workspace *ws, hipStream_t s) {
    if (!variant_listed(n, prec, B, variant))
        return fail(LB_EINVAL, "chain variant " + std::to_string(variant) + " does not exist for this shape");
    if (nsteps == 0) return LB_OK;
    const int prm = variant_param(variant) % kGraphVariant;
    const bool graph = variant_param(variant) >= kGraphVariant;
    switch (variant_family(variant)) {
        case VF_BASELINE: return chain_baseline(n, P, B, rho, nsteps, ws, s, graph);
        case VF_WAVE: return chain_wave(n, P, prec, B, rho, nsteps, s);
        case VF_FUSED: return chain_fused(n, P, prec, prm, B, rho, nsteps, s);
        case VF_BF16_FUSED: return chain_bf16_fused(n, P, prec, B, rho, nsteps, s);
        case VF_GEMM: return chain_gemm(n, P, prec, prm, B, rho, nsteps, ws, s, graph);
        case VF_MATVEC: return chain_matvec(n, P, prec, B, rho, nsteps, ws, s, graph);
        case VF_PLANES: return chain_planes(n, P, prec, B, rho, nsteps, ws, s, graph);
        case VF_BALANCED: return chain_balanced(n, P, prec, B, rho, nsteps, s);
        case VF_Q15: return chain_q15(n, P, B, rho, nsteps, prm == 0, graph, ws, s);
        case VF_TAIL: return chain_tail(n, P, prec, prm, B, rho, nsteps, s);
        case VF_TGEMM: return chain_tgemm(n, P, prec, prm, B, rho, nsteps, ws, s, graph);
        case VF_TPLANES: return chain_planes(n, P, prec, B, rho, nsteps, ws, s, graph, prm == 0 ? 1 : prm + 1);
        case VF_I8_FUSED:
            return chain_i8_fused(n, P, B, rho, nsteps, s, prm == 1 ? 4 : 8, prm == 2, prec == LB_I8_HERM);
        case VF_FX_I8: return chain_fx_i8(n, P, prec, B, rho, nsteps, s);
        case VF_I8_GEMM: return chain_i8_gemm(n, P, B, rho, nsteps, ws, s, graph, prm, prec == LB_I8_HERM);
        default: return fail(LB_EINVAL, "unknown chain variant");
    }
}

int chain_run(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s) {
    if (nsteps == 0 || B == 0) return LB_OK;
    int v = tuned_variant(n, prec, B);
    if (v == 0) v = chain_heuristic(n, prec, B);
    if (v == 0) return fail(LB_ENOTSUP, "no chain kernel for this precision at n = " + std::to_string(n));
    return chain_run_variant(n, P, prec, B, rho, nsteps, v, ws, s);
}

}  // namespace lb

using namespace lb;

static int check_prec(const char *who, lb_precision prec) {
    if ((int)prec < LB_C128 || (int)prec > LB_I8_HERM) return fail(LB_EINVAL, std::string(who) + ": bad precision");
    return LB_OK;
}

extern "C" int lindblad_propagate(int n, const void *P, lb_precision prec, int B, void *rho, long long nsteps,
                                  lb_workspace *ws, hipStream_t stream) {
    LB_TRY(validate_chain("lindblad_propagate", n, P, B, rho, nsteps));
    LB_TRY(check_prec("lindblad_propagate", prec));
    Workspace *w = ws_resolve(ws);
    ws_begin(w, stream);
    return chain_run(n, static_cast<const cd *>(P), prec, B, static_cast<cd *>(rho), nsteps, w, stream);
}

extern "C" int lindblad_propagate_variant(int n, const void *P, lb_precision prec, int B, void *rho,
                                          long long nsteps, int variant, lb_workspace *ws, hipStream_t stream) {
    LB_TRY(validate_chain("lindblad_propagate_variant", n, P, B, rho, nsteps));
    LB_TRY(check_prec("lindblad_propagate_variant", prec));
    Workspace *w = ws_resolve(ws);
    ws_begin(w, stream);
    return chain_run_variant(n, static_cast<const cd *>(P), prec, B, static_cast<cd *>(rho), nsteps, variant, w,
                             stream);
}

extern "C" int lindblad_chain_variants(int n, lb_precision prec, int B, int *ids, int max_ids, int *count) {
    if (n < 1 || n > 4096 || B < 1) return fail(LB_ESHAPE, "lindblad_chain_variants: bad n or B");
    LB_TRY(check_prec("lindblad_chain_variants", prec));
    if (!count || (max_ids > 0 && !ids) || max_ids < 0) return fail(LB_EINVAL, "lindblad_chain_variants: bad output");
    *count = chain_variants(n, prec, B, ids, max_ids);
    return LB_OK;
}

extern "C" int lindblad_chain_variant(int n, lb_precision prec, int B, int *variant) {
    if (n < 1 || n > 4096 || B < 1) return fail(LB_ESHAPE, "lindblad_chain_variant: bad n or B");
    LB_TRY(check_prec("lindblad_chain_variant", prec));
    if (!variant) return fail(LB_EINVAL, "lindblad_chain_variant: NULL output");
    const int v = tuned_variant(n, prec, B);
    *variant = v ? v : chain_heuristic(n, prec, B);
    return LB_OK;
}

extern "C" int lindblad_tune_set(int n, lb_precision prec, int B, int variant) {
    if (n < 1 || n > 4096 || B < 1) return fail(LB_ESHAPE, "lindblad_tune_set: bad n or B");
    LB_TRY(check_prec("lindblad_tune_set", prec));
    if (variant != 0 && !variant_listed(n, prec, B, variant))
        return fail(LB_EINVAL, "lindblad_tune_set: variant " + std::to_string(variant) + " does not exist for this shape");
    set_tuned(n, prec, B, variant);
    return LB_OK;
}

extern "C" int lindblad_tune(int n, const void *P, lb_precision prec, int B, const void *rho, long long probe_steps,
                             int repeats, lb_workspace *ws, hipStream_t stream, int *best_variant, float *best_ms) {
    LB_TRY(validate_chain("lindblad_tune", n, P, B, rho, probe_steps));
    LB_TRY(check_prec("lindblad_tune", prec));
    if (probe_steps < 1 || repeats < 1) return fail(LB_EINVAL, "lindblad_tune: probe_steps and repeats must be >= 1");
    int ids[32];
    const int nv = chain_variants(n, prec, B, ids, 32);
    if (nv < 1 || nv > 32) return fail(LB_ENOTSUP, "lindblad_tune: no variants for this shape");
    Workspace *w = ws_resolve(ws);
    ws_begin(w, stream);
    const size_t xbytes = (size_t)B * n * sizeof(cd);
    size_t need = 0;
    for (int i = 0; i < nv; ++i) need = std::max(need, chain_ws_bytes(n, prec, B, ids[i]));
    LB_TRY(ws_ensure(w, align256(xbytes) + need));
    cd *x = (cd *)ws_take(w, xbytes);
    LB_HIP(hipMemcpyAsync(x, rho, xbytes, hipMemcpyDeviceToDevice, stream));
    const size_t base = w->used;
    hipEvent_t e0, e1;
    LB_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(LB_EHIP, "lindblad_tune: hipEventCreate failed");
    }
    int best = 0, st = LB_OK;
    float best_t = 0.f;
    const cd *Pc = static_cast<const cd *>(P);
    for (int i = 0; i < nv && st == LB_OK; ++i) {
        // a probe too short to replay a graph would time the direct twin again
        if (variant_param(ids[i]) >= kGraphVariant && probe_steps <= 2 * kGraphSteps &&
            (variant_family(ids[i]) == VF_BASELINE || variant_family(ids[i]) == VF_GEMM ||
             variant_family(ids[i]) == VF_MATVEC || variant_family(ids[i]) == VF_PLANES ||
             variant_family(ids[i]) == VF_Q15 || variant_family(ids[i]) == VF_TGEMM ||
             variant_family(ids[i]) == VF_TPLANES))
            continue;
        w->used = base;
        st = chain_run_variant(n, Pc, prec, B, x, probe_steps, ids[i], w, stream);  // warm-up
        float tmin = 0.f;
        for (int r = 0; r < repeats && st == LB_OK; ++r) {  // fastest of the repeats
            w->used = base;
            float ms = 0.f;
            if (hipEventRecord(e0, stream) != hipSuccess) {
                st = fail(LB_EHIP, "lindblad_tune: hipEventRecord failed");
                break;
            }
            st = chain_run_variant(n, Pc, prec, B, x, probe_steps, ids[i], w, stream);
            if (st != LB_OK) break;
            if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = fail(LB_EHIP, "lindblad_tune: timing failed");
                break;
            }
            if (r == 0 || ms < tmin) tmin = ms;
        }
        if (st != LB_OK) break;
        if (best == 0 || tmin < best_t) {
            best = ids[i];
            best_t = tmin;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != LB_OK) return st;
    set_tuned(n, prec, B, best);
    if (best_variant) *best_variant = best;
    if (best_ms) *best_ms = best_t;
    return LB_OK;
}
