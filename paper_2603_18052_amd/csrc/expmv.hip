// Action of the exponential: rho_b <- (e^{tL})^nsteps rho_b without forming
// the propagator (no Pade products, no LU solve) -- the follow-on direction
// the paper's GRAPE section names for removing the dense solve.  This leaves
// the fixed-propagator regime of the chain: every step applies a truncated
// Taylor series of t (L - mu I) with scaling and shifting (the approach of
// Al-Mohy & Higham, SIAM J. Sci. Comput. 33 (2011)):
//   mu = tr(L) / n,  X = t (L - mu I),  a = ||X||_1,
//   s sub-steps, m terms:  F <- e^{t mu / s} sum_{j <= m} (X / s)^j F / j!,
// with (s, m) minimising the number of products s m over theta in a fixed set
// subject to ||X / s||_1 <= theta and the remainder bound
//   e^{2 theta} theta^{m+1} / (m+1)!  <=  2^-53
// (the tail of the exponential series relative to a lower bound on
// ||e^{X/s}||), so each sub-step is accurate to FP64 rounding.  Fixed m, no
// early termination: the number of products per step is known up front.
#include <cmath>
#include <vector>

#include "chain.hpp"

namespace lb {
namespace {

__global__ void diag_kernel(int n, const cd *__restrict__ L, cd *__restrict__ diag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) diag[i] = L[(size_t)i * n + i];
}

// colsum[j] = sum_i |L[i][j] - mu delta_ij|, one workgroup per column,
// fixed-order reduction
__global__ void __launch_bounds__(256) shifted_colsum_kernel(int n, const cd *__restrict__ L, double mur, double mui,
                                                             double *__restrict__ colsum) {
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        cd v = L[(size_t)i * n + j];
        if (i == j) v = {v.re - mur, v.im - mui};
        acc += hypot(v.re, v.im);
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) colsum[j] = red[0];
}

const double kThetas[] = {0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0};
constexpr int kMaxTerms = 80;
constexpr long long kMaxProducts = 1 << 22;  // per step; larger norms are rejected

// smallest m with e^{2 theta} theta^{m+1} / (m+1)! <= 2^-53, in logs
int terms_for(double theta) {
    const double lim = -53.0 * std::log(2.0);
    for (int m = 1; m <= kMaxTerms; ++m)
        if (2.0 * theta + (m + 1) * std::log(theta) - std::lgamma((double)m + 2.0) <= lim) return m;
    return kMaxTerms;
}

}  // namespace

int expmv_params(double a, int *s_out, int *m_out) {
    if (!std::isfinite(a) || a < 0.0) return fail(LB_EINVAL, "expmv: norm must be finite and >= 0");
    if (a == 0.0) {  // X = 0: e^X = I
        *s_out = 1;
        *m_out = 1;
        return LB_OK;
    }
    long long best = -1;
    int bs = 1, bm = 1;
    for (double th : kThetas) {
        const double sd = std::ceil(a / th);
        if (sd > (double)kMaxProducts) continue;
        const long long sv = sd < 1.0 ? 1 : (long long)sd;
        const int m = terms_for(th);
        const long long cost = sv * m;
        if (cost <= kMaxProducts && (best < 0 || cost < best)) best = cost, bs = (int)sv, bm = m;
    }
    if (best < 0) return fail(LB_EINVAL, "expmv: ||t (L - mu I)||_1 too large for the series");
    *s_out = bs;
    *m_out = bm;
    return LB_OK;
}

}  // namespace lb

using namespace lb;

extern "C" int lindblad_expmv_params(double a, int *s, int *m) {
    if (!s || !m) return fail(LB_EINVAL, "lindblad_expmv_params: NULL output");
    return expmv_params(a, s, m);
}

extern "C" int lindblad_expmv(int n, const void *L, double t, int B, void *rho, long long nsteps, int *products,
                              lb_workspace *ws, hipStream_t stream) {
    LB_TRY(validate_chain("lindblad_expmv", n, L, B, rho, nsteps));
    if (!std::isfinite(t)) return fail(LB_EINVAL, "lindblad_expmv: t must be finite");
    Workspace *w = ws_resolve(ws);
    ws_begin(w, stream);
    const cd *Lc = static_cast<const cd *>(L);
    // shift and norm (host synchronisation: the series length depends on them)
    LB_TRY(ws_ensure(w, align256((size_t)n * sizeof(cd)) + align256((size_t)n * sizeof(double))));
    const size_t mark = w->used;
    cd *d_diag = (cd *)ws_take(w, (size_t)n * sizeof(cd));
    double *d_col = (double *)ws_take(w, (size_t)n * sizeof(double));
    diag_kernel<<<(n + 255) / 256, 256, 0, stream>>>(n, Lc, d_diag);
    LB_TRY(check_launch("expmv_diag"));
    std::vector<cd> diag(n);
    LB_HIP(hipMemcpyAsync(diag.data(), d_diag, n * sizeof(cd), hipMemcpyDeviceToHost, stream));
    LB_HIP(hipStreamSynchronize(stream));
    double tr_re = 0.0, tr_im = 0.0;
    for (int i = 0; i < n; ++i) tr_re += diag[i].re, tr_im += diag[i].im;
    const double mur = tr_re / n, mui = tr_im / n;
    shifted_colsum_kernel<<<n, 256, 0, stream>>>(n, Lc, mur, mui, d_col);
    LB_TRY(check_launch("expmv_colsum"));
    std::vector<double> col(n);
    LB_HIP(hipMemcpyAsync(col.data(), d_col, n * sizeof(double), hipMemcpyDeviceToHost, stream));
    LB_HIP(hipStreamSynchronize(stream));
    w->used = mark;
    double nrm = 0.0;
    for (int j = 0; j < n; ++j) nrm = col[j] > nrm ? col[j] : nrm;
    int s = 1, m = 1;
    LB_TRY(expmv_params(std::fabs(t) * nrm, &s, &m));
    if (products) *products = s * m;
    return expmv_run(n, Lc, t, mur, mui, s, m, B, static_cast<cd *>(rho), nsteps, w, stream);
}
