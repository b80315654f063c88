/*
 * lindblad.h -- C-ABI of liblindblad.so, dense time-independent Lindblad
 * propagation on one AMD Instinct MI355X (gfx950).
 *
 * Paper: "Hardware-Aware Performance Characterization of Small Dense Lindblad
 * Propagation for Near-Term Quantum Control", arXiv 2603.18052.
 *
 * Conventions (every call):
 *  - Matrices are row-major.  Complex numbers are interleaved {double re, im}
 *    (numpy/torch complex128).  A d x d density matrix stored row-major IS the
 *    length-n vector of the vectorised equation (n = d*d); the paper's step
 *    (Sec. 3, Alg. 2 storage note) uses the same row-major vectorisation.
 *  - Every array pointer is a DEVICE pointer owned by the caller, unless the
 *    argument is marked "host".  The library never frees, reallocates or
 *    keeps caller memory after a call returns.
 *  - `stream` is the caller's hipStream_t (NULL = the legacy default stream).
 *    Work is enqueued on it in order.  Calls that document a host
 *    synchronisation block the host until their own work on `stream` ends.
 *  - The return value is an lb_status.  Validation errors are detected before
 *    anything is enqueued and leave every output untouched.  On any non-zero
 *    status lindblad_last_error() returns a message (thread-local, valid until
 *    the next call on the same thread).  No C++ exception crosses the ABI.
 *  - Scratch memory comes from an lb_workspace.  Passing NULL selects the
 *    library's per-device default workspace (grown on demand, cap 64 GiB).
 *    Growth is stream-ordered on the call's stream (the old buffer goes back
 *    with hipFreeAsync after the work already enqueued there, the new one
 *    comes from hipMallocAsync) and does not block the host.  Calls that
 *    share one workspace must be ordered (same stream, or synchronised by the
 *    caller): the workspace is not locked.
 */
#ifndef LINDBLAD_H
#define LINDBLAD_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LB_OK = 0,
    LB_EINVAL = -1,      /* bad argument value (NULL pointer, negative count, bad enum) */
    LB_ESHAPE = -2,      /* unsupported size (d, n, B, K, C out of the supported range) */
    LB_ENOMEM = -3,      /* workspace cap exceeded or device allocation failed */
    LB_EHIP = -4,        /* a HIP runtime call failed (launch, copy, synchronise) */
    LB_ESINGULAR = -5,   /* zero pivot in the LU of the Pade denominator V - U */
    LB_ENONFINITE = -6,  /* NaN or Inf in ||L dt||_1: the scaling exponent is undefined */
    LB_ENOTSUP = -7      /* valid request this build does not implement */
} lb_status;

/* Arithmetic of the propagation chain (lindblad_propagate).  The state is
 * always handed over as complex128; the variants differ in how P and the
 * in-flight state are represented inside the kernel. */
typedef enum {
    LB_C128 = 0,        /* complex FP64: P and states FP64, FP64 MFMA accumulation */
    LB_C64 = 1,         /* complex FP32: P rounded to FP32 (nearest-even), FP32 MFMA accumulation,
                           state rounded to FP32 after every step */
    LB_BF16_HILO = 2,   /* split BF16: P = Phi + Plo and x = xhi + xlo in BF16, products
                           Phi xhi + Phi xlo + Plo xhi on BF16 MFMA with FP32 accumulation */
    LB_BF16_SLICED = 3, /* exponent-aligned BF16 integer slices of P (per row) and of each
                           state (per state): every slice product sums exactly in the FP32
                           MFMA accumulator; slice pairs are combined in FP64.  One digit
                           set for every call (5 digits of P, 4 of the state, levels <= 4),
                           so a run split into several calls keeps the bound of one call */
    LB_Q15 = 4          /* the paper's fixed-point step (Alg. 5): P and the state quantised to
                           Q1.15 (16-bit, 15 fractional bits; round to nearest, ties to even,
                           saturating, so 1.0 becomes 1 - 2^-15), each step's sums exact in
                           64-bit integers, then floor(acc / 2^15) saturated.  Results are
                           integers / 2^15, bitwise reproducible and independent of the kernel */,
    LB_I8_SLICED = 5    /* exponent-aligned INT8 digit slices on the INT8 matrix cores: the step
                           as its real embedding [[Re P, -Im P], [Im P, Re P]] (2n x 2n); rows of
                           that matrix scaled by their own power of two and rounded to 38
                           fraction bits, five balanced base-256 digits; each state scaled by
                           its own power of two, rounded to 30 fraction bits, four digits; the
                           14 digit pairs of levels <= 4 summed EXACTLY in int32 accumulators
                           over the whole k range, levels combined in FP64 and the state
                           re-sliced every step.  One digit set for every call length.  One
                           fused launch for n <= 96; beyond, one INT8 GEMM launch per step, the
                           next state sliced below 2^(M + g) with M the exponent of the previous
                           state's largest entry and 2^g the largest row sum of the embedding */,
    LB_Q31 = 6,         /* the paper's fixed-point step at 31 fraction bits (its Q1.31 drift
                           curve): LB_Q15's rules with 32-bit codes, sums exact in 128 bits,
                           floor(acc / 2^31) saturated.  Bitwise reproducible; n <= 96 */
    LB_I8_HERM = 7      /* LB_I8_SLICED's digits and rules on the real coordinates of a
                           HERMITIAN state (a density matrix; n = d^2).  The Lindblad
                           generator (Eq. 1), exp(L dt) and its Pade approximant map rho^dagger
                           to (P rho)^dagger, so the step is one real n x n matrix R on the
                           coordinates h_(i,j) = Re rho_ij (i <= j), Im rho_ij (i > j):
                           half the rows and half the k of the 2n x 2n embedding.  The call
                           reads only those entries of each state (the Hermitian matrix they
                           define) and writes a Hermitian result.  One fused launch for
                           n <= 192, beyond one INT8 GEMM launch per step as LB_I8_SLICED.
                           No kernel (LB_ENOTSUP) unless n is a perfect square */
} lb_precision;

typedef struct lb_workspace lb_workspace;

/* Library-owned device scratch on the current device (the paper's reusable
 * matrix-exponential workspace, Sec. 2 "Reusable Propagator Construction").
 * Memory is allocated on first need and grown up to `max_bytes` (stream-
 * ordered, see above); a request beyond the cap fails with LB_ENOMEM.
 * destroy synchronises the device before freeing.  Thread-compatible, not
 * thread-safe. */
int lb_workspace_create(size_t max_bytes, lb_workspace **ws);
int lb_workspace_destroy(lb_workspace *ws);
/* Bytes currently allocated by the workspace (host query, no device work). */
size_t lb_workspace_bytes(const lb_workspace *ws);

/* Message of the last failing call on this thread ("" if none). */
const char *lindblad_last_error(void);

/* Superoperator of the Lindblad master equation, Eq. (1), vectorised row-major
 * (Eqs. (2)-(3)):
 *   L = -i (H (x) I - I (x) H^T)
 *       + sum_k [ Lk (x) conj(Lk) - 1/2 (Lk^dag Lk) (x) I - 1/2 I (x) (Lk^dag Lk)^T ]
 * so that L vec(rho) = vec(-i[H, rho] + sum_k D[Lk] rho) for every rho.
 *   d     : Hilbert-space dimension, 1 <= d <= 64 (n = d*d <= 4096)
 *   H     : d x d complex128 (need not be Hermitian; used as given)
 *   K     : number of collapse operators, 0 <= K <= 64
 *   Lk    : K x d x d complex128 (may be NULL when K = 0)
 *   Lout  : n x n complex128, written completely
 * Asynchronous; no workspace. */
int lindblad_liouvillian(int d, const void *H, int K, const void *Lk, void *Lout, hipStream_t stream);

/* Control-affine slice generators (Eq. (5), one generator per segment):
 *   Lout[m] = L0 + sum_c u[m*C + c] * Lc[c],   m = 0..M-1
 *   n     : superoperator size, 1 <= n <= 4096
 *   L0    : n x n complex128 (drift incl. dissipators); Lc: C x n x n complex128
 *   u     : M x C double (device); Lout: M x n x n complex128
 *   0 <= C <= 64, M >= 0.  Asynchronous; no workspace. */
int lindblad_generators(int n, int M, int C, const void *L0, const void *Lc, const double *u,
                        void *Lout, hipStream_t stream);

/* Propagators P[m] = exp(L[m] dt[m]) by Alg. 1: scaling exponent
 * s = smallest s >= 0 with ||A||_1 <= theta 2^s (A = L dt, ||.||_1 the largest
 * column sum of complex moduli), Pade [13/13] numerator V + U and denominator
 * V - U of A / 2^s (three powers, three products), LU with partial pivoting of
 * V - U (largest modulus, lowest row on ties) solving for P with the n columns
 * of V + U as right-hand sides, then s squarings.  FP64 throughout.
 *   n      : 1 <= n <= 4096;  M >= 1 generators, L is M x n x n complex128
 *   dt     : HOST array of M finite step lengths (read before the call
 *            returns; the values travel to the device as kernel arguments)
 *   theta  : threshold, > 0 (the paper uses 0.25; Higham's is 5.37)
 *   P      : M x n x n complex128 output (may alias nothing else)
 *   s_used : DEVICE array of M ints receiving s, or NULL
 *   status : DEVICE int, or NULL.  The caller sets it to LB_OK (0) before the
 *            call; the build lowers it (atomic min, so the smallest code
 *            wins) to LB_ENOTSUP if some s exceeds 24 (||A||_1 > 2^22: the
 *            squarings are enqueued up to that cap), LB_ENONFINITE if some
 *            ||A||_1 is not finite, LB_ESINGULAR if some denominator has an
 *            exactly zero pivot.  P of such a generator is unspecified.
 * Stream-ordered and asynchronous: nothing blocks the host.  s and the
 * status stay on the device; the squarings run as masked launches up to the
 * cap, each skipping on the device the matrices whose s it exceeds.  The
 * return value covers argument checks, workspace limits and launch errors
 * only. */
int lindblad_propagator(int n, int M, const void *L, const double *dt, double theta, void *P,
                        int *s_used, int *status, lb_workspace *ws, hipStream_t stream);

/* The build of lindblad_propagator timed by stage, the method of the paper's
 * build-time breakdown (Table "Build-time breakdown per landscape point"):
 * HIP events recorded on `stream` at the stage boundaries give
 *   stage_ms[0] the LU solve of the Pade denominator (Alg. 1),
 *   stage_ms[1] the Pade products (powers, V, W, U: Alg. 1),
 *   stage_ms[2] the s squarings,
 *   stage_ms[3] everything else (norm and scaling, V -/+ U, copies and the
 *               host's part of the scaling stage),
 * summed over the chunks the workspace splits the batch into.  Same
 * arguments and result P as lindblad_propagator except: s_host is a HOST
 * array of M ints (or NULL), the call synchronises the stream (a
 * measurement call, not for pipelines) and data-dependent failures are
 * returned (LB_ENONFINITE, LB_ESINGULAR) instead of written to a status
 * word.  stage_ms: HOST array of 4 doubles. */
int lindblad_propagator_stages(int n, int M, const void *L, const double *dt, double theta, void *P,
                               int *s_host, double *stage_ms, lb_workspace *ws, hipStream_t stream);

/* lindblad_propagator for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same build, arguments, results and status word, with no
 * workspace argument.  Its scratch is a fixed device array inside the
 * library, 80 MiB per device (lindblad_propagator_noalloc_scratch_bytes()),
 * held until the process ends; the call itself allocates nothing
 * (no hipMalloc / hipFree / hipMallocAsync, no library allocation).
 *   n      : 1 <= n <= 809 (one n x n build needs 128 n^2 bytes plus a
 *            little; larger n fail with LB_ENOMEM before anything runs)
 *   M      : any M >= 1; batches are built in chunks that fit the scratch
 *            (one after another on `stream`)
 * Stream-ordered and asynchronous like lindblad_propagator.  Every call on a
 * device shares that device's scratch and leaves its contents behind: calls
 * that overlap on one device (several streams or threads) race and must be
 * serialised by the caller. */
int lindblad_propagator_noalloc(int n, int M, const void *L, const double *dt, double theta, void *P,
                                int *s_used, int *status, hipStream_t stream);
size_t lindblad_propagator_noalloc_scratch_bytes(void);

/* The step chain, Alg. 2 applied nsteps times to each of B independent states
 * (Alg. 3 parallelism): rho_b <- P^nsteps rho_b.
 *   n      : 1 <= n <= 4096 (n = d*d)
 *   P      : n x n complex128 (converted once per call to `prec`'s format)
 *   prec   : lb_precision
 *   B      : number of states, >= 1
 *   rho    : B x n complex128, in place (row b = vec of state b)
 *   nsteps : >= 0
 * Asynchronous.  Every precision runs for every n.  The kernel ("variant")
 * is the one lindblad_tune recorded for (n, prec, B) on this device, else
 * the built-in rule: one wavefront per state with P rows in registers for
 * n <= 16 (LB_C128, LB_C64); the plain per-state matvec for LB_C128 when
 * B n^2 <= 1.1e6; the whole chain in one launch with P on chip while it fits
 * one compute unit's LDS (n <= 84 LB_C128, 124 LB_C64, 85 LB_BF16_SLICED,
 * 96 LB_BF16_HILO; for n = 81 rows and columns 0..79 on MFMA and row and
 * column 80 on the vector ALUs, else the SIMD-balanced layout for
 * 81 <= n <= 84 / 96); beyond
 * that one MFMA GEMM launch per step (B >= 16; the ring-pipelined LDS-tiled
 * one, variant 1101, once ceil(B / 64) ceil(n / 48) >= 240) or a per-state
 * matvec (B < 16); for the
 * BF16 precisions the ring-pipelined plane GEMM, its k range split over
 * workgroups when the batch has fewer than 256 tiles. */
int lindblad_propagate(int n, const void *P, lb_precision prec, int B, void *rho, long long nsteps,
                       lb_workspace *ws, hipStream_t stream);

/* The plain per-state FP64 matvec chain the fast paths are measured against:
 * one launch per step, each wavefront reads rows of P from memory (coalesced)
 * for one state and reduces with cross-lane shuffles.  Same arguments and
 * result as lindblad_propagate with LB_C128.  Asynchronous. */
int lindblad_propagate_baseline(int n, const void *P, int B, void *rho, long long nsteps,
                                lb_workspace *ws, hipStream_t stream);

/* Action of the exponential without forming the propagator -- the
 * alternative the paper's GRAPE section names for removing the dense LU
 * solve; it leaves the fixed-propagator regime (every step re-applies a
 * series in L):  rho_b <- (e^{tL})^nsteps rho_b  for b < B.
 *   n      : 1 <= n <= 4096
 *   L      : n x n complex128 generator (row-major), DEVICE memory
 *   t      : finite step length
 *   B, rho : B x n complex128 states, DEVICE memory, in place
 *   nsteps : >= 0
 *   products (optional HOST int*): receives s m, the number of products
 *            L V per step
 * FP64 throughout: mu = tr(L) / n, X = t (L - mu I); s sub-steps of the
 * m-term Taylor series of X / s, each times e^{t mu / s}; (s, m) from
 * lindblad_expmv_params(||X||_1).  Synchronises the stream once (the series
 * length depends on ||X||_1), then enqueues the steps.  LB_EINVAL if
 * ||X||_1 is not finite or too large for the series. */
int lindblad_expmv(int n, const void *L, double t, int B, void *rho, long long nsteps, int *products,
                   lb_workspace *ws, hipStream_t stream);

/* Host only: the sub-steps s and terms m lindblad_expmv uses for
 * ||t (L - mu I)||_1 = a >= 0: the smallest product count s m over theta in
 * {0.5, 1, ..., 4} with a / s <= theta and
 * e^{2 theta} theta^{m+1} / (m+1)! <= 2^-53 (a = 0: s = m = 1). */
int lindblad_expmv_params(double a, int *s, int *m);

/* Chain variants and their autotuner (Alg. 2 / Alg. 3: the same steps, a
 * choice of kernel and tile shape).  A variant id is family * 100 + tile
 * parameter:
 *   100       plain FP64 per-state matvec (LB_C128 only)
 *   200       one wavefront per state, P rows in registers (n <= 16)
 *   300 + k   whole chain in one launch, P as MFMA fragments in registers,
 *             k = 4-deep k steps per work unit (n within the fused limit)
 *   400       whole BF16 chain in one launch (BF16 precisions, fused limit)
 *   500 + w   one MFMA GEMM launch per step, w = 16-output tiles per wavefront
 *   600       per-state FP32 matvec, one launch per step (LB_C64 only)
 *   700       one BF16 plane-GEMM launch per step (BF16 precisions)
 *   800       whole chain in one launch, the two wavefronts of every SIMD
 *             balanced (81 <= n <= 84 LB_C128, <= 96 LB_C64)
 *   900       LB_Q15, one wavefront per state (n <= 16)
 *   901       LB_Q15, one per-row matvec launch per step
 *   1000      whole chain in one launch, rows 0..79 on MFMA in three k parts
 *             per tile, row 80 on the vector ALUs (n = 81, LB_C128 / LB_C64)
 *   1001      the same with 16 wavefronts per workgroup, one part each
 *   1002      whole chain in one launch, rows and columns 0..79 on MFMA with
 *             one whole 16-row tile per wavefront, row and column 80 on the
 *             vector ALUs (n = 81, LB_C128 / LB_C64)
 *   1003      the same with the partial sums of rows 64..80 formed once a
 *             step by the last wavefront to finish them
 *   1100 + w  one LDS-tiled MFMA GEMM launch per step, 64 states x 48 outputs
 *             per workgroup, w = 4 or 8 wavefronts (LB_C128 / LB_C64)
 *   1101      the same tile with k chunks loaded straight into an LDS ring a few
 *             chunks ahead (four wavefronts)
 *   1102      1101 with the k range split over workgroups (FP64 partial sums
 *             added in a fixed order)
 *   1200      one LDS-tiled BF16 plane-GEMM launch per step, 64 states x 48
 *             outputs per workgroup, direct global-to-LDS loads (BF16 precisions)
 *   1201      the same tile with each wavefront's state planes staged per 64-k
 *             pair and a ring of propagator chunks loaded 2-3 chunks ahead
 *   1202      1201 with the k range split over workgroups when the batch has
 *             fewer than 256 tiles (partial sums added in a fixed order)
 *   1300      LB_I8_SLICED, whole chain in one launch (n <= 96), eight
 *             wavefronts of up to two 16-row tiles, a barrier per step;
 *             1300 .. 1302 are also LB_I8_HERM's variants (n = d^2 <= 192), and
 *             so are 1500 .. 1503 (any n = d^2)
 *   1301      the same with four wavefronts of up to three tiles
 *   1302      eight wavefronts, steps synchronised by per-tile progress words
 *             in LDS instead of a barrier (three state digit buffers)
 *   1400      LB_Q15 / LB_Q31, whole chain in one launch on the INT8 matrix
 *             cores (n <= 96)
 *   1500      LB_I8_SLICED, one INT8-digit GEMM launch per step, 96 rows x 64
 *             states per workgroup, three LDS ring slots
 *   1501      96 rows x 32 states, four ring slots
 *   1502      64 rows x 16 states, six ring slots
 *   1503      96 rows x 32 states, two ring slots, two workgroups per CU
 * 1300 .. 1302 give the same bits, and so do 1500 .. 1503.
 * Adding 50 to a per-step family (100, 500 + w, 600, 700, 901, 1100 + w,
 * 1101, 1102, 1200 .. 1202, 1500 .. 1503) replays its steps
 * from a HIP graph captured once per call (32 steps, replayed over all but
 * the last step).  Variants of one shape differ only in summation order. */

/* Variants that exist for (n, prec, B): up to max_ids ids written to the HOST
 * array ids, the total number to *count. */
int lindblad_chain_variants(int n, lb_precision prec, int B, int *ids, int max_ids, int *count);

/* The variant lindblad_propagate runs for (n, prec, B) on the current device
 * (tuned, else the built-in rule), to the HOST int *variant. */
int lindblad_chain_variant(int n, lb_precision prec, int B, int *variant);

/* lindblad_propagate with an explicit variant; LB_EINVAL if the variant does
 * not exist for the shape.  Asynchronous. */
int lindblad_propagate_variant(int n, const void *P, lb_precision prec, int B, void *rho, long long nsteps,
                               int variant, lb_workspace *ws, hipStream_t stream);

/* Autotuner: runs every variant of (n, prec, B) for probe_steps steps on a
 * workspace copy of rho (rho itself is only read), `repeats` times after one
 * warm-up run (graph-replayed twins only when probe_steps > 64, since a
 * shorter probe replays nothing), times each with HIP events on `stream`, and
 * records the
 * fastest for (current device, n, prec, B) for the rest of the process.
 * *best_variant and *best_ms (its fastest probe run in ms; both HOST, may be
 * NULL) receive the winner.  Synchronises the host with `stream`.  Thread-safe
 * table; calls that share a workspace must still be ordered. */
int lindblad_tune(int n, const void *P, lb_precision prec, int B, const void *rho, long long probe_steps,
                  int repeats, lb_workspace *ws, hipStream_t stream, int *best_variant, float *best_ms);

/* Record `variant` for (current device, n, prec, B) without timing (e.g. a
 * choice saved from an earlier tuning run); 0 removes the record. */
int lindblad_tune_set(int n, lb_precision prec, int B, int variant);

/* GRAPE fidelity and its gradient for piecewise-constant controls.
 * (Not in the paper, which runs only the forward landscape point of Eq. (5).)
 *   L0 : n x n complex128 generator of the drift (coherent + dissipative)
 *   Lc : C x n x n complex128 control generators (coherent, -i[Hc, .])
 *   u  : M x C double amplitudes (device); dt: slice length
 *   x0 : n complex128 initial state; w: n complex128 target (vec of sigma)
 *   A_m = dt (L0 + sum_c u[m,c] Lc[c]),  P_m = exp(A_m)  (Alg. 1)
 *   x_m = P_m x_{m-1},  F = Re <w, x_M>
 *   dF/du[m,c] = Re Tr(dt Lc[c] G_m),  G_m = L(A_m, x_{m-1} lambda_m^dag)
 *   lambda_M = w, lambda_{m-1} = P_m^dag lambda_m
 * where L(A, E) is the Frechet derivative of exp at A in direction E,
 * evaluated with the Pade [13/13] derivative recurrences that share the LU of
 * V - U, followed by the squaring recurrence L <- R L + L R.
 *   F    : HOST double;  grad: M x C double (device)
 *   checkpoint_bytes : if the propagators of all slices (M n^2 16 bytes) do not
 *          fit in this budget, they are not kept; each backward slice is rebuilt
 *          (forward states x_m are always kept: (M+1) n 16 bytes).  <= 0: no limit.
 * Synchronises the host with `stream`.  Returns the propagator's statuses. */
int grape_gradient(int n, int M, int C, const void *L0, const void *Lc, const double *u, double dt,
                   double theta, const void *x0, const void *w, double *F, double *grad,
                   long long checkpoint_bytes, lb_workspace *ws, hipStream_t stream);

/* One entry of a mixed batch: its own generator, step and state. */
typedef struct lb_problem {
    int d;                /* 3, 9 or 27 (any d with d*d <= 4096 is accepted) */
    const void *L;        /* n x n complex128 generator (device) */
    double dt;            /* step length */
    long long nsteps;     /* >= 0 */
    void *rho;            /* n complex128 state, in place (device) */
} lb_problem;

/* Mixed serving batch: builds every problem's propagator in FP64 (Alg. 1,
 * problems of one size batched together) and runs every chain in `prec`
 * (problems of one size advance together; states whose step count is reached
 * stop being updated).  probs is a HOST array.  Synchronises the host. */
int lindblad_batch_run(const lb_problem *probs, int nprob, lb_precision prec, double theta,
                       lb_workspace *ws, hipStream_t stream);

/* lindblad_batch_run without any host synchronisation, so that a caller can
 * capture the whole batch into one HIP graph and replay it: every small host
 * array (problem pointers, step counts, the window schedule) reaches the
 * device as kernel arguments, the builds take their scaling exponents on the
 * device, and the size groups that fit one workgroup per problem (n <= 128)
 * run on a second, library-owned stream of the device beside the larger ones
 * (forked from and joined back into `stream` with events).  Data-dependent
 * failures (a non-finite ||L dt||_1, a zero pivot, a scaling exponent above
 * 24) lower the DEVICE int `status` (the caller sets it to LB_OK first; NULL
 * drops them).  The workspace must already hold the batch's buffers when the
 * call is captured (a first, eager call of the same batch grows it).  Results
 * are bitwise those of lindblad_batch_run.  Calls that overlap on one device
 * share the side stream. */
int lindblad_batch_enqueue(const lb_problem *probs, int nprob, lb_precision prec, double theta, int *status,
                           lb_workspace *ws, hipStream_t stream);

/* Byte budget of the propagators that lindblad_batch_run keeps running at
 * once for sizes past its one-workgroup-per-problem limit (n > 128): problems
 * run longest first in a sliding window of floor(bytes / P_bytes) (at least
 * one), which bounds the propagator bytes streamed per step.  0 restores the
 * default (192 MiB, the fastest measured budget).  Process-wide; results do
 * not depend on it (bitwise). */
int lindblad_batch_set_window(size_t bytes);

#ifdef __cplusplus
}
#endif
#endif /* LINDBLAD_H */
