// GRAPE fidelity gradient (adjoint + Frechet derivative of the propagator).
#include "lb_internal.hpp"

using namespace lb;

extern "C" int grape_gradient(int n, int M, int C, const void *L0, const void *Lc, const double *u, double dt,
                              double theta, const void *x0, const void *w, double *F, double *grad,
                              long long checkpoint_bytes, lb_workspace *ws, hipStream_t stream) {
    (void)n; (void)M; (void)C; (void)L0; (void)Lc; (void)u; (void)dt; (void)theta; (void)x0; (void)w;
    (void)F; (void)grad; (void)checkpoint_bytes; (void)ws; (void)stream;
    return fail(LB_ENOTSUP, "grape_gradient: not built yet");
}

extern "C" int lindblad_batch_run(const lb_problem *probs, int nprob, lb_precision prec, double theta,
                                  lb_workspace *ws, hipStream_t stream) {
    (void)probs; (void)nprob; (void)prec; (void)theta; (void)ws; (void)stream;
    return fail(LB_ENOTSUP, "lindblad_batch_run: not built yet");
}
