// Internal launchers of the propagation chain (lindblad_propagate).
#pragma once
#include "lb_internal.hpp"

namespace lb {

// Largest n whose fused, LDS-resident chain exists for each precision.
int fused_max_n(lb_precision prec);

int chain_baseline(int n, const cd *P, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s);
int bf16_fused_max_n(lb_precision prec);
int chain_bf16_fused(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, hipStream_t s);
int chain_run(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s);

}  // namespace lb
