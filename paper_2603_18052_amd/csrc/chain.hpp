// Internal launchers of the propagation chain (lindblad_propagate).
#pragma once
#include "lb_internal.hpp"

namespace lb {

// Largest n whose fused, LDS-resident chain exists for each precision.
int fused_max_n(lb_precision prec);

int chain_baseline(int n, const cd *P, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s);
// Longest chain that runs with the 4 x 4-digit slice set (10 slice pairs);
// longer chains use 5 x 4 digits (14 pairs).  Emulated and measured trace
// distances of the short set grow about linearly with the step count and
// reach ~8e-7 at 1e3 steps for d = 27, so the switch sits well before that.
constexpr long long kSlicedShortRun = 600;
int bf16_fused_max_n(lb_precision prec);
int chain_bf16_fused(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, hipStream_t s);
int chain_large(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, Workspace *ws,
                hipStream_t s);
int chain_run(int n, const cd *P, lb_precision prec, int B, cd *rho, long long nsteps, Workspace *ws, hipStream_t s);

}  // namespace lb
