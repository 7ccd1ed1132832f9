// ADMM-TV step: internal interface between the plan and the ADMM kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "lam.h"

namespace lam {
void* plan_ws(lam_plan p, size_t* off_p);
const lam_params& plan_params(lam_plan p);
int plan_fwd_hat_real(lam_plan p, const void* u, const void* dhat, void* r, hipStream_t s);
int plan_adj_hat_real(lam_plan p, const void* r, void* u, hipStream_t s);
int set_error(int code, const char* msg);
// the plan's u1 stage buffer (complex, h x n1 x n2)
void* plan_u1(lam_plan p);
// one stage of L^ / L^* with memoized chunks skipped: 0 F_u1D (real volume in -> u1), 1 F_u2D (u1 -> out,
// no subtraction), 2 F*_u2D (in -> u1), 3 F*_u1D (u1 -> real volume out); chunks of 2^log2chunk volume
// rows (0, 3) or k_v slices (1, 2) whose hit flag is nonzero are skipped (hit = nullptr: none)
int plan_stage(lam_plan p, int stage, const void* in, void* out, const int* hit, int log2chunk, hipStream_t s);
}  // namespace lam
