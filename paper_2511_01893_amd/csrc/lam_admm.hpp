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
}  // namespace lam
