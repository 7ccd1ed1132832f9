// ADMM-TV step (placeholder until the device kernels land).
#include "lam_admm.hpp"

extern "C" size_t lam_admm_work_bytes(lam_plan p) { return p ? 0 : 0; }

extern "C" int lam_admm_step(lam_plan p, const lam_admm_state* s, const void* dhat, int n_inner, void* stream) {
  (void)p; (void)s; (void)dhat; (void)n_inner; (void)stream;
  return lam::set_error(LAM_ERR_STATE, "lam_admm_step is not available in this build");
}
