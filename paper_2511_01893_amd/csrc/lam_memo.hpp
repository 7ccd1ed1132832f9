// Memoized LSP operators: internal interface between the memoization and the ADMM step.
#pragma once
#include <hip/hip_runtime.h>

#include "lam.h"

namespace lam {
// Validates the memoization parameters (and, with state, the work and counter pointers).
int memo_check(lam_plan p, const lam_memo* m, bool state);
size_t memo_bytes(lam_plan p, const lam_memo* m);
// Builds the sign tables at the first step on a zero-filled work buffer (no-op afterwards).
int memo_prepare(lam_plan p, const lam_memo& m, hipStream_t s);
// One memoized operator application: 0 F_u1D (real volume in -> plan u1), 1 F_u2D (plan u1 -> out, then
// out -= sub), 2 F*_u2D (in -> plan u1), 3 F*_u1D (plan u1 -> real volume out).
template <typename T>
int memo_apply(lam_plan p, const lam_memo& m, int op, const void* in, void* out, const void* sub, hipStream_t s);
}  // namespace lam
