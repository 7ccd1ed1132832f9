// Host-side exercise of liblam's C ABI under AddressSanitizer and UBSan (built host-only: no device
// code, no GPU).  Every entry point that does host work without a device runs here: parameter
// validation and its error paths, plan construction (every FP64 table, the inverse z runs, the
// workspace layout) on power-of-two and 3 2^k sizes and every kernel half-width, the compute entry
// points' argument and state checks (no workspace set), the memoization layout, and the
// ADMM-Offload planner on random timelines.  Prints one line per group and exits non-zero on the
// first unexpected status; the sanitizers abort on the first memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>

#include "lam.h"

namespace {

int g_fail = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL: %s (%s)\n", what, lam_last_error());
    g_fail = 1;
  }
}

lam_params params(int n0, int n1, int n2, int nt, int h, int w, int m, lam_dtype dt, int slab = 0) {
  lam_params p;
  std::memset(&p, 0, sizeof p);
  p.n0 = n0; p.n1 = n1; p.n2 = n2; p.ntheta = nt; p.theta = nullptr; p.phi = 0.35;
  p.h = h; p.w = w; p.oversample = 2; p.m = m; p.dtype = dt; p.slab = slab;
  return p;
}

void plans() {
  struct Case { int n0, n1, n2, nt, h, w, m, slab; };
  const Case cs[] = {
      {16, 16, 16, 7, 16, 16, 4, 0},   {32, 64, 16, 33, 48, 24, 1, 3}, {24, 48, 96, 5, 96, 48, 8, 0},
      {64, 32, 128, 13, 32, 64, 3, 5}, {48, 48, 48, 19, 48, 48, 4, 0}, {16, 96, 32, 1, 24, 16, 6, 1},
  };
  int n = 0;
  for (const Case& c : cs)
    for (lam_dtype dt : {LAM_C64, LAM_C128}) {
      lam_params p = params(c.n0, c.n1, c.n2, c.nt, c.h, c.w, c.m, dt, c.slab);
      lam_plan h = nullptr;
      expect(lam_init(&h, &p) == LAM_OK && h, "lam_init");
      if (!h) continue;
      expect(lam_workspace_bytes(h) > 0, "lam_workspace_bytes");
      expect(lam_admm_work_bytes(h) > 0, "lam_admm_work_bytes");
      // compute calls before a workspace: state / argument errors, nothing enqueued
      expect(lam_fwd(h, nullptr, nullptr, nullptr) != LAM_OK, "lam_fwd without workspace");
      expect(lam_adj(h, nullptr, nullptr, nullptr) != LAM_OK, "lam_adj without workspace");
      expect(lam_fwd_hat(h, nullptr, nullptr, nullptr, nullptr) != LAM_OK, "lam_fwd_hat without workspace");
      expect(lam_data_hat(h, nullptr, nullptr, nullptr) != LAM_OK, "lam_data_hat without workspace");
      expect(lam_fwd_streamed(h, nullptr, 1, nullptr, nullptr) != LAM_OK, "streamed null");
      expect(lam_stream_slabs(h, 0, 1) == LAM_ERR_ARG, "stream slabs 0 rows");
      expect(lam_stream_slabs(h, 1, c.nt + 1) == LAM_ERR_ARG, "stream slabs too many projections");
      expect(lam_stream_slabs(h, 1, 1) == LAM_OK, "stream slabs 1, 1");
      expect(lam_set_workspace(h, nullptr, 0) != LAM_OK, "null workspace");
      lam_destroy(h);
      ++n;
    }
  // explicit angles, tomography (phi = 0)
  double th[5] = {0.0, M_PI / 2, M_PI, 1.25 * M_PI, 0.3};
  lam_params p = params(32, 32, 32, 5, 32, 32, 4, LAM_C64);
  p.theta = th;
  p.phi = 0.0;
  lam_plan h = nullptr;
  expect(lam_init(&h, &p) == LAM_OK, "lam_init with angles");
  lam_destroy(h);
  lam_destroy(nullptr);
  std::printf("plans: %d built and destroyed\n", n + 1);
}

void rejects() {
  const lam_params good = params(32, 32, 32, 8, 32, 32, 4, LAM_C64);
  int n = 0;
  auto bad = [&](lam_params p, const char* what) {
    lam_plan h = reinterpret_cast<lam_plan>(&n);   // must be overwritten with null
    expect(lam_init(&h, &p) == LAM_ERR_ARG && h == nullptr, what);
    expect(std::strlen(lam_last_error()) > 0, "error text");
    ++n;
  };
  lam_params p;
  p = good; p.n0 = 40; bad(p, "n0 = 40");
  p = good; p.n1 = 12; bad(p, "n1 = 12");
  p = good; p.n2 = 8192; bad(p, "n2 = 8192");
  p = good; p.h = 80; bad(p, "h = 80");
  p = good; p.w = 0; bad(p, "w = 0");
  p = good; p.ntheta = 0; bad(p, "ntheta = 0");
  p = good; p.phi = M_PI / 2; bad(p, "phi = pi/2");
  p = good; p.phi = NAN; bad(p, "phi = NaN");
  p = good; p.oversample = 3; bad(p, "oversample 3");
  p = good; p.m = 9; bad(p, "m = 9");
  p = good; p.dtype = (lam_dtype)7; bad(p, "dtype");
  p = good; p.slab = -1; bad(p, "slab");
  double th[3] = {0.0, INFINITY, 1.0};
  p = good; p.ntheta = 3; p.theta = th; bad(p, "theta inf");
  expect(lam_init(nullptr, &good) == LAM_ERR_ARG, "null out");
  for (int c = 0; c <= 6; ++c) expect(lam_error_string(c) != nullptr, "error string");
  for (int k = 0; k < 12; ++k) (void)lam_kernel_name(k);
  std::printf("rejects: %d invalid problems refused\n", n);
}

void memo() {
  lam_params p = params(64, 64, 64, 16, 64, 64, 4, LAM_C64);
  lam_plan h = nullptr;
  expect(lam_init(&h, &p) == LAM_OK, "memo plan");
  int n = 0;
  for (int cy : {1, 4, 16, 64})
    for (int ck : {1, 8, 64})
      for (int kd : {64, 1024, 4096}) {
        lam_memo m;
        std::memset(&m, 0, sizeof m);
        m.tau = 0.9; m.chunk_y = cy; m.chunk_kv = ck; m.key_dim = kd; m.seed = 3;
        expect(lam_memo_bytes(h, &m) > 0, "memo bytes");
        ++n;
      }
  lam_memo m;
  std::memset(&m, 0, sizeof m);
  m.tau = 0.9; m.chunk_y = 3; m.chunk_kv = 8; m.key_dim = 64;
  expect(lam_memo_bytes(h, &m) == 0, "memo chunk_y 3 refused");
  lam_destroy(h);
  // 3 2^k sizes: memoization refused
  p = params(48, 48, 48, 8, 48, 48, 4, LAM_C64);
  expect(lam_init(&h, &p) == LAM_OK, "memo plan 48");
  m.chunk_y = 16;
  expect(lam_memo_bytes(h, &m) == 0, "memo on 3 2^k refused");
  lam_destroy(h);
  std::printf("memo: %d layouts\n", n);
}

void offload() {
  std::mt19937_64 rng(11);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  int n = 0, plans_found = 0;
  for (int trial = 0; trial < 400; ++trial) {
    const int np = 1 + (int)(rng() % LAM_OFFLOAD_MAX_PHASES), nv = 1 + (int)(rng() % 10);
    double ph[LAM_OFFLOAD_MAX_PHASES];
    for (int k = 0; k < np; ++k) ph[k] = 0.001 + 0.05 * U(rng);
    lam_offload_var v[16];
    std::memset(v, 0, sizeof v);
    for (int i = 0; i < nv; ++i) {
      v[i].bytes = 1e6 + 1e9 * U(rng);
      v[i].candidate = (int)(rng() % 4 != 0);
      bool any = false;
      for (int k = 0; k < np; ++k) {
        v[i].accessed[k] = (int)(rng() % 2);
        if (k == np - 1 && !any) v[i].accessed[k] = 1;
        if (!v[i].accessed[k]) continue;
        any = true;
        const double a = ph[k] * U(rng), b = ph[k] * U(rng);
        v[i].first[k] = a < b ? a : b;
        v[i].last[k] = a < b ? b : a;
        v[i].writes_first[k] = (int)(rng() % 3 == 0);
      }
    }
    lam_offload_result r;
    const double budget = (trial % 3 == 0) ? 0.0 : 1e9 * U(rng);
    expect(lam_offload_plan(ph, np, v, nv, 2e9, 5e10, budget, &r) == LAM_OK, "offload plan");
    if (r.MT >= 0) ++plans_found;
    for (unsigned mask = 0; mask < (1u << (nv < 6 ? nv : 6)); ++mask) {
      lam_offload_result e;
      expect(lam_offload_evaluate(ph, np, v, nv, 2e9, 5e10, mask, &e) == LAM_OK, "offload evaluate");
      expect(std::isfinite(e.M) && std::isfinite(e.T) && e.T >= 0.0, "evaluate finite");
    }
    ++n;
  }
  // errors
  double ph[2] = {0.01, 0.02};
  lam_offload_var v[1];
  std::memset(v, 0, sizeof v);
  v[0].bytes = 1.0;
  lam_offload_result r;
  expect(lam_offload_plan(ph, 2, v, 1, 0.0, 1e9, 0.0, &r) == LAM_ERR_ARG, "variable with no access");
  v[0].accessed[0] = 1; v[0].first[0] = 0.02; v[0].last[0] = 0.01;
  expect(lam_offload_plan(ph, 2, v, 1, 0.0, 1e9, 0.0, &r) == LAM_ERR_ARG, "first > last");
  expect(lam_offload_plan(ph, 0, v, 1, 0.0, 1e9, 0.0, &r) == LAM_ERR_ARG, "no phases");
  expect(lam_offload_evaluate(ph, 2, v, 1, 0.0, 1e9, 2u, &r) == LAM_ERR_ARG, "mask beyond nvars");
  std::printf("offload: %d random timelines planned (%d with a plan in budget)\n", n, plans_found);
}

}  // namespace

int main() {
  plans();
  rejects();
  memo();
  offload();
  std::printf(g_fail ? "abi host checks FAILED\n" : "abi host checks ok\n");
  return g_fail;
}
