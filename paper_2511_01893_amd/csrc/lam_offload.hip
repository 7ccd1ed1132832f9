// ADMM-Offload planning (Section 5.1): choose which ADMM variables to move out of device memory
// between their accesses, and when to prefetch them back, by the largest MT = M x 1/T over all
// plans that keep the paper's four constraints.  Host code only (lam_offload_plan in lam.h).
//
// Model.  One ADMM iteration is the phases run back to back and repeated.  For an offloaded
// variable and each phase k accessing it, with k' the next phase accessing it (cyclically), the
// gap runs from its last access in k (L) to its first access in k' (F); k' starts at S.  A gap
// whose next phase overwrites the variable first is dead: the variable is absent from L to S with
// no transfer.  Otherwise the offload starts at L (or when the link is free) and the gap is dropped
// if it cannot end by F (the maximum prefetch distance, constraint 3); the prefetch starts after
// the offload (constraint 1), as late as lets it end at S (constraint 4), or when the link is free,
// and the gap is dropped if no prefetch distance is left (constraint 2); the variable is absent
// from the offload's end to the prefetch's start, and a prefetch ending after F delays the
// iteration by the difference (T sums the delays).  Offloads take the link in the order of their
// gaps' last accesses, then prefetches in the order of their planned starts.  M is the total size
// of the variables less the plan's peak of resident sizes over the iteration (a dead gap's absence
// ends exactly at its phase's start when folded onto one iteration, not at a rounded start + period).
#include <algorithm>
#include <cmath>
#include <vector>

#include "lam.h"
#include "lam_admm.hpp"

namespace {

#pragma clang fp contract(off)

struct Gap {
  double L, F, S;
  bool dead;
  int v;
};
struct Absence {
  int v;
  double a, z;
  double z0;   // >= 0: the end folded onto [0, Ttot) exactly (a dead gap ends where its phase starts)
};

struct Plan {
  double M = 0, T = 0;
};

Plan evaluate(const std::vector<int>& plan, const double* start, int P, const lam_offload_var* vars, double link,
              double total) {
  const double Ttot = start[P];
  std::vector<Gap> live;
  std::vector<Absence> absent;
  for (int v : plan) {
    std::vector<int> ks;
    for (int k = 0; k < P; ++k)
      if (vars[v].accessed[k]) ks.push_back(k);
    for (size_t i = 0; i < ks.size(); ++i) {
      const int k = ks[i], kn = ks[(i + 1) % ks.size()];
      const double shift = kn <= k ? Ttot : 0.0;
      const double L = start[k] + vars[v].last[k];
      const double F = start[kn] + vars[v].first[kn] + shift;
      const double S = start[kn] + shift;
      if (vars[v].writes_first[kn]) absent.push_back({v, L, S, start[kn]});
      else live.push_back({L, F, S, false, v});
    }
  }
  std::stable_sort(live.begin(), live.end(), [](const Gap& a, const Gap& b) { return a.L < b.L; });
  struct Kept { double ps, oe, F; int v; };
  struct Busy { double b, e; };
  std::vector<Kept> kept;
  std::vector<Busy> busy;
  double free = 0.0;
  for (const Gap& g : live) {                       // offloads, in order of last access
    const double dur = vars[g.v].bytes / link;
    const double b = std::max(g.L, free), e = b + dur;
    if (!(e < g.F)) continue;                       // constraints 2 and 3
    free = e;
    busy.push_back({b, e});
    kept.push_back({std::max(e, g.S - dur), e, g.F, g.v});   // constraints 1 and 4
  }
  auto by_start = [](const Busy& x, const Busy& y) { return x.b != y.b ? x.b < y.b : x.e < y.e; };
  std::sort(busy.begin(), busy.end(), by_start);
  std::stable_sort(kept.begin(), kept.end(), [](const Kept& a, const Kept& b) { return a.ps < b.ps; });
  Plan r;
  for (const Kept& k : kept) {                      // prefetches: first free stretch at or after the planned start
    const double dur = vars[k.v].bytes / link;
    double t = k.ps;
    for (const Busy& x : busy) {
      if (t + dur <= x.b) break;
      if (t < x.e) t = x.e;
    }
    busy.push_back({t, t + dur});
    std::sort(busy.begin(), busy.end(), by_start);
    r.T += std::max(0.0, t + dur - k.F);
    absent.push_back({k.v, k.oe, t, -1.0});
  }
  // peak of the resident sizes over one iteration (absences folded onto [0, Ttot))
  struct Ev { double t, d; };
  std::vector<Ev> ev;
  for (const Absence& a : absent) {
    const double s = vars[a.v].bytes;
    if (a.z - a.a >= Ttot) {
      ev.push_back({0.0, -s});
      ev.push_back({Ttot, s});
      continue;
    }
    const double a0 = std::fmod(a.a, Ttot), z0 = a.z0 >= 0.0 ? a.z0 : std::fmod(a.z, Ttot);
    if (z0 >= a0) {
      ev.push_back({a0, -s});
      ev.push_back({z0, s});
    } else {
      ev.push_back({a0, -s});
      ev.push_back({Ttot, s});
      ev.push_back({0.0, -s});
      ev.push_back({z0, s});
    }
  }
  std::stable_sort(ev.begin(), ev.end(), [](const Ev& x, const Ev& y) { return x.t != y.t ? x.t < y.t : x.d < y.d; });
  std::vector<double> times{0.0};
  for (const Ev& e : ev)
    if (e.t < Ttot) times.push_back(e.t);
  std::sort(times.begin(), times.end());
  times.erase(std::unique(times.begin(), times.end()), times.end());
  double cur = total, peak = -INFINITY;
  size_t i = 0;
  for (double t : times) {                          // resident just after each event time
    while (i < ev.size() && ev[i].t <= t) cur += ev[i++].d;
    peak = std::max(peak, cur);
  }
  r.M = total - peak;
  return r;
}


// Validates the problem; fills the phase starts and the total size.
int check(const double* phase_s, int nphases, const lam_offload_var* vars, int nvars, double resident, double link_bps,
          double* start, double& total) {
  if (!phase_s || !vars) return lam::set_error(LAM_ERR_ARG, "null argument");
  if (nphases < 1 || nphases > LAM_OFFLOAD_MAX_PHASES || nvars < 1 || nvars > LAM_OFFLOAD_MAX_VARS)
    return lam::set_error(LAM_ERR_ARG, "nphases in [1, 8] and nvars in [1, 16]");
  if (!(link_bps > 0.0) || !(resident >= 0.0)) return lam::set_error(LAM_ERR_ARG, "link_bps > 0 and resident >= 0");
  start[0] = 0.0;
  for (int k = 0; k < nphases; ++k) {
    if (!(phase_s[k] > 0.0)) return lam::set_error(LAM_ERR_ARG, "phase durations must be positive");
    start[k + 1] = start[k] + phase_s[k];
  }
  total = 0.0;
  for (int v = 0; v < nvars; ++v) {
    const lam_offload_var& x = vars[v];
    bool any = false;
    for (int k = 0; k < nphases; ++k) {
      if (!x.accessed[k]) continue;
      any = true;
      if (!(x.first[k] >= 0.0 && x.last[k] >= x.first[k] && x.last[k] <= phase_s[k]))
        return lam::set_error(LAM_ERR_ARG, "access offsets must satisfy 0 <= first <= last <= phase duration");
    }
    if (!any || !(x.bytes >= 0.0)) return lam::set_error(LAM_ERR_ARG, "every variable needs a size and an access");
    total += x.bytes;
  }
  return LAM_OK;
}

}  // namespace

extern "C" int lam_offload_evaluate(const double* phase_s, int nphases, const lam_offload_var* vars, int nvars,
                                    double resident, double link_bps, unsigned mask, lam_offload_result* out) {
  double start[LAM_OFFLOAD_MAX_PHASES + 1], total = 0.0;
  if (!out) return lam::set_error(LAM_ERR_ARG, "null argument");
  int rc = check(phase_s, nphases, vars, nvars, resident, link_bps, start, total);
  if (rc) return rc;
  if (nvars < 32 && (mask >> nvars)) return lam::set_error(LAM_ERR_ARG, "mask names a variable beyond nvars");
  std::vector<int> plan;
  for (int v = 0; v < nvars; ++v)
    if (mask >> v & 1u) plan.push_back(v);
  const Plan r = evaluate(plan, start, nphases, vars, link_bps, total);
  out->mask = mask;
  out->M = r.M;
  out->T = r.T;
  out->MT = r.M / std::max(r.T, 1e-6);
  out->peak = resident + total - r.M;
  return LAM_OK;
}

extern "C" int lam_offload_plan(const double* phase_s, int nphases, const lam_offload_var* vars, int nvars,
                                double resident, double link_bps, double budget, lam_offload_result* out) {
  if (!phase_s || !vars || !out) return lam::set_error(LAM_ERR_ARG, "null argument");
  double start[LAM_OFFLOAD_MAX_PHASES + 1], total = 0.0;
  int rc = check(phase_s, nphases, vars, nvars, resident, link_bps, start, total);
  if (rc) return rc;
  std::vector<int> cand;
  for (int v = 0; v < nvars; ++v)
    if (vars[v].candidate) cand.push_back(v);
  auto fits = [&](double M) { return budget <= 0.0 || resident + total - M <= budget; };
  lam_offload_result best{};
  best.mask = 0;
  best.M = best.T = 0.0;
  best.MT = fits(0.0) ? 0.0 : -1.0;
  best.peak = resident + total;
  const unsigned nplans = 1u << cand.size();
  for (unsigned mask = 1; mask < nplans; ++mask) {
    std::vector<int> plan;
    unsigned vmask = 0;
    for (size_t j = 0; j < cand.size(); ++j)
      if (mask >> j & 1u) { plan.push_back(cand[j]); vmask |= 1u << cand[j]; }
    const Plan r = evaluate(plan, start, nphases, vars, link_bps, total);
    const double MT = r.M / std::max(r.T, 1e-6);
    if (fits(r.M) && MT > best.MT) {
      best.mask = vmask;
      best.M = r.M;
      best.T = r.T;
      best.MT = MT;
      best.peak = resident + total - r.M;
    }
  }
  *out = best;
  return LAM_OK;
}
