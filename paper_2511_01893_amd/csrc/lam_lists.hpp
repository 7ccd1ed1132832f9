// Target-list geometry shared by the device list builder (count, fill and
// check kernels) and host code: which detector bins (theta, k_u) of one k_v
// slice have their Gaussian stencil base floor(s) in a band of TS rows of the
// oversampled grid, and in which tile and border class.
//
// The targets of one angle and slice lie on a line, s = A k_u + C (k_v/h)
// per axis (the plan's per-angle line parameters), so the candidates of a band
// are one or two k_u intervals; every candidate is then re-checked with the
// exact FP64 coordinate function that the gather and spread use.
#pragma once
#include "lam_internal.hpp"

namespace lam {

// k_u interval of one angle's targets whose floor(s) lies in [lo_s, hi_s) along
// one axis, s = A k_u + B (iA = 1/A, 0 when |A| < 1e-8).  Bounds are generous;
// callers re-check every candidate exactly.
__host__ __device__ inline void interval_1d(double A, double iA, double B, double lo_s, double hi_s, int kmin,
                                            int kmax, int& a, int& b) {
  if (iA == 0.0) {
    if (B >= lo_s - 1.0 && B < hi_s + 1.0) { a = kmin; b = kmax; }
    else { a = 1; b = 0; }
    return;
  }
  double k1 = (lo_s - B) * iA, k2 = (hi_s - B) * iA;
  if (k1 > k2) { const double t = k1; k1 = k2; k2 = t; }
  k1 = fmax(k1, (double)kmin - 2.0);
  k2 = fmin(k2, (double)kmax + 2.0);
  const int ca = (int)ceil(k1 - 1e-3), cb = (int)floor(k2 + 1e-3);
  a = ca > kmin ? ca : kmin;
  b = cb < kmax ? cb : kmax;
}

// The same modulo the grid period M: the band [X0, X0 + LX) and its periodic
// images.  At most two intervals (the line meets the images of a band only near
// its ends); overlapping intervals are merged so that no k_u comes twice.
__host__ __device__ inline int axis_intervals(double A, double iA, double B, int X0, int LX, int M, int kmin, int kmax,
                                              int* lo, int* hi) {
  const double half = fabs(A) * (double)(kmax - kmin) * 0.5 + fabs(A);
  const double mid = B + A * 0.5 * (double)(kmin + kmax);
  const double smin = mid - half - 1.0, smax = mid + half + 1.0;
  int n = 0;
  for (int i = -2; i <= 2; ++i) {
    const double l = (double)X0 + (double)i * M, h = l + LX;
    if (h < smin || l > smax) continue;
    int a, b;
    interval_1d(A, iA, B, l, h, kmin, kmax, a, b);
    if (a > b) continue;
    if (n < 2) { lo[n] = a; hi[n] = b; ++n; }
    else { lo[1] = a < lo[1] ? a : lo[1]; hi[1] = b > hi[1] ? b : hi[1]; }
  }
  if (n == 2 && lo[1] <= hi[0] + 1 && lo[0] <= hi[1] + 1) {
    lo[0] = lo[1] < lo[0] ? lo[1] : lo[0];
    hi[0] = hi[1] > hi[0] ? hi[1] : hi[0];
    n = 1;
  }
  return n;
}

// Border class along one axis of a stencil whose base sits at offset o in a
// tile of TS: 0 if it reaches across the low border, 2 across the high one, 1
// if it stays inside.
__host__ __device__ inline int border_class(int o, int TS, int MH) {
  return o < MH - 1 ? 0 : (o >= TS - MH ? 2 : 1);
}

// Candidate k_u intervals (centred k_u) of angle t's targets on slice k whose
// base row lies in the band of rows [Y0, Y0 + 2^log2TS) (modulo M1).  ln: the
// angle's six line parameters A_x, 1/A_x, C_x, A_y, 1/A_y, C_y.
__host__ __device__ inline int band_intervals(const Dims& D, const double* ln, int k, int Y0, int log2TS, int* lo,
                                              int* hi) {
  const double kv = (double)(k - D.h / 2) * D.xy.inv_h;
  return axis_intervals(ln[3], ln[4], ln[5] * kv, Y0, 1 << log2TS, D.M1, -D.w / 2, D.w / 2 - 1, lo, hi);
}

// v modulo M in [0, M), for any sign of v
__host__ __device__ inline int pmod(int v, int M) {
  const int r = v % M;
  return r < 0 ? r + M : r;
}

// Exact test of one candidate (array indices k, aku; angle cos/sin ct, st): true
// when its base row lies in the band at Y0; then tx is its tile column and c
// its border class (3 x row class + column class).
__host__ __device__ inline bool classify_target(const Dims& D, double ct, double st, int k, int aku, int Y0,
                                                int log2TS, int MH, int& tx, int& c) {
  const int TS = 1 << log2TS;
  double sx, sy;
  target_coords(D.xy, ct, st, k, aku, sx, sy);
  const int oy = pmod((int)floor(sy) - Y0, D.M1);
  const int fx = pmod((int)floor(sx), D.M2);
  tx = fx >> log2TS;
  c = border_class(oy, TS, MH) * 3 + border_class(fx & (TS - 1), TS, MH);
  return oy < TS;
}

}  // namespace lam
