// Host emulation of the per-tile target-list enumeration (the candidate
// intervals and the exact classification the device count/fill kernels run
// for every (slice, tile row, angle)), on geometries chosen for their edge
// cases: angles at multiples of pi/2 and within 1e-9 of them (a line parallel
// to a grid axis, |A| < 1e-8), phi = 0 (targets on integer coordinates), one
// tile spanning the whole grid period, detectors wider than the volume (lines
// spanning the period), odd angle counts, m = 1 and m = 8.
//
// For each geometry: every target (theta, k_u) of every slice must be
// enumerated exactly once over all tile rows, in the tile row, tile column and
// border class that its coordinates give directly.  Prints one line per
// geometry and exits non-zero on the first failure.
#include <cmath>
#include <cstdio>
#include <vector>

#include "lam_lists.hpp"

using namespace lam;

namespace {

struct Geo {
  int n1, n2, h, w, m;
  double phi;
  std::vector<double> theta;
};

int ilog2(int v) { int r = 0; while ((1 << r) < v) ++r; return r; }

int run(const Geo& g, const char* name) {
  const int R = 2, M1 = R * g.n1, M2 = R * g.n2, nt = (int)g.theta.size();
  int TS = 64;
  while (M1 % TS || M2 % TS) TS >>= 1;   // the plan's tile: the largest power of two <= 64 dividing both
  const int log2TS = ilog2(TS), ntx = M2 / TS, nty = M1 / TS;
  Dims D{};
  D.n1 = g.n1; D.n2 = g.n2; D.h = g.h; D.w = g.w; D.ntheta = nt; D.m = g.m;
  D.M1 = M1; D.M2 = M2;
  D.xy.Rn2 = (double)R * g.n2; D.xy.Rn1 = (double)R * g.n1;
  D.xy.inv_w = 1.0 / g.w; D.xy.inv_h = 1.0 / g.h; D.xy.sphi = std::sin(g.phi);
  D.xy.w = g.w; D.xy.h = g.h;
  std::vector<double> cth(nt), sth(nt), line(6 * (size_t)nt);
  for (int t = 0; t < nt; ++t) {
    cth[t] = std::cos(g.theta[t]);
    sth[t] = std::sin(g.theta[t]);
    const double Ax = R * (double)g.n2 * cth[t] / g.w, Ay = R * (double)g.n1 * sth[t] / g.w;
    double* l = &line[6 * (size_t)t];
    l[0] = Ax; l[1] = std::fabs(Ax) < 1e-8 ? 0.0 : 1.0 / Ax; l[2] = R * (double)g.n2 * D.xy.sphi * sth[t];
    l[3] = Ay; l[4] = std::fabs(Ay) < 1e-8 ? 0.0 : 1.0 / Ay; l[5] = -R * (double)g.n1 * D.xy.sphi * cth[t];
  }
  long listed = 0;
  for (int k = 0; k < g.h; ++k) {
    std::vector<int> seen((size_t)nt * g.w, 0);
    for (int ty = 0; ty < nty; ++ty) {
      const int Y0 = ty * TS;
      for (int t = 0; t < nt; ++t) {
        int lo[2], hi[2];
        const int n = band_intervals(D, &line[6 * (size_t)t], k, Y0, log2TS, lo, hi);
        for (int j = 0; j < n; ++j)
          for (int ku = lo[j]; ku <= hi[j]; ++ku) {
            int tx, c;
            const int aku = ku + g.w / 2;
            if (!classify_target(D, cth[t], sth[t], k, aku, Y0, log2TS, g.m, tx, c)) continue;
            // the direct classification of the same target
            double sx, sy;
            target_coords(D.xy, cth[t], sth[t], k, aku, sx, sy);
            const int by = (int)(std::floor(sy) - M1 * std::floor(std::floor(sy) / M1));
            const int bx = (int)(std::floor(sx) - M2 * std::floor(std::floor(sx) / M2));
            const int oy = by % TS, ox = bx % TS;
            const int cy = oy < g.m - 1 ? 0 : (oy >= TS - g.m ? 2 : 1), cx = ox < g.m - 1 ? 0 : (ox >= TS - g.m ? 2 : 1);
            if (by / TS != ty || bx / TS != tx || c != 3 * cy + cx || tx >= ntx) {
              std::printf("%s: slice %d theta %d k_u %d misfiled (tile %d,%d class %d)\n", name, k, t, aku, ty, tx, c);
              return 1;
            }
            if (seen[(size_t)t * g.w + aku]++) {
              std::printf("%s: slice %d theta %d k_u %d listed twice\n", name, k, t, aku);
              return 1;
            }
            ++listed;
          }
      }
    }
    for (int t = 0; t < nt; ++t)
      for (int a = 0; a < g.w; ++a)
        if (!seen[(size_t)t * g.w + a]) {
          std::printf("%s: slice %d theta %d k_u %d missed\n", name, k, t, a);
          return 1;
        }
  }
  std::printf("%s: %ld targets, each listed once\n", name, listed);
  return 0;
}

std::vector<double> uniform(int n) {
  std::vector<double> t(n);
  for (int i = 0; i < n; ++i) t[i] = 2.0 * M_PI * i / n;
  return t;
}

}  // namespace

int main() {
  const double pi = M_PI, deg = pi / 180.0;
  const std::vector<double> edge = {0.0, pi / 2, pi, 1.5 * pi, 1e-9, pi / 2 + 1e-9, pi - 1e-9, 2 * pi - 1e-12,
                                    pi / 4, 3 * pi / 4, 1e-7, 0.3};
  int rc = 0;
  rc |= run({32, 32, 32, 32, 4, 20 * deg, edge}, "one tile per period, edge angles");
  rc |= run({128, 128, 64, 128, 4, 20 * deg, edge}, "4 x 4 tiles, edge angles");
  rc |= run({64, 64, 64, 64, 4, 0.0, edge}, "phi = 0, edge angles");
  rc |= run({64, 256, 16, 512, 4, 35 * deg, edge}, "detector wider than the volume");
  rc |= run({256, 64, 32, 64, 4, 60 * deg, uniform(97)}, "97 angles, rectangular grid");
  rc |= run({128, 128, 32, 128, 8, 30 * deg, edge}, "m = 8");
  rc |= run({128, 64, 32, 64, 1, 30 * deg, uniform(41)}, "m = 1");
  // grids of 3 2^k points: tiles of 16 (M = 48) and 32 (M1 = 96 beside M2 = 192)
  rc |= run({24, 24, 24, 24, 4, 20 * deg, edge}, "3 2^k: 48 x 48 grid, edge angles");
  rc |= run({48, 96, 48, 96, 4, 30 * deg, uniform(61)}, "3 2^k: 96 x 192 grid, 61 angles");
  rc |= run({96, 64, 24, 128, 4, 35 * deg, edge}, "3 2^k rows beside 2^k columns, wide detector");
  return rc;
}
