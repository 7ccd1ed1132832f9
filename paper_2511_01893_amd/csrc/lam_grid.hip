// The unequally-spaced part of F_u2D and its adjoint on the oversampled grid
// of one k_v slice: the 2m x 2m Gaussian gather (forward) and spread
// (adjoint) at the n_theta x w targets of the slice.
//
// The targets' coordinates depend only on the geometry, so the plan sorts
// them once (at lam_set_workspace): for every slice, every TS x TS tile of
// the M1 x M2 grid gets the list of targets whose stencil base floor(s)
// lies in the tile, sub-sorted into 3 x 3 classes by whether the stencil
// reaches across the tile's low / high border in x and y.  Each target is
// listed exactly once (checked on the host: every slice holds n_theta w
// entries).
//   k_gather   stages a tile plus its (2m-1) halo in LDS and walks the tile's
//              list: FP64 coordinates and weights, 2m x 2m FMA gather,
//              optional fused "- d^" (Algorithm 2).
//   k_scatter  accumulates one tile in LDS in FP64: its own list plus the
//              border classes of the 8 neighbouring tiles whose stencils
//              reach in.  Phase 1 turns a round of targets into records
//              (weights, sample, stencil corner); phase 2 gives every
//              stencil tap of a record its own lane, so the 2m x 2m adds of a
//              target hit distinct cells in distinct banks (native
//              ds_add_f64; gfx950 runs FP64 LDS atomics ~20x faster than
//              FP32 ones).  Every cell of the tile is then written once.
#include "lam_internal.hpp"

namespace lam {

extern __shared__ __align__(16) unsigned char lam_smem[];

namespace {

// k_u interval(s) of one angle's targets whose floor(s) lies, modulo M, in
// [X0, X0 + LX) along one axis; s = A k_u + B.  At most two intervals (the
// line meets the periodic images of a band only near its ends).  Bounds are
// generous; callers re-check every candidate exactly.
__device__ __forceinline__ void interval_1d(double A, double iA, double B, double lo_s, double hi_s, int kmin,
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
  a = max(kmin, (int)ceil(k1 - 1e-3));
  b = min(kmax, (int)floor(k2 + 1e-3));
}

__device__ __forceinline__ int axis_intervals(double A, double iA, double B, int X0, int LX, int M, int kmin, int kmax,
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
    else { lo[1] = min(lo[1], a); hi[1] = max(hi[1], b); }
  }
  // the generous bounds let the intervals of neighbouring images overlap when
  // the band spans most of the period; visit their union so no k_u comes twice
  if (n == 2 && lo[1] <= hi[0] + 1 && lo[0] <= hi[1] + 1) {
    lo[0] = min(lo[0], lo[1]);
    hi[0] = max(hi[0], hi[1]);
    n = 1;
  }
  return n;
}

__device__ __forceinline__ int border_class(int o, int TS, int MH) {
  return o < MH - 1 ? 0 : (o >= TS - MH ? 2 : 1);
}

// Visit every target of slice k whose base row lies in the band of tile row
// ty; calls f(t, aku, tx, class) with its tile column and border class.
template <int MH, class F>
__device__ __forceinline__ void band_targets(const Dims& D, const double* cth, const double* sth, const double* line,
                                             int k, int ty, int log2TS, F&& f) {
  const int TS = 1 << log2TS, M1 = 1 << D.log2M1, M2 = 1 << D.log2M2;
  const int Y0 = ty * TS;
  const int kmin = -D.w / 2, kmax = D.w / 2 - 1;
  const double kv = (double)(k - D.h / 2) * D.xy.inv_h;
  for (int t = threadIdx.x; t < D.ntheta; t += blockDim.x) {
    const double* ln = line + 6 * t;
    int lo[2], hi[2];
    const int n = axis_intervals(ln[3], ln[4], ln[5] * kv, Y0, TS, M1, kmin, kmax, lo, hi);
    for (int j = 0; j < n; ++j)
      for (int ku = lo[j]; ku <= hi[j]; ++ku) {
        double sx, sy;
        target_coords(D.xy, cth[t], sth[t], k, ku + D.w / 2, sx, sy);
        const int oy = ((int)floor(sy) - Y0) & (M1 - 1);
        if (oy >= TS) continue;
        const int fx = (int)floor(sx) & (M2 - 1);
        const int tx = fx >> log2TS, ox = fx & (TS - 1);
        f(t, ku + D.w / 2, tx, border_class(oy, TS, MH) * 3 + border_class(ox, TS, MH));
      }
  }
}

// counts[k][ty][tx][class] for the slices [k0, k0 + gridDim.y), tile row blockIdx.x
template <typename T, int MH>
__global__ __launch_bounds__(256) void k_list_count(Dims D, Tables<T> tb, int log2TS, int k0, int* __restrict__ counts) {
  const int ntx = (1 << D.log2M2) >> log2TS, nty = (1 << D.log2M1) >> log2TS;
  const int ty = blockIdx.x, k = k0 + blockIdx.y;
  int* cnt = reinterpret_cast<int*>(lam_smem);                 // [ntx * 9]
  for (int i = threadIdx.x; i < ntx * 9; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  band_targets<MH>(D, tb.cth, tb.sth, tb.line, k, ty, log2TS,
                   [&](int, int, int tx, int c) { atomicAdd(&cnt[tx * 9 + c], 1); });
  __syncthreads();
  const size_t per_slice = (size_t)ntx * nty * 9 + 1;
  int* out = counts + (size_t)k * per_slice + (size_t)ty * ntx * 9;
  for (int i = threadIdx.x; i < ntx * 9; i += blockDim.x) out[i] = cnt[i];
}

// lists[k][offset] = t * 4096 + aku, placed from the per-slice offsets
template <typename T, int MH>
__global__ __launch_bounds__(256) void k_list_fill(Dims D, Tables<T> tb, int log2TS, int k0, const int* __restrict__ offs,
                                                   int* __restrict__ lists) {
  const int ntx = (1 << D.log2M2) >> log2TS, nty = (1 << D.log2M1) >> log2TS;
  const int ty = blockIdx.x, k = k0 + blockIdx.y;
  int* cur = reinterpret_cast<int*>(lam_smem);                 // [ntx * 9]
  const size_t per_slice = (size_t)ntx * nty * 9 + 1;
  const int* of = offs + (size_t)k * per_slice + (size_t)ty * ntx * 9;
  for (int i = threadIdx.x; i < ntx * 9; i += blockDim.x) cur[i] = of[i];
  __syncthreads();
  int* L = lists + (size_t)k * D.ntheta * D.w;
  band_targets<MH>(D, tb.cth, tb.sth, tb.line, k, ty, log2TS, [&](int t, int aku, int tx, int c) {
    const int pos = atomicAdd(&cur[tx * 9 + c], 1);
    L[pos] = t * 4096 + aku;
  });
}

}  // namespace

// ---------------------------------------------------------------------------
// F_u2D gather over one tile of the oversampled grid
// ---------------------------------------------------------------------------
template <typename T, int MH>
__global__ __launch_bounds__(256) void k_gather(const cpx<T>* __restrict__ Gb, cpx<T>* out, const cpx<T>* dhat, int k0,
                                                Dims D, Tables<T> tb, int log2TS) {
  constexpr int W = 2 * MH;
  const int TS = 1 << log2TS, P = TS + W - 1;
  const int M1 = 1 << D.log2M1, M2 = 1 << D.log2M2;
  const int ntx = M2 >> log2TS, nty = M1 >> log2TS;
  const int tid = threadIdx.x, nth = blockDim.x;
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(lam_smem);
  // blocks run rank-major over the slab's slices: the heaviest tile of every slice first
  const int ns = gridDim.x / (ntx * nty), rank = blockIdx.x / ns, kk = blockIdx.x - rank * ns, k = k0 + kk;
  const int tix = tb.gperm[(size_t)k * ntx * nty + rank];
  const int tx = tix % ntx, ty = tix / ntx;
  const int x0 = tx * TS, y0 = ty * TS;
  const cpx<T>* G = Gb + (size_t)kk * M1 * M2;
  // e / P by multiplication: exact for e < 2^16 with P < 2^8
  const unsigned magicP = 0xffffffffu / (unsigned)P + 1u;
  for (int e0 = 0; e0 < P * P; e0 += vpt<T>() * nth) {
    cpx<T> v[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = min(e0 + tid + it * nth, P * P - 1);
      const int r = (int)(((unsigned long long)(unsigned)e * magicP) >> 32), c = e - r * P;
      v[it] = G[(size_t)((y0 - MH + 1 + r) & (M1 - 1)) * M2 + ((x0 - MH + 1 + c) & (M2 - 1))];
    }
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = e0 + tid + it * nth;
      if (e < P * P) tile[e] = v[it];
    }
  }
  __syncthreads();
  const size_t per_slice = (size_t)ntx * nty * 9 + 1;
  const int* of = tb.toff + (size_t)k * per_slice + (size_t)(ty * ntx + tx) * 9;
  const int beg = of[0], end = of[9];
  const int* L = tb.tlist + (size_t)k * D.ntheta * D.w;
  for (int i = beg + tid; i < end; i += nth) {
    const int p = L[i];
    const int t = p >> 12, aku = p & 4095;
    double sx, sy;
    target_coords(D.xy, tb.cth[t], tb.sth[t], k, aku, sx, sy);
    T wx[W], wy[W];
    int bx, by;
    stencil_weights<T, MH>(sx, D.beta, tb.rc, bx, wx);
    stencil_weights<T, MH>(sy, D.beta, tb.rc, by, wy);
    const int ox = (bx - x0) & (M2 - 1), oy = (by - y0) & (M1 - 1);
    T ax = 0, ay = 0;
#pragma unroll
    for (int iy = 0; iy < W; ++iy) {
      const cpx<T>* row = tile + (oy + iy) * P + ox;
      T rx = 0, ry = 0;
#pragma unroll
      for (int ix = 0; ix < W; ++ix) {
        const cpx<T> g = row[ix];
        rx += wx[ix] * g.x;
        ry += wx[ix] * g.y;
      }
      ax += wy[iy] * rx;
      ay += wy[iy] * ry;
    }
    const size_t o = ((size_t)t * D.h + k) * D.w + aku;
    if (dhat) {
      const cpx<T> dd = dhat[o];
      ax -= dd.x;
      ay -= dd.y;
    }
    out[o] = mk(ax, ay);
  }
}

// ---------------------------------------------------------------------------
// F*_u2D spread into one tile of the oversampled grid
// ---------------------------------------------------------------------------
template <typename T, int MH>
__global__ __launch_bounds__(1024) void k_scatter(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ Gb, int k0,
                                                  Dims D, Tables<T> tb, int log2TS) {
  constexpr int W = 2 * MH;
  constexpr int TPL = (W * W + 63) / 64;     // stencil taps per lane
  constexpr int RS = 2 * W + 2;              // record: wy[W], wx[W], sample (re, im)
  const int TS = 1 << log2TS, PA = TS + 8;   // PA = 8 (mod 32): 2 rows of 8 FP64 cells fill 32 banks
  const int M1 = 1 << D.log2M1, M2 = 1 << D.log2M2;
  const int ntx = M2 >> log2TS, nty = M1 >> log2TS;
  const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wave = tid >> 6, nwave = nth >> 6;
  double* are = reinterpret_cast<double*>(lam_smem);           // [TS][PA]
  double* aim = are + TS * PA;                                  // [TS][PA]
  T* rec = reinterpret_cast<T*>(aim + TS * PA);                 // [nth][RS]
  int* corner = reinterpret_cast<int*>(rec + (size_t)nth * RS); // [nth]
  int* rng = corner + nth;                                      // [2][14]: starts, prefix counts
  // blocks run rank-major over the slab's slices: the heaviest tile of every slice first
  const int ns = gridDim.x / (ntx * nty), rank = blockIdx.x / ns, kk = blockIdx.x - rank * ns, k = k0 + kk;
  const int tile = tb.sperm[(size_t)k * ntx * nty + rank];
  const int tx = tile % ntx, ty = tile / ntx;
  const int x0 = tx * TS, y0 = ty * TS;
  for (int e = tid; e < 2 * TS * PA; e += nth) are[e] = 0.0;
  const size_t per_slice = (size_t)ntx * nty * 9 + 1;
  const int* of = tb.toff + (size_t)k * per_slice;
  if (tid == 0) {
    int b[13], e[13];
    const int nr = spread_ranges(of, ntx, nty, ty, tx, b, e);
    int tot = 0;
    for (int j = 0; j < nr; ++j) { rng[j] = b[j]; rng[14 + j] = tot; tot += e[j] - b[j]; }
    rng[14 + nr] = tot;
    rng[13] = nr;
  }
  __syncthreads();
  const int nr = rng[13], total = rng[14 + nr];
  const int* L = tb.tlist + (size_t)k * D.ntheta * D.w;
  for (int r0 = 0; r0 < total; r0 += nth) {
    // phase 1: one record per target
    const int i = r0 + tid;
    if (i < total) {
      int j = 0;
      while (j + 1 < nr && rng[14 + j + 1] <= i) ++j;
      const int p = L[rng[j] + (i - rng[14 + j])];
      const int t = p >> 12, aku = p & 4095;
      double sx, sy;
      target_coords(D.xy, tb.cth[t], tb.sth[t], k, aku, sx, sy);
      T* rr = rec + (size_t)tid * RS;
      int bx, by;
      stencil_weights<T, MH>(sy, D.beta, tb.rc, by, rr);
      stencil_weights<T, MH>(sx, D.beta, tb.rc, bx, rr + W);
      const cpx<T> v = in[((size_t)t * D.h + k) * D.w + aku];
      rr[2 * W] = v.x;
      rr[2 * W + 1] = v.y;
      corner[tid] = (((by - MH + 1 - y0) & (M1 - 1)) << 16) | ((bx - MH + 1 - x0) & (M2 - 1));
    }
    __syncthreads();
    // phase 2: one lane per stencil tap
    const int nrec = min(nth, total - r0);
    for (int q = wave; q < nrec; q += nwave) {
      const int c = corner[q];
      const int ry0 = c >> 16, rx0 = c & 0xffff;
      const T* rr = rec + (size_t)q * RS;
      const T vx = rr[2 * W], vy = rr[2 * W + 1];
#pragma unroll
      for (int kt = 0; kt < TPL; ++kt) {
        const int tap = lane + 64 * kt;
        if (tap < W * W) {
          const int iy = tap / W, ix = tap - iy * W;
          const int row = (ry0 + iy) & (M1 - 1), col = (rx0 + ix) & (M2 - 1);
          if (row < TS && col < TS) {
            const T w = rr[iy] * rr[W + ix];
            atomicAdd(are + row * PA + col, (double)(w * vx));
            atomicAdd(aim + row * PA + col, (double)(w * vy));
          }
        }
      }
    }
    __syncthreads();
  }
  cpx<T>* G = Gb + (size_t)kk * M1 * M2;
  for (int e = tid; e < TS * TS; e += nth) {
    const int r = e >> log2TS, c = e & (TS - 1);
    G[(size_t)(y0 + r) * M2 + x0 + c] = mk((T)are[r * PA + c], (T)aim[r * PA + c]);
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
namespace {
template <typename Kern>
hipError_t prep(Kern k, size_t lds) {
  if (lds > 64 * 1024)
    return hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}
}  // namespace

#define LAM_MH_SWITCH(MHV, ...)                                   \
  switch (MHV) {                                                  \
    case 1: { constexpr int MH = 1; __VA_ARGS__; } break;         \
    case 2: { constexpr int MH = 2; __VA_ARGS__; } break;         \
    case 3: { constexpr int MH = 3; __VA_ARGS__; } break;         \
    case 4: { constexpr int MH = 4; __VA_ARGS__; } break;         \
    case 5: { constexpr int MH = 5; __VA_ARGS__; } break;         \
    case 6: { constexpr int MH = 6; __VA_ARGS__; } break;         \
    case 7: { constexpr int MH = 7; __VA_ARGS__; } break;         \
    default: { constexpr int MH = 8; __VA_ARGS__; } break;        \
  }

template <typename T>
hipError_t launch_list_count(const LaunchCfg& c, int k0, int ns, const Dims& D, const Tables<T>& tb, int* counts,
                             hipStream_t s) {
  const int ntx = (1 << D.log2M2) >> c.g_log2TS, nty = (1 << D.log2M1) >> c.g_log2TS;
  LAM_MH_SWITCH(D.m, {
    hipLaunchKernelGGL((k_list_count<T, MH>), dim3(nty, ns), dim3(256), ntx * 9 * sizeof(int), s, D, tb, c.g_log2TS,
                       k0, counts);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_list_fill(const LaunchCfg& c, int k0, int ns, const Dims& D, const Tables<T>& tb, const int* offs,
                            int* lists, hipStream_t s) {
  const int ntx = (1 << D.log2M2) >> c.g_log2TS, nty = (1 << D.log2M1) >> c.g_log2TS;
  LAM_MH_SWITCH(D.m, {
    hipLaunchKernelGGL((k_list_fill<T, MH>), dim3(nty, ns), dim3(256), ntx * 9 * sizeof(int), s, D, tb, c.g_log2TS,
                       k0, offs, lists);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const LaunchCfg& c, const cpx<T>* Gb, cpx<T>* out, const cpx<T>* dhat, int k0, int ns,
                         const Dims& D, const Tables<T>& tb, hipStream_t s) {
  hipError_t e = hipSuccess;
  LAM_MH_SWITCH(D.m, {
    auto k = k_gather<T, MH>;
    if ((e = prep(k, c.g_lds)) != hipSuccess) return e;
    const int ntiles = ((1 << D.log2M2) >> c.g_log2TS) * ((1 << D.log2M1) >> c.g_log2TS);
    hipLaunchKernelGGL(k, dim3(ntiles * ns), dim3(c.g_threads), c.g_lds, s, Gb, out, dhat, k0, D, tb, c.g_log2TS);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scatter(const LaunchCfg& c, const cpx<T>* in, cpx<T>* Gb, int k0, int ns, const Dims& D,
                          const Tables<T>& tb, hipStream_t s) {
  hipError_t e = hipSuccess;
  LAM_MH_SWITCH(D.m, {
    auto k = k_scatter<T, MH>;
    if ((e = prep(k, c.s_lds)) != hipSuccess) return e;
    const int ntiles = ((1 << D.log2M2) >> c.g_log2TS) * ((1 << D.log2M1) >> c.g_log2TS);
    hipLaunchKernelGGL(k, dim3(ntiles * ns), dim3(c.s_threads), c.s_lds, s, in, Gb, k0, D, tb, c.g_log2TS);
  });
  return hipGetLastError();
}

#define LAM_GRID_INST(T)                                                                                          \
  template hipError_t launch_list_count<T>(const LaunchCfg&, int, int, const Dims&, const Tables<T>&, int*,       \
                                           hipStream_t);                                                         \
  template hipError_t launch_list_fill<T>(const LaunchCfg&, int, int, const Dims&, const Tables<T>&, const int*,  \
                                          int*, hipStream_t);                                                    \
  template hipError_t launch_gather<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, const cpx<T>*, int, int,        \
                                       const Dims&, const Tables<T>&, hipStream_t);                              \
  template hipError_t launch_scatter<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, int, int, const Dims&,         \
                                        const Tables<T>&, hipStream_t);

LAM_GRID_INST(float)
LAM_GRID_INST(double)

}  // namespace lam
