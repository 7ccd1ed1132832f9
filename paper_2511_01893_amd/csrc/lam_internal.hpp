// Internal declarations shared by the kernels and the host plan.
#pragma once
#include <hip/hip_runtime.h>

#include "lam_device.hpp"

namespace lam {

// Sizes passed by value to every kernel.
struct Dims {
  int n0, n1, n2, h, w, ntheta, m;
  int log2M0, log2M1, log2M2;
  double beta;      // Gaussian exponent in grid units, pi (R - 1/2) / (R m)
  XYGeom xy;
};

// Device tables (inside the caller's workspace), built in FP64 on the host.
template <typename T>
struct Tables {
  const cpx<T>* tw;   // exp(-2 pi i t / 2^log2tw)
  int log2tw;
  const T* cz;        // deconvolution factors along z, y, x
  const T* cy;
  const T* cx;
  const int* zbase;   // [h] floor(R xi_z)
  const T* zw;        // [h][2m] z-gather weights
  const double* cth;  // [ntheta] cos(theta)
  const double* sth;  // [ntheta] sin(theta)
  const double* rc;   // [2m] exp(-beta (2 o + 1)), o = -m+1 ..
  const double* line; // [ntheta][6] per angle: A_x, 1/A_x, C_x, A_y, 1/A_y, C_y (s = A k_u + C k_v/h-units, 1/A = 0 if |A| < 1e-8)
  const int* zq_ptr;  // [M0 + 1] inverse z table: for grid point q, entries zq_ptr[q] .. zq_ptr[q+1]
  const int* zq_av;   // [h 2m] k_v index of each entry
  const T* zq_w;      // [h 2m] weight of each entry
  const int* tlist;   // per slice [n_theta w]: targets sorted by (tile, border class), t * 4096 + k_u index
  const int* toff;    // per slice [n_tiles 9 + 1]: offsets of the (tile, class) lists within the slice
  const int* gperm;   // per slice [n_tiles]: tiles in decreasing order of gather work
  const int* sperm;   // per slice [n_tiles]: tiles in decreasing order of spread work
};

// The list ranges [b, e) of one slice that tile (ty, tx) consumes in the adjoint
// spread: its own list (all border classes), then the border classes of the
// neighbouring tiles whose stencils reach into it (the facing column of a left /
// right neighbour, the facing row of an upper / lower one, the facing corner of
// a diagonal one).  of: the slice's [n_tiles 9 + 1] offsets.  Returns the number
// of non-empty ranges (at most 13).
__host__ __device__ inline int spread_ranges(const int* of, int ntx, int nty, int ty, int tx, int* b, int* e) {
  int nr = 0;
  auto add = [&](int tyy, int txx, int c0, int c1) {
    const int* o = of + (tyy * ntx + txx) * 9;
    if (o[c1] > o[c0]) { b[nr] = o[c0]; e[nr] = o[c1]; ++nr; }
  };
  add(ty, tx, 0, 9);
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      if ((dx == 0 && dy == 0) || (dx != 0 && ntx == 1) || (dy != 0 && nty == 1)) continue;
      const int ny_ = (ty + dy + nty) % nty, nx_ = (tx + dx + ntx) % ntx;
      const int cx = dx < 0 ? 2 : 0, cy = dy < 0 ? 2 : 0;     // the neighbour's border facing this tile
      if (dy == 0) {
        for (int c = 0; c < 3; ++c) add(ny_, nx_, 3 * c + cx, 3 * c + cx + 1);
      } else if (dx == 0) {
        add(ny_, nx_, 3 * cy, 3 * cy + 3);
      } else {
        add(ny_, nx_, 3 * cy + cx, 3 * cy + cx + 1);
      }
    }
  return nr;
}

// Launch shapes chosen by the host plan.
struct LaunchCfg {
  int z_log2TX, z_threads; size_t z_lds;    // F_u1D column blocks
  int y_log2TX, y_threads; size_t y_lds;    // y-FFT column blocks
  int x_log2RB, x_threads; size_t x_lds;    // x-FFT row blocks
  int g_log2TS, g_threads; size_t g_lds;    // gather tiles (TS = 2^g_log2TS, also the scatter's)
  int s_threads; size_t s_lds;              // scatter tiles
  int r_log2RB, r_threads; size_t r_lds;    // 2D FFT row pass
  int c_log2TX, c_threads; size_t c_lds;    // 2D FFT column pass
};

template <typename T>
// z step over the volume rows [y0, y0 + ny); the slab buffer holds those rows with z stride zs elements
// (zs = n1 n2 for the whole volume)
hipError_t launch_zfwd(const LaunchCfg& c, const void* u, bool real_in, cpx<T>* u1, int y0, int ny, size_t in_zs,
                       const Dims& D, const Tables<T>& tb, hipStream_t s);
template <typename T>
hipError_t launch_zadj(const LaunchCfg& c, const cpx<T>* u1, void* u, bool real_out, int y0, int ny, size_t out_zs,
                       const Dims& D, const Tables<T>& tb, hipStream_t s);
template <typename T>
hipError_t launch_ycol_fwd(const LaunchCfg& c, const cpx<T>* u1, cpx<T>* Tb, int k0, int ns, const Dims& D,
                           const Tables<T>& tb, hipStream_t s);
template <typename T>
hipError_t launch_xrow_fwd(const LaunchCfg& c, const cpx<T>* Tb, cpx<T>* Gb, int ns, const Dims& D,
                           const Tables<T>& tb, hipStream_t s);
template <typename T>
hipError_t launch_gather(const LaunchCfg& c, const cpx<T>* Gb, cpx<T>* out, const cpx<T>* dhat, int k0, int ns,
                         const Dims& D, const Tables<T>& tb, hipStream_t s);
template <typename T>
hipError_t launch_scatter(const LaunchCfg& c, const cpx<T>* in, cpx<T>* Gb, int k0, int ns, const Dims& D,
                          const Tables<T>& tb, hipStream_t s);
template <typename T>
hipError_t launch_xrow_adj(const LaunchCfg& c, const cpx<T>* Gb, cpx<T>* Tb, int ns, const Dims& D,
                           const Tables<T>& tb, hipStream_t s);
template <typename T>
hipError_t launch_ycol_adj(const LaunchCfg& c, const cpx<T>* Tb, cpx<T>* u1, int k0, int ns, const Dims& D,
                           const Tables<T>& tb, hipStream_t s);
template <typename T>
hipError_t launch_list_count(const LaunchCfg& c, int k0, int ns, const Dims& D, const Tables<T>& tb, int* counts,
                             hipStream_t s);
template <typename T>
hipError_t launch_list_fill(const LaunchCfg& c, int k0, int ns, const Dims& D, const Tables<T>& tb, const int* offs,
                            int* lists, hipStream_t s);
template <typename T>
hipError_t launch_rowfft(const LaunchCfg& c, const cpx<T>* in, cpx<T>* out, bool inverse, int nproj, const Dims& D,
                         const Tables<T>& tb, hipStream_t s);
template <typename T>
hipError_t launch_colfft(const LaunchCfg& c, const cpx<T>* in, cpx<T>* out, bool inverse, double scale, int nproj,
                         const Dims& D, const Tables<T>& tb, hipStream_t s);

}  // namespace lam
