// Internal declarations shared by the kernels and the host plan.
#pragma once
#include <hip/hip_runtime.h>

#include "lam_device.hpp"

namespace lam {

// Chunks whose memoized output is taken from the cache: a kernel whose unit (volume row y of the z
// steps, slab-local k_v slice of the 2D steps) lies in chunk ((unit + off) >> log2chunk) with a
// nonzero hit flag returns at once.  hit = nullptr: nothing is skipped.
struct SkipMap {
  const int* hit;
  int log2chunk, off;
  __device__ __forceinline__ bool skip(int unit) const { return hit && hit[(unit + off) >> log2chunk]; }
};

// Sizes passed by value to every kernel.  Every transform length (the oversampled grids M0, M1, M2
// and the detector h, w) is 2^l or 3 2^l; lM* is that l (the count of trailing zero bits).
struct Dims {
  int n0, n1, n2, h, w, ntheta, m;
  int M0, M1, M2;
  int lM0, lM1, lM2;
  double beta;      // Gaussian exponent in grid units, pi (R - 1/2) / (R m)
  XYGeom xy;
  SkipMap skip;     // memoized chunks (lam_admm_step_memo); empty otherwise
  // slice of row r of a slab of M1-row grids
  __device__ __forceinline__ int slice_of(int r) const { return M1 == (1 << lM1) ? r >> lM1 : div3(r >> lM1); }
};

// Periodic index arithmetic on a grid of M points: P2 when M is a power of two (a mask), otherwise
// M = 3 2^k (compares and selects).  wrap1 takes -M <= v < 2M, wrap2 -2M <= v < 2M.
template <bool P2> __host__ __device__ __forceinline__ int wrap1(int v, int M) {
  if constexpr (P2) return v & (M - 1);
  else return v < 0 ? v + M : (v >= M ? v - M : v);
}
template <bool P2> __host__ __device__ __forceinline__ int wrap2(int v, int M) {
  if constexpr (P2) return v & (M - 1);
  else {
    v = v < 0 ? v + 2 * M : v;
    return v >= M ? v - M : v;
  }
}
// e / N and N = 2^l (P2) or 3 2^l
template <bool P2> __device__ __forceinline__ int div_len(int e, int l) { return P2 ? e >> l : div3(e >> l); }

// Device tables (inside the caller's workspace), built in FP64 on the host.
template <typename T>
struct Tables {
  const cpx<T>* tw;   // exp(-2 pi i t / 2^log2tw): the power-of-two transforms
  int log2tw;
  const cpx<T>* tw3;  // exp(-2 pi i t / (3 2^log2tw3)): the 3 2^k transforms (null when the plan has none)
  int log2tw3;
  const T* cz;        // deconvolution factors along z, y, x
  const T* cy;
  const T* cx;
  const int* zbase;   // [h] floor(R xi_z) of detector row k_v
  const T* zdelta;    // [h] R xi_z - floor(R xi_z)
  const double* cth;  // [ntheta] cos(theta)
  const double* sth;  // [ntheta] sin(theta)
  const double* rc;   // [2m] exp(-beta (2 o + 1)), o = -m+1 ..
  const double* line; // [ntheta][6] per angle: A_x, 1/A_x, C_x, A_y, 1/A_y, C_y (s = A k_u + C k_v/h-units, 1/A = 0 if |A| < 1e-8)
  const unsigned* zrun; // [M0][2] rows whose z stencil covers grid point q: runs start | count << 16
  const int* tlist;   // per slice [n_theta w]: targets sorted by (tile, border class), t * 4096 + k_u index
  const int* toff;    // per slice [n_tiles 9 + 1]: offsets of the (tile, class) lists within the slice
  const int* gperm;   // per slice [n_tiles]: tiles in decreasing order of gather work
  const int* sperm;   // per slice [n_tiles]: tiles in decreasing order of spread work
  const unsigned char* sblk;   // aligned with tlist: the 8 x 8 block (8 by + bx) of each target's stencil
                               // base within its own tile (complex64 fixed-point spread only; else null)
};

// The list ranges [b, e) of one slice that tile (ty, tx) consumes in the adjoint
// spread, in 13 fixed slots (empty where a slot does not apply): its own list
// (all border classes); the facing border column of the left and right
// neighbours (3 classes each); the facing border row of the upper and lower
// neighbours; the facing corner of the 4 diagonal neighbours.  Neighbours along
// an axis with a single tile are skipped.  of: the slice's [n_tiles 9 + 1]
// offsets.  Fixed slots keep the arrays in registers on the device.
constexpr int kSpreadSlots = 13;
__host__ __device__ inline void spread_ranges(const int* of, int ntx, int nty, int ty, int tx, int* b, int* e) {
  auto set = [&](int slot, int tyy, int txx, int c0, int c1) {
    const int* o = of + (tyy * ntx + txx) * 9;
    b[slot] = o[c0];
    e[slot] = o[c1];
  };
  for (int s = 0; s < kSpreadSlots; ++s) b[s] = e[s] = 0;
  set(0, ty, tx, 0, 9);
  const int xl = (tx + ntx - 1) % ntx, xr = (tx + 1) % ntx, yu = (ty + nty - 1) % nty, yd = (ty + 1) % nty;
  if (ntx > 1)
    for (int c = 0; c < 3; ++c) {
      set(1 + c, ty, xl, 3 * c + 2, 3 * c + 3);    // left neighbour: its high-x border column
      set(4 + c, ty, xr, 3 * c, 3 * c + 1);        // right neighbour: its low-x border column
    }
  if (nty > 1) {
    set(7, yu, tx, 6, 9);                          // upper neighbour: its high-y border row
    set(8, yd, tx, 0, 3);                          // lower neighbour: its low-y border row
  }
  if (ntx > 1 && nty > 1) {
    set(9, yu, xl, 8, 9);
    set(10, yu, xr, 6, 7);
    set(11, yd, xl, 2, 3);
    set(12, yd, xr, 0, 1);
  }
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
hipError_t launch_list_blocks(const LaunchCfg& c, int k0, int ns, const Dims& D, const Tables<T>& tb,
                              unsigned char* sblk, hipStream_t s);
template <typename T>
hipError_t launch_list_check(const LaunchCfg& c, int k0, int ns, const Dims& D, const Tables<T>& tb, unsigned* seen,
                             int* bad, hipStream_t s);
template <typename T>
hipError_t launch_rowfft(const LaunchCfg& c, const cpx<T>* in, cpx<T>* out, bool inverse, int nproj, const Dims& D,
                         const Tables<T>& tb, hipStream_t s);
template <typename T>
hipError_t launch_colfft(const LaunchCfg& c, const cpx<T>* in, cpx<T>* out, bool inverse, double scale, int nproj,
                         const Dims& D, const Tables<T>& tb, hipStream_t s);

}  // namespace lam
