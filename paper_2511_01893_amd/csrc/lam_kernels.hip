// HIP kernels (gfx950) of the laminography operator L = F*_2D F_u2D F_u1D
// and its adjoint, and their host-side launchers.
//
// Stage map (forward; the adjoint runs the transposed stages in reverse):
//   k_zfwd      F_u1D: per (y, x-tile) column block: deconvolve by c_z, zero-pad
//               n0 -> M0 = R n0, FFT along z in LDS, gather the h targets
//               xi_z = n0 (k_v/h) cos(phi) with 2m table weights.
//   k_ycol_fwd  F_u2D part 1: per k_v slice and x-tile: deconvolve by c_y c_x,
//               zero-pad n1 -> M1, FFT along y.
//   k_xrow_fwd  F_u2D part 2: zero-pad rows n2 -> M2, FFT along x: the
//               oversampled grid G of one slice.
//   k_gather    F_u2D part 3: per (slice, TSxTS tile of G): stage the tile plus
//               a (2m-1) halo in LDS, enumerate the (theta, k_u) targets whose
//               stencil base falls in the tile, 2m x 2m Gaussian gather with
//               FP64 coordinates and weights; optional fused "- d^".
//   k_rowfft / k_colfft   F*_2D (and the adjoint's F_2D): centred 2D DFT per
//               projection as a row pass and a column pass.
// Adjoint: k_scatter (type-1 spreading into an LDS-privatised tile; each
// tile is owned by one work-group, so G is written with plain stores),
// k_xrow_adj, k_ycol_adj (inverse FFTs + crop + deconvolution), k_zadj.
#include "lam_internal.hpp"

namespace lam {

extern __shared__ __align__(16) unsigned char lam_smem[];

constexpr int VPT = 16;   // complex values per thread per FFT stage

__device__ __forceinline__ int sgn_parity(int k) { return (k & 1) ? -1 : 1; }

// ---------------------------------------------------------------------------
// F_u1D
// ---------------------------------------------------------------------------
template <typename T, int MH, bool REAL_IN>
__global__ __launch_bounds__(1024) void k_zfwd(const void* __restrict__ uin, cpx<T>* __restrict__ u1, Dims D,
                                               Tables<T> tb, int log2TX) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  const int TX = 1 << log2TX, M0 = 1 << D.log2M0, n0 = D.n0;
  const int x0 = blockIdx.x * TX, y = blockIdx.y;
  const int tid = threadIdx.x, nth = blockDim.x;
  const size_t plane = (size_t)D.n1 * D.n2;
  const cpx<T> zero = mk((T)0, (T)0);
  for (int e = tid; e < (M0 - n0) * TX; e += nth) buf[(n0 / 2) * TX + e] = zero;
  for (int e = tid; e < n0 * TX; e += nth) {
    const int a = e >> log2TX, b = e & (TX - 1);
    const size_t gi = (size_t)a * plane + (size_t)y * D.n2 + x0 + b;
    cpx<T> v;
    if constexpr (REAL_IN) v = mk(reinterpret_cast<const T*>(uin)[gi], (T)0);
    else v = reinterpret_cast<const cpx<T>*>(uin)[gi];
    buf[((a - n0 / 2) & (M0 - 1)) * TX + b] = v * tb.cz[a];
  }
  __syncthreads();
  lds_fft<T, VPT>(buf, D.log2M0, log2TX, TX, 1, true, tb.tw, tb.log2tw);
  for (int e = tid; e < D.h * TX; e += nth) {
    const int av = e >> log2TX, b = e & (TX - 1);
    const int base = tb.zbase[av] - MH + 1;
    const T* w = tb.zw + av * 2 * MH;
    T ax = 0, ay = 0;
#pragma unroll
    for (int i = 0; i < 2 * MH; ++i) {
      const cpx<T> g = buf[((base + i) & (M0 - 1)) * TX + b];
      ax += w[i] * g.x;
      ay += w[i] * g.y;
    }
    u1[(size_t)av * plane + (size_t)y * D.n2 + x0 + b] = mk(ax, ay);
  }
}

// F*_u1D: the transpose of the z gather, evaluated as a gather through the
// inverse table (for every grid point q of the oversampled line, the (k_v,
// weight) pairs whose stencil covers q), so no atomics are needed: stage the
// h samples of TX columns in LDS, form each grid value in registers, write
// the grid over the staging area, inverse FFT (conj-FFT-conj), crop,
// deconvolve.
template <typename T, int MH, bool REAL_OUT>
__global__ __launch_bounds__(1024) void k_zadj(const cpx<T>* __restrict__ u1, void* __restrict__ uout, Dims D,
                                               Tables<T> tb, int log2TX) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  const int TX = 1 << log2TX, M0 = 1 << D.log2M0, n0 = D.n0;
  const int x0 = blockIdx.x * TX, y = blockIdx.y;
  const int tid = threadIdx.x, nth = blockDim.x;
  const size_t plane = (size_t)D.n1 * D.n2;
  for (int e = tid; e < D.h * TX; e += nth) {
    const int av = e >> log2TX, b = e & (TX - 1);
    buf[e] = conj(u1[(size_t)av * plane + (size_t)y * D.n2 + x0 + b]);
  }
  __syncthreads();
  cpx<T> v[VPT];
  const int total = M0 * TX;
#pragma unroll
  for (int it = 0; it < VPT; ++it) {
    const int e = tid + it * nth;
    T ax = 0, ay = 0;
    if (e < total) {
      const int q = e >> log2TX, b = e & (TX - 1);
      const int beg = tb.zq_ptr[q], end = tb.zq_ptr[q + 1];
      for (int j = beg; j < end; ++j) {
        const T w = tb.zq_w[j];
        const cpx<T> g = buf[tb.zq_av[j] * TX + b];
        ax += w * g.x;
        ay += w * g.y;
      }
    }
    v[it] = mk(ax, ay);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < VPT; ++it) {
    const int e = tid + it * nth;
    if (e < total) buf[e] = v[it];
  }
  __syncthreads();
  lds_fft<T, VPT>(buf, D.log2M0, log2TX, TX, 1, true, tb.tw, tb.log2tw);
  for (int e = tid; e < n0 * TX; e += nth) {
    const int a = e >> log2TX, b = e & (TX - 1);
    const cpx<T> g = buf[((a - n0 / 2) & (M0 - 1)) * TX + b];
    const T c = tb.cz[a];
    const size_t gi = (size_t)a * plane + (size_t)y * D.n2 + x0 + b;
    if constexpr (REAL_OUT) reinterpret_cast<T*>(uout)[gi] = g.x * c;
    else reinterpret_cast<cpx<T>*>(uout)[gi] = mk(g.x * c, -g.y * c);
  }
}

// ---------------------------------------------------------------------------
// F_u2D / F*_u2D equispaced parts
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void k_ycol_fwd(const cpx<T>* __restrict__ u1, cpx<T>* __restrict__ Tb, int k0,
                                                   Dims D, Tables<T> tb, int log2TX) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  const int TX = 1 << log2TX, M1 = 1 << D.log2M1, n1 = D.n1, n2 = D.n2;
  const int x0 = blockIdx.x * TX, kk = blockIdx.y, k = k0 + kk;
  const int tid = threadIdx.x, nth = blockDim.x;
  const cpx<T> zero = mk((T)0, (T)0);
  for (int e = tid; e < (M1 - n1) * TX; e += nth) buf[(n1 / 2) * TX + e] = zero;
  for (int e = tid; e < n1 * TX; e += nth) {
    const int a = e >> log2TX, b = e & (TX - 1);
    const cpx<T> v = u1[((size_t)k * n1 + a) * n2 + x0 + b];
    buf[((a - n1 / 2) & (M1 - 1)) * TX + b] = v * (tb.cy[a] * tb.cx[x0 + b]);
  }
  __syncthreads();
  lds_fft<T, VPT>(buf, D.log2M1, log2TX, TX, 1, true, tb.tw, tb.log2tw);
  for (int e = tid; e < M1 * TX; e += nth) {
    const int q = e >> log2TX, b = e & (TX - 1);
    Tb[((size_t)kk * M1 + q) * n2 + x0 + b] = buf[e];
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_ycol_adj(const cpx<T>* __restrict__ Tb, cpx<T>* __restrict__ u1, int k0,
                                                   Dims D, Tables<T> tb, int log2TX) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  const int TX = 1 << log2TX, M1 = 1 << D.log2M1, n1 = D.n1, n2 = D.n2;
  const int x0 = blockIdx.x * TX, kk = blockIdx.y, k = k0 + kk;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int e = tid; e < M1 * TX; e += nth) {
    const int q = e >> log2TX, b = e & (TX - 1);
    buf[e] = conj(Tb[((size_t)kk * M1 + q) * n2 + x0 + b]);
  }
  __syncthreads();
  lds_fft<T, VPT>(buf, D.log2M1, log2TX, TX, 1, true, tb.tw, tb.log2tw);
  for (int e = tid; e < n1 * TX; e += nth) {
    const int a = e >> log2TX, b = e & (TX - 1);
    const cpx<T> v = buf[((a - n1 / 2) & (M1 - 1)) * TX + b];
    const T c = tb.cy[a] * tb.cx[x0 + b];
    u1[((size_t)k * n1 + a) * n2 + x0 + b] = mk(v.x * c, -v.y * c);
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_xrow_fwd(const cpx<T>* __restrict__ Tb, cpx<T>* __restrict__ Gb, Dims D,
                                                   Tables<T> tb, int log2RB) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  const int RB = 1 << log2RB, M2 = 1 << D.log2M2, n2 = D.n2, log2n2 = D.log2M2 - 1;
  const size_t r0 = (size_t)blockIdx.x * RB;
  const int tid = threadIdx.x, nth = blockDim.x;
  const cpx<T> zero = mk((T)0, (T)0);
  // R = 2: the padded positions of each row are [n2/2, M2 - n2/2), n2 of them
  for (int e = tid; e < RB * n2; e += nth) {
    const int b = e >> log2n2, a = e & (n2 - 1);
    buf[b * M2 + n2 / 2 + a] = zero;
    buf[b * M2 + ((a - n2 / 2) & (M2 - 1))] = Tb[(r0 + b) * n2 + a];
  }
  __syncthreads();
  lds_fft<T, VPT>(buf, D.log2M2, log2RB, 1, M2, false, tb.tw, tb.log2tw);
  for (int e = tid; e < RB * M2; e += nth) Gb[r0 * M2 + e] = buf[e];
}

template <typename T>
__global__ __launch_bounds__(1024) void k_xrow_adj(const cpx<T>* __restrict__ Gb, cpx<T>* __restrict__ Tb, Dims D,
                                                   Tables<T> tb, int log2RB) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  const int RB = 1 << log2RB, M2 = 1 << D.log2M2, n2 = D.n2, log2n2 = D.log2M2 - 1;
  const size_t r0 = (size_t)blockIdx.x * RB;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int e = tid; e < RB * M2; e += nth) buf[e] = conj(Gb[r0 * M2 + e]);
  __syncthreads();
  lds_fft<T, VPT>(buf, D.log2M2, log2RB, 1, M2, false, tb.tw, tb.log2tw);
  for (int e = tid; e < RB * n2; e += nth) {
    const int b = e >> log2n2, a = e & (n2 - 1);
    Tb[(r0 + b) * n2 + a] = conj(buf[b * M2 + ((a - n2 / 2) & (M2 - 1))]);
  }
}

// ---------------------------------------------------------------------------
// Target enumeration for a tile of the oversampled grid.
//
// For one angle the targets k_u lie on a line, s(k_u) = A k_u + B (per axis).
// cand_range returns a superset [lo, hi] (array indices) of the k_u whose
// stencil base floor(s) lies, modulo M, in [X0, X0+LX) along x and in
// [Y0, Y0+LY) along y.  The caller re-evaluates every candidate with
// target_coords and keeps only the ones that really qualify, so the bounds
// only need to be generous.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void interval_1d(double A, double B, double lo_s, double hi_s, int kmin, int kmax,
                                            int& a, int& b) {
  if (fabs(A) < 1e-8) {
    if (B >= lo_s - 1.0 && B < hi_s + 1.0) { a = kmin; b = kmax; }
    else { a = 1; b = 0; }
    return;
  }
  double k1 = (lo_s - B) / A, k2 = (hi_s - B) / A;
  if (k1 > k2) { const double t = k1; k1 = k2; k2 = t; }
  k1 = fmax(k1, (double)kmin - 2.0);
  k2 = fmin(k2, (double)kmax + 2.0);
  a = max(kmin, (int)ceil(k1 - 1e-3));
  b = min(kmax, (int)floor(k2 + 1e-3));
}

__device__ __forceinline__ void hull_axis(double A, double B, int X0, int LX, int M, int kmin, int kmax,
                                          int& lo, int& hi) {
  lo = kmax + 1;
  hi = kmin - 1;
  const double s_a = A * kmin + B, s_b = A * kmax + B;
  const double smin = fmin(s_a, s_b) - 1.0, smax = fmax(s_a, s_b) + 1.0;
  for (int i = -2; i <= 2; ++i) {
    const double l = (double)X0 + (double)i * M, h = l + LX;
    if (h < smin || l > smax) continue;
    int a, b;
    interval_1d(A, B, l, h, kmin, kmax, a, b);
    if (a <= b) { lo = min(lo, a); hi = max(hi, b); }
  }
}

__device__ __forceinline__ void cand_range(const XYGeom& g, double ct, double st, int akv, int X0, int LX, int M2,
                                           int Y0, int LY, int M1, int& lo, int& hi) {
  const double kv = (double)(akv - g.h / 2) * g.inv_h;
  const double Ax = g.Rn2 * ct * g.inv_w, Bx = g.Rn2 * (kv * g.sphi * st);
  const double Ay = g.Rn1 * st * g.inv_w, By = g.Rn1 * (-(kv * g.sphi * ct));
  const int kmin = -g.w / 2, kmax = g.w / 2 - 1;
  int xl, xh, yl, yh;
  hull_axis(Ax, Bx, X0, LX, M2, kmin, kmax, xl, xh);
  hull_axis(Ay, By, Y0, LY, M1, kmin, kmax, yl, yh);
  lo = max(xl, yl) + g.w / 2;
  hi = min(xh, yh) + g.w / 2;
}

// exclusive scan of a[0..n) in place, a[n] = total; part has blockDim.x*2 ints
__device__ void block_exclusive_scan(int* a, int n, int* part) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int per = (n + nth - 1) / nth;
  const int beg = min(n, tid * per), end = min(n, beg + per);
  int s = 0;
  for (int i = beg; i < end; ++i) s += a[i];
  part[tid] = s;
  __syncthreads();
  int* src = part;
  int* dst = part + nth;
  for (int off = 1; off < nth; off <<= 1) {
    dst[tid] = src[tid] + (tid >= off ? src[tid - off] : 0);
    __syncthreads();
    int* t = src; src = dst; dst = t;
  }
  int run = src[tid] - s;       // exclusive prefix of this thread's chunk
  for (int i = beg; i < end; ++i) { const int c = a[i]; a[i] = run; run += c; }
  if (tid == nth - 1) a[n] = src[nth - 1];
  __syncthreads();
}

// largest t in [0, n) with scan[t] <= i
__device__ __forceinline__ int find_theta(const int* scan, int n, int i) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (scan[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Shared by gather and scatter: FP64 coordinates, bases and weights of one target.
template <typename T, int MH>
__device__ __forceinline__ void target_stencil(const Dims& D, const Tables<T>& tb, double ct, double st, int akv,
                                               int aku, int& bx, int& by, T* wx, T* wy) {
  double sx, sy;
  target_coords(D.xy, ct, st, akv, aku, sx, sy);
  stencil_weights<T, MH>(sx, D.beta, tb.rc, bx, wx);
  stencil_weights<T, MH>(sy, D.beta, tb.rc, by, wy);
}

// ---------------------------------------------------------------------------
// F_u2D gather over one tile of the oversampled grid
// ---------------------------------------------------------------------------
template <typename T, int MH>
__global__ __launch_bounds__(256) void k_gather(const cpx<T>* __restrict__ Gb, cpx<T>* out,
                                                const cpx<T>* dhat, int k0, Dims D, Tables<T> tb,
                                                int log2TS) {
  const int TS = 1 << log2TS, P = TS + 2 * MH - 1;
  const int M1 = 1 << D.log2M1, M2 = 1 << D.log2M2;
  const int nt = D.ntheta;
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(lam_smem);
  int* scan = reinterpret_cast<int*>(tile + P * P);      // nt + 1
  int* lo = scan + nt + 1;                               // nt
  int* part = lo + nt;                                   // 2 * blockDim.x
  const int kk = blockIdx.z, k = k0 + kk;
  const int x0 = blockIdx.x * TS, y0 = blockIdx.y * TS;
  const int tid = threadIdx.x, nth = blockDim.x;
  const cpx<T>* G = Gb + (size_t)kk * M1 * M2;
  for (int e = tid; e < P * P; e += nth) {
    const int r = e / P, c = e - r * P;
    const int gy = (y0 - MH + 1 + r) & (M1 - 1), gx = (x0 - MH + 1 + c) & (M2 - 1);
    tile[e] = G[(size_t)gy * M2 + gx];
  }
  for (int t = tid; t < nt; t += nth) {
    int l, h;
    cand_range(D.xy, tb.cth[t], tb.sth[t], k, x0, TS, M2, y0, TS, M1, l, h);
    scan[t] = h >= l ? h - l + 1 : 0;
    lo[t] = l;
  }
  __syncthreads();
  block_exclusive_scan(scan, nt, part);
  const int total = scan[nt];
  for (int i = tid; i < total; i += nth) {
    const int t = find_theta(scan, nt, i);
    const int aku = lo[t] + (i - scan[t]);
    const double ct = tb.cth[t], st = tb.sth[t];
    double sx, sy;
    target_coords(D.xy, ct, st, k, aku, sx, sy);
    const int ox = ((int)floor(sx) - x0) & (M2 - 1), oy = ((int)floor(sy) - y0) & (M1 - 1);
    if (ox >= TS || oy >= TS) continue;
    T wx[2 * MH], wy[2 * MH];
    int bx, by;
    stencil_weights<T, MH>(sx, D.beta, tb.rc, bx, wx);
    stencil_weights<T, MH>(sy, D.beta, tb.rc, by, wy);
    T ax = 0, ay = 0;
#pragma unroll
    for (int iy = 0; iy < 2 * MH; ++iy) {
      const cpx<T>* row = tile + (oy + iy) * P + ox;
      T rx = 0, ry = 0;
#pragma unroll
      for (int ix = 0; ix < 2 * MH; ++ix) {
        const cpx<T> g = row[ix];
        rx += wx[ix] * g.x;
        ry += wx[ix] * g.y;
      }
      ax += wy[iy] * rx;
      ay += wy[iy] * ry;
    }
    const size_t o = ((size_t)t * D.h + k) * D.w + aku;
    if (dhat) {
      const cpx<T> q = dhat[o];
      ax -= q.x;
      ay -= q.y;
    }
    out[o] = mk(ax, ay);
  }
}

// ---------------------------------------------------------------------------
// F*_u2D scatter into one tile of the oversampled grid (owner computes).
//
// One lane per candidate target: FP64 coordinates and weights, then the 2m x
// 2m taps that land in the tile are added into an FP64 LDS accumulator with
// native ds_add_f64 (gfx950 executes FP64 LDS atomics at close to the rate
// of plain stores, unlike FP32 LDS atomics).  Accumulating in FP64 also
// makes the sum insensitive to the arrival order.  Every cell of the tile is
// finally rounded to T and written once to the grid, so G needs no clearing
// and no global atomics.
// ---------------------------------------------------------------------------
template <typename T, int MH>
__global__ __launch_bounds__(256) void k_scatter(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ Gb, int k0,
                                                 Dims D, Tables<T> tb, int log2TS) {
  constexpr int W = 2 * MH;
  const int TS = 1 << log2TS, PA = TS + 1;
  const int M1 = 1 << D.log2M1, M2 = 1 << D.log2M2;
  const int nt = D.ntheta;
  const int tid = threadIdx.x, nth = blockDim.x;
  double* acc = reinterpret_cast<double*>(lam_smem);          // [TS][PA] complex as (re, im) doubles
  int* scan = reinterpret_cast<int*>(acc + 2 * TS * PA);
  int* lo = scan + nt + 1;
  int* part = lo + nt;
  const int kk = blockIdx.z, k = k0 + kk;
  const int x0 = blockIdx.x * TS, y0 = blockIdx.y * TS;
  const int LX = TS + W - 1;
  for (int e = tid; e < 2 * TS * PA; e += nth) acc[e] = 0.0;
  for (int t = tid; t < nt; t += nth) {
    int l, h;
    cand_range(D.xy, tb.cth[t], tb.sth[t], k, x0 - MH, LX, M2, y0 - MH, LX, M1, l, h);
    scan[t] = h >= l ? h - l + 1 : 0;
    lo[t] = l;
  }
  __syncthreads();
  block_exclusive_scan(scan, nt, part);
  const int total = scan[nt];
  for (int i = tid; i < total; i += nth) {
    const int t = find_theta(scan, nt, i);
    const int aku = lo[t] + (i - scan[t]);
    double sx, sy;
    target_coords(D.xy, tb.cth[t], tb.sth[t], k, aku, sx, sy);
    // stencil corner relative to the tile, modulo the grid; the stencil
    // touches the tile if it starts inside it or wraps into it
    const int rx0 = ((int)floor(sx) - MH + 1 - x0) & (M2 - 1);
    const int ry0 = ((int)floor(sy) - MH + 1 - y0) & (M1 - 1);
    if (!((rx0 < TS || rx0 > M2 - W) && (ry0 < TS || ry0 > M1 - W))) continue;
    T wx[W], wy[W];
    int bx, by;
    stencil_weights<T, MH>(sx, D.beta, tb.rc, bx, wx);
    stencil_weights<T, MH>(sy, D.beta, tb.rc, by, wy);
    const cpx<T> v = in[((size_t)t * D.h + k) * D.w + aku];
#pragma unroll
    for (int iy = 0; iy < W; ++iy) {
      const int row = (ry0 + iy) & (M1 - 1);
      if (row >= TS) continue;
      const double vx = (double)(wy[iy] * v.x), vy = (double)(wy[iy] * v.y);
#pragma unroll
      for (int ix = 0; ix < W; ++ix) {
        const int col = (rx0 + ix) & (M2 - 1);
        if (col >= TS) continue;
        double* cell = acc + 2 * (row * PA + col);
        atomicAdd(cell, (double)wx[ix] * vx);
        atomicAdd(cell + 1, (double)wx[ix] * vy);
      }
    }
  }
  __syncthreads();
  cpx<T>* G = Gb + (size_t)kk * M1 * M2;
  for (int e = tid; e < TS * TS; e += nth) {
    const int r = e >> log2TS, c = e & (TS - 1);
    const double* cell = acc + 2 * (r * PA + c);
    G[(size_t)(y0 + r) * M2 + x0 + c] = mk((T)cell[0], (T)cell[1]);
  }
}

// ---------------------------------------------------------------------------
// Centred 2D DFT per projection: row pass (along k_u / p) and column pass
// (along k_v / v).  Centring is the checkerboard (-1)^(row+col) applied
// before the row pass and after the column pass (h, w multiples of 4).
// The inverse transform is conj(FFT(conj(.))).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void k_rowfft(const cpx<T>* in, cpx<T>* out, int log2L,
                                                 int log2h, int log2RB, int inverse, Tables<T> tb) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  const int RB = 1 << log2RB, L = 1 << log2L;
  const size_t r0 = (size_t)blockIdx.x * RB;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int hmask = (1 << log2h) - 1;
  for (int e = tid; e < RB * L; e += nth) {
    const int b = e >> log2L, p = e & (L - 1);
    const int arow = (int)((r0 + b) & hmask);
    cpx<T> v = in[r0 * L + e];
    if (inverse) v = conj(v);
    buf[e] = sgn_parity(arow + p) > 0 ? v : mk(-v.x, -v.y);
  }
  __syncthreads();
  lds_fft<T, VPT>(buf, log2L, log2RB, 1, L, false, tb.tw, tb.log2tw);
  for (int e = tid; e < RB * L; e += nth) {
    const cpx<T> v = buf[e];
    out[r0 * L + e] = inverse ? conj(v) : v;
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_colfft(const cpx<T>* in, cpx<T>* out, int log2h,
                                                 int log2w, int log2TX, int inverse, T scale, Tables<T> tb) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  const int TX = 1 << log2TX, H = 1 << log2h, W = 1 << log2w;
  const int p0 = blockIdx.x * TX;
  const size_t base = (size_t)blockIdx.y * H * W;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int e = tid; e < H * TX; e += nth) {
    const int a = e >> log2TX, b = e & (TX - 1);
    const cpx<T> v = in[base + (size_t)a * W + p0 + b];
    buf[e] = inverse ? conj(v) : v;
  }
  __syncthreads();
  lds_fft<T, VPT>(buf, log2h, log2TX, TX, 1, true, tb.tw, tb.log2tw);
  for (int e = tid; e < H * TX; e += nth) {
    const int a = e >> log2TX, b = e & (TX - 1);
    cpx<T> v = buf[e];
    if (inverse) v = conj(v);
    const T s = sgn_parity(a + p0 + b) > 0 ? scale : -scale;
    out[base + (size_t)a * W + p0 + b] = v * s;
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <typename Kern>
static hipError_t prep(Kern k, size_t lds) {
  if (lds > 64 * 1024) return hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

#define LAM_MH_SWITCH(MHV, ...)                     \
  switch (MHV) {                                    \
    case 1: { constexpr int MH = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int MH = 2; __VA_ARGS__; } break; \
    case 3: { constexpr int MH = 3; __VA_ARGS__; } break; \
    case 4: { constexpr int MH = 4; __VA_ARGS__; } break; \
    case 5: { constexpr int MH = 5; __VA_ARGS__; } break; \
    case 6: { constexpr int MH = 6; __VA_ARGS__; } break; \
    case 7: { constexpr int MH = 7; __VA_ARGS__; } break; \
    default: { constexpr int MH = 8; __VA_ARGS__; } break; \
  }

template <typename T>
hipError_t launch_zfwd(const LaunchCfg& c, const void* u, bool real_in, cpx<T>* u1, const Dims& D, const Tables<T>& tb,
                       hipStream_t s) {
  dim3 grid(D.n2 >> c.z_log2TX, D.n1);
  hipError_t e = hipSuccess;
  LAM_MH_SWITCH(D.m, {
    if (real_in) {
      auto k = k_zfwd<T, MH, true>;
      if ((e = prep(k, c.z_lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k, grid, dim3(c.z_threads), c.z_lds, s, u, u1, D, tb, c.z_log2TX);
    } else {
      auto k = k_zfwd<T, MH, false>;
      if ((e = prep(k, c.z_lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k, grid, dim3(c.z_threads), c.z_lds, s, u, u1, D, tb, c.z_log2TX);
    }
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zadj(const LaunchCfg& c, const cpx<T>* u1, void* u, bool real_out, const Dims& D,
                       const Tables<T>& tb, hipStream_t s) {
  dim3 grid(D.n2 >> c.z_log2TX, D.n1);
  hipError_t e = hipSuccess;
  LAM_MH_SWITCH(D.m, {
    if (real_out) {
      auto k = k_zadj<T, MH, true>;
      if ((e = prep(k, c.z_lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k, grid, dim3(c.z_threads), c.z_lds, s, u1, u, D, tb, c.z_log2TX);
    } else {
      auto k = k_zadj<T, MH, false>;
      if ((e = prep(k, c.z_lds)) != hipSuccess) return e;
      hipLaunchKernelGGL(k, grid, dim3(c.z_threads), c.z_lds, s, u1, u, D, tb, c.z_log2TX);
    }
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ycol_fwd(const LaunchCfg& c, const cpx<T>* u1, cpx<T>* Tb, int k0, int ns, const Dims& D,
                           const Tables<T>& tb, hipStream_t s) {
  auto k = k_ycol_fwd<T>;
  hipError_t e = prep(k, c.y_lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(D.n2 >> c.y_log2TX, ns), dim3(c.y_threads), c.y_lds, s, u1, Tb, k0, D, tb, c.y_log2TX);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xrow_fwd(const LaunchCfg& c, const cpx<T>* Tb, cpx<T>* Gb, int ns, const Dims& D,
                           const Tables<T>& tb, hipStream_t s) {
  auto k = k_xrow_fwd<T>;
  hipError_t e = prep(k, c.x_lds);
  if (e != hipSuccess) return e;
  const size_t rows = (size_t)ns << D.log2M1;
  hipLaunchKernelGGL(k, dim3((unsigned)(rows >> c.x_log2RB)), dim3(c.x_threads), c.x_lds, s, Tb, Gb, D, tb,
                     c.x_log2RB);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const LaunchCfg& c, const cpx<T>* Gb, cpx<T>* out, const cpx<T>* dhat, int k0, int ns,
                         const Dims& D, const Tables<T>& tb, hipStream_t s) {
  hipError_t e = hipSuccess;
  LAM_MH_SWITCH(D.m, {
    auto k = k_gather<T, MH>;
    if ((e = prep(k, c.g_lds)) != hipSuccess) return e;
    dim3 grid((1 << D.log2M2) >> c.g_log2TS, (1 << D.log2M1) >> c.g_log2TS, ns);
    hipLaunchKernelGGL(k, grid, dim3(c.g_threads), c.g_lds, s, Gb, out, dhat, k0, D, tb, c.g_log2TS);
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
    dim3 grid((1 << D.log2M2) >> c.g_log2TS, (1 << D.log2M1) >> c.g_log2TS, ns);
    hipLaunchKernelGGL(k, grid, dim3(c.s_threads), c.s_lds, s, in, Gb, k0, D, tb, c.g_log2TS);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xrow_adj(const LaunchCfg& c, const cpx<T>* Gb, cpx<T>* Tb, int ns, const Dims& D,
                           const Tables<T>& tb, hipStream_t s) {
  auto k = k_xrow_adj<T>;
  hipError_t e = prep(k, c.x_lds);
  if (e != hipSuccess) return e;
  const size_t rows = (size_t)ns << D.log2M1;
  hipLaunchKernelGGL(k, dim3((unsigned)(rows >> c.x_log2RB)), dim3(c.x_threads), c.x_lds, s, Gb, Tb, D, tb,
                     c.x_log2RB);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ycol_adj(const LaunchCfg& c, const cpx<T>* Tb, cpx<T>* u1, int k0, int ns, const Dims& D,
                           const Tables<T>& tb, hipStream_t s) {
  auto k = k_ycol_adj<T>;
  hipError_t e = prep(k, c.y_lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(D.n2 >> c.y_log2TX, ns), dim3(c.y_threads), c.y_lds, s, Tb, u1, k0, D, tb, c.y_log2TX);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rowfft(const LaunchCfg& c, const cpx<T>* in, cpx<T>* out, bool inverse, const Dims& D,
                         const Tables<T>& tb, hipStream_t s) {
  const int log2h = __builtin_ctz(D.h), log2w = __builtin_ctz(D.w);
  auto k = k_rowfft<T>;
  hipError_t e = prep(k, c.r_lds);
  if (e != hipSuccess) return e;
  const size_t rows = (size_t)D.ntheta * D.h;
  hipLaunchKernelGGL(k, dim3((unsigned)(rows >> c.r_log2RB)), dim3(c.r_threads), c.r_lds, s, in, out, log2w, log2h,
                     c.r_log2RB, inverse ? 1 : 0, tb);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_colfft(const LaunchCfg& c, const cpx<T>* in, cpx<T>* out, bool inverse, double scale_d,
                         const Dims& D, const Tables<T>& tb, hipStream_t s) {
  const int log2h = __builtin_ctz(D.h), log2w = __builtin_ctz(D.w);
  auto k = k_colfft<T>;
  hipError_t e = prep(k, c.c_lds);
  if (e != hipSuccess) return e;
  const T scale = (T)scale_d;
  hipLaunchKernelGGL(k, dim3(D.w >> c.c_log2TX, D.ntheta), dim3(c.c_threads), c.c_lds, s, in, out, log2h, log2w,
                     c.c_log2TX, inverse ? 1 : 0, scale, tb);
  return hipGetLastError();
}

#define LAM_INST(T)                                                                                              \
  template hipError_t launch_zfwd<T>(const LaunchCfg&, const void*, bool, cpx<T>*, const Dims&, const Tables<T>&, \
                                     hipStream_t);                                                               \
  template hipError_t launch_zadj<T>(const LaunchCfg&, const cpx<T>*, void*, bool, const Dims&, const Tables<T>&, \
                                     hipStream_t);                                                               \
  template hipError_t launch_ycol_fwd<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, int, int, const Dims&,        \
                                         const Tables<T>&, hipStream_t);                                         \
  template hipError_t launch_xrow_fwd<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, int, const Dims&,             \
                                         const Tables<T>&, hipStream_t);                                         \
  template hipError_t launch_gather<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, const cpx<T>*, int, int,        \
                                       const Dims&, const Tables<T>&, hipStream_t);                              \
  template hipError_t launch_scatter<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, int, int, const Dims&,         \
                                        const Tables<T>&, hipStream_t);                                          \
  template hipError_t launch_xrow_adj<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, int, const Dims&,             \
                                         const Tables<T>&, hipStream_t);                                         \
  template hipError_t launch_ycol_adj<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, int, int, const Dims&,        \
                                         const Tables<T>&, hipStream_t);                                         \
  template hipError_t launch_rowfft<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, bool, const Dims&,              \
                                       const Tables<T>&, hipStream_t);                                           \
  template hipError_t launch_colfft<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, bool, double, const Dims&,      \
                                       const Tables<T>&, hipStream_t);

LAM_INST(float)
LAM_INST(double)

}  // namespace lam
