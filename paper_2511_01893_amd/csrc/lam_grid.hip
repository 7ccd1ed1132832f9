// The unequally-spaced part of F_u2D and its adjoint on the oversampled grid
// of one k_v slice: the 2m x 2m Gaussian gather (forward) and spread
// (adjoint) at the n_theta x w targets of the slice.
//
// The targets' coordinates depend only on the geometry, so the plan sorts
// them once (at lam_set_workspace): for every slice, every TS x TS tile of
// the M1 x M2 grid gets the list of targets whose stencil base floor(s)
// lies in the tile, sub-sorted into 3 x 3 classes by whether the stencil
// reaches across the tile's low / high border in x and y.  Each target is
// listed exactly once (checked when the lists are built: every slice holds
// n_theta w entries, and k_list_check re-classifies every entry and marks it
// in a per-target bitmap, so a duplicate or a misplaced entry is an error).
//   k_gather   stages a tile plus its (2m-1) halo in LDS and walks the tile's
//              list, one lane per target: FP64 coordinates, weights, 2m x 2m
//              FMA gather, optional fused "- d^" (Algorithm 2).
//   k_scatter_fx  (complex64, grids of at least 128 x 128, m <= 4) accumulates
//              one tile in LDS in 64-bit fixed point, re and im packed in one
//              integer per cell: its own list plus the border classes of the 8
//              neighbouring tiles whose stencils reach in, one lane per stencil
//              column, one integer LDS atomic per tap; bit-reproducible.
//   k_scatter  the same in FP64 LDS atomics (complex128, and complex64 on
//              smaller grids or for m > 4; for m = 4 on large grids laid out
//              so that each atomic instruction adds two adjacent rows of 4
//              targets, which spreads it evenly over the LDS banks).  Every
//              cell of the tile is then written once.
#include <type_traits>

#include "lam_lists.hpp"

namespace lam {

extern __shared__ __align__(16) unsigned char lam_smem[];

namespace {

// Visit every target of slice k whose base row lies in the band of tile row
// ty.  One wave per angle; its lanes take consecutive k_u, so each call of
// f(ok, t, aku, tx, class) (made by all lanes of the wave together; ok
// marks the lanes holding a target of the band, tx its tile column) sees a
// run of neighbouring targets along one line of the slice.
template <int MH, class F>
__device__ __forceinline__ void band_targets(const Dims& D, const double* cth, const double* sth, const double* line,
                                             int k, int ty, int log2TS, F&& f) {
  const int Y0 = ty << log2TS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  for (int t = wave; t < D.ntheta; t += nwave) {
    int lo[2], hi[2];
    const int n = band_intervals(D, line + 6 * t, k, Y0, log2TS, lo, hi);
    for (int jj = 0; jj < n; ++jj)
      for (int ku0 = lo[jj]; ku0 <= hi[jj]; ku0 += 64) {
        const int ku = ku0 + lane;
        bool ok = ku <= hi[jj];
        int tx = 0, c = 0;
        if (ok) ok = classify_target(D, cth[t], sth[t], k, ku + D.w / 2, Y0, log2TS, MH, tx, c);
        f(ok, t, ku + D.w / 2, tx, c);
      }
  }
}

// counts[k][ty][tx][class] for the slices [k0, k0 + gridDim.y), tile row blockIdx.x
template <typename T, int MH>
__global__ __launch_bounds__(256) void k_list_count(Dims D, Tables<T> tb, int log2TS, int k0, int* __restrict__ counts) {
  const int ntx = D.M2 >> log2TS, nty = D.M1 >> log2TS;
  const int ty = blockIdx.x, k = k0 + blockIdx.y;
  int* cnt = reinterpret_cast<int*>(lam_smem);                 // [ntx * 9]
  for (int i = threadIdx.x; i < ntx * 9; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  band_targets<MH>(D, tb.cth, tb.sth, tb.line, k, ty, log2TS, [&](bool ok, int, int, int tx, int c) {
    if (ok) atomicAdd(&cnt[tx * 9 + c], 1);
  });
  __syncthreads();
  const size_t per_slice = (size_t)ntx * nty * 9 + 1;
  int* out = counts + (size_t)k * per_slice + (size_t)ty * ntx * 9;
  for (int i = threadIdx.x; i < ntx * 9; i += blockDim.x) out[i] = cnt[i];
}

// lists[k][offset] = t * 4096 + aku, placed from the per-slice offsets.  The
// lanes of a wave that share a (tile, class) list take one contiguous block
// of it in lane order, so each list holds runs of targets that are
// neighbours along a line (the gather's LDS reads of a run overlap).
template <typename T, int MH>
__global__ __launch_bounds__(256) void k_list_fill(Dims D, Tables<T> tb, int log2TS, int k0, const int* __restrict__ offs,
                                                   int* __restrict__ lists) {
  const int ntx = D.M2 >> log2TS, nty = D.M1 >> log2TS;
  const int ty = blockIdx.x, k = k0 + blockIdx.y;
  int* cur = reinterpret_cast<int*>(lam_smem);                 // [ntx * 9]
  const size_t per_slice = (size_t)ntx * nty * 9 + 1;
  const int* of = offs + (size_t)k * per_slice + (size_t)ty * ntx * 9;
  for (int i = threadIdx.x; i < ntx * 9; i += blockDim.x) cur[i] = of[i];
  __syncthreads();
  int* L = lists + (size_t)k * D.ntheta * D.w;
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  band_targets<MH>(D, tb.cth, tb.sth, tb.line, k, ty, log2TS, [&](bool ok, int t, int aku, int tx, int c) {
    const int dest = tx * 9 + c;
    unsigned long long pending = __ballot(ok);
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const int d = __shfl(dest, leader);
      const bool mine = ok && dest == d;
      const unsigned long long m = __ballot(mine);
      int base = 0;
      if (lane == leader) base = atomicAdd(&cur[d], __popcll(m));
      base = __shfl(base, leader);
      if (mine) L[base + __popcll(m & below)] = t * 4096 + aku;
      pending &= ~m;
    }
  });
}

// sblk[k][i] for the lists of slices [k0, k0 + gridDim.y), one block per (tile, slice): the 8 x 8 block
// (8 by + bx) of each listed target's stencil base within its own tile (the same FP64 coordinates as the
// kernels), so that the complex64 spread's first pass places a sample without evaluating them.
template <typename T, int MH>
__global__ __launch_bounds__(256) void k_list_blocks(Dims D, Tables<T> tb, int log2TS, int k0,
                                                     unsigned char* __restrict__ sblk) {
  const int ntx = D.M2 >> log2TS, nty = D.M1 >> log2TS;
  const int tile = blockIdx.x, k = k0 + blockIdx.y, tx = tile % ntx, ty = tile / ntx;
  const int* of = tb.toff + (size_t)k * ((size_t)ntx * nty * 9 + 1) + (size_t)tile * 9;
  const size_t base = (size_t)k * D.ntheta * D.w;
  for (int i = of[0] + (int)threadIdx.x; i < of[9]; i += blockDim.x) {
    const int id = tb.tlist[base + i], t = id >> 12, aku = id & 4095;
    double sx, sy;
    target_coords(D.xy, tb.cth[t], tb.sth[t], k, aku, sx, sy);
    const int oy = pmod((int)floor(sy) - (ty << log2TS), D.M1), ox = pmod((int)floor(sx) - (tx << log2TS), D.M2);
    sblk[base + i] = (unsigned char)(((oy >> 3) << 3) | (ox >> 3));
  }
}

// Exact check of the lists of slices [k0, k0 + gridDim.y), one block per (tile, slice): every entry
// must name a target in range, classify (by the same FP64 coordinates) into the tile and border
// class whose list holds it, and appear only once in its slice (a bit per target in `seen`, cleared
// by the caller).  With the per-slice counts equal to n_theta w this makes each slice's lists a
// permutation of its targets.  Every violation adds one to *bad.
template <typename T, int MH>
__global__ __launch_bounds__(256) void k_list_check(Dims D, Tables<T> tb, int log2TS, int k0,
                                                    unsigned* __restrict__ seen, int* __restrict__ bad) {
  const int ntx = D.M2 >> log2TS, nty = D.M1 >> log2TS;
  const int tile = blockIdx.x, k = k0 + blockIdx.y, tx = tile % ntx, ty = tile / ntx;
  const int* of = tb.toff + (size_t)k * ((size_t)ntx * nty * 9 + 1) + (size_t)tile * 9;
  const int* L = tb.tlist + (size_t)k * D.ntheta * D.w;
  int nbad = 0;
  for (int c = 0; c < 9; ++c)
    for (int i = of[c] + (int)threadIdx.x; i < of[c + 1]; i += blockDim.x) {
      const int id = L[i], t = id >> 12, aku = id & 4095;
      if (id < 0 || t >= D.ntheta || aku >= D.w) { ++nbad; continue; }
      int tx2 = -1, c2 = -1;
      if (!classify_target(D, tb.cth[t], tb.sth[t], k, aku, ty << log2TS, log2TS, MH, tx2, c2) || tx2 != tx || c2 != c)
        ++nbad;
      const size_t bit = ((size_t)k * D.ntheta + t) * D.w + aku;
      const unsigned m = 1u << (bit & 31);
      if (atomicOr(&seen[bit >> 5], m) & m) ++nbad;
    }
  if (nbad) atomicAdd(bad, nbad);
}

}  // namespace

// ---------------------------------------------------------------------------
// Lane layout of the spread: a wave takes NG = 64 / GW targets
// at a time, GW = the stencil width 2m rounded up to a power of two; lane j of
// a target's group owns stencil column j, so one stencil row is GW adjacent
// cells of the tile.  Every lane computes its target's FP64 coordinates, the
// 2m y-weights and its own x-weight.
// ---------------------------------------------------------------------------
template <int MH> constexpr int group_width() { return 2 * MH <= 2 ? 2 : (2 * MH <= 4 ? 4 : (2 * MH <= 8 ? 8 : 16)); }

// The weights exp(-beta (delta - o)^2), o = -m+1 .. m, of one axis come from
// three exponentials (fast Gaussian gridding, Greengard & Lee): the centre tap
// o = 0 (a = delta in [0, 1)) and the ratios to its two neighbours,
// exp(beta (2 delta - 1)) towards o = 1 and exp(-beta (2 delta + 1)) towards
// o = -1; each further ratio is the previous one times exp(-2 beta).  The
// fractional offset delta comes from the FP64 coordinate.  For complex64 the
// exponentials are single-precision 2^x; the gather runs the recurrence in
// FP32 (relative weight error below 5e-7), the spread in FP64 on its products
// with the sample (it accumulates in FP64 anyway).  For complex128 everything
// is FP64.
template <typename T>
struct Fgg;
template <>
struct Fgg<float> {
  float b;    // beta log2(e)
  double q;   // exp(-2 beta)
  float e2m, e4m, e4p;   // exp(-2 beta), exp(-4 beta), exp(4 beta)
  __device__ explicit Fgg(double beta)
      : b((float)(beta * 1.4426950408889634074)), q(exp(-2.0 * beta)), e2m((float)exp(-2.0 * beta)),
        e4m((float)exp(-4.0 * beta)), e4p((float)exp(4.0 * beta)) {}
  __device__ __forceinline__ void seeds(float d, float& wc, float& up, float& dn) const {
    wc = __builtin_amdgcn_exp2f(-b * d * d);
    up = __builtin_amdgcn_exp2f(b * (2.f * d - 1.f));
    dn = __builtin_amdgcn_exp2f(-b * (2.f * d + 1.f));
  }
  // one weight exp(-beta a^2), evaluated directly
  __device__ __forceinline__ float one(float a) const { return __builtin_amdgcn_exp2f(-b * a * a); }
  // exp(-beta d^2), exp(-beta (2d + 1)), exp(4 beta (d - 1))
  __device__ __forceinline__ void three(float d, float& w, float& dn, float& up2) const {
    w = __builtin_amdgcn_exp2f(-b * d * d);
    dn = __builtin_amdgcn_exp2f(-b * (2.f * d + 1.f));
    up2 = __builtin_amdgcn_exp2f(4.f * b * (d - 1.f));
  }
};
template <>
struct Fgg<double> {
  double beta, q;
  double e2m, e4m, e4p;
  __device__ explicit Fgg(double beta_)
      : beta(beta_), q(exp(-2.0 * beta_)), e2m(exp(-2.0 * beta_)), e4m(exp(-4.0 * beta_)), e4p(exp(4.0 * beta_)) {}
  __device__ __forceinline__ void seeds(double d, double& wc, double& up, double& dn) const {
    wc = exp(-beta * d * d);
    up = exp(beta * (2.0 * d - 1.0));
    dn = exp(-beta * (2.0 * d + 1.0));
  }
  __device__ __forceinline__ double one(double a) const { return exp(-beta * a * a); }
  __device__ __forceinline__ void three(double d, double& w, double& dn, double& up2) const {
    w = exp(-beta * d * d);
    dn = exp(-beta * (2.0 * d + 1.0));
    up2 = exp(4.0 * beta * (d - 1.0));
  }
};

// Value of lane U of the lane's quad (DPP quad_perm broadcast).
template <int U>
__device__ __forceinline__ int quad_bcast(int v) {
  return __builtin_amdgcn_update_dpp(0, v, U * 0x55, 0xf, 0xf, false);
}
template <int U>
__device__ __forceinline__ float quad_bcast(float v) { return __int_as_float(quad_bcast<U>(__float_as_int(v))); }
template <int U>
__device__ __forceinline__ double quad_bcast(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = quad_bcast<U>((int)(b & 0xffffffff)), hi = quad_bcast<U>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Half-row exchange through DPP (row rotate by 8 within each row of 16 lanes, no LDS traffic):
// from_half<H>(own, send) gives lanes of half H their own value and lanes of the other half the
// value `send` of the lane 8 places away (bank mask: only the other half's two banks are written).
template <int H>
__device__ __forceinline__ int from_half(int own, int send) {
  return __builtin_amdgcn_update_dpp(own, send, 0x128, 0xf, H == 0 ? 0xc : 0x3, false);
}
template <int H>
__device__ __forceinline__ float from_half(float own, float send) {
  return __int_as_float(from_half<H>(__float_as_int(own), __float_as_int(send)));
}
template <int H>
__device__ __forceinline__ double from_half(double own, double send) {
  const long long o = __double_as_longlong(own), s = __double_as_longlong(send);
  const int lo = from_half<H>((int)(o & 0xffffffff), (int)(s & 0xffffffff));
  const int hi = from_half<H>((int)(o >> 32), (int)(s >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// All 2m weights of one axis; w[i] belongs to grid point floor(s) - m + 1 + i.
template <typename T, int MH>
__device__ __forceinline__ void fgg_taps(const Fgg<T>& g, T d, T* w) {
  T wc, up, dn;
  g.seeds(d, wc, up, dn);
  const T q = (T)g.q;
  w[MH - 1] = wc;
  T x = wc;
#pragma unroll
  for (int i = MH; i < 2 * MH; ++i) {
    x *= up;
    w[i] = x;
    up *= q;
  }
  x = wc;
#pragma unroll
  for (int i = MH - 2; i >= 0; --i) {
    x *= dn;
    w[i] = x;
    dn *= q;
  }
}

// Position v (-2M <= v < 2M) relative to a tile origin, folded by the grid period M into
// [-16, M - 16): with TS + 16 <= M and at most 16 taps, a stencil point lies in
// the tile exactly when its folded position is in [0, TS).  P2: M is a power of two.
template <bool P2>
__device__ __forceinline__ int fold_rel(int v, int M) {
  const int r = wrap2<P2>(v, M);
  return r >= M - 16 ? r - M : r;
}

// ---------------------------------------------------------------------------
// F_u2D gather over one tile of the oversampled grid
// ---------------------------------------------------------------------------
// P2: M1 and M2 are powers of two (index masks); otherwise either may be 3 2^k (compares).  Target
// coordinates satisfy |s| < 0.71 M (|k_u|, |k_v| <= 1/2 of the detector, sin(phi) < 1), so a base
// relative to a tile origin lies in (-2M, M).
template <typename T, int MH, bool P2>
__global__ __launch_bounds__(256) void k_gather(const cpx<T>* __restrict__ Gb, cpx<T>* out, const cpx<T>* dhat, int k0,
                                                Dims D, Tables<T> tb, int log2TS) {
  constexpr int W = 2 * MH;
  const int TS = 1 << log2TS, P = TS + W - 1;
  const int M1 = D.M1, M2 = D.M2;
  const int ntx = M2 >> log2TS, nty = M1 >> log2TS;
  const int tid = threadIdx.x, nth = blockDim.x;
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(lam_smem);
  // blocks run rank-major over the slab's slices: the heaviest tile of every slice first
  const int ns = gridDim.x / (ntx * nty), rank = blockIdx.x / ns, kk = blockIdx.x - rank * ns, k = k0 + kk;
  if (D.skip.skip(kk)) return;
  const int tix = tb.gperm[(size_t)k * ntx * nty + rank];
  const int tx = tix % ntx, ty = tix / ntx;
  const int x0 = tx * TS, y0 = ty * TS;
  const cpx<T>* G = Gb + (size_t)kk * M1 * M2;
  const Fgg<T> fg(D.beta);
  // e / P by multiplication: exact for e < 2^16 with P < 2^8
  const unsigned magicP = 0xffffffffu / (unsigned)P + 1u;
  for (int e0 = 0; e0 < P * P; e0 += vpt<T>() * nth) {
    cpx<T> v[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = min(e0 + tid + it * nth, P * P - 1);
      const int r = (int)(((unsigned long long)(unsigned)e * magicP) >> 32), c = e - r * P;
      v[it] = G[(size_t)wrap1<P2>(y0 - MH + 1 + r, M1) * M2 + wrap1<P2>(x0 - MH + 1 + c, M2)];
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
  // one lane per target; consecutive lanes take neighbouring targets of a run along a line, and each
  // lane takes UG targets per step whose loads are in flight together (complex128 keeps two: four
  // would take it past 128 registers)
  constexpr int UG = sizeof(T) == 4 ? 4 : 2;
  for (int i0 = beg + tid; i0 < end; i0 += UG * nth) {
    int t[UG], uk[UG];
    double c[UG], sn[UG];
    cpx<T> dd[UG];
#pragma unroll
    for (int u = 0; u < UG; ++u) {
      const int pe = L[min(i0 + u * nth, end - 1)];
      t[u] = pe >> 12;
      uk[u] = pe & 4095;
    }
#pragma unroll
    for (int u = 0; u < UG; ++u) {
      c[u] = tb.cth[t[u]];
      sn[u] = tb.sth[t[u]];
      dd[u] = dhat ? dhat[((size_t)t[u] * D.h + k) * D.w + uk[u]] : mk((T)0, (T)0);
    }
#pragma unroll
    for (int u = 0; u < UG; ++u) {
      double sx, sy;
      target_coords(D.xy, c[u], sn[u], k, uk[u], sx, sy);
      const double fy = floor(sy), fx = floor(sx);
      const int by = (int)fy, bx = (int)fx;
      T wx[W], wy[W];
      fgg_taps<T, MH>(fg, (T)(sx - fx), wx);
      fgg_taps<T, MH>(fg, (T)(sy - fy), wy);
      const int ox = wrap2<P2>(bx - x0, M2), oy = wrap2<P2>(by - y0, M1);
      T ax = 0, ay = 0;
#pragma unroll
      for (int iy = 0; iy < W; ++iy) {
        const cpx<T>* row = tile + (oy + iy) * P + ox;
        T rx = 0, ry = 0;
#pragma unroll
        for (int ix = 0; ix < W; ++ix) {
          const cpx<T> v = row[ix];
          rx += wx[ix] * v.x;
          ry += wx[ix] * v.y;
        }
        ax += wy[iy] * rx;
        ay += wy[iy] * ry;
      }
      if (i0 + u * nth < end) out[((size_t)t[u] * D.h + k) * D.w + uk[u]] = mk(ax - dd[u].x, ay - dd[u].y);
    }
  }
}

// ---------------------------------------------------------------------------
// F*_u2D spread into one tile of the oversampled grid in FP64 (complex128; complex64 on grids
// below 128 x 128 or for m > 4).  Each lane adds its column's 2m taps, one stencil row per FP64
// LDS atomic (native ds_add_f64; gfx950 runs FP64 LDS atomics ~20x faster than FP32 ones); a
// wave's 64 adds cover NG targets' rows, GW adjacent cells each.
//
// LTS > 0 (with PAIRS, m = 4) fixes the tile size 2^LTS at compile time and requires M1, M2 >=
// 2^LTS + 16: stencil rows and columns are then folded positions relative to the tile, so a row's
// cell is the row base plus a constant (immediate LDS offsets) and the test for the tile is one
// compare.
//
// PAIRS changes how the adds are laid out.  An atomic
// instruction whose 8-lane groups each add one row of a different target hits the banks at
// random (~16 cycles per 64-lane FP64 add); one whose 16-lane rows each add two adjacent
// rows of one target covers every bank equally (PA = 8 (mod 32) doubles puts the second row
// 16 banks on) and runs at the minimum (~9 cycles).  So the two 8-lane groups of a 16-lane
// row evaluate their own targets as before, trade what the other needs through DPP, and then
// add both targets in turn: lane (h, j) adds column j of the rows of parity h.
// ---------------------------------------------------------------------------
template <typename T, int MH, bool P2, int LTS = 0, bool PAIRS = false>
__global__ __launch_bounds__(512) void k_scatter(const cpx<T>* __restrict__ in, cpx<T>* __restrict__ Gb, int k0,
                                                 Dims D, Tables<T> tb, int log2TS_) {
  constexpr int W = 2 * MH, GW = group_width<MH>(), NG = 64 / GW;
  static_assert(LTS == 0 || W <= 16, "folded positions assume at most 16 taps");
  static_assert(PAIRS == (LTS > 0) && (!PAIRS || MH == 4), "the folded path is the row-pair path, m = 4");
  const int log2TS = LTS > 0 ? LTS : log2TS_;
  const int TS = 1 << log2TS, PA = TS + 8;   // PA = 8 (mod 32): stencil rows of a target fall in distinct banks
  const int M1 = D.M1, M2 = D.M2;
  const int ntx = M2 >> log2TS, nty = M1 >> log2TS;
  const int tid = threadIdx.x, nth = blockDim.x;
  double* are = reinterpret_cast<double*>(lam_smem);           // [TS][PA]
  double* aim = are + TS * PA;                                  // [TS][PA]
  // blocks run rank-major over the slab's slices: the heaviest tile of every slice first
  const int ns = gridDim.x / (ntx * nty), rank = blockIdx.x / ns, kk = blockIdx.x - rank * ns, k = k0 + kk;
  if (D.skip.skip(kk)) return;
  const int tix = tb.sperm[(size_t)k * ntx * nty + rank];
  const int tx = tix % ntx, ty = tix / ntx;
  const int x0 = tx * TS, y0 = ty * TS;
  for (int e = tid; e < 2 * TS * PA; e += nth) are[e] = 0.0;
  // the tile's list ranges (uniform over the block): fixed slots and their prefix counts
  int rb[kSpreadSlots], re[kSpreadSlots], pre[kSpreadSlots + 1];
  spread_ranges(tb.toff + (size_t)k * ((size_t)ntx * nty * 9 + 1), ntx, nty, ty, tx, rb, re);
  pre[0] = 0;
#pragma unroll
  for (int q = 0; q < kSpreadSlots; ++q) pre[q + 1] = pre[q] + (re[q] - rb[q]);
  const int total = pre[kSpreadSlots];
  const int* L = tb.tlist + (size_t)k * D.ntheta * D.w;
  const int lane = tid & 63, wave = tid >> 6, nwave = nth >> 6;
  const int g = lane / GW, j = lane & (GW - 1);
  __syncthreads();
  // Add the targets of list positions [0, n) (position -> list index by idx_of): the NG * U
  // targets of a wave step come from NG * U far-apart stretches of the positions (the lists hold
  // runs of neighbouring targets, whose stencils overlap, and adds to one cell within an
  // instruction serialise); the U targets of a lane group are independent load chains.
  constexpr int U = 4;
  const unsigned hw = (unsigned)D.h * D.w;   // < 2^24: a 32 x 32 -> 64-bit product per sample
  const int kw = k * D.w;
  const Fgg<T> fg(D.beta);
  const double qd = fg.q;
  auto spread = [&](int n, auto idx_of) {
    const int stretch = (n + NG * U - 1) / (NG * U);
    for (int i0 = wave; i0 < stretch; i0 += nwave) {
      if constexpr (PAIRS) {
        // Lane (g, j) evaluates target j & 3 of its group's four (coordinates, bases, offsets,
        // sample); each quad then broadcasts them, so every lane of the group has all four.
        static_assert(U == 4, "one target per lane of a quad");
        const int is = ((j & 3) * NG + g) * stretch + i0;
        const bool oks = is < n;
        const int pe = oks ? L[idx_of(is)] : 0;
        const unsigned ts = (unsigned)pe >> 12;
        const int uks = pe & 4095;
        const cpx<T> vs = in[(size_t)ts * hw + (unsigned)(kw + uks)];
        double sx, sy;
        target_coords(D.xy, tb.cth[ts], tb.sth[ts], k, uks, sx, sy);
        const double fy = floor(sy), fx = floor(sx);
        const int c0s = oks ? fold_rel<P2>((int)fx - MH + 1 - x0, M2) : TS;   // TS: no target
        const int r0s = fold_rel<P2>((int)fy - MH + 1 - y0, M1);
        const T dxs = (T)(sx - fx);
        // row weights by parity, from d = delta_y: odd rows start at the centre row m - 1
        // (offset d), even rows at row m - 2 (offset d + 1); two-row ratios up and down.  The
        // group's lanes all have parity h = g & 1: keep parity h, the other half needs 1 - h.
        const int h = g & 1;
        T w1, dn1, up1;
        fg.three((T)(sy - fy), w1, dn1, up1);
        const T dn1r = dn1 * dn1 * (T)fg.e2m;   // exp(-4 beta (d + 1))
        const T w0 = w1 * dn1, up0 = up1 * (T)fg.e4p, dn0r = dn1r * (T)fg.e4m;
        const T wshs = h ? w1 : w0, uphs = h ? up1 : up0, dnhs = h ? dn1r : dn0r;
        const T wsxs = h ? w0 : w1, upxs = h ? up0 : up1, dnxs = h ? dn0r : dn1r;
        auto target = [&](auto UC) {
          constexpr int u = decltype(UC)::value;
          const int col = quad_bcast<u>(c0s) + j, r0 = quad_bcast<u>(r0s);
          const T dx = quad_bcast<u>(dxs);
          const T vx = quad_bcast<u>(vs.x), vy = quad_bcast<u>(vs.y);
          const T ws_h = quad_bcast<u>(wshs), up_h = quad_bcast<u>(uphs), dn_h = quad_bcast<u>(dnhs);
          const T ws_x = quad_bcast<u>(wsxs), up_x = quad_bcast<u>(upxs), dn_x = quad_bcast<u>(dnxs);
          // this lane's target (valid or not, every lane takes part in the DPP exchange)
          const bool valid = (unsigned)col < (unsigned)TS;
          const T wxj = fg.one(dx - (T)(j + 1 - MH));
          const T pvx = wxj * vx, pvy = wxj * vy;
          const int col_o = valid ? col : TS;
          // target of the row's first half, then of its second half
          auto phase = [&](auto H) {
            constexpr int ph = decltype(H)::value;
            const int cc = from_half<ph>(col_o, col_o), rs = from_half<ph>(r0, r0) + MH - 2 + h;
            const T ax = from_half<ph>(pvx, pvx), ay = from_half<ph>(pvy, pvy);
            const T ws = from_half<ph>(ws_h, ws_x), up = from_half<ph>(up_h, up_x), dn = from_half<ph>(dn_h, dn_x);
            if ((unsigned)cc < (unsigned)TS) {
              const int as = rs * PA + cc;
              auto add = [&](int k2, double x, double y) {   // row rs + k2 (same parity)
                if ((unsigned)(rs + k2) >= (unsigned)TS) return;
                atomicAdd(are + as + k2 * PA, x);
                atomicAdd(aim + as + k2 * PA, y);
              };
              const double cx = (double)ax * (double)ws, cy = (double)ay * (double)ws;
              add(0, cx, cy);
              const double ru = (double)up, px = cx * ru, py = cy * ru;
              add(2, px, py);
              const double ru2 = ru * (double)fg.e4m * (double)fg.e4m;   // next two-row ratio up
              add(4, px * ru2, py * ru2);
              add(-2, cx * (double)dn, cy * (double)dn);
            }
          };
          phase(std::integral_constant<int, 0>());
          phase(std::integral_constant<int, 1>());
        };
        target(std::integral_constant<int, 0>());
        target(std::integral_constant<int, 1>());
        target(std::integral_constant<int, 2>());
        target(std::integral_constant<int, 3>());
      } else {
        int t[U], uk[U];
        bool ok[U];
        double c[U], sn[U];
        cpx<T> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = (u * NG + g) * stretch + i0;
          ok[u] = i < n;
          const int pe = ok[u] ? L[idx_of(i)] : 0;
          t[u] = (int)((unsigned)pe >> 12);
          uk[u] = pe & 4095;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          c[u] = tb.cth[t[u]];
          sn[u] = tb.sth[t[u]];
          v[u] = in[(size_t)(unsigned)t[u] * hw + (unsigned)(kw + uk[u])];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          double sx, sy;
          target_coords(D.xy, c[u], sn[u], k, uk[u], sx, sy);
          const double fy = floor(sy), fx = floor(sx);
          const int by = (int)fy, bx = (int)fx;
          const int col = wrap2<P2>(bx - MH + 1 + j - x0, M2), r0 = by - MH + 1 - y0;
          if (ok[u] && j < W && (unsigned)col < (unsigned)TS) {
            const T wxj = fg.one((T)(sx - fx) - (T)(j + 1 - MH));
            T wc, up, dn;
            fg.seeds((T)(sy - fy), wc, up, dn);
            auto add = [&](int iy, double x, double y) {
              const int row = wrap2<P2>(r0 + iy, M1);
              if (row >= TS) return;
              const int a = __umul24(row, PA) + col;
              atomicAdd(are + a, x);
              atomicAdd(aim + a, y);
            };
            // the column's products with the row weights, by the weight recurrence in FP64 from the
            // centre row outwards
            const double cx = (double)(wxj * v[u].x) * (double)wc, cy = (double)(wxj * v[u].y) * (double)wc;
            add(MH - 1, cx, cy);
            double px = cx, py = cy, r = (double)up;
#pragma unroll
            for (int iy = MH; iy < W; ++iy) {
              px *= r;
              py *= r;
              add(iy, px, py);
              r *= qd;
            }
            px = cx;
            py = cy;
            r = (double)dn;
#pragma unroll
            for (int iy = MH - 2; iy >= 0; --iy) {
              px *= r;
              py *= r;
              add(iy, px, py);
              r *= qd;
            }
          }
        }
      }
    }
  };
  // the tile's own list, then the neighbours' border classes (the last slot starting at or before
  // position i holds it; empty slots share their successor's start)
  spread(pre[1], [&](int i) { return rb[0] + i; });
  spread(total - pre[1], [&](int i0) {
    const int i = i0 + pre[1];
    int idx = rb[1] + i0;
#pragma unroll
    for (int q = 2; q < kSpreadSlots; ++q)
      if (i >= pre[q]) idx = rb[q] + (i - pre[q]);
    return idx;
  });
  __syncthreads();
  cpx<T>* G = Gb + (size_t)kk * M1 * M2;
  for (int e = tid; e < TS * TS; e += nth) {
    const int r = e >> log2TS, c = e & (TS - 1);
    G[(size_t)(y0 + r) * M2 + x0 + c] = mk((T)are[r * PA + c], (T)aim[r * PA + c]);
  }
}

// ---------------------------------------------------------------------------
// F*_u2D spread of complex64 samples into one 64 x 64 tile (grids of at least 128 x 128, m <= 4)
// in 64-bit fixed point.  Each cell accumulates re * 2^32 + im as one 64-bit integer, re and im
// being the tap's contribution scaled by the tile's power-of-two scale S and rounded to 32-bit
// integers: one integer LDS atomic (ds_add_u64) per tap instead of two FP64 ones, and integer sums
// do not depend on the order of the adds, so the spread is bit-reproducible.  The low word of a sum
// is exactly the sum of the im parts, the high word the sum of the re parts less one where the im
// sum is negative, as long as both sums stay inside 32 bits; S keeps them below 2^30:
//   pass 1  every target adds max(|re|, |im|) of its sample to the 8 x 8 block of the tile that
//           holds its stencil base (clamped to the tile's edge blocks); a target's stencil reaches
//           only the blocks next to its base block, and |weight| <= 1, so the 3 x 3 sum around a
//           block bounds |re| and |im| of every cell of that block; S = 2^(30 - e) with 2^e above
//           the largest such bound;
//   pass 2  8 lanes per target, lane j adding stencil column j for all 2m rows (each target's
//           coordinates evaluated by one lane of a quad and broadcast).  The accumulator
//           carries a guard band of 2m - 1 cells on every side, so taps that leave the tile land in
//           the guard (the neighbouring tile adds them) and no tap needs a bounds test.
// A tile whose bound is not finite (NaN or Inf samples) is written as NaN.
// ---------------------------------------------------------------------------
// Value of lane U of the lane's quad (DPP quad_perm; every lane is written, so no old value).
template <int U>
__device__ __forceinline__ int quad_copy(int v) { return __builtin_amdgcn_mov_dpp(v, U * 0x55, 0xf, 0xf, false); }
template <int U>
__device__ __forceinline__ float quad_copy(float v) { return __int_as_float(quad_copy<U>(__float_as_int(v))); }

// floor(a b + 1/2) as an integer: one FMA and one floor conversion (v_cvt_flr_i32_f32, which the
// compiler does not form from floorf), i.e. a b rounded to the nearest integer.  Truncation would
// bias every tap towards zero, and the bias of coherent taps adds up.
__device__ __forceinline__ int round_to_int(float a, float b) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(__builtin_fmaf(a, b, 0.5f)));
  return r;
}

template <int MH>
constexpr int fx_pitch() { return 64 + 2 * (2 * MH - 1); }
template <int MH>
constexpr size_t fx_lds() { return (size_t)fx_pitch<MH>() * fx_pitch<MH>() * 8 + 64 * 8 + 16; }

template <int MH, bool P2>
__global__ __launch_bounds__(512) void k_scatter_fx(const cpx<float>* __restrict__ in, cpx<float>* __restrict__ Gb,
                                                    int k0, Dims D, Tables<float> tb) {
  constexpr int W = 2 * MH, GD = W - 1, PT = fx_pitch<MH>(), TS = 64, LTS = 6, GW = 8, NG = 64 / GW;
  static_assert(W <= GW, "one lane per stencil column");
  const int M1 = D.M1, M2 = D.M2;
  const int ntx = M2 >> LTS, nty = M1 >> LTS;
  const int tid = threadIdx.x, nth = blockDim.x;
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(lam_smem);   // [PT][PT], cell (r, c) at (r + GD) PT + c + GD
  double* blk = reinterpret_cast<double*>(acc + PT * PT);                       // [8][8] block sums
  float* scal = reinterpret_cast<float*>(blk + 64);                             // S, 1 / S, finite flag
  // blocks run rank-major over the slab's slices: the heaviest tile of every slice first
  const int ns = gridDim.x / (ntx * nty), rank = blockIdx.x / ns, kk = blockIdx.x - rank * ns, k = k0 + kk;
  if (D.skip.skip(kk)) return;
  const int tix = tb.sperm[(size_t)k * ntx * nty + rank];
  const int tx = tix % ntx, ty = tix / ntx;
  const int x0 = tx * TS, y0 = ty * TS;
  for (int e = tid; e < PT * PT; e += nth) acc[e] = 0ull;
  for (int e = tid; e < 64; e += nth) blk[e] = 0.0;
  int rb[kSpreadSlots], re[kSpreadSlots], pre[kSpreadSlots + 1];
  spread_ranges(tb.toff + (size_t)k * ((size_t)ntx * nty * 9 + 1), ntx, nty, ty, tx, rb, re);
  pre[0] = 0;
#pragma unroll
  for (int q = 0; q < kSpreadSlots; ++q) pre[q + 1] = pre[q] + (re[q] - rb[q]);
  const int total = pre[kSpreadSlots];
  // list index of position i of the tile's ranges (the last slot starting at or before i holds it)
  auto idx_of = [&](int i) {
    int idx = rb[0] + i;
#pragma unroll
    for (int q = 1; q < kSpreadSlots; ++q)
      if (i >= pre[q]) idx = rb[q] + (i - pre[q]);
    return idx;
  };
  const int* L = tb.tlist + (size_t)k * D.ntheta * D.w;
  const unsigned hw = (unsigned)D.h * D.w;   // < 2^24
  const int kw = k * D.w;
  __syncthreads();
  // pass 1: block sums of max(|re|, |im|) at the stencil bases.  A target's block in this tile is its
  // block in its own tile (the plan's byte), or for a neighbour's border class the facing edge block:
  // slots 1-3 / 4-6 the left / right neighbour (bx 0 / 7), 7 / 8 the upper / lower one (by 0 / 7),
  // 9-12 the corners.
  const unsigned char* SB = tb.sblk + (size_t)k * D.ntheta * D.w;
  for (int i = tid; i < total; i += nth) {
    int q = 0, idx = rb[0] + i;
#pragma unroll
    for (int s = 1; s < kSpreadSlots; ++s)
      if (i >= pre[s]) { q = s; idx = rb[s] + (i - pre[s]); }
    const int pe = L[idx];
    const unsigned b = SB[idx];
    const cpx<float> v = in[(size_t)((unsigned)pe >> 12) * hw + (unsigned)(kw + (pe & 4095))];
    const int bx = (q == 0 || q == 7 || q == 8) ? (int)(b & 7u) : ((q >= 4 && q <= 6) || q == 10 || q == 12 ? 7 : 0);
    const int by = q <= 6 ? (int)(b >> 3) : (q == 8 || q == 11 || q == 12 ? 7 : 0);
    atomicAdd(blk + by * 8 + bx, (double)fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  __syncthreads();
  if (tid < 64) {
    const int bx = tid & 7, by = tid >> 3;
    double b = 0.0;
    for (int yy = max(by - 1, 0); yy <= min(by + 1, 7); ++yy)
      for (int xx = max(bx - 1, 0); xx <= min(bx + 1, 7); ++xx) b += blk[yy * 8 + xx];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) b = fmax(b, __shfl_xor(b, o));
    if (tid == 0) {
      int e = 0;
      if (b > 0.0 && b <= 1e300) (void)frexp(b, &e);   // b < 2^e
      const int sh = min(max(30 - e, -126), 126);
      scal[0] = ldexpf(1.0f, sh);
      scal[1] = ldexpf(1.0f, -sh);
      scal[2] = (b <= 1e300) ? 1.0f : 0.0f;   // NaN fails the test too
    }
  }
  __syncthreads();
  const float S = scal[0];
  // pass 2: the taps, over the tile's own list and then the neighbours' border classes.  A lane
  // group of 8 takes U = 4 targets per wave step; lane j of the group evaluates target j & 3
  // (FP64 coordinates, cell address, row weights, scaled sample; the group's two quads evaluate
  // the same four), and a quad broadcast (DPP) hands each target's values to every lane in turn.
  // The NG targets of one instruction come from NG far-apart stretches of the positions: the lists
  // hold runs of neighbouring targets, whose stencils overlap, and adds to one cell within an
  // instruction serialise.
  constexpr int U = 4;
  const int lane = tid & 63, wave = tid >> 6, nwave = nth >> 6;
  const int g = lane / GW, j = lane & (GW - 1), js = j & 3;
  const Fgg<float> fg(D.beta);
  auto spread = [&](int n, auto list_idx) {
    const int stretch = (n + NG * U - 1) / (NG * U);
    for (int i0 = wave; i0 < stretch; i0 += nwave) {
      // this lane's target: the group's js-th
      const int is = (js * NG + g) * stretch + i0;
      const bool oks = is < n;
      const int pe = oks ? L[list_idx(is)] : 0;
      const unsigned ts = (unsigned)pe >> 12;
      const int uks = pe & 4095;
      const cpx<float> vs = in[(size_t)ts * hw + (unsigned)(kw + uks)];
      double sx, sy;
      target_coords(D.xy, tb.cth[ts], tb.sth[ts], k, uks, sx, sy);
      const double fy = floor(sy), fx = floor(sx);
      // address of the stencil's first cell, -1: no target
      const int as = oks ? __umul24(fold_rel<P2>((int)fy - MH + 1 - y0, M1) + GD, PT) +
                               fold_rel<P2>((int)fx - MH + 1 - x0, M2) + GD
                         : -1;
      const float dxs = (float)(sx - fx);
      float wys[W];
      fgg_taps<float, MH>(fg, (float)(sy - fy), wys);
      const float vxs = vs.x * S, vys = vs.y * S;
      auto target = [&](auto UC) {
        constexpr int u = decltype(UC)::value;
        const int a0 = quad_copy<u>(as);
        const float dx = quad_copy<u>(dxs), vx = quad_copy<u>(vxs), vy = quad_copy<u>(vys);
        float wy[W];
#pragma unroll
        for (int i = 0; i < W; ++i) wy[i] = quad_copy<u>(wys[i]);
        if (a0 < 0 || j >= W) return;
        const float wxj = fg.one(dx - (float)(j + 1 - MH));
        const float pvx = wxj * vx, pvy = wxj * vy;
        unsigned long long* a = acc + a0 + j;
#pragma unroll
        for (int iy = 0; iy < W; ++iy) {
          const int xi = round_to_int(pvx, wy[iy]), yi = round_to_int(pvy, wy[iy]);
          const unsigned long long pk = ((unsigned long long)(unsigned)(xi + (yi >> 31)) << 32) | (unsigned)yi;
          atomicAdd(a + iy * PT, pk);
        }
      };
      target(std::integral_constant<int, 0>());
      target(std::integral_constant<int, 1>());
      target(std::integral_constant<int, 2>());
      target(std::integral_constant<int, 3>());
    }
  };
  spread(pre[1], [&](int i) { return rb[0] + i; });
  spread(total - pre[1], [&](int i) { return idx_of(i + pre[1]); });
  __syncthreads();
  const float iS = scal[1];
  const bool finite = scal[2] != 0.0f;
  cpx<float>* G = Gb + (size_t)kk * M1 * M2;
  for (int e = tid; e < TS * TS; e += nth) {
    const int r = e >> LTS, cc = e & (TS - 1);
    const unsigned long long X = acc[(r + GD) * PT + cc + GD];
    const int im = (int)(unsigned)X, rl = (int)(unsigned)(X >> 32) - (im >> 31);
    G[(size_t)(y0 + r) * M2 + x0 + cc] =
        finite ? mk((float)rl * iS, (float)im * iS) : mk(__builtin_nanf(""), __builtin_nanf(""));
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
namespace {
// 64 x 64 tiles on a grid of at least 128 x 128: the compile-time tile kernels apply
bool fast_tiles(const LaunchCfg& c, const Dims& D) { return c.g_log2TS == 6 && D.M1 >= 128 && D.M2 >= 128; }
// both grid periods are powers of two: the tile kernels index with masks
bool pow2_grid(const Dims& D) { return (D.M1 & (D.M1 - 1)) == 0 && (D.M2 & (D.M2 - 1)) == 0; }

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
  const int ntx = D.M2 >> c.g_log2TS, nty = D.M1 >> c.g_log2TS;
  LAM_MH_SWITCH(D.m, {
    hipLaunchKernelGGL((k_list_count<T, MH>), dim3(nty, ns), dim3(256), ntx * 9 * sizeof(int), s, D, tb, c.g_log2TS,
                       k0, counts);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_list_fill(const LaunchCfg& c, int k0, int ns, const Dims& D, const Tables<T>& tb, const int* offs,
                            int* lists, hipStream_t s) {
  const int ntx = D.M2 >> c.g_log2TS, nty = D.M1 >> c.g_log2TS;
  LAM_MH_SWITCH(D.m, {
    hipLaunchKernelGGL((k_list_fill<T, MH>), dim3(nty, ns), dim3(256), ntx * 9 * sizeof(int), s, D, tb, c.g_log2TS,
                       k0, offs, lists);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_list_blocks(const LaunchCfg& c, int k0, int ns, const Dims& D, const Tables<T>& tb,
                              unsigned char* sblk, hipStream_t s) {
  const int ntx = D.M2 >> c.g_log2TS, nty = D.M1 >> c.g_log2TS;
  LAM_MH_SWITCH(D.m, {
    hipLaunchKernelGGL((k_list_blocks<T, MH>), dim3(ntx * nty, ns), dim3(256), 0, s, D, tb, c.g_log2TS, k0, sblk);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_list_check(const LaunchCfg& c, int k0, int ns, const Dims& D, const Tables<T>& tb, unsigned* seen,
                             int* bad, hipStream_t s) {
  const int ntx = D.M2 >> c.g_log2TS, nty = D.M1 >> c.g_log2TS;
  LAM_MH_SWITCH(D.m, {
    hipLaunchKernelGGL((k_list_check<T, MH>), dim3(ntx * nty, ns), dim3(256), 0, s, D, tb, c.g_log2TS, k0, seen,
                       bad);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const LaunchCfg& c, const cpx<T>* Gb, cpx<T>* out, const cpx<T>* dhat, int k0, int ns,
                         const Dims& D, const Tables<T>& tb, hipStream_t s) {
  hipError_t e = hipSuccess;
  LAM_MH_SWITCH(D.m, {
    auto k = pow2_grid(D) ? k_gather<T, MH, true> : k_gather<T, MH, false>;
    if ((e = prep(k, c.g_lds)) != hipSuccess) return e;
    const int ntiles = (D.M2 >> c.g_log2TS) * (D.M1 >> c.g_log2TS);
    hipLaunchKernelGGL(k, dim3(ntiles * ns), dim3(c.g_threads), c.g_lds, s, Gb, out, dhat, k0, D, tb, c.g_log2TS);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scatter(const LaunchCfg& c, const cpx<T>* in, cpx<T>* Gb, int k0, int ns, const Dims& D,
                          const Tables<T>& tb, hipStream_t s) {
  hipError_t e = hipSuccess;
  const int ntiles = (D.M2 >> c.g_log2TS) * (D.M1 >> c.g_log2TS);
  const bool p2 = pow2_grid(D);
  LAM_MH_SWITCH(D.m, {
    if constexpr (std::is_same<T, float>::value && MH <= 4) {
      if (fast_tiles(c, D) && tb.sblk) {   // complex64: fixed-point accumulation (needs the plan's block bytes)
        auto kf = p2 ? k_scatter_fx<MH, true> : k_scatter_fx<MH, false>;
        if ((e = prep(kf, fx_lds<MH>())) != hipSuccess) return e;
        hipLaunchKernelGGL(kf, dim3(ntiles * ns), dim3(512), fx_lds<MH>(), s, in, Gb, k0, D, tb);
        return hipGetLastError();
      }
    }
    auto k = p2 ? k_scatter<T, MH, true> : k_scatter<T, MH, false>;
    if constexpr (MH == 4)
      if (fast_tiles(c, D)) k = p2 ? k_scatter<T, MH, true, 6, true> : k_scatter<T, MH, false, 6, true>;
    if ((e = prep(k, c.s_lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(ntiles * ns), dim3(c.s_threads), c.s_lds, s, in, Gb, k0, D, tb, c.g_log2TS);
  });
  return hipGetLastError();
}

#define LAM_GRID_INST(T)                                                                                          \
  template hipError_t launch_list_count<T>(const LaunchCfg&, int, int, const Dims&, const Tables<T>&, int*,       \
                                           hipStream_t);                                                         \
  template hipError_t launch_list_fill<T>(const LaunchCfg&, int, int, const Dims&, const Tables<T>&, const int*,  \
                                          int*, hipStream_t);                                                    \
  template hipError_t launch_list_blocks<T>(const LaunchCfg&, int, int, const Dims&, const Tables<T>&,          \
                                           unsigned char*, hipStream_t);                                         \
  template hipError_t launch_list_check<T>(const LaunchCfg&, int, int, const Dims&, const Tables<T>&, unsigned*, \
                                          int*, hipStream_t);                                                    \
  template hipError_t launch_gather<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, const cpx<T>*, int, int,        \
                                       const Dims&, const Tables<T>&, hipStream_t);                              \
  template hipError_t launch_scatter<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, int, int, const Dims&,         \
                                        const Tables<T>&, hipStream_t);

LAM_GRID_INST(float)
LAM_GRID_INST(double)

}  // namespace lam
