// HIP kernels (gfx950) of the laminography operator L = F*_2D F_u2D F_u1D
// and its adjoint, and their host-side launchers.
//
// Stage map (forward; the adjoint runs the transposed stages in reverse):
//   k_zfwd      F_u1D: per (y, x-tile) column block: deconvolve by c_z, zero-pad
//               n0 -> M0 = R n0, FFT along z in LDS, gather the h targets
//               xi_z = n0 (k_v/h) cos(phi) with 2m Gaussian weights evaluated
//               from each row's tabulated base and offset.
//   k_ycol_fwd  F_u2D part 1: per k_v slice and x-tile: deconvolve by c_y c_x,
//               zero-pad n1 -> M1, FFT along y.
//   k_xrow_fwd  F_u2D part 2: zero-pad rows n2 -> M2, FFT along x: the
//               oversampled grid G of one slice.
//   (F_u2D part 3, the Gaussian gather, and its adjoint spread live in
//   lam_grid.hip)
//   k_rowfft / k_colfft   F*_2D (and the adjoint's F_2D): centred 2D DFT per
//               projection as a row pass and a column pass.
// Adjoint: k_xrow_adj, k_ycol_adj (inverse FFTs + crop + deconvolution), k_zadj.
#include "lam_internal.hpp"

namespace lam {

extern __shared__ __align__(16) unsigned char lam_smem[];


__device__ __forceinline__ int sgn_parity(int k) { return (k & 1) ? -1 : 1; }

// Block (bx, by) of a 2D grid of column blocks, in an XCD-aware order.  The dispatcher deals
// work-groups to the 8 XCDs round robin by linear id, and each XCD has its own L2; neighbouring
// x-tiles of a column kernel read neighbouring pieces of the same HBM lines (a tile row is TX
// values, 16 to 128 bytes).  So each XCD is given a contiguous run of the logical blocks: logical id
// (lin mod 8) (total / 8) + lin / 8 for linear id lin (the last total mod 8 keep theirs).
__device__ __forceinline__ void xcd_block(int& bx, int& by) {
  const int gx = gridDim.x, total = gx * gridDim.y, lin = blockIdx.x + blockIdx.y * gx;
  const int per = total >> 3;
  const int l = lin < per * 8 ? (lin & 7) * per + (lin >> 3) : lin;
  by = l / gx;
  bx = l - by * gx;
}

// 16 bytes of a z block's row of TX columns (two complex64 or one complex128 values): the z
// stencil kernels move a row as NCH = TX / CW such chunks (ds_read_b128 / global 16-byte stores).
template <typename T>
struct alignas(16) Chunk16 {
  static constexpr int CW = 16 / (int)sizeof(cpx<T>);
  cpx<T> c[CW];
};
template <typename T>
__device__ __forceinline__ void fma_chunk(Chunk16<T>& a, T w, const Chunk16<T>& g) {
#pragma unroll
  for (int e = 0; e < Chunk16<T>::CW; ++e) {
    a.c[e].x += w * g.c[e].x;
    a.c[e].y += w * g.c[e].y;
  }
}
// Chunk order of this lane: a thread handles whole rows (64 bytes for eight complex64 columns), so
// lanes reading chunk c of different rows at once would meet on the banks of that chunk's
// position; instead lane l starts at chunk s(l), with s sweeping 0 .. NCH - 1 over every 16 lanes,
// and lane l's c-th access is chunk (c + s(l)) mod NCH.
template <int NCH>
__device__ __forceinline__ int chunk_skew() {
  return (((int)(threadIdx.x & 15) * NCH) >> 4) & (NCH - 1);
}

// The FFT kernels take a template length code LN and LB (log2 of the transforms per block):
// LN = 0 selects the general kernel for power-of-two lengths (sizes from the arguments), LN = -1 the
// general kernel for lengths 3 2^l (the mixed-radix LDS FFT); otherwise the sizes are compile-time
// constants (the hot sizes): LN in 1..31 the length 2^LN, LN >= 32 the length 3 2^(LN - 32).
template <int LN> constexpr bool p2_len() { return LN >= 0 && LN < 32; }
template <int LN> constexpr int ct_l() { return LN >= 32 ? LN - 32 : LN; }
template <int LN> constexpr int ct_n() {   // 0 for the run-time codes
  if constexpr (LN >= 32) return 3 << (LN - 32);
  else if constexpr (LN > 0) return 1 << LN;
  else return 0;
}
template <typename T, int LN, int LB> constexpr int ct_threads() {
  if constexpr (LN >= 32) return fft3_threads<vpt<T>(), LN - 32, LB>();
  else return ((1 << (LN + LB)) / vpt<T>()) < 64 ? 64 : ((1 << (LN + LB)) / vpt<T>());
}
template <typename T, int LN, int LB> __device__ __forceinline__ int block_threads() {
  if constexpr (LN > 0) return ct_threads<T, LN, LB>();
  else return (int)blockDim.x;
}
// column blocks: element (p, b) at p 2^log2TX + b; the length is 2^lN, or 3 2^lN for LN = -1
template <typename T, int LN, int LB>
__device__ __forceinline__ void fft_cols(cpx<T>* buf, int lN, int log2TX, const Tables<T>& tb, int nth) {
  if constexpr (LN >= 32) lds_fft3_ct<T, vpt<T>(), false, LN - 32, LB, true>(buf, tb.tw3, tb.log2tw3);
  else if constexpr (LN > 0) lds_fft_ct<T, vpt<T>(), false, LN, LB, true>(buf, tb.tw, tb.log2tw);
  else if constexpr (LN < 0) lds_fft3<T, vpt<T>()>(buf, lN, log2TX, 1 << log2TX, 1, true, tb.tw3, tb.log2tw3, nth);
  else lds_fft<T, vpt<T>()>(buf, lN, log2TX, 1 << log2TX, 1, true, tb.tw, tb.log2tw, nth);
}
// Row kernels with one wave per row (or per few rows): compile-time power-of-two lengths whose rows
// fit a wave (N <= 64 VPT) and blocks of whole waves' rows.  The staging, the FFT stages and the store
// then touch only the wave's own rows, ordered by wave-level fences (no work-group barrier).
template <typename T, int LN, int LB> constexpr bool wave_rows() {
  if constexpr (LN > 0 && LN < 32) return (64 * vpt<T>() >= (1 << LN)) && ((1 << LB) * (1 << LN) >= 64 * vpt<T>());
  else return false;
}

// Column kernels with one wave per column (or per few columns): the same condition on the column
// length; the block's coalesced loads stage the columns into a column-major buffer (pitch
// wave_pitch<LN>(true)), one work-group barrier, the wave-ordered stages, one barrier, the stores.
template <typename T, int LN, int LB> constexpr bool wave_cols() { return wave_rows<T, LN, LB>(); }

// row blocks: element (p, b) at b N + p, one pad slot per 8 elements; N = 2^lN, or 3 2^lN for LN = -1
template <typename T, int LN, int LB>
__device__ __forceinline__ void fft_rows(cpx<T>* buf, int lN, int N, int log2RB, const Tables<T>& tb, int nth) {
  if constexpr (LN >= 32) lds_fft3_ct<T, vpt<T>(), true, LN - 32, LB, false>(buf, tb.tw3, tb.log2tw3);
  else if constexpr (LN > 0) lds_fft_ct<T, vpt<T>(), true, LN, LB, false>(buf, tb.tw, tb.log2tw);
  else if constexpr (LN < 0) lds_fft3<T, vpt<T>(), true>(buf, lN, log2RB, 1, N, false, tb.tw3, tb.log2tw3, nth);
  else lds_fft<T, vpt<T>(), true>(buf, lN, log2RB, 1, N, false, tb.tw, tb.log2tw, nth);
}

// ---------------------------------------------------------------------------
// F_u1D
// ---------------------------------------------------------------------------
template <typename T, int MH, bool REAL_IN, int LN = 0, int LB = 0>
__global__ __launch_bounds__(1024) void k_zfwd(const void* __restrict__ uin, cpx<T>* __restrict__ u1, Dims D,
                                               Tables<T> tb, int log2TX_, int y0, size_t in_zs) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  constexpr bool P2 = p2_len<LN>();
  const int log2TX = LN > 0 ? LB : log2TX_, lM0 = LN > 0 ? ct_l<LN>() : D.lM0;
  const int TX = 1 << log2TX, M0 = LN > 0 ? ct_n<LN>() : D.M0, n0 = LN > 0 ? M0 / 2 : D.n0;   // R = 2
  // block row yl is the row within the input slab; y the row of the volume
  int bx, yl;
  xcd_block(bx, yl);
  const int x0 = bx * TX, y = y0 + yl;
  if (D.skip.skip(y)) return;
  const int tid = threadIdx.x, nth = block_threads<T, LN, LB>();
  const size_t plane = (size_t)D.n1 * D.n2;
  const cpx<T> zero = mk((T)0, (T)0);
  // per-row stencil bases and offsets, after the buffer (its size is shared with the z adjoint)
  int* zb = reinterpret_cast<int*>(buf + (size_t)max(M0, D.h) * TX);
  T* zd = reinterpret_cast<T*>(zb + D.h);
  for (int e = tid; e < D.h; e += nth) {
    zb[e] = tb.zbase[e];
    zd[e] = tb.zdelta[e];
  }
  for (int e = tid; e < (M0 - n0) * TX; e += nth) buf[(n0 / 2) * TX + e] = zero;
  {
    // all global loads of this thread are issued before the first LDS store
    cpx<T> v[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      if (it * nth >= n0 * TX) break;   // the input fills n0 of the M0 rows
      const int e = min(tid + it * nth, n0 * TX - 1);    // clamped: every load is issued unconditionally
      const int a = e >> log2TX, b = e & (TX - 1);
      const size_t gi = (size_t)a * in_zs + (size_t)yl * D.n2 + x0 + b;
      if constexpr (REAL_IN) v[it] = mk(reinterpret_cast<const T*>(uin)[gi], (T)0);
      else v[it] = reinterpret_cast<const cpx<T>*>(uin)[gi];
    }
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      if (it * nth >= n0 * TX) break;
      const int e = tid + it * nth;
      if (e < n0 * TX) {
        const int a = e >> log2TX, b = e & (TX - 1);
        buf[wrap1<P2>(a - n0 / 2, M0) * TX + b] = v[it] * tb.cz[a];
      }
    }
  }
  __syncthreads();
  fft_cols<T, LN, LB>(buf, lM0, log2TX, tb, nth);
  const GaussW gw{D.beta};
  if constexpr (LN > 0) {
    if (D.h <= nth) {
      // one thread per detector row: its 2m weights once, then the TX columns of each stencil row
      // as 16-byte chunks; the rows go back through LDS (over the grid, after a barrier) so that the
      // stores are coalesced.  (With more rows than threads the loop below is faster: each thread's
      // rows would have to be stored straight from registers, one 16-byte piece per plane.)
      using C = Chunk16<T>;
      constexpr int NCH = (1 << LB) / C::CW;
      static_assert(NCH >= 1 && ((1 << LB) % C::CW) == 0, "whole chunks per block row");
      const int s = chunk_skew<NCH>();
      const int av = tid;
      C acc[NCH];
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int e = 0; e < C::CW; ++e) acc[c].c[e] = mk((T)0, (T)0);
      if (av < D.h) {
        const int base = zb[av] - MH + 1;
        const T dl = zd[av];
#pragma unroll
        for (int i = 0; i < 2 * MH; ++i) {
          const T w = gw(dl - (T)(i + 1 - MH), T());
          const C* row = reinterpret_cast<const C*>(buf + wrap1<P2>(base + i, M0) * (1 << LB));
#pragma unroll
          for (int c = 0; c < NCH; ++c) fma_chunk(acc[c], w, row[(c + s) & (NCH - 1)]);
        }
      }
      __syncthreads();
      if (av < D.h) {
        C* dst = reinterpret_cast<C*>(buf + av * (1 << LB));
#pragma unroll
        for (int c = 0; c < NCH; ++c) dst[(c + s) & (NCH - 1)] = acc[c];
      }
      __syncthreads();
      for (int e = tid; e < D.h * TX; e += nth) {
        const int a = e >> LB, b = e & (TX - 1);
        u1[(size_t)a * plane + (size_t)y * D.n2 + x0 + b] = buf[e];
      }
      return;
    }
  }
  for (int e = tid; e < D.h * TX; e += nth) {
    const int av = e >> log2TX, b = e & (TX - 1);
    const int base = zb[av] - MH + 1;
    const T dl = zd[av];
    T ax = 0, ay = 0;
#pragma unroll
    for (int i = 0; i < 2 * MH; ++i) {
      const T w = gw(dl - (T)(i + 1 - MH), T());
      const cpx<T> g = buf[wrap1<P2>(base + i, M0) * TX + b];
      ax += w * g.x;
      ay += w * g.y;
    }
    u1[(size_t)av * plane + (size_t)y * D.n2 + x0 + b] = mk(ax, ay);
  }
}

// F*_u1D: the transpose of the z gather, evaluated as a gather through the
// inverse map (for every grid point q of the oversampled line, the run(s) of
// detector rows whose stencil covers q; the weights are evaluated from the
// rows' fractional offsets exactly as the forward does), so no atomics are
// needed: stage the h samples of TX columns in LDS, form each grid value in
// registers, write the grid over the staging area, inverse FFT
// (conj-FFT-conj), crop, deconvolve.
template <typename T, int MH, bool REAL_OUT, int LN = 0, int LB = 0>
__global__ __launch_bounds__(1024) void k_zadj(const cpx<T>* __restrict__ u1, void* __restrict__ uout, Dims D,
                                               Tables<T> tb, int log2TX_, int y0, size_t out_zs) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  constexpr bool P2 = p2_len<LN>();
  const int log2TX = LN > 0 ? LB : log2TX_, lM0 = LN > 0 ? ct_l<LN>() : D.lM0;
  const int TX = 1 << log2TX, M0 = LN > 0 ? ct_n<LN>() : D.M0, n0 = LN > 0 ? M0 / 2 : D.n0;   // R = 2
  // block row yl is the row within the output slab; y the row of the volume
  int bx, yl;
  xcd_block(bx, yl);
  const int x0 = bx * TX, y = y0 + yl;
  if (D.skip.skip(y)) return;
  const int tid = threadIdx.x, nth = block_threads<T, LN, LB>();
  const size_t plane = (size_t)D.n1 * D.n2;
  // per-row stencil bases and offsets and the inverse runs, after the buffer
  int* zb = reinterpret_cast<int*>(buf + (size_t)max(M0, D.h) * TX);
  T* zd = reinterpret_cast<T*>(zb + D.h);
  unsigned* zr = reinterpret_cast<unsigned*>(zd + D.h);
  for (int e = tid; e < D.h; e += nth) {
    zb[e] = tb.zbase[e];
    zd[e] = tb.zdelta[e];
  }
  for (int e = tid; e < 2 * M0; e += nth) zr[e] = tb.zrun[e];
  for (int e0 = 0; e0 < D.h * TX; e0 += vpt<T>() * nth) {
    cpx<T> g[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      if (e0 + it * nth >= D.h * TX) break;
      const int e = min(e0 + tid + it * nth, D.h * TX - 1);
      const int av = e >> log2TX, b = e & (TX - 1);
      g[it] = u1[(size_t)av * plane + (size_t)y * D.n2 + x0 + b];
    }
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      if (e0 + it * nth >= D.h * TX) break;
      const int e = e0 + tid + it * nth;
      if (e < D.h * TX) buf[e] = conj(g[it]);
    }
  }
  __syncthreads();
  const GaussW gw{D.beta};
  if constexpr (LN > 0) {
    // one thread per grid point q (QPT of them): each covering row's weight once, then its TX
    // columns as 16-byte chunks; the grid replaces the staging area after a barrier
    using C = Chunk16<T>;
    constexpr int NCH = (1 << LB) / C::CW, NTH = ct_threads<T, LN, LB>(), QPT = (ct_n<LN>() + NTH - 1) / NTH;
    static_assert(NCH >= 1 && ((1 << LB) % C::CW) == 0, "whole chunks per block row");
    const int s = chunk_skew<NCH>();
    C acc[QPT][NCH];
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
#pragma unroll
      for (int c = 0; c < NCH; ++c)
#pragma unroll
        for (int e = 0; e < C::CW; ++e) acc[j][c].c[e] = mk((T)0, (T)0);
      const int q = tid + j * NTH;
      if (q >= M0) continue;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const unsigned run = zr[2 * q + r];
        const int a0 = (int)(run & 0xffffu), a1 = a0 + (int)(run >> 16);
        for (int av = a0; av < a1; ++av) {
          // the stencil tap of row av that lands on q
          const int i = wrap1<P2>(q - zb[av] + MH - 1, M0);
          const T w = gw(zd[av] - (T)(i + 1 - MH), T());
          const C* row = reinterpret_cast<const C*>(buf + av * (1 << LB));
#pragma unroll
          for (int c = 0; c < NCH; ++c) fma_chunk(acc[j][c], w, row[(c + s) & (NCH - 1)]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
      const int q = tid + j * NTH;
      if (q >= M0) continue;
      C* dst = reinterpret_cast<C*>(buf + q * (1 << LB));
#pragma unroll
      for (int c = 0; c < NCH; ++c) dst[(c + s) & (NCH - 1)] = acc[j][c];
    }
  } else {
    cpx<T> v[vpt<T>()];
    const int total = M0 * TX;
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = tid + it * nth;
      T ax = 0, ay = 0;
      if (e < total) {
        const int q = e >> log2TX, b = e & (TX - 1);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const unsigned run = zr[2 * q + r];
          const int a0 = (int)(run & 0xffffu), a1 = a0 + (int)(run >> 16);
          for (int av = a0; av < a1; ++av) {
            // the stencil tap of row av that lands on q
            const int i = wrap1<P2>(q - zb[av] + MH - 1, M0);
            const T w = gw(zd[av] - (T)(i + 1 - MH), T());
            const cpx<T> g = buf[av * TX + b];
            ax += w * g.x;
            ay += w * g.y;
          }
        }
      }
      v[it] = mk(ax, ay);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = tid + it * nth;
      if (e < total) buf[e] = v[it];
    }
  }
  __syncthreads();
  fft_cols<T, LN, LB>(buf, lM0, log2TX, tb, nth);
  for (int e = tid; e < n0 * TX; e += nth) {
    const int a = e >> log2TX, b = e & (TX - 1);
    const cpx<T> g = buf[wrap1<P2>(a - n0 / 2, M0) * TX + b];
    const T c = tb.cz[a];
    const size_t gi = (size_t)a * out_zs + (size_t)yl * D.n2 + x0 + b;
    if constexpr (REAL_OUT) reinterpret_cast<T*>(uout)[gi] = g.x * c;
    else reinterpret_cast<cpx<T>*>(uout)[gi] = mk(g.x * c, -g.y * c);
  }
}

// ---------------------------------------------------------------------------
// F_u2D / F*_u2D equispaced parts
// ---------------------------------------------------------------------------
template <typename T, int LN = 0, int LB = 0>
__global__ __launch_bounds__(1024) void k_ycol_fwd(const cpx<T>* __restrict__ u1, cpx<T>* __restrict__ Tb, int k0,
                                                   Dims D, Tables<T> tb, int log2TX_) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  constexpr bool P2 = p2_len<LN>();
  const int log2TX = LN > 0 ? LB : log2TX_, lM1 = LN > 0 ? ct_l<LN>() : D.lM1;
  const int TX = 1 << log2TX, M1 = LN > 0 ? ct_n<LN>() : D.M1, n1 = LN > 0 ? M1 / 2 : D.n1, n2 = D.n2;   // R = 2
  int bx, kk;
  xcd_block(bx, kk);
  const int x0 = bx * TX, k = k0 + kk;
  if (D.skip.skip(kk)) return;
  const int tid = threadIdx.x, nth = block_threads<T, LN, LB>();
  const cpx<T> zero = mk((T)0, (T)0);
  if constexpr (wave_cols<T, LN, LB>()) {
    constexpr int PC = wave_pitch<LN>(true);
    cpx<T> v[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>() / 2; ++it)   // the input fills n1 = M1 / 2 rows
      v[it] = u1[((size_t)k * n1 + ((tid + it * nth) >> LB)) * n2 + x0 + ((tid + it * nth) & (TX - 1))];
#pragma unroll
    for (int it = 0; it < vpt<T>() / 2; ++it) {
      const int e = tid + it * nth, a = e >> LB, b = e & (TX - 1);
      buf[b * PC + lpad<true>(n1 / 2 + a)] = zero;
      buf[b * PC + lpad<true>((a - n1 / 2) & (M1 - 1))] = v[it] * (tb.cy[a] * tb.cx[x0 + b]);
    }
    __syncthreads();
    lds_fft_wave<T, vpt<T>(), LN, PC>(buf, tb.tw, tb.log2tw);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = tid + it * nth, q = e >> LB, b = e & (TX - 1);
      Tb[((size_t)kk * M1 + q) * n2 + x0 + b] = buf[b * PC + lpad<true>(q)];
    }
    return;
  }
  for (int e = tid; e < (M1 - n1) * TX; e += nth) buf[(n1 / 2) * TX + e] = zero;
  {
    cpx<T> v[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      if (it * nth >= n1 * TX) break;   // the input fills n1 of the M1 rows
      const int e = min(tid + it * nth, n1 * TX - 1);
      v[it] = u1[((size_t)k * n1 + (e >> log2TX)) * n2 + x0 + (e & (TX - 1))];
    }
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      if (it * nth >= n1 * TX) break;
      const int e = tid + it * nth;
      if (e < n1 * TX) {
        const int a = e >> log2TX, b = e & (TX - 1);
        buf[wrap1<P2>(a - n1 / 2, M1) * TX + b] = v[it] * (tb.cy[a] * tb.cx[x0 + b]);
      }
    }
  }
  __syncthreads();
  fft_cols<T, LN, LB>(buf, lM1, log2TX, tb, nth);
  for (int e = tid; e < M1 * TX; e += nth) {
    const int q = e >> log2TX, b = e & (TX - 1);
    Tb[((size_t)kk * M1 + q) * n2 + x0 + b] = buf[e];
  }
}

template <typename T, int LN = 0, int LB = 0>
__global__ __launch_bounds__(1024) void k_ycol_adj(const cpx<T>* __restrict__ Tb, cpx<T>* __restrict__ u1, int k0,
                                                   Dims D, Tables<T> tb, int log2TX_) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  constexpr bool P2 = p2_len<LN>();
  const int log2TX = LN > 0 ? LB : log2TX_, lM1 = LN > 0 ? ct_l<LN>() : D.lM1;
  const int TX = 1 << log2TX, M1 = LN > 0 ? ct_n<LN>() : D.M1, n1 = LN > 0 ? M1 / 2 : D.n1, n2 = D.n2;   // R = 2
  int bx, kk;
  xcd_block(bx, kk);
  const int x0 = bx * TX, k = k0 + kk;
  if (D.skip.skip(kk)) return;
  const int tid = threadIdx.x, nth = block_threads<T, LN, LB>();
  if constexpr (wave_cols<T, LN, LB>()) {
    constexpr int PC = wave_pitch<LN>(true);
    cpx<T> v[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it)
      v[it] = Tb[((size_t)kk * M1 + ((tid + it * nth) >> LB)) * n2 + x0 + ((tid + it * nth) & (TX - 1))];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = tid + it * nth;
      buf[(e & (TX - 1)) * PC + lpad<true>(e >> LB)] = conj(v[it]);
    }
    __syncthreads();
    lds_fft_wave<T, vpt<T>(), LN, PC>(buf, tb.tw, tb.log2tw);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < vpt<T>() / 2; ++it) {
      const int e = tid + it * nth, a = e >> LB, b = e & (TX - 1);
      const cpx<T> w = buf[b * PC + lpad<true>((a - n1 / 2) & (M1 - 1))];
      const T c = tb.cy[a] * tb.cx[x0 + b];
      u1[((size_t)k * n1 + a) * n2 + x0 + b] = mk(w.x * c, -w.y * c);
    }
    return;
  }
  {
    cpx<T> v[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = min(tid + it * nth, M1 * TX - 1);
      v[it] = Tb[((size_t)kk * M1 + (e >> log2TX)) * n2 + x0 + (e & (TX - 1))];
    }
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = tid + it * nth;
      if (e < M1 * TX) buf[e] = conj(v[it]);
    }
  }
  __syncthreads();
  fft_cols<T, LN, LB>(buf, lM1, log2TX, tb, nth);
  for (int e = tid; e < n1 * TX; e += nth) {
    const int a = e >> log2TX, b = e & (TX - 1);
    const cpx<T> v = buf[wrap1<P2>(a - n1 / 2, M1) * TX + b];
    const T c = tb.cy[a] * tb.cx[x0 + b];
    u1[((size_t)k * n1 + a) * n2 + x0 + b] = mk(v.x * c, -v.y * c);
  }
}

template <typename T, int LN = 0, int LB = 0>
__global__ __launch_bounds__(1024) void k_xrow_fwd(const cpx<T>* __restrict__ Tb, cpx<T>* __restrict__ Gb, Dims D,
                                                   Tables<T> tb, int log2RB_) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  constexpr bool P2 = p2_len<LN>();
  const int log2RB = LN > 0 ? LB : log2RB_, lM2 = LN > 0 ? ct_l<LN>() : D.lM2;
  const int RB = 1 << log2RB, M2 = LN > 0 ? ct_n<LN>() : D.M2, n2 = M2 / 2, ln2 = lM2 - 1;
  const int r0 = blockIdx.x * RB;   // slab rows: at most h M1 < 2^31
  if (D.skip.hit && D.skip.skip(D.slice_of(r0))) return;
  const int tid = threadIdx.x, nth = block_threads<T, LN, LB>();
  const cpx<T> zero = mk((T)0, (T)0);
  if constexpr (wave_rows<T, LN, LB>()) {
    // the wave's rows: RPW rows of M2 points from RPW rows of n2 inputs, contiguous in memory
    constexpr int RPW = (64 * vpt<T>()) >> LN, NI = RPW * (M2 / 2) / 64;
    const int lane = tid & 63, row0 = (tid >> 6) * RPW;
    cpx<T> v[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) v[it] = Tb[((size_t)r0 + row0) * n2 + lane + 64 * it];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int e = lane + 64 * it, b = row0 + e / n2, a = e % n2;
      buf[lpad<true>(b * M2 + n2 / 2 + a)] = zero;
      buf[lpad<true>(b * M2 + ((a - n2 / 2) & (M2 - 1)))] = v[it];
    }
    wave_lds_sync();
    lds_fft_wave<T, vpt<T>(), LN>(buf, tb.tw, tb.log2tw);
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = row0 * M2 + lane + 64 * it;
      Gb[(size_t)r0 * M2 + e] = buf[lpad<true>(e)];
    }
    return;
  }
  // R = 2: the padded positions of each row are [n2/2, M2 - n2/2), n2 of them
  {
    cpx<T> v[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      if (it * nth >= RB * n2) break;   // the input fills n2 of the M2 points of each row
      const int e = min(tid + it * nth, RB * n2 - 1);
      v[it] = Tb[(size_t)r0 * n2 + e];
    }
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      if (it * nth >= RB * n2) break;
      const int e = tid + it * nth;
      if (e < RB * n2) {
        const int b = div_len<P2>(e, ln2), a = e - b * n2;
        buf[lpad<true>(b * M2 + n2 / 2 + a)] = zero;
        buf[lpad<true>(b * M2 + wrap1<P2>(a - n2 / 2, M2))] = v[it];
      }
    }
  }
  __syncthreads();
  fft_rows<T, LN, LB>(buf, lM2, M2, log2RB, tb, nth);
  for (int e = tid; e < RB * M2; e += nth) Gb[(size_t)r0 * M2 + e] = buf[lpad<true>(e)];
}

template <typename T, int LN = 0, int LB = 0>
__global__ __launch_bounds__(1024) void k_xrow_adj(const cpx<T>* __restrict__ Gb, cpx<T>* __restrict__ Tb, Dims D,
                                                   Tables<T> tb, int log2RB_) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  constexpr bool P2 = p2_len<LN>();
  const int log2RB = LN > 0 ? LB : log2RB_, lM2 = LN > 0 ? ct_l<LN>() : D.lM2;
  const int RB = 1 << log2RB, M2 = LN > 0 ? ct_n<LN>() : D.M2, n2 = M2 / 2, ln2 = lM2 - 1;
  const int r0 = blockIdx.x * RB;   // slab rows: at most h M1 < 2^31
  if (D.skip.hit && D.skip.skip(D.slice_of(r0))) return;
  const int tid = threadIdx.x, nth = block_threads<T, LN, LB>();
  if constexpr (wave_rows<T, LN, LB>()) {
    constexpr int RPW = (64 * vpt<T>()) >> LN, NO = RPW * (M2 / 2) / 64;
    const int lane = tid & 63, row0 = (tid >> 6) * RPW;
    cpx<T> v[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) v[it] = Gb[((size_t)r0 + row0) * M2 + lane + 64 * it];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) buf[lpad<true>(row0 * M2 + lane + 64 * it)] = conj(v[it]);
    wave_lds_sync();
    lds_fft_wave<T, vpt<T>(), LN>(buf, tb.tw, tb.log2tw);
#pragma unroll
    for (int it = 0; it < NO; ++it) {
      const int e = lane + 64 * it, b = row0 + e / n2, a = e % n2;
      Tb[((size_t)r0 + b) * n2 + a] = conj(buf[lpad<true>(b * M2 + ((a - n2 / 2) & (M2 - 1)))]);
    }
    return;
  }
  {
    cpx<T> v[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = min(tid + it * nth, RB * M2 - 1);
      v[it] = Gb[(size_t)r0 * M2 + e];
    }
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = tid + it * nth;
      if (e < RB * M2) buf[lpad<true>(e)] = conj(v[it]);
    }
  }
  __syncthreads();
  fft_rows<T, LN, LB>(buf, lM2, M2, log2RB, tb, nth);
  for (int e = tid; e < RB * n2; e += nth) {
    const int b = div_len<P2>(e, ln2), a = e - b * n2;
    Tb[((size_t)r0 + b) * n2 + a] = conj(buf[lpad<true>(b * M2 + wrap1<P2>(a - n2 / 2, M2))]);
  }
}

// ---------------------------------------------------------------------------
// Centred 2D DFT per projection: row pass (along k_u / p) and column pass
// (along k_v / v).  Centring is the checkerboard (-1)^(row+col) applied
// before the row pass and after the column pass (h, w multiples of 4; h even,
// so the parity of a row within its projection is that of its slab row).
// The inverse transform is conj(FFT(conj(.))).
// ---------------------------------------------------------------------------
template <typename T, int LN = 0, int LB = 0>
__global__ __launch_bounds__(1024) void k_rowfft(const cpx<T>* in, cpx<T>* out, int L_, int lL_, int log2RB_,
                                                 int inverse, Tables<T> tb) {
  constexpr bool P2 = p2_len<LN>();
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  const int log2RB = LN > 0 ? LB : log2RB_, lL = LN > 0 ? ct_l<LN>() : lL_;
  const int RB = 1 << log2RB, L = LN > 0 ? ct_n<LN>() : L_;
  const size_t r0 = (size_t)blockIdx.x * RB;
  const int tid = threadIdx.x, nth = block_threads<T, LN, LB>();
  if constexpr (wave_rows<T, LN, LB>()) {
    constexpr int RPW = (64 * vpt<T>()) >> LN;
    const int lane = tid & 63, row0 = (tid >> 6) * RPW;
    const size_t base = (r0 + row0) * L;
    cpx<T> w[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) w[it] = in[base + lane + 64 * it];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = lane + 64 * it, b = row0 + (e >> LN), p = e & (L - 1);
      const cpx<T> v = inverse ? conj(w[it]) : w[it];
      buf[lpad<true>(row0 * L + e)] = sgn_parity((int)(r0 & 1) + b + p) > 0 ? v : mk(-v.x, -v.y);
    }
    wave_lds_sync();
    lds_fft_wave<T, vpt<T>(), LN>(buf, tb.tw, tb.log2tw);
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const cpx<T> v = buf[lpad<true>(row0 * L + lane + 64 * it)];
      out[base + lane + 64 * it] = inverse ? conj(v) : v;
    }
    return;
  }
  {
    cpx<T> w[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = min(tid + it * nth, RB * L - 1);
      w[it] = in[r0 * L + e];
    }
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = tid + it * nth;
      if (e < RB * L) {
        const int b = div_len<P2>(e, lL), p = e - b * L;
        cpx<T> v = inverse ? conj(w[it]) : w[it];
        buf[lpad<true>(e)] = sgn_parity((int)(r0 & 1) + b + p) > 0 ? v : mk(-v.x, -v.y);
      }
    }
  }
  __syncthreads();
  fft_rows<T, LN, LB>(buf, lL, L, log2RB, tb, nth);
  for (int e = tid; e < RB * L; e += nth) {
    const cpx<T> v = buf[lpad<true>(e)];
    out[r0 * L + e] = inverse ? conj(v) : v;
  }
}

template <typename T, int LN = 0, int LB = 0>
__global__ __launch_bounds__(1024) void k_colfft(const cpx<T>* in, cpx<T>* out, int H_, int lH_, int W,
                                                 int log2TX_, int inverse, T scale, Tables<T> tb) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lam_smem);
  const int log2TX = LN > 0 ? LB : log2TX_, lH = LN > 0 ? ct_l<LN>() : lH_;
  const int TX = 1 << log2TX, H = LN > 0 ? ct_n<LN>() : H_;
  int bx, by;
  xcd_block(bx, by);
  const int p0 = bx * TX;
  const size_t base = (size_t)by * H * W;
  const int tid = threadIdx.x, nth = block_threads<T, LN, LB>();
  if constexpr (wave_cols<T, LN, LB>()) {
    constexpr int PC = wave_pitch<LN>(true);
    cpx<T> w[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it)
      w[it] = in[base + (size_t)((tid + it * nth) >> LB) * W + p0 + ((tid + it * nth) & (TX - 1))];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = tid + it * nth;
      buf[(e & (TX - 1)) * PC + lpad<true>(e >> LB)] = inverse ? conj(w[it]) : w[it];
    }
    __syncthreads();
    lds_fft_wave<T, vpt<T>(), LN, PC>(buf, tb.tw, tb.log2tw);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = tid + it * nth, a = e >> LB, b = e & (TX - 1);
      cpx<T> v = buf[b * PC + lpad<true>(a)];
      if (inverse) v = conj(v);
      const T sg = sgn_parity(a + p0 + b) > 0 ? scale : -scale;
      out[base + (size_t)a * W + p0 + b] = v * sg;
    }
    return;
  }
  {
    cpx<T> w[vpt<T>()];
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = min(tid + it * nth, H * TX - 1);
      w[it] = in[base + (size_t)(e >> log2TX) * W + p0 + (e & (TX - 1))];
    }
#pragma unroll
    for (int it = 0; it < vpt<T>(); ++it) {
      const int e = tid + it * nth;
      if (e < H * TX) buf[e] = inverse ? conj(w[it]) : w[it];
    }
  }
  __syncthreads();
  fft_cols<T, LN, LB>(buf, lH, log2TX, tb, nth);
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

// Compile-time-size kernels for the hot (log2 N, log2 batch) pairs, when the configured work-group
// size matches; the general kernel otherwise.  L2N is the length code: log2 N for a power of two,
// 32 + l for N = 3 2^l.  STMT names LN and LB.
#define LAM_CT_CASE(T_, L2N, L2B, THR, ln, lb, STMT)                          \
  else if (L2N == ln && L2B == lb && THR == ct_threads<T_, ln, lb>()) {      \
    constexpr int LN = ln, LB = lb;                                          \
    STMT;                                                                    \
  }
#define LAM_CT_COLS(T_, L2N, L2B, THR, STMT)                                  \
  if (false) {}                                                              \
  LAM_CT_CASE(T_, L2N, L2B, THR, 10, 4, STMT)                                \
  LAM_CT_CASE(T_, L2N, L2B, THR, 10, 3, STMT)                                \
  LAM_CT_CASE(T_, L2N, L2B, THR, 9, 4, STMT)                                 \
  LAM_CT_CASE(T_, L2N, L2B, THR, 9, 3, STMT)                                 \
  LAM_CT_CASE(T_, L2N, L2B, THR, 11, 3, STMT)                                \
  LAM_CT_CASE(T_, L2N, L2B, THR, 42, 2, STMT)                                \
  LAM_CT_CASE(T_, L2N, L2B, THR, 42, 1, STMT)                                \
  LAM_CT_CASE(T_, L2N, L2B, THR, 41, 3, STMT)                                \
  LAM_CT_CASE(T_, L2N, L2B, THR, 41, 2, STMT)                                \
  else if (L2N >= 32) {                                                        \
    constexpr int LN = -1, LB = 0;                                           \
    STMT;                                                                    \
  }                                                                          \
  else {                                                                     \
    constexpr int LN = 0, LB = 0;                                            \
    STMT;                                                                    \
  }
#define LAM_CT_ROWS(T_, L2N, L2B, THR, STMT)                                  \
  if (false) {}                                                              \
  LAM_CT_CASE(T_, L2N, L2B, THR, 10, 2, STMT)                                \
  LAM_CT_CASE(T_, L2N, L2B, THR, 10, 1, STMT)                                \
  LAM_CT_CASE(T_, L2N, L2B, THR, 9, 3, STMT)                                 \
  LAM_CT_CASE(T_, L2N, L2B, THR, 9, 2, STMT)                                 \
  LAM_CT_CASE(T_, L2N, L2B, THR, 11, 1, STMT)                                \
  LAM_CT_CASE(T_, L2N, L2B, THR, 42, 0, STMT)                                \
  LAM_CT_CASE(T_, L2N, L2B, THR, 41, 1, STMT)                                \
  LAM_CT_CASE(T_, L2N, L2B, THR, 41, 0, STMT)                                \
  else if (L2N >= 32) {                                                        \
    constexpr int LN = -1, LB = 0;                                           \
    STMT;                                                                    \
  }                                                                          \
  else {                                                                     \
    constexpr int LN = 0, LB = 0;                                            \
    STMT;                                                                    \
  }

// length code of a transform of N = 2^l or 3 2^l points (l = its trailing zero bits): l, or 32 + l
static int len_code(int N) {
  const int l = __builtin_ctz((unsigned)N);
  return N == (1 << l) ? l : 32 + l;
}

template <typename Kern, typename... Args>
static hipError_t launch(Kern k, dim3 grid, int threads, size_t lds, hipStream_t s, Args... args) {
  const hipError_t e = prep(k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, grid, dim3(threads), lds, s, args...);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zfwd(const LaunchCfg& c, const void* u, bool real_in, cpx<T>* u1, int y0, int ny, size_t in_zs,
                       const Dims& D, const Tables<T>& tb, hipStream_t s) {
  const dim3 grid(D.n2 >> c.z_log2TX, ny);
  const int code = len_code(D.M0);
  hipError_t e = hipSuccess;
  LAM_MH_SWITCH(D.m, {
    if constexpr (MH == 4) {
      if (real_in) {
        LAM_CT_COLS(T, code, c.z_log2TX, c.z_threads,
                    e = launch(k_zfwd<T, MH, true, LN, LB>, grid, c.z_threads, c.z_lds, s, u, u1, D, tb, c.z_log2TX,
                               y0, in_zs))
      } else {
        LAM_CT_COLS(T, code, c.z_log2TX, c.z_threads,
                    e = launch(k_zfwd<T, MH, false, LN, LB>, grid, c.z_threads, c.z_lds, s, u, u1, D, tb, c.z_log2TX,
                               y0, in_zs))
      }
    } else {
      if (code >= 32)
        e = real_in ? launch(k_zfwd<T, MH, true, -1>, grid, c.z_threads, c.z_lds, s, u, u1, D, tb, c.z_log2TX, y0, in_zs)
                    : launch(k_zfwd<T, MH, false, -1>, grid, c.z_threads, c.z_lds, s, u, u1, D, tb, c.z_log2TX, y0, in_zs);
      else
        e = real_in ? launch(k_zfwd<T, MH, true>, grid, c.z_threads, c.z_lds, s, u, u1, D, tb, c.z_log2TX, y0, in_zs)
                    : launch(k_zfwd<T, MH, false>, grid, c.z_threads, c.z_lds, s, u, u1, D, tb, c.z_log2TX, y0, in_zs);
    }
  });
  return e;
}

template <typename T>
hipError_t launch_zadj(const LaunchCfg& c, const cpx<T>* u1, void* u, bool real_out, int y0, int ny, size_t out_zs,
                       const Dims& D, const Tables<T>& tb, hipStream_t s) {
  const dim3 grid(D.n2 >> c.z_log2TX, ny);
  const int code = len_code(D.M0);
  hipError_t e = hipSuccess;
  LAM_MH_SWITCH(D.m, {
    if constexpr (MH == 4) {
      if (real_out) {
        LAM_CT_COLS(T, code, c.z_log2TX, c.z_threads,
                    e = launch(k_zadj<T, MH, true, LN, LB>, grid, c.z_threads, c.z_lds, s, u1, u, D, tb, c.z_log2TX,
                               y0, out_zs))
      } else {
        LAM_CT_COLS(T, code, c.z_log2TX, c.z_threads,
                    e = launch(k_zadj<T, MH, false, LN, LB>, grid, c.z_threads, c.z_lds, s, u1, u, D, tb, c.z_log2TX,
                               y0, out_zs))
      }
    } else {
      if (code >= 32)
        e = real_out ? launch(k_zadj<T, MH, true, -1>, grid, c.z_threads, c.z_lds, s, u1, u, D, tb, c.z_log2TX, y0, out_zs)
                     : launch(k_zadj<T, MH, false, -1>, grid, c.z_threads, c.z_lds, s, u1, u, D, tb, c.z_log2TX, y0, out_zs);
      else
        e = real_out ? launch(k_zadj<T, MH, true>, grid, c.z_threads, c.z_lds, s, u1, u, D, tb, c.z_log2TX, y0, out_zs)
                     : launch(k_zadj<T, MH, false>, grid, c.z_threads, c.z_lds, s, u1, u, D, tb, c.z_log2TX, y0, out_zs);
    }
  });
  return e;
}

template <typename T>
hipError_t launch_ycol_fwd(const LaunchCfg& c, const cpx<T>* u1, cpx<T>* Tb, int k0, int ns, const Dims& D,
                           const Tables<T>& tb, hipStream_t s) {
  const dim3 grid(D.n2 >> c.y_log2TX, ns);
  hipError_t e = hipSuccess;
  LAM_CT_COLS(T, len_code(D.M1), c.y_log2TX, c.y_threads,
              e = launch(k_ycol_fwd<T, LN, LB>, grid, c.y_threads, c.y_lds, s, u1, Tb, k0, D, tb, c.y_log2TX))
  return e;
}

template <typename T>
hipError_t launch_xrow_fwd(const LaunchCfg& c, const cpx<T>* Tb, cpx<T>* Gb, int ns, const Dims& D,
                           const Tables<T>& tb, hipStream_t s) {
  const dim3 grid((unsigned)(((size_t)ns * D.M1) >> c.x_log2RB));
  hipError_t e = hipSuccess;
  LAM_CT_ROWS(T, len_code(D.M2), c.x_log2RB, c.x_threads,
              e = launch(k_xrow_fwd<T, LN, LB>, grid, c.x_threads, c.x_lds, s, Tb, Gb, D, tb, c.x_log2RB))
  return e;
}

template <typename T>
hipError_t launch_xrow_adj(const LaunchCfg& c, const cpx<T>* Gb, cpx<T>* Tb, int ns, const Dims& D,
                           const Tables<T>& tb, hipStream_t s) {
  const dim3 grid((unsigned)(((size_t)ns * D.M1) >> c.x_log2RB));
  hipError_t e = hipSuccess;
  LAM_CT_ROWS(T, len_code(D.M2), c.x_log2RB, c.x_threads,
              e = launch(k_xrow_adj<T, LN, LB>, grid, c.x_threads, c.x_lds, s, Gb, Tb, D, tb, c.x_log2RB))
  return e;
}

template <typename T>
hipError_t launch_ycol_adj(const LaunchCfg& c, const cpx<T>* Tb, cpx<T>* u1, int k0, int ns, const Dims& D,
                           const Tables<T>& tb, hipStream_t s) {
  const dim3 grid(D.n2 >> c.y_log2TX, ns);
  hipError_t e = hipSuccess;
  LAM_CT_COLS(T, len_code(D.M1), c.y_log2TX, c.y_threads,
              e = launch(k_ycol_adj<T, LN, LB>, grid, c.y_threads, c.y_lds, s, Tb, u1, k0, D, tb, c.y_log2TX))
  return e;
}

template <typename T>
hipError_t launch_rowfft(const LaunchCfg& c, const cpx<T>* in, cpx<T>* out, bool inverse, int nproj, const Dims& D,
                         const Tables<T>& tb, hipStream_t s) {
  const int lw = __builtin_ctz((unsigned)D.w);
  const dim3 grid((unsigned)(((size_t)nproj * D.h) >> c.r_log2RB));
  const int inv = inverse ? 1 : 0;
  hipError_t e = hipSuccess;
  LAM_CT_ROWS(T, len_code(D.w), c.r_log2RB, c.r_threads,
              e = launch(k_rowfft<T, LN, LB>, grid, c.r_threads, c.r_lds, s, in, out, D.w, lw, c.r_log2RB, inv, tb))
  return e;
}

template <typename T>
hipError_t launch_colfft(const LaunchCfg& c, const cpx<T>* in, cpx<T>* out, bool inverse, double scale_d, int nproj,
                         const Dims& D, const Tables<T>& tb, hipStream_t s) {
  const int lh = __builtin_ctz((unsigned)D.h);
  const dim3 grid(D.w >> c.c_log2TX, nproj);
  const T scale = (T)scale_d;
  const int inv = inverse ? 1 : 0;
  hipError_t e = hipSuccess;
  LAM_CT_COLS(T, len_code(D.h), c.c_log2TX, c.c_threads,
              e = launch(k_colfft<T, LN, LB>, grid, c.c_threads, c.c_lds, s, in, out, D.h, lh, D.w, c.c_log2TX, inv,
                         scale, tb))
  return e;
}

#define LAM_INST(T)                                                                                              \
  template hipError_t launch_zfwd<T>(const LaunchCfg&, const void*, bool, cpx<T>*, int, int, size_t, const Dims&,  \
                                     const Tables<T>&, hipStream_t);                                             \
  template hipError_t launch_zadj<T>(const LaunchCfg&, const cpx<T>*, void*, bool, int, int, size_t, const Dims&,  \
                                     const Tables<T>&, hipStream_t);                                             \
  template hipError_t launch_ycol_fwd<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, int, int, const Dims&,        \
                                         const Tables<T>&, hipStream_t);                                         \
  template hipError_t launch_xrow_fwd<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, int, const Dims&,             \
                                         const Tables<T>&, hipStream_t);                                         \
  template hipError_t launch_xrow_adj<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, int, const Dims&,             \
                                         const Tables<T>&, hipStream_t);                                         \
  template hipError_t launch_ycol_adj<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, int, int, const Dims&,        \
                                         const Tables<T>&, hipStream_t);                                         \
  template hipError_t launch_rowfft<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, bool, int, const Dims&,         \
                                       const Tables<T>&, hipStream_t);                                           \
  template hipError_t launch_colfft<T>(const LaunchCfg&, const cpx<T>*, cpx<T>*, bool, double, int, const Dims&, \
                                       const Tables<T>&, hipStream_t);

LAM_INST(float)
LAM_INST(double)

}  // namespace lam
