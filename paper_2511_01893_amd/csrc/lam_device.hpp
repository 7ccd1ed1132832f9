// Device building blocks for gfx950: complex arithmetic, an in-LDS batched
// Stockham FFT (radix 8/4/2, and a radix-3 stage for lengths 3 2^a), and the
// Gaussian-gridding stencil.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lam {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

// complex values per thread per FFT stage (and per batched load): 16 for
// complex64, 8 for complex128, so the register arrays stay in VGPRs
template <typename T> constexpr int vpt() { return sizeof(T) == 4 ? 16 : 8; }

template <typename T> __device__ __forceinline__ cpx<T> mk(T a, T b) { cpx<T> r; r.x = a; r.y = b; return r; }
template <typename T> __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cpx<T> operator*(cpx<T> a, T s) { return mk(a.x * s, a.y * s); }
template <typename T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ cpx<T> conj(cpx<T> a) { return mk(a.x, -a.y); }
// a * (-i)
template <typename T> __device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) { return mk(a.y, -a.x); }

// ---------------------------------------------------------------------------
// Forward DFT butterflies (exponent sign -), natural-order outputs.
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ void dft2(cpx<T>* v) {
  cpx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename T> __device__ __forceinline__ void dft4(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2, cpx<T>& a3) {
  cpx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_mi(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

template <typename T> __device__ __forceinline__ void dft4(cpx<T>* v) { dft4(v[0], v[1], v[2], v[3]); }

template <typename T> __device__ __forceinline__ void dft8(cpx<T>* v) {
  const T r = (T)0.70710678118654752440084436210484904;
  cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cpx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  o1 = mk((o1.x + o1.y) * r, (o1.y - o1.x) * r);     // * e^{-i pi/4}
  o2 = mul_mi(o2);                                  // * e^{-i pi/2}
  o3 = mk((o3.y - o3.x) * r, -(o3.x + o3.y) * r);    // * e^{-3 i pi/4}
  v[0] = e0 + o0; v[4] = e0 - o0;
  v[1] = e1 + o1; v[5] = e1 - o1;
  v[2] = e2 + o2; v[6] = e2 - o2;
  v[3] = e3 + o3; v[7] = e3 - o3;
}

// 3-point DFT: y0 = a0 + a1 + a2, y1,2 = a0 - (a1 + a2)/2 -/+ i sin(pi/3) (a1 - a2)
template <typename T> __device__ __forceinline__ void dft3(cpx<T>* v) {
  const T s = (T)0.86602540378443864676372317075293618;
  const cpx<T> a0 = v[0], t = v[1] + v[2], d = v[1] - v[2];
  const cpx<T> c = mk(a0.x - (T)0.5 * t.x, a0.y - (T)0.5 * t.y);
  const cpx<T> r = mk(d.y * s, -d.x * s);          // -i sin(pi/3) (a1 - a2)
  v[0] = a0 + t;
  v[1] = c + r;
  v[2] = c - r;
}

template <typename T, int R> __device__ __forceinline__ void dftR(cpx<T>* v) {
  if constexpr (R == 2) dft2(v);
  else if constexpr (R == 3) dft3(v);
  else if constexpr (R == 4) dft4(v);
  else dft8(v);
}

// floor(q / 3) for any 32-bit unsigned q: the high word of q (2^33 + 1) / 3, shifted once
__host__ __device__ __forceinline__ int div3(int q) {
  return (int)((unsigned)(((unsigned long long)(unsigned)q * 0xAAAAAAABull) >> 33));
}

// ---------------------------------------------------------------------------
// Batched in-place Stockham FFT in LDS.
//
// Element (point p, batch b) lives at buf[p*sp + b*sb].  N = 2^log2n points,
// NB = 2^log2nb transforms.  Each radix-R stage reads every value into
// registers, synchronises, applies twiddles and the R-point DFT and writes
// the results to their autosorted positions, then synchronises again, so
// one buffer suffices.  nth is the work-group size.  Values per thread per
// stage = N*NB/nth, which
// must not exceed VPT.  tw[t] = exp(-2 pi i t / 2^log2tw), 2^log2tw >= N,
// generated in FP64 on the host and rounded to T.  bfast selects the thread
// to (j, b) map: batch index fastest (for interleaved [p][b] layouts) or
// butterfly index fastest (for contiguous rows).
// ---------------------------------------------------------------------------
// LDS element index of the FFT buffers, optionally with one pad slot per 8
// elements.  Without it, a row-major buffer's first Stockham stages store at
// strides of 8 and 64 elements, which puts a wave's 64 lanes on a handful of
// banks; with it, those stores spread over every bank.
template <bool PAD> __device__ __forceinline__ int lpad(int e) { return PAD ? e + (e >> 3) : e; }

// Multiply v[1..R-1] by the twiddles w^r, w = exp(-2 pi i k / span), then the
// R-point DFT.  w and w^4 come from the FP64-built table, the other powers by
// at most two complex products (two table loads per radix-8 butterfly instead
// of seven).
template <typename T, int R>
__device__ __forceinline__ void twiddle_dft(cpx<T>* v, const cpx<T>* __restrict__ tw, int k, int twsh) {
  cpx<T> tw_r[R];
  tw_r[1] = tw[k << twsh];
  if constexpr (R >= 4) {
    tw_r[2] = cmul(tw_r[1], tw_r[1]);
    tw_r[3] = cmul(tw_r[2], tw_r[1]);
  }
  if constexpr (R == 8) {
    tw_r[4] = tw[(4 * k) << twsh];
    tw_r[5] = cmul(tw_r[4], tw_r[1]);
    tw_r[6] = cmul(tw_r[4], tw_r[2]);
    tw_r[7] = cmul(tw_r[4], tw_r[3]);
  }
#pragma unroll
  for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw_r[r]);
  dftR<T, R>(v);
}

template <typename T, int R, int VPT, bool PAD = false>
__device__ __forceinline__ void fft_stage(cpx<T>* buf, int log2n, int log2nb, int Ns, int log2span, int sp, int sb,
                                          bool bfast, const cpx<T>* __restrict__ tw, int log2tw, int nth) {
  constexpr int IT = VPT / R;
  constexpr int LR = (R == 8) ? 3 : (R == 4 ? 2 : 1);
  const int tid = threadIdx.x;
  const int log2nbf = log2n - LR;                      // butterflies per transform = N / R
  const int total = 1 << (log2nbf + log2nb);
  const int nbf = 1 << log2nbf;
  cpx<T> v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int t = tid + it * nth;
    if (t < total) {
      int j, b;
      if (bfast) { b = t & ((1 << log2nb) - 1); j = t >> log2nb; }
      else { j = t & (nbf - 1); b = t >> log2nbf; }
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = buf[lpad<PAD>((j + r * nbf) * sp + b * sb)];
    }
  }
  __syncthreads();
  const int twsh = log2tw - log2span;                  // span = Ns * R
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int t = tid + it * nth;
    if (t < total) {
      int j, b;
      if (bfast) { b = t & ((1 << log2nb) - 1); j = t >> log2nb; }
      else { j = t & (nbf - 1); b = t >> log2nbf; }
      const int k = j & (Ns - 1);
      twiddle_dft<T, R>(v[it], tw, k, twsh);
      const int idxD = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lpad<PAD>((idxD + r * Ns) * sp + b * sb)] = v[it][r];
    }
  }
  __syncthreads();
}

template <typename T, int VPT, bool PAD = false>
__device__ __forceinline__ void lds_fft(cpx<T>* buf, int log2n, int log2nb, int sp, int sb, bool bfast,
                        const cpx<T>* __restrict__ tw, int log2tw, int nth) {
  int Ns = 1, lspan = 0, rem = log2n;
  while (rem > 0) {
    if (rem >= 3) {
      fft_stage<T, 8, VPT, PAD>(buf, log2n, log2nb, Ns, lspan + 3, sp, sb, bfast, tw, log2tw, nth);
      Ns <<= 3; lspan += 3; rem -= 3;
    } else if (rem == 2) {
      fft_stage<T, 4, VPT, PAD>(buf, log2n, log2nb, Ns, lspan + 2, sp, sb, bfast, tw, log2tw, nth);
      Ns <<= 2; lspan += 2; rem -= 2;
    } else {
      fft_stage<T, 2, VPT, PAD>(buf, log2n, log2nb, Ns, lspan + 1, sp, sb, bfast, tw, log2tw, nth);
      Ns <<= 1; lspan += 1; rem -= 1;
    }
  }
}

// The same FFT for lengths N = 3 2^a (the grids of 3 2^k voxels): a radix-3
// stage first (span 3, no twiddles), then radix 8/4/2 stages with Ns = 3 2^s
// values already combined.  Index arithmetic divides by 3 with div3.  tw3[t]
// = exp(-2 pi i t / Ntw3), Ntw3 = 3 2^log2tw3 >= N, so the twiddle of a stage
// of span 3 2^(s + log2 R) sits at a stride 2^(log2tw3 - s - log2 R).  The
// per-thread register arrays hold ceil(VPT / R) butterflies, which covers a
// stage when nth >= N NB / VPT.
template <typename T, int R, int VPT, bool PAD = false>
__device__ __forceinline__ void fft_stage3(cpx<T>* buf, int a, int log2nb, int ls, int sp, int sb, bool bfast,
                                           const cpx<T>* __restrict__ tw3, int log2tw3, int nth) {
  constexpr int IT = (VPT + R - 1) / R;
  constexpr int LR = R == 3 ? 0 : (R == 8 ? 3 : (R == 4 ? 2 : 1));
  // butterflies per transform: N / 3 = 2^a for the radix-3 stage, N / R = 3 2^(a - LR) otherwise
  const int la = a - LR, nbf = R == 3 ? (1 << a) : 3 << la;
  const int total = nbf << log2nb;
  const int tid = threadIdx.x;
  auto map = [&](int t, int& j, int& b) {
    if (bfast) { b = t & ((1 << log2nb) - 1); j = t >> log2nb; }
    else if (R == 3) { j = t & (nbf - 1); b = t >> a; }
    else { b = div3(t >> la); j = t - b * nbf; }
  };
  cpx<T> v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int t = tid + it * nth;
    if (t < total) {
      int j, b;
      map(t, j, b);
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = buf[lpad<PAD>((j + r * nbf) * sp + b * sb)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int t = tid + it * nth;
    if (t < total) {
      int j, b;
      map(t, j, b);
      int idxD, Ns;
      if constexpr (R == 3) {          // Ns = 1: k = 0, outputs at 3 j + r
        dft3(v[it]);
        idxD = 3 * j;
        Ns = 1;
      } else {                         // Ns = 3 2^ls
        const int hi = div3(j >> ls);
        Ns = 3 << ls;
        const int k = j - hi * Ns;
        twiddle_dft<T, R>(v[it], tw3, k, log2tw3 - ls - LR);
        idxD = hi * Ns * R + k;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lpad<PAD>((idxD + r * Ns) * sp + b * sb)] = v[it][r];
    }
  }
  __syncthreads();
}

template <typename T, int VPT, bool PAD = false>
__device__ __forceinline__ void lds_fft3(cpx<T>* buf, int a, int log2nb, int sp, int sb, bool bfast,
                                         const cpx<T>* __restrict__ tw3, int log2tw3, int nth) {
  fft_stage3<T, 3, VPT, PAD>(buf, a, log2nb, 0, sp, sb, bfast, tw3, log2tw3, nth);
  int ls = 0, rem = a;
  while (rem > 0) {
    if (rem >= 3) {
      fft_stage3<T, 8, VPT, PAD>(buf, a, log2nb, ls, sp, sb, bfast, tw3, log2tw3, nth);
      ls += 3; rem -= 3;
    } else if (rem == 2) {
      fft_stage3<T, 4, VPT, PAD>(buf, a, log2nb, ls, sp, sb, bfast, tw3, log2tw3, nth);
      ls += 2; rem -= 2;
    } else {
      fft_stage3<T, 2, VPT, PAD>(buf, a, log2nb, ls, sp, sb, bfast, tw3, log2tw3, nth);
      ls += 1; rem -= 1;
    }
  }
}

// Row FFTs with one wave per row (or per few rows): when a wave's 64 lanes hold whole rows
// (RPW = 64 VPT / N rows of N = 2^LOG2N points, row-major with one pad slot per 8 elements), each
// wave runs every stage on its own rows, and the stages are ordered by wave-level fences instead of
// work-group barriers: the LDS operations of one wave complete in order, so its reads after a fence
// see its writes before it, and no wave waits for another.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// PITCH: elements from one row to the next (lpad(N) for row-major buffers; column kernels hold each
// column as a row of a column-major buffer and skew the pitch by one slot, lpad(N) + 1, so that the
// staging writes of neighbouring columns fall in different banks).
template <int LOG2N> constexpr int wave_pitch(bool skew) { return (1 << LOG2N) + ((1 << LOG2N) >> 3) + (skew ? 1 : 0); }

template <typename T, int R, int VPT, int LOG2N, int LOG2NS, int PITCH>
__device__ __forceinline__ void fft_stage_wave(cpx<T>* buf, const cpx<T>* __restrict__ tw, int log2tw) {
  constexpr int LR = (R == 8) ? 3 : (R == 4 ? 2 : 1);
  constexpr int LOG2NBF = LOG2N - LR, NBF = 1 << LOG2NBF, NS = 1 << LOG2NS;
  constexpr int RPW = (64 * VPT) >> LOG2N;         // rows per wave
  constexpr int IT = VPT / R;                      // butterflies per lane: RPW NBF / 64
  static_assert(RPW >= 1 && (RPW << LOG2NBF) == 64 * IT, "a wave holds whole rows");
  const int lane = threadIdx.x & 63, row0 = (threadIdx.x >> 6) * RPW;
  cpx<T> v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int q = lane + 64 * it, b = row0 + (q >> LOG2NBF), j = q & (NBF - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) v[it][r] = buf[b * PITCH + lpad<true>(j + r * NBF)];
  }
  wave_lds_sync();
  const int twsh = log2tw - (LOG2NS + LR);
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int q = lane + 64 * it, b = row0 + (q >> LOG2NBF), j = q & (NBF - 1);
    const int k = j & (NS - 1);
    twiddle_dft<T, R>(v[it], tw, k, twsh);
    const int idxD = ((j >> LOG2NS) << (LOG2NS + LR)) + k;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[b * PITCH + lpad<true>(idxD + r * NS)] = v[it][r];
  }
  wave_lds_sync();
}

template <typename T, int VPT, int LOG2N, int PITCH = wave_pitch<LOG2N>(false), int REM = LOG2N, int LOG2NS = 0>
__device__ __forceinline__ void lds_fft_wave(cpx<T>* buf, const cpx<T>* __restrict__ tw, int log2tw) {
  if constexpr (REM >= 3) {
    fft_stage_wave<T, 8, VPT, LOG2N, LOG2NS, PITCH>(buf, tw, log2tw);
    lds_fft_wave<T, VPT, LOG2N, PITCH, REM - 3, LOG2NS + 3>(buf, tw, log2tw);
  } else if constexpr (REM == 2) {
    fft_stage_wave<T, 4, VPT, LOG2N, LOG2NS, PITCH>(buf, tw, log2tw);
  } else if constexpr (REM == 1) {
    fft_stage_wave<T, 2, VPT, LOG2N, LOG2NS, PITCH>(buf, tw, log2tw);
  }
}

// The 3 2^A-point FFT with A, the batch NB = 2^LOG2NB and the layout fixed at compile time (the
// hot sizes of the 3 2^k grids): every division by 3 2^s is by a constant, the stages unroll, and
// the work-group size is the launch's, max(64, N NB / VPT rounded up to whole waves).  COLS as for
// lds_fft_ct.
template <int VPT, int A, int LOG2NB> constexpr int fft3_threads() {
  return ((3 << (A + LOG2NB)) + 64 * VPT - 1) / (64 * VPT) * 64 < 64
             ? 64
             : ((3 << (A + LOG2NB)) + 64 * VPT - 1) / (64 * VPT) * 64;
}

template <typename T, int R, int VPT, bool PAD, int A, int LOG2NB, bool COLS, int LS>
__device__ __forceinline__ void fft_stage3_ct(cpx<T>* buf, const cpx<T>* __restrict__ tw3, int log2tw3) {
  constexpr int LR = R == 3 ? 0 : (R == 8 ? 3 : (R == 4 ? 2 : 1));
  constexpr int N = 3 << A;
  constexpr int NBF = R == 3 ? (1 << A) : (3 << (A - LR));   // butterflies per transform
  constexpr int TOTAL = NBF << LOG2NB;
  constexpr int NTH = fft3_threads<VPT, A, LOG2NB>();
  constexpr int IT = (TOTAL + NTH - 1) / NTH;
  constexpr int NS = R == 3 ? 1 : 3 << LS;                   // values combined by earlier stages
  auto at = [](int p, int b) { return lpad<PAD>(COLS ? (p << LOG2NB) + b : b * N + p); };
  auto map = [](int t, int& j, int& b) {
    if (COLS) { b = t & ((1 << LOG2NB) - 1); j = t >> LOG2NB; }
    else { b = (int)((unsigned)t / (unsigned)NBF); j = t - b * NBF; }
  };
  const int tid = threadIdx.x;
  cpx<T> v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int t = tid + it * NTH;
    if (TOTAL % NTH == 0 || t < TOTAL) {
      int j, b;
      map(t, j, b);
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = buf[at(j + r * NBF, b)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int t = tid + it * NTH;
    if (TOTAL % NTH == 0 || t < TOTAL) {
      int j, b;
      map(t, j, b);
      int idxD;
      if constexpr (R == 3) {
        dft3(v[it]);
        idxD = 3 * j;
      } else {
        const int hi = (int)((unsigned)j / (unsigned)NS), k = j - hi * NS;
        twiddle_dft<T, R>(v[it], tw3, k, log2tw3 - LS - LR);
        idxD = hi * NS * R + k;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) buf[at(idxD + r * NS, b)] = v[it][r];
    }
  }
  __syncthreads();
}

template <typename T, int VPT, bool PAD, int A, int LOG2NB, bool COLS, int REM, int LS>
__device__ __forceinline__ void lds_fft3_ct_rest(cpx<T>* buf, const cpx<T>* __restrict__ tw3, int log2tw3) {
  if constexpr (REM >= 3) {
    fft_stage3_ct<T, 8, VPT, PAD, A, LOG2NB, COLS, LS>(buf, tw3, log2tw3);
    lds_fft3_ct_rest<T, VPT, PAD, A, LOG2NB, COLS, REM - 3, LS + 3>(buf, tw3, log2tw3);
  } else if constexpr (REM == 2) {
    fft_stage3_ct<T, 4, VPT, PAD, A, LOG2NB, COLS, LS>(buf, tw3, log2tw3);
  } else if constexpr (REM == 1) {
    fft_stage3_ct<T, 2, VPT, PAD, A, LOG2NB, COLS, LS>(buf, tw3, log2tw3);
  }
}

template <typename T, int VPT, bool PAD, int A, int LOG2NB, bool COLS>
__device__ __forceinline__ void lds_fft3_ct(cpx<T>* buf, const cpx<T>* __restrict__ tw3, int log2tw3) {
  fft_stage3_ct<T, 3, VPT, PAD, A, LOG2NB, COLS, 0>(buf, tw3, log2tw3);
  lds_fft3_ct_rest<T, VPT, PAD, A, LOG2NB, COLS, A, 0>(buf, tw3, log2tw3);
}

// The same FFT with the transform length N = 2^LOG2N and the batch NB =
// 2^LOG2NB fixed at compile time (the hot sizes): every index is a shift or a
// constant, the stage sequence is unrolled and the work-group size is the
// launch's, max(64, N NB / VPT).  COLS selects the layout: element (p, b) at
// p NB + b with the batch index fastest across threads (column blocks), or at
// b N + p with the butterfly index fastest (row blocks).
template <typename T, int R, int VPT, bool PAD, int LOG2N, int LOG2NB, bool COLS, int LOG2NS>
__device__ __forceinline__ void fft_stage_ct(cpx<T>* buf, const cpx<T>* __restrict__ tw, int log2tw) {
  constexpr int LR = (R == 8) ? 3 : (R == 4 ? 2 : 1);
  constexpr int LOG2NBF = LOG2N - LR, NBF = 1 << LOG2NBF, NS = 1 << LOG2NS;
  constexpr int TOTAL = 1 << (LOG2NBF + LOG2NB);                       // butterflies of the stage
  constexpr int NTH = ((1 << (LOG2N + LOG2NB)) / VPT) < 64 ? 64 : ((1 << (LOG2N + LOG2NB)) / VPT);
  constexpr int IT = (TOTAL + NTH - 1) / NTH;
  auto at = [](int p, int b) { return lpad<PAD>(COLS ? (p << LOG2NB) + b : (b << LOG2N) + p); };
  const int tid = threadIdx.x;
  cpx<T> v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int t = tid + it * NTH;
    if (TOTAL % NTH == 0 || t < TOTAL) {
      const int j = COLS ? t >> LOG2NB : t & (NBF - 1), b = COLS ? t & ((1 << LOG2NB) - 1) : t >> LOG2NBF;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = buf[at(j + r * NBF, b)];
    }
  }
  __syncthreads();
  const int twsh = log2tw - (LOG2NS + LR);
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int t = tid + it * NTH;
    if (TOTAL % NTH == 0 || t < TOTAL) {
      const int j = COLS ? t >> LOG2NB : t & (NBF - 1), b = COLS ? t & ((1 << LOG2NB) - 1) : t >> LOG2NBF;
      const int k = j & (NS - 1);
      twiddle_dft<T, R>(v[it], tw, k, twsh);
      const int idxD = ((j >> LOG2NS) << (LOG2NS + LR)) + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[at(idxD + r * NS, b)] = v[it][r];
    }
  }
  __syncthreads();
}

template <typename T, int VPT, bool PAD, int LOG2N, int LOG2NB, bool COLS, int REM = LOG2N, int LOG2NS = 0>
__device__ __forceinline__ void lds_fft_ct(cpx<T>* buf, const cpx<T>* __restrict__ tw, int log2tw) {
  if constexpr (REM >= 3) {
    fft_stage_ct<T, 8, VPT, PAD, LOG2N, LOG2NB, COLS, LOG2NS>(buf, tw, log2tw);
    lds_fft_ct<T, VPT, PAD, LOG2N, LOG2NB, COLS, REM - 3, LOG2NS + 3>(buf, tw, log2tw);
  } else if constexpr (REM == 2) {
    fft_stage_ct<T, 4, VPT, PAD, LOG2N, LOG2NB, COLS, LOG2NS>(buf, tw, log2tw);
  } else if constexpr (REM == 1) {
    fft_stage_ct<T, 2, VPT, PAD, LOG2N, LOG2NB, COLS, LOG2NS>(buf, tw, log2tw);
  }
}

// ---------------------------------------------------------------------------
// Gaussian-gridding stencil: for s = R xi (FP64), base = floor(s),
// delta = s - base and the 2m weights exp(-beta (delta - o)^2),
// o = -m+1 .. m, by the two-exponential recurrence
//   w_{o+1} = w_o * exp(2 beta delta) * exp(-beta (2o + 1))
// (Greengard & Lee 2004, fast Gaussian gridding), all in FP64, rounded to T.
// rc[i] = exp(-beta (2 o_i + 1)) for o_i = -m+1+i, precomputed on the host.
// ---------------------------------------------------------------------------
template <typename T, int MH>
__device__ __forceinline__ void stencil_weights(double s, double beta, const double* rc, int& base, T* w) {
  const double b = floor(s);
  const double d = s - b;
  base = (int)b;
  const double o0 = (double)(1 - MH);
  double cur = exp(-beta * (d - o0) * (d - o0));
  const double e = exp(2.0 * beta * d);
  w[0] = (T)cur;
#pragma unroll
  for (int i = 1; i < 2 * MH; ++i) {
    cur = cur * e * rc[i - 1];
    w[i] = (T)cur;
  }
}

// Gaussian weight exp(-beta a^2) of a stencil offset a: for complex64 as a
// single-precision 2^x of -beta log2(e) a^2 (a itself comes from an FP64
// coordinate, so only the exponential is single precision: relative error
// below 2e-6 at the stencil edge, 1e-7 at its centre); for complex128 in FP64.
// Every forward gather and its adjoint spread use this same function, so they
// stay an exact adjoint pair.
struct GaussW {
  double beta;
  __device__ __forceinline__ float operator()(float a, float) const {
    return __builtin_amdgcn_exp2f(-(float)(beta * 1.4426950408889634074) * a * a);
  }
  __device__ __forceinline__ double operator()(double a, double) const { return exp(-beta * a * a); }
};

// Oversampled coordinates (R n nu) of detector bin (k_v, k_u) at angle with
// cos/sin (ct, st): the same expression in the forward gather and the
// adjoint scatter, so both see identical bases and weights.
struct XYGeom {
  double Rn2, Rn1;        // R * n2, R * n1
  double inv_w, inv_h;    // 1/w, 1/h
  double sphi;            // sin(phi)
  int w, h;
};

// Contraction is off so the coordinate is the plain sequence of correctly
// rounded products and sums: at angles where s lands on an integer (multiples
// of pi/2), a fused multiply-add would round differently and move floor(s).
// For the same reason k_u / w and k_v / h are correctly rounded quotients: the
// product with 1/w is one only when w is a power of two (1/w exact); for
// w = 3 2^k it can fall an ulp below an integer coordinate.
__host__ __device__ inline void target_coords(const XYGeom& g, double ct, double st, int akv, int aku,
                                              double& sx, double& sy) {
#pragma clang fp contract(off)
  const double nu = (double)(aku - g.w / 2), nv = (double)(akv - g.h / 2);
  const double ku = (g.w & (g.w - 1)) == 0 ? nu * g.inv_w : nu / (double)g.w;
  const double kv = (g.h & (g.h - 1)) == 0 ? nv * g.inv_h : nv / (double)g.h;
  sx = g.Rn2 * (ku * ct + kv * g.sphi * st);
  sy = g.Rn1 * (ku * st - kv * g.sphi * ct);
}

}  // namespace lam
