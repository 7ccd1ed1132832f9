// Memoization of the LSP's operator applications on the device (Section 4.4 "Memoization Cache",
// Section 4.5 Equation (cs)).
//
// Each of the four operators of the cancelled LSP (F_u1D, F_u2D, F*_u2D, F*_u1D) keeps a private
// cache per chunk location: one (key, value) item, replaced first-in-first-out.  A chunk is a range
// of 2^k volume rows y (F_u1D, F*_u1D act on whole z columns) or k_v slices (F_u2D, F*_u2D act on
// whole slices).  For every application of the operator:
//   sketch   the key of each input chunk, a signed random projection (count sketch) standing in for
//            the paper's CNN encoder: value q of the chunk (C order, complex values as (re, im)) adds
//            to bucket q mod d with sign -1 when the top bit of SplitMix64 output number
//            chunk 2^40 + q (state seed + operator index) is set, else +1; FP64 sums.  The signs are
//            kept as a bit table built on the device at the first step;
//   compare  cosine similarity of the query key and the chunk's cached key (Equation (cs)), FP64;
//            a hit where the cache holds an item and the similarity exceeds tau;
//   operator the operator's kernels skip the chunks that hit (lam::SkipMap);
//   commit   a hit copies the cached value into the output, a miss stores the output and the query
//            key as the chunk's new item.
// Everything stays on the device (hit flags, counters): the host never synchronises.
#include "lam_admm.hpp"
#include "lam_internal.hpp"
#include "lam_memo.hpp"

namespace lam {
namespace {

constexpr int MT = 256;           // threads per block
constexpr int SKETCH_BLOCKS = 16; // blocks per chunk in the sketch's first pass

int ilog2i(long v) { int r = 0; while ((1L << r) < v) ++r; return r; }
size_t al(size_t v) { return (v + 255) / 256 * 256; }

// View of a C-order array [A][B][C] of real (ncomp 1) or complex (ncomp 2) values, split along B
// into chunks of 2^lcb.  Positions are counted in reals: row length Lr = C ncomp = 2^lr.
struct View {
  int A, lB, lr, lcb;
  __host__ __device__ size_t reals() const { return (size_t)A << (lB + lr); }
  __host__ __device__ int chunks() const { return 1 << (lB - lcb); }
  __host__ __device__ size_t chunk_reals() const { return (size_t)A << (lcb + lr); }
  // real position of value q of chunk c
  __device__ __forceinline__ size_t at(int c, size_t q) const {
    const size_t rho = q >> lr, o = q & ((((size_t)1) << lr) - 1);
    const size_t a = rho >> lcb, bb = rho & ((((size_t)1) << lcb) - 1);
    return ((((a << lB) + ((size_t)c << lcb) + bb)) << lr) | o;
  }
  // chunk and within-chunk number of the value at real position g
  __device__ __forceinline__ void of(size_t g, int& c, size_t& q) const {
    const size_t row = g >> lr, o = g & ((((size_t)1) << lr) - 1);
    const size_t a = row >> lB, b = row & ((((size_t)1) << lB) - 1);
    c = (int)(b >> lcb);
    q = ((((a << lcb) + (b & ((((size_t)1) << lcb) - 1)))) << lr) | o;
  }
};

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long state, unsigned long long counter) {
  unsigned long long z = state + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Sign bits of one operator's input positions (bit set: sign -1); once, while *built is 0.
__global__ __launch_bounds__(MT) void k_memo_signs(View v, unsigned long long state, unsigned* __restrict__ bits,
                                                   const int* __restrict__ built) {
  if (*built) return;
  const size_t words = (v.reals() + 31) / 32;
  for (size_t w = (size_t)blockIdx.x * MT + threadIdx.x; w < words; w += (size_t)gridDim.x * MT) {
    unsigned word = 0;
    for (int k = 0; k < 32; ++k) {
      const size_t g = w * 32 + k;
      if (g >= v.reals()) break;
      int c;
      size_t q;
      v.of(g, c, q);
      word |= (unsigned)(splitmix64(state, ((unsigned long long)c << 40) + q) >> 63) << k;
    }
    bits[w] = word;
  }
}

__global__ void k_memo_flag(int* built) { *built = 1; }

// Partial keys: block x of chunk c sums spans x, x + SKETCH_BLOCKS, ... of d consecutive values;
// thread t owns buckets t + MT k of its block's accumulator.
template <typename T>
__global__ __launch_bounds__(MT) void k_memo_sketch(const T* __restrict__ x, View v, const unsigned* __restrict__ bits,
                                                    int d, double* __restrict__ partial) {
  extern __shared__ double acc[];   // [d]
  const int c = blockIdx.y, t = threadIdx.x;
  for (int i = t; i < d; i += MT) acc[i] = 0.0;
  const size_t n = v.chunk_reals();
  for (size_t q0 = (size_t)blockIdx.x * d; q0 < n; q0 += (size_t)SKETCH_BLOCKS * d)
    for (int i = t; i < d; i += MT) {
      const size_t q = q0 + i;
      if (q >= n) break;
      const size_t g = v.at(c, q);
      const double val = (double)x[g];
      acc[i] += ((bits[g >> 5] >> (g & 31)) & 1u) ? -val : val;
    }
  double* out = partial + ((size_t)c * SKETCH_BLOCKS + blockIdx.x) * d;
  for (int i = t; i < d; i += MT) out[i] = acc[i];
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < MT / 64; ++w) s += sh[w];
  return s;
}

// Query key of chunk blockIdx.x (sum of the partial keys), its cosine similarity with the cached key
// (Equation (cs)) and the hit flag; counters[0] += hits, counters[1] += misses.
__global__ __launch_bounds__(MT) void k_memo_compare(const double* __restrict__ partial, int d, double* __restrict__ kq,
                                                     const double* __restrict__ kc, const int* __restrict__ valid,
                                                     int* __restrict__ hit, double tau, long long* counters) {
  __shared__ double sh[MT / 64];
  const int c = blockIdx.x;
  double dot = 0, nq = 0, nc = 0;
  for (int i = threadIdx.x; i < d; i += MT) {
    double s = 0;
    for (int b = 0; b < SKETCH_BLOCKS; ++b) s += partial[((size_t)c * SKETCH_BLOCKS + b) * d + i];
    kq[(size_t)c * d + i] = s;
    const double k = kc[(size_t)c * d + i];
    dot += s * k;
    nq += s * s;
    nc += k * k;
  }
  dot = block_sum(dot, sh);
  nq = block_sum(nq, sh);
  nc = block_sum(nc, sh);
  if (threadIdx.x == 0) {
    const double cs = (nq > 0.0 && nc > 0.0) ? dot / (sqrt(nq) * sqrt(nc)) : 0.0;
    const int h = (valid[c] && cs > tau) ? 1 : 0;
    hit[c] = h;
    atomicAdd((unsigned long long*)(counters + (h ? 0 : 1)), 1ull);
  }
}

// Hit: output <- cached value (less sub, if given); miss: cached value <- output, output -= sub, and the
// query key becomes the chunk's key.  Real positions of the output's chunk blockIdx.y.
template <typename T>
__global__ __launch_bounds__(MT) void k_memo_commit(T* __restrict__ out, T* __restrict__ cache, const T* __restrict__ sub,
                                                    View v, const int* __restrict__ hit, int d,
                                                    const double* __restrict__ kq, double* __restrict__ kc,
                                                    int* __restrict__ valid) {
  const int c = blockIdx.y;
  const bool h = hit[c] != 0;
  const size_t n = v.chunk_reals();
  for (size_t q = (size_t)blockIdx.x * MT + threadIdx.x; q < n; q += (size_t)gridDim.x * MT) {
    const size_t g = v.at(c, q);
    if (h) {
      out[g] = sub ? cache[g] - sub[g] : cache[g];
    } else {
      const T o = out[g];
      cache[g] = o;
      if (sub) out[g] = o - sub[g];
    }
  }
  if (!h && blockIdx.x == 0) {
    for (int i = threadIdx.x; i < d; i += MT) kc[(size_t)c * d + i] = kq[(size_t)c * d + i];
    if (threadIdx.x == 0) valid[c] = 1;
  }
}

// The views of operator o's input and output, and its chunk size (log2).
void views(const lam_params& q, const lam_memo& m, int o, View& in, View& out, int& lcb) {
  const int lcy = ilog2i(m.chunk_y), lck = ilog2i(m.chunk_kv);
  const int l0 = ilog2i(q.n0), l1 = ilog2i(q.n1), l2 = ilog2i(q.n2), lh = ilog2i(q.h), lw = ilog2i(q.w);
  (void)l0;
  const View vol{q.n0, l1, l2, lcy};                       // u[z][y][x], real, chunks along y
  const View u1y{q.h, l1, l2 + 1, lcy};                    // u1[k_v][y][x], complex, chunks along y
  const View u1k{1, lh, l1 + l2 + 1, lck};                 // u1 as [1][k_v][y x], chunks along k_v
  const View dat{q.ntheta, lh, lw + 1, lck};               // r[theta][k_v][k_u], complex, chunks along k_v
  switch (o) {
    case 0: in = vol; out = u1y; lcb = lcy; break;
    case 1: in = u1k; out = dat; lcb = lck; break;
    case 2: in = dat; out = u1k; lcb = lck; break;
    default: in = u1y; out = vol; lcb = lcy; break;
  }
}

struct OpLayout {
  size_t bits, kc, kq, valid, hit, cache;
};
struct MemoLayout {
  OpLayout op[4];
  size_t partial, built, total;
};

MemoLayout memo_layout(const lam_params& q, const lam_memo& m) {
  const size_t rs = q.dtype == LAM_C64 ? 4 : 8;
  MemoLayout L{};
  size_t o = 0;
  int maxch = 1;
  for (int k = 0; k < 4; ++k) {
    View in, out;
    int lcb;
    views(q, m, k, in, out, lcb);
    const int nch = in.chunks();
    maxch = nch > maxch ? nch : maxch;
    OpLayout& p = L.op[k];
    p.bits = o; o += al((in.reals() + 31) / 32 * 4);
    p.kc = o; o += al((size_t)nch * m.key_dim * 8);
    p.kq = o; o += al((size_t)nch * m.key_dim * 8);
    p.valid = o; o += al((size_t)nch * 4);
    p.hit = o; o += al((size_t)nch * 4);
    p.cache = o; o += al(out.reals() * rs);
  }
  L.partial = o; o += al((size_t)maxch * SKETCH_BLOCKS * m.key_dim * 8);
  L.built = o; o += al(4);
  L.total = o;
  return L;
}

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

template <typename T>
int apply(lam_plan pl, const lam_memo& m, int o, const void* in, void* out, const void* sub, hipStream_t s) {
  const lam_params& q = plan_params(pl);
  const MemoLayout L = memo_layout(q, m);
  const OpLayout& op = L.op[o];
  unsigned char* w = static_cast<unsigned char*>(m.work);
  View vin, vout;
  int lcb;
  views(q, m, o, vin, vout, lcb);
  const int nch = vin.chunks(), d = m.key_dim;
  unsigned* bits = reinterpret_cast<unsigned*>(w + op.bits);
  double* kc = reinterpret_cast<double*>(w + op.kc);
  double* kq = reinterpret_cast<double*>(w + op.kq);
  int* valid = reinterpret_cast<int*>(w + op.valid);
  int* hit = reinterpret_cast<int*>(w + op.hit);
  T* cache = reinterpret_cast<T*>(w + op.cache);
  double* partial = reinterpret_cast<double*>(w + L.partial);
  hipLaunchKernelGGL(k_memo_sketch<T>, dim3(SKETCH_BLOCKS, nch), dim3(MT), (size_t)d * 8, s, static_cast<const T*>(in),
                     vin, bits, d, partial);
  hipLaunchKernelGGL(k_memo_compare, dim3(nch), dim3(MT), 0, s, partial, d, kq, kc, valid, hit, m.tau,
                     m.counters + 2 * o);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(LAM_ERR_HIP, hipGetErrorString(e));
  const int rc = plan_stage(pl, o, in, out, hit, lcb, s);
  if (rc) return rc;
  const int blocks = (int)std::min<size_t>(1024, (vout.chunk_reals() + MT - 1) / MT);
  hipLaunchKernelGGL(k_memo_commit<T>, dim3(blocks, nch), dim3(MT), 0, s, static_cast<T*>(out), cache,
                     static_cast<const T*>(sub), vout, hit, d, kq, kc, valid);
  e = hipGetLastError();
  return e == hipSuccess ? LAM_OK : set_error(LAM_ERR_HIP, hipGetErrorString(e));
}

}  // namespace

int memo_check(lam_plan p, const lam_memo* m, bool state) {
  if (!m) return set_error(LAM_ERR_ARG, "null memoization state");
  if (state && (!m->work || !m->counters)) return set_error(LAM_ERR_ARG, "null memoization work or counters");
  const lam_params& q = plan_params(p);
  // the chunk views index with shifts
  for (int v : {q.n0, q.n1, q.n2, q.h, q.w})
    if (!pow2_in(v, 1, 1 << 30)) return set_error(LAM_ERR_ARG, "memoization needs power-of-two n0, n1, n2, h, w");
  if (!pow2_in(m->chunk_y, 1, q.n1)) return set_error(LAM_ERR_ARG, "chunk_y must be a power of two in [1, n1]");
  if (!pow2_in(m->chunk_kv, 1, q.h)) return set_error(LAM_ERR_ARG, "chunk_kv must be a power of two in [1, h]");
  if (!pow2_in(m->key_dim, 64, 4096)) return set_error(LAM_ERR_ARG, "key_dim must be a power of two in [64, 4096]");
  if (!(m->tau == m->tau)) return set_error(LAM_ERR_ARG, "tau must not be NaN");
  return LAM_OK;
}

size_t memo_bytes(lam_plan p, const lam_memo* m) { return memo_layout(plan_params(p), *m).total; }

int memo_prepare(lam_plan p, const lam_memo& m, hipStream_t s) {
  const lam_params& q = plan_params(p);
  const MemoLayout L = memo_layout(q, m);
  unsigned char* w = static_cast<unsigned char*>(m.work);
  const int* built = reinterpret_cast<const int*>(w + L.built);
  for (int o = 0; o < 4; ++o) {
    View in, out;
    int lcb;
    views(q, m, o, in, out, lcb);
    const size_t words = (in.reals() + 31) / 32;
    const int blocks = (int)std::min<size_t>(4096, (words + MT - 1) / MT);
    hipLaunchKernelGGL(k_memo_signs, dim3(blocks), dim3(MT), 0, s, in, (unsigned long long)(m.seed + o),
                       reinterpret_cast<unsigned*>(w + L.op[o].bits), built);
  }
  hipLaunchKernelGGL(k_memo_flag, dim3(1), dim3(1), 0, s, reinterpret_cast<int*>(w + L.built));
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LAM_OK : set_error(LAM_ERR_HIP, hipGetErrorString(e));
}

template <typename T>
int memo_apply(lam_plan p, const lam_memo& m, int op, const void* in, void* out, const void* sub, hipStream_t s) {
  return apply<T>(p, m, op, in, out, sub, s);
}
template int memo_apply<float>(lam_plan, const lam_memo&, int, const void*, void*, const void*, hipStream_t);
template int memo_apply<double>(lam_plan, const lam_memo&, int, const void*, void*, const void*, hipStream_t);

}  // namespace lam

extern "C" size_t lam_memo_bytes(lam_plan p, const lam_memo* m) {
  if (!p || !m || lam::memo_check(p, m, false) != LAM_OK) return 0;
  return lam::memo_bytes(p, m);
}
