// Host plan and C ABI of liblam.so (declared in include/lam.h).
//
// lam_init validates the problem statement and builds every table in FP64
// on the host; lam_set_workspace copies them into the caller's device
// workspace; the compute entry points only enqueue kernels on the caller's
// stream.  The 2D step runs over slabs of k_v slices so that the
// oversampled grids never need more than `slab` slices of scratch.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <algorithm>
#include <atomic>
#include <mutex>
#include <utility>
#include <vector>

#include "lam.h"
#include "lam_internal.hpp"
#include "lam_admm.hpp"

using namespace lam;

namespace {

thread_local std::string g_last_error;
std::atomic<unsigned long long> g_next_uid{0};

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }
// a transform length the kernels support: 2^k or 3 2^k, in [lo, hi]
bool is_len_in(int v, int lo, int hi) { return v >= lo && v <= hi && (is_pow2(v) || (v % 3 == 0 && is_pow2(v / 3))); }
int ilog2(long v) { int r = 0; while ((1L << r) < v) ++r; return r; }
size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

constexpr size_t kLdsMax = 160 * 1024;
constexpr size_t kScratchBytes = LAM_SCRATCH_BYTES;
// complex values per thread per FFT stage (as the kernels are built): 16 for complex64, 8 for complex128
int vpt_of(size_t csize) { return csize == 8 ? 16 : 8; }

}  // namespace

// Host buffers of the target-list build (counts and offsets, tile orders).
struct ListHost {
  std::vector<int> cnt, gperm, sperm, work;
};

struct lam_plan_s {
  lam_params p{};
  unsigned long long uid = 0;  // unique per plan (lam_init), names the owner of a device's scratch
  std::vector<double> theta;
  int M0 = 0, M1 = 0, M2 = 0, Ntw = 0, Ntw3 = 0, slab = 0;
  bool sblk = false;           // the workspace holds the spread's per-target block bytes
  double beta = 0;
  size_t csize = 8, rsize = 4;
  // host tables (FP64)
  std::vector<double> tw, tw3, cz, cy, cx, zdelta, cth, sth, rc, line;
  std::vector<int> zbase;
  std::vector<unsigned> zrun;
  // the tables as the device holds them (type per dtype), at their workspace offsets
  std::vector<std::pair<size_t, std::vector<unsigned char>>> blobs;
  // list-build buffers kept for plans that fit the static scratch (their rebuilds allocate nothing)
  ListHost lh;
  // workspace layout (byte offsets)
  size_t off_tw = 0, off_tw3 = 0, off_cz = 0, off_cy = 0, off_cx = 0, off_zbase = 0, off_zdelta = 0, off_cth = 0, off_sth = 0,
         off_rc = 0, off_line = 0, off_zrun = 0, off_tlist = 0, off_toff = 0, off_gperm = 0, off_sperm = 0, off_sblk = 0, off_u1 = 0, off_p = 0, off_t = 0, off_g = 0, ws_need = 0;
  unsigned char* ws = nullptr;
  size_t ws_bytes = 0;
  int ntx = 1, nty = 1;        // tiles of the oversampled grid per slice
  // host streaming (lam_fwd_streamed / lam_adj_streamed)
  int ys = 1, ts = 1;          // volume rows per y-slab, projections per theta-slab
  size_t off_stage = 0, stage_bytes = 0;   // two staging buffers for y-slabs
  hipStream_t copy = nullptr;
  hipEvent_t ev_ready[2] = {nullptr, nullptr}, ev_freed[2] = {nullptr, nullptr}, ev_start = nullptr, ev_done = nullptr;
  Dims D{};
  LaunchCfg cfg{};
  // optional per-kernel timing (lam_profile)
  bool prof_on = false;
  struct Rec { int slot; hipEvent_t a, b; };
  std::vector<hipEvent_t> ev_pool;
  std::vector<Rec> recs;
  ~lam_plan_s() {
    for (auto& r : recs) { ev_pool.push_back(r.a); ev_pool.push_back(r.b); }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : {ev_ready[0], ev_ready[1], ev_freed[0], ev_freed[1], ev_start, ev_done})
      if (e) (void)hipEventDestroy(e);
    // copies of a streamed call may still be in flight on the plan's copy stream
    if (copy) {
      (void)hipStreamSynchronize(copy);
      (void)hipStreamDestroy(copy);
    }
  }
};

namespace {

std::vector<double> deconv(int n, int R, int m) {
  const double M = (double)R * n;
  const double tau = M_PI * m / ((double)n * n * R * (R - 0.5));
  std::vector<double> c(n);
  for (int a = 0; a < n; ++a) {
    const double j = a - n / 2;
    c[a] = std::sqrt(M_PI / tau) * std::exp(tau * j * j) / M;
  }
  return c;
}

// work-group size of an LDS FFT over N points x B transforms: N B / VPT values per thread and stage
// (rounded up to whole waves for lengths 3 2^k), at least one wave
int fft_threads(long N, long B, size_t csize) {
  const long vp = vpt_of(csize);
  return (int)std::max<long>(64, (N * B + vp * 64 - 1) / (vp * 64) * 64);
}

// column blocks of TX <= txmax transforms of length N (TX a power of two dividing ncols)
void col_cfg(long N, int ncols, size_t csize, int& log2TX, int& threads, size_t& lds, int txmax = 16) {
  int TX = txmax;
  const int vp = vpt_of(csize);
  while (TX > 1 && (TX > ncols || ncols % TX || N * TX * (long)csize > 131072 || N * TX / vp > 1024)) TX >>= 1;
  log2TX = ilog2(TX);
  threads = fft_threads(N, TX, csize);
  lds = (size_t)N * TX * csize;
}

void row_cfg(long N, long nrows, size_t csize, int& log2RB, int& threads, size_t& lds) {
  int RB = 16;
  // rows are contiguous in memory, so small row blocks stay coalesced: cap LDS at 32 KB so that
  // several work-groups share a CU and one's loads overlap another's FFT (the row kernels are
  // at most 1024 threads)
  const int vp = vpt_of(csize);
  while (RB > 1 && (RB > nrows || N * RB * (long)csize > 32768 || N * RB / vp > 1024 || nrows % RB)) RB >>= 1;
  log2RB = ilog2(RB);
  threads = fft_threads(N, RB, csize);
  lds = (size_t)N * RB * csize * 9 / 8;     // one pad slot per 8 elements (bank spreading)
}

template <typename T>
std::vector<unsigned char> pack(const std::vector<double>& v) {
  std::vector<unsigned char> out(v.size() * sizeof(T));
  T* o = reinterpret_cast<T*>(out.data());
  for (size_t i = 0; i < v.size(); ++i) o[i] = (T)v[i];
  return out;
}

int build(lam_plan_s* P) {
  const lam_params& p = P->p;
  const int R = p.oversample, m = p.m;
  P->csize = p.dtype == LAM_C64 ? 8 : 16;
  P->rsize = P->csize / 2;
  P->M0 = R * p.n0; P->M1 = R * p.n1; P->M2 = R * p.n2;
  P->beta = M_PI * (R - 0.5) / (R * (double)m);
  // twiddles exp(-2 pi i t / Ntw) in FP64: one table for the power-of-two transform lengths (Ntw the
  // largest of them, at least 8) and one for the lengths 3 2^k (Ntw3 the largest, 0: none)
  P->Ntw = 8;
  P->Ntw3 = 0;
  for (int N : {P->M0, P->M1, P->M2, p.h, p.w}) {
    if (is_pow2(N)) P->Ntw = std::max(P->Ntw, N);
    else P->Ntw3 = std::max(P->Ntw3, N);
  }
  auto twiddles = [](int n, std::vector<double>& tw) {
    tw.resize(2 * (size_t)n);
    for (int t = 0; t < n; ++t) {
      const double a = 2.0 * M_PI * (double)t / (double)n;
      tw[2 * (size_t)t] = std::cos(a);
      tw[2 * (size_t)t + 1] = -std::sin(a);
    }
  };
  twiddles(P->Ntw, P->tw);
  twiddles(P->Ntw3, P->tw3);
  P->cz = deconv(p.n0, R, m);
  P->cy = deconv(p.n1, R, m);
  P->cx = deconv(p.n2, R, m);
  // z-gather: targets xi_z = n0 (k_v / h) cos(phi), s = R xi_z; per detector row the stencil base
  // floor(s) and the fractional offset (the kernels evaluate the weights from it)
  P->zbase.resize(p.h);
  P->zdelta.resize(p.h);
  for (int av = 0; av < p.h; ++av) {
    const double kv = (double)(av - p.h / 2) / (double)p.h;
    const double s = R * (p.n0 * (kv * std::cos(p.phi)));
    const double b = std::floor(s);
    P->zbase[av] = (int)b;
    P->zdelta[av] = s - b;
  }
  // inverse z map for the adjoint's gather form: for each oversampled grid point q, the detector
  // rows whose stencil covers q.  The bases grow with the row, so these rows form one run (two when
  // the stencils of the first rows wrap around the periodic grid); packed as start | count << 16.
  {
    std::vector<std::vector<int>> rows(P->M0);
    for (int av = 0; av < p.h; ++av)
      for (int i = 0; i < 2 * m; ++i) rows[(P->zbase[av] - m + 1 + i + 2 * P->M0) % P->M0].push_back(av);
    P->zrun.assign(2 * (size_t)P->M0, 0u);
    for (int q = 0; q < P->M0; ++q) {
      std::vector<int>& r = rows[q];
      std::sort(r.begin(), r.end());
      int nrun = 0;
      for (size_t a = 0; a < r.size();) {
        size_t e = a + 1;
        while (e < r.size() && r[e] == r[e - 1] + 1) ++e;
        if (nrun == 2) return fail(LAM_ERR_ARG, "z stencil map has more than two runs per grid point");
        P->zrun[2 * (size_t)q + nrun++] = (unsigned)r[a] | ((unsigned)(e - a) << 16);
        a = e;
      }
    }
  }
  P->cth.resize(p.ntheta);
  P->sth.resize(p.ntheta);
  for (int t = 0; t < p.ntheta; ++t) {
    P->cth[t] = std::cos(P->theta[t]);
    P->sth[t] = std::sin(P->theta[t]);
  }
  // per-angle line parameters of the 2D targets: s_x = A_x k_u + C_x (k_v/h), s_y = A_y k_u + C_y (k_v/h),
  // k_u, k_v centred integers; used only to bound the candidate k_u range of a tile
  P->line.assign(6 * (size_t)p.ntheta, 0.0);
  for (int t = 0; t < p.ntheta; ++t) {
    const double sphi = std::sin(p.phi);
    const double Ax = R * (double)p.n2 * P->cth[t] / p.w, Ay = R * (double)p.n1 * P->sth[t] / p.w;
    double* l = &P->line[6 * (size_t)t];
    l[0] = Ax; l[1] = std::fabs(Ax) < 1e-8 ? 0.0 : 1.0 / Ax; l[2] = R * (double)p.n2 * sphi * P->sth[t];
    l[3] = Ay; l[4] = std::fabs(Ay) < 1e-8 ? 0.0 : 1.0 / Ay; l[5] = -R * (double)p.n1 * sphi * P->cth[t];
  }
  P->rc.assign(16, 0.0);
  for (int i = 0; i < 2 * m - 1; ++i) {
    const double o = (double)(i - m + 1);
    P->rc[i] = std::exp(-P->beta * (2.0 * o + 1.0));
  }
  // slab: k_v slices per pass of the 2D step; automatic: the largest power of two whose grids (T and G)
  // take at most 2 GiB (128 slices at 512^3 complex64, 16 at 1536^3: launches of ten to thirty thousand
  // work-groups, whose tails cost ~1 % of the pair against 1 GiB slabs)
  const size_t per_slice = ((size_t)P->M1 * p.n2 + (size_t)P->M1 * P->M2) * P->csize;
  int S = p.slab;
  if (S <= 0) {
    S = 1;
    while (S * 2 <= p.h && per_slice * S * 2 <= ((size_t)2 << 30)) S *= 2;
  }
  if (S > p.h) S = p.h;
  P->slab = S;
  // workspace layout
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + bytes); return at; };
  P->off_tw = take((size_t)P->Ntw * P->csize);
  P->off_tw3 = take((size_t)P->Ntw3 * P->csize);
  P->off_cz = take((size_t)p.n0 * P->rsize);
  P->off_cy = take((size_t)p.n1 * P->rsize);
  P->off_cx = take((size_t)p.n2 * P->rsize);
  P->off_zbase = take((size_t)p.h * sizeof(int));
  P->off_zdelta = take((size_t)p.h * P->rsize);
  P->off_cth = take((size_t)p.ntheta * sizeof(double));
  P->off_sth = take((size_t)p.ntheta * sizeof(double));
  P->off_rc = take(16 * sizeof(double));
  P->off_line = take(6 * (size_t)p.ntheta * sizeof(double));
  P->off_zrun = take(2 * (size_t)P->M0 * sizeof(unsigned));
  // per-slice target lists of the tiles (built on the device by lam_set_workspace); tiles of TS x TS,
  // TS the largest power of two up to 64 that divides both grid periods
  int TS = 64;
  while (P->M1 % TS || P->M2 % TS) TS >>= 1;
  P->ntx = P->M2 / TS;
  P->nty = P->M1 / TS;
  P->off_tlist = take((size_t)p.h * p.ntheta * p.w * sizeof(int));
  P->off_toff = take((size_t)p.h * ((size_t)P->ntx * P->nty * 9 + 1) * sizeof(int));
  P->off_gperm = take((size_t)p.h * P->ntx * P->nty * sizeof(int));
  P->off_sperm = take((size_t)p.h * P->ntx * P->nty * sizeof(int));
  // the complex64 fixed-point spread (64 x 64 tiles on grids of at least 128 x 128, m <= 4) reads one
  // byte per target: its stencil base's 8 x 8 block within its own tile
  P->sblk = p.dtype == LAM_C64 && TS == 64 && P->M1 >= 128 && P->M2 >= 128 && m <= 4;
  P->off_sblk = P->sblk ? take((size_t)p.h * p.ntheta * p.w) : 0;
  P->off_u1 = take((size_t)p.h * p.n1 * p.n2 * P->csize);
  P->off_p = take((size_t)p.ntheta * p.h * p.w * P->csize);
  P->off_t = take((size_t)S * P->M1 * p.n2 * P->csize);
  P->off_g = take((size_t)S * P->M1 * P->M2 * P->csize);
  // host streaming: y-slabs of the volume (real or complex) through two staging buffers of
  // about 64 MiB; theta-slabs of the data go straight to / from the resident data buffer
  {
    const size_t row = (size_t)p.n0 * p.n2 * P->csize;          // one volume row (all z, all x)
    P->ys = (int)std::max<size_t>(1, std::min<size_t>(p.n1, ((size_t)64 << 20) / row));
    const size_t proj = (size_t)p.h * p.w * P->csize;
    P->ts = (int)std::max<size_t>(1, std::min<size_t>(p.ntheta, ((size_t)64 << 20) / proj));
    P->stage_bytes = align_up((size_t)P->ys * row);
    P->off_stage = take(2 * P->stage_bytes);
  }
  P->ws_need = o;
  // the tables as the device holds them (FP32 or FP64 per dtype where the kernels read T)
  {
    const bool f = p.dtype == LAM_C64;
    auto real = [&](const std::vector<double>& v) { return f ? pack<float>(v) : pack<double>(v); };
    auto ints = [](const void* src, size_t bytes) {
      std::vector<unsigned char> b(bytes);
      std::memcpy(b.data(), src, bytes);
      return b;
    };
    P->blobs.clear();
    P->blobs.emplace_back(P->off_tw, real(P->tw));
    if (P->Ntw3) P->blobs.emplace_back(P->off_tw3, real(P->tw3));
    P->blobs.emplace_back(P->off_cz, real(P->cz));
    P->blobs.emplace_back(P->off_cy, real(P->cy));
    P->blobs.emplace_back(P->off_cx, real(P->cx));
    P->blobs.emplace_back(P->off_zdelta, real(P->zdelta));
    P->blobs.emplace_back(P->off_cth, pack<double>(P->cth));
    P->blobs.emplace_back(P->off_sth, pack<double>(P->sth));
    P->blobs.emplace_back(P->off_rc, pack<double>(P->rc));
    P->blobs.emplace_back(P->off_line, pack<double>(P->line));
    P->blobs.emplace_back(P->off_zbase, ints(P->zbase.data(), P->zbase.size() * sizeof(int)));
    P->blobs.emplace_back(P->off_zrun, ints(P->zrun.data(), P->zrun.size() * sizeof(unsigned)));
  }
  // plans that fit the static scratch keep their list-build buffers, so that rebuilding the
  // lists there (lam_fwd_scratch) allocates nothing
  if (P->off_stage <= kScratchBytes) {
    const size_t ntiles = (size_t)P->ntx * P->nty;
    P->lh.cnt.resize((size_t)p.h * (ntiles * 9 + 1));
    P->lh.gperm.resize((size_t)p.h * ntiles);
    P->lh.sperm.resize((size_t)p.h * ntiles);
    P->lh.work.resize(ntiles);
  }
  // kernel dimensions
  Dims& D = P->D;
  D.n0 = p.n0; D.n1 = p.n1; D.n2 = p.n2; D.h = p.h; D.w = p.w; D.ntheta = p.ntheta; D.m = m;
  D.M0 = P->M0; D.M1 = P->M1; D.M2 = P->M2;
  D.lM0 = __builtin_ctz((unsigned)P->M0); D.lM1 = __builtin_ctz((unsigned)P->M1); D.lM2 = __builtin_ctz((unsigned)P->M2);
  D.beta = P->beta;
  D.xy.Rn2 = (double)R * p.n2;
  D.xy.Rn1 = (double)R * p.n1;
  D.xy.inv_w = 1.0 / p.w;
  D.xy.inv_h = 1.0 / p.h;
  D.xy.sphi = std::sin(p.phi);
  D.xy.w = p.w;
  D.xy.h = p.h;
  // launch shapes
  LaunchCfg& c = P->cfg;
  // z and y steps: at most 8 columns per block, so that two blocks share a CU (one loads while the
  // other runs its FFT); with the XCD-aware block order the 64-byte row pieces of neighbouring blocks
  // meet in one L2 (measured at 512^3: z steps 2.64 -> 2.38 ms, y steps 2.05 -> 1.93 ms per pair)
  col_cfg(P->M0, p.n2, P->csize, c.z_log2TX, c.z_threads, c.z_lds, 8);
  // the z adjoint stages h samples per column in the same LDS, and both z kernels stage the per-row
  // bases and offsets and the inverse runs after it: shrink the tile until everything fits
  const size_t z_tables = (size_t)p.h * (sizeof(int) + P->rsize) + 2 * (size_t)P->M0 * sizeof(unsigned);
  while (c.z_log2TX > 0 && ((size_t)std::max(P->M0, p.h) * ((size_t)1 << c.z_log2TX) * P->csize > 131072 ||
                            (size_t)std::max(P->M0, p.h) * ((size_t)1 << c.z_log2TX) * P->csize + z_tables > kLdsMax)) {
    --c.z_log2TX;
    c.z_threads = fft_threads(P->M0, 1L << c.z_log2TX, P->csize);
  }
  c.z_lds = (size_t)std::max(P->M0, p.h) * ((size_t)1 << c.z_log2TX) * P->csize + z_tables;
  if (c.z_lds > kLdsMax) return fail(LAM_ERR_ARG, "z kernels do not fit the LDS");
  col_cfg(P->M1, p.n2, P->csize, c.y_log2TX, c.y_threads, c.y_lds, 8);
  // y kernels whose columns each fit one wave hold them column-major with a skewed pitch of
  // N + N/8 + 1 elements (one pad slot per 8, plus one)
  c.y_lds = std::max(c.y_lds, ((size_t)1 << c.y_log2TX) * ((size_t)P->M1 + P->M1 / 8 + 1) * P->csize);
  row_cfg(P->M2, (long)S * P->M1, P->csize, c.x_log2RB, c.x_threads, c.x_lds);
  row_cfg(p.w, p.h, P->csize, c.r_log2RB, c.r_threads, c.r_lds);
  col_cfg(p.h, p.w, P->csize, c.c_log2TX, c.c_threads, c.c_lds);
  c.c_lds = std::max(c.c_lds, ((size_t)1 << c.c_log2TX) * ((size_t)p.h + p.h / 8 + 1) * P->csize);
  c.g_log2TS = ilog2(TS);
  // gather: the tile plus its (2m-1) halo; scatter: two FP64 planes of the tile (pitch TS + 8)
  const size_t Pt = TS + 2 * m - 1;
  c.g_threads = 256;
  c.g_lds = (Pt * Pt + (Pt * Pt & 1)) * P->csize;
  c.s_threads = 512;
  c.s_lds = 2 * (size_t)TS * (TS + 8) * sizeof(double);
  if (c.g_lds > kLdsMax || c.s_lds > kLdsMax) return fail(LAM_ERR_ARG, "tile kernels do not fit the LDS");
  return LAM_OK;
}

template <typename T>
Tables<T> tables(const lam_plan_s* P, const unsigned char* w) {
  Tables<T> t;
  t.tw = reinterpret_cast<const cpx<T>*>(w + P->off_tw);
  t.log2tw = ilog2(P->Ntw);
  t.tw3 = P->Ntw3 ? reinterpret_cast<const cpx<T>*>(w + P->off_tw3) : nullptr;
  t.log2tw3 = P->Ntw3 ? ilog2(P->Ntw3 / 3) : 0;
  t.cz = reinterpret_cast<const T*>(w + P->off_cz);
  t.cy = reinterpret_cast<const T*>(w + P->off_cy);
  t.cx = reinterpret_cast<const T*>(w + P->off_cx);
  t.zbase = reinterpret_cast<const int*>(w + P->off_zbase);
  t.zdelta = reinterpret_cast<const T*>(w + P->off_zdelta);
  t.cth = reinterpret_cast<const double*>(w + P->off_cth);
  t.sth = reinterpret_cast<const double*>(w + P->off_sth);
  t.rc = reinterpret_cast<const double*>(w + P->off_rc);
  t.line = reinterpret_cast<const double*>(w + P->off_line);
  t.tlist = reinterpret_cast<const int*>(w + P->off_tlist);
  t.toff = reinterpret_cast<const int*>(w + P->off_toff);
  t.gperm = reinterpret_cast<const int*>(w + P->off_gperm);
  t.sperm = reinterpret_cast<const int*>(w + P->off_sperm);
  t.sblk = P->sblk ? w + P->off_sblk : nullptr;
  t.zrun = reinterpret_cast<const unsigned*>(w + P->off_zrun);
  return t;
}
template <typename T>
Tables<T> tables(const lam_plan_s* P) { return tables<T>(P, P->ws); }

// Sort every slice's targets into per-tile lists on the device (once per
// workspace): count per (slice, tile, border class), exclusive scan on the
// host with the invariant that each slice lists exactly n_theta w targets,
// then fill.  Runs on the null stream and waits for it.  ws: the device base
// holding the plan's layout; lh: host buffers (sized here on first use).
template <typename T>
int build_lists(lam_plan_s* P, unsigned char* ws, ListHost& lh);

int hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return LAM_OK;
  return fail(LAM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int check_ready(const lam_plan_s* P) {
  if (!P) return fail(LAM_ERR_ARG, "null plan");
  if (!P->ws) return fail(LAM_ERR_WORKSPACE, "no workspace set (call lam_set_workspace)");
  return LAM_OK;
}

enum { K_ZFWD, K_YCOL_FWD, K_XROW_FWD, K_GATHER, K_ROWFFT, K_COLFFT, K_SCATTER, K_XROW_ADJ, K_YCOL_ADJ, K_ZADJ };
const char* const kKernelNames[LAM_NUM_KERNELS] = {"zfwd", "ycol_fwd", "xrow_fwd", "gather", "rowfft",
                                                  "colfft", "scatter", "xrow_adj", "ycol_adj", "zadj"};

hipEvent_t take_event(lam_plan_s* P) {
  if (!P->ev_pool.empty()) { hipEvent_t e = P->ev_pool.back(); P->ev_pool.pop_back(); return e; }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch one kernel; with profiling on, bracket it with events on its stream.
template <class F>
int timed(lam_plan_s* P, int slot, hipStream_t s, const char* what, F&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (P->prof_on) {
    a = take_event(P);
    b = take_event(P);
    if (!a || !b || hipEventRecord(a, s) != hipSuccess) return fail(LAM_ERR_HIP, "profiling event");
  }
  const hipError_t e = launch();
  if (P->prof_on) {
    if (hipEventRecord(b, s) != hipSuccess) return fail(LAM_ERR_HIP, "profiling event");
    P->recs.push_back({slot, a, b});
  }
  return hip_status(e, what);
}

double inv_hw(const lam_plan_s* P) { return 1.0 / ((double)P->p.h * (double)P->p.w); }

template <typename T>
int build_lists(lam_plan_s* P, unsigned char* ws, ListHost& lh) {
  const Tables<T> tb = tables<T>(P, ws);
  int* toff = reinterpret_cast<int*>(ws + P->off_toff);
  int* tlist = reinterpret_cast<int*>(ws + P->off_tlist);
  const size_t per_slice = (size_t)P->ntx * P->nty * 9 + 1;
  const int h = P->p.h;
  const int chunk = 256;   // slices per launch
  for (int k0 = 0; k0 < h; k0 += chunk) {
    const int rc = hip_status(launch_list_count<T>(P->cfg, k0, std::min(chunk, h - k0), P->D, tb, toff, nullptr),
                              "target count");
    if (rc) return rc;
  }
  const int ntiles = P->ntx * P->nty;
  lh.cnt.resize((size_t)h * per_slice);
  lh.gperm.resize((size_t)h * ntiles);
  lh.sperm.resize((size_t)h * ntiles);
  lh.work.resize(ntiles);
  std::vector<int>& cnt = lh.cnt;
  hipError_t e = hipMemcpy(cnt.data(), toff, cnt.size() * sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_status(e, "target count copy");
  const long expect = (long)P->p.ntheta * P->p.w;
  for (int k = 0; k < h; ++k) {
    int* c = &cnt[(size_t)k * per_slice];
    long run = 0;
    for (size_t i = 0; i + 1 < per_slice; ++i) { const int v = c[i]; c[i] = (int)run; run += v; }
    c[per_slice - 1] = (int)run;
    if (run != expect)
      return fail(LAM_ERR_STATE, "target lists: slice " + std::to_string(k) + " holds " + std::to_string(run) +
                                     " targets, expected " + std::to_string(expect));
  }
  e = hipMemcpy(toff, cnt.data(), cnt.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_status(e, "target offset copy");
  // per slice, the tiles in decreasing order of work (targets gathered, targets spread): the
  // kernels start the heaviest tiles first so that the dense tiles near the frequency origin do
  // not form the tail of a launch (ties in tile order)
  std::vector<int>& work = lh.work;
  auto heavier = [&](int a, int b) { return work[a] != work[b] ? work[a] > work[b] : a < b; };
  for (int k = 0; k < h; ++k) {
    const int* of = &cnt[(size_t)k * per_slice];
    int* gp = &lh.gperm[(size_t)k * ntiles];
    int* sp = &lh.sperm[(size_t)k * ntiles];
    for (int i = 0; i < ntiles; ++i) {
      gp[i] = sp[i] = i;
      work[i] = of[i * 9 + 9] - of[i * 9];
    }
    std::sort(gp, gp + ntiles, heavier);
    for (int i = 0; i < ntiles; ++i) {
      int b[kSpreadSlots], en[kSpreadSlots];
      spread_ranges(of, P->ntx, P->nty, i / P->ntx, i % P->ntx, b, en);
      work[i] = 0;
      for (int j = 0; j < kSpreadSlots; ++j) work[i] += en[j] - b[j];
    }
    std::sort(sp, sp + ntiles, heavier);
  }
  e = hipMemcpy(ws + P->off_gperm, lh.gperm.data(), lh.gperm.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(ws + P->off_sperm, lh.sperm.data(), lh.sperm.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_status(e, "tile order copy");
  for (int k0 = 0; k0 < h; k0 += chunk) {
    const int rc = hip_status(launch_list_fill<T>(P->cfg, k0, std::min(chunk, h - k0), P->D, tb, toff, tlist, nullptr),
                              "target fill");
    if (rc) return rc;
  }
  // exact check: one bit per target in the (still unused) data buffer, a violation counter after it
  const size_t nbits = (size_t)h * P->p.ntheta * P->p.w, words = (nbits + 31) / 32;
  unsigned* seen = reinterpret_cast<unsigned*>(ws + P->off_p);
  int* bad = reinterpret_cast<int*>(seen + words);
  e = hipMemset(seen, 0, words * sizeof(unsigned) + sizeof(int));
  if (e != hipSuccess) return hip_status(e, "target check clear");
  for (int k0 = 0; k0 < h; k0 += chunk) {
    const int rc = hip_status(launch_list_check<T>(P->cfg, k0, std::min(chunk, h - k0), P->D, tb, seen, bad, nullptr),
                              "target check");
    if (rc) return rc;
  }
  int nbad = 0;
  e = hipMemcpy(&nbad, bad, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_status(e, "target check copy");
  if (nbad)
    return fail(LAM_ERR_STATE, "target lists: " + std::to_string(nbad) +
                                   " entries out of range, misfiled or listed twice");
  if (P->sblk)
    for (int k0 = 0; k0 < h; k0 += chunk) {
      const int rc = hip_status(launch_list_blocks<T>(P->cfg, k0, std::min(chunk, h - k0), P->D, tb,
                                                      ws + P->off_sblk, nullptr),
                                "target blocks");
      if (rc) return rc;
    }
  return hip_status(hipDeviceSynchronize(), "target list build");
}

// Copy the plan's tables to the device base ws (synchronous).
int upload_tables(const lam_plan_s* P, unsigned char* ws) {
  for (auto& b : P->blobs) {
    const hipError_t e = hipMemcpy(ws + b.first, b.second.data(), b.second.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(LAM_ERR_HIP, std::string("table upload: ") + hipGetErrorString(e));
  }
  return LAM_OK;
}

// ---------------------------------------------------------------- operators
// ws: the device base holding the plan's layout (its workspace, or the static scratch)
template <typename T>
int run_fwd(lam_plan_s* P, unsigned char* ws, const void* u, bool real_in, const void* dhat, void* out, bool to_space,
            hipStream_t s) {
  const Tables<T> tb = tables<T>(P, ws);
  const LaunchCfg& c = P->cfg;
  const Dims& D = P->D;
  cpx<T>* U1 = reinterpret_cast<cpx<T>*>(ws + P->off_u1);
  cpx<T>* Tb = reinterpret_cast<cpx<T>*>(ws + P->off_t);
  cpx<T>* Gb = reinterpret_cast<cpx<T>*>(ws + P->off_g);
  cpx<T>* o = reinterpret_cast<cpx<T>*>(out);
  const cpx<T>* dh = reinterpret_cast<const cpx<T>*>(dhat);
  int rc = timed(P, K_ZFWD, s, "F_u1D",
                 [&] { return launch_zfwd<T>(c, u, real_in, U1, 0, P->p.n1, (size_t)P->p.n1 * P->p.n2, D, tb, s); });
  for (int k0 = 0; !rc && k0 < P->p.h; k0 += P->slab) {
    const int ns = std::min(P->slab, P->p.h - k0);
    rc = timed(P, K_YCOL_FWD, s, "F_u2D y-FFT", [&] { return launch_ycol_fwd<T>(c, U1, Tb, k0, ns, D, tb, s); });
    if (!rc) rc = timed(P, K_XROW_FWD, s, "F_u2D x-FFT", [&] { return launch_xrow_fwd<T>(c, Tb, Gb, ns, D, tb, s); });
    if (!rc) rc = timed(P, K_GATHER, s, "F_u2D gather", [&] { return launch_gather<T>(c, Gb, o, dh, k0, ns, D, tb, s); });
  }
  if (!rc && to_space) {
    rc = timed(P, K_ROWFFT, s, "F*_2D rows", [&] { return launch_rowfft<T>(c, o, o, true, P->p.ntheta, D, tb, s); });
    if (!rc)
      rc = timed(P, K_COLFFT, s, "F*_2D columns",
                 [&] { return launch_colfft<T>(c, o, o, true, inv_hw(P), P->p.ntheta, D, tb, s); });
  }
  return rc;
}

template <typename T>
int run_adj(lam_plan_s* P, const void* in, bool from_space, void* u, bool real_out, hipStream_t s) {
  const Tables<T> tb = tables<T>(P);
  const LaunchCfg& c = P->cfg;
  const Dims& D = P->D;
  cpx<T>* U1 = reinterpret_cast<cpx<T>*>(P->ws + P->off_u1);
  cpx<T>* Pb = reinterpret_cast<cpx<T>*>(P->ws + P->off_p);
  cpx<T>* Tb = reinterpret_cast<cpx<T>*>(P->ws + P->off_t);
  cpx<T>* Gb = reinterpret_cast<cpx<T>*>(P->ws + P->off_g);
  const cpx<T>* r = reinterpret_cast<const cpx<T>*>(in);
  int rc = 0;
  if (from_space) {
    rc = timed(P, K_ROWFFT, s, "F_2D rows", [&] { return launch_rowfft<T>(c, r, Pb, false, P->p.ntheta, D, tb, s); });
    if (!rc)
      rc = timed(P, K_COLFFT, s, "F_2D columns",
                 [&] { return launch_colfft<T>(c, Pb, Pb, false, inv_hw(P), P->p.ntheta, D, tb, s); });
    r = Pb;
  }
  for (int k0 = 0; !rc && k0 < P->p.h; k0 += P->slab) {
    const int ns = std::min(P->slab, P->p.h - k0);
    rc = timed(P, K_SCATTER, s, "F*_u2D scatter", [&] { return launch_scatter<T>(c, r, Gb, k0, ns, D, tb, s); });
    if (!rc) rc = timed(P, K_XROW_ADJ, s, "F*_u2D x-FFT", [&] { return launch_xrow_adj<T>(c, Gb, Tb, ns, D, tb, s); });
    if (!rc) rc = timed(P, K_YCOL_ADJ, s, "F*_u2D y-FFT", [&] { return launch_ycol_adj<T>(c, Tb, U1, k0, ns, D, tb, s); });
  }
  if (!rc)
    rc = timed(P, K_ZADJ, s, "F*_u1D",
               [&] { return launch_zadj<T>(c, U1, u, real_out, 0, P->p.n1, (size_t)P->p.n1 * P->p.n2, D, tb, s); });
  return rc;
}

// One stage of L^ / L^* with the chunks whose hit flag is set skipped (memoized LSP): 0 F_u1D of a real
// volume into the u1 buffer; 1 F_u2D of u1 into out (no subtraction); 2 F*_u2D of in into u1; 3 F*_u1D of
// u1 into a real volume.  Chunks of 2^log2chunk volume rows (stages 0, 3) or k_v slices (1, 2).
template <typename T>
int run_stage(lam_plan_s* P, int stage, const void* in, void* out, const int* hit, int log2chunk, hipStream_t s) {
  const Tables<T> tb = tables<T>(P);
  const LaunchCfg& c = P->cfg;
  Dims D = P->D;
  D.skip = SkipMap{hit, log2chunk, 0};
  cpx<T>* U1 = reinterpret_cast<cpx<T>*>(P->ws + P->off_u1);
  cpx<T>* Tb = reinterpret_cast<cpx<T>*>(P->ws + P->off_t);
  cpx<T>* Gb = reinterpret_cast<cpx<T>*>(P->ws + P->off_g);
  const size_t zs = (size_t)P->p.n1 * P->p.n2;
  if (stage == 0)
    return timed(P, K_ZFWD, s, "F_u1D", [&] { return launch_zfwd<T>(c, in, true, U1, 0, P->p.n1, zs, D, tb, s); });
  if (stage == 3)
    return timed(P, K_ZADJ, s, "F*_u1D", [&] { return launch_zadj<T>(c, U1, out, true, 0, P->p.n1, zs, D, tb, s); });
  int rc = 0;
  for (int k0 = 0; !rc && k0 < P->p.h; k0 += P->slab) {
    const int ns = std::min(P->slab, P->p.h - k0);
    D.skip.off = k0;
    if (stage == 1) {
      cpx<T>* o = reinterpret_cast<cpx<T>*>(out);
      rc = timed(P, K_YCOL_FWD, s, "F_u2D y-FFT", [&] { return launch_ycol_fwd<T>(c, U1, Tb, k0, ns, D, tb, s); });
      if (!rc) rc = timed(P, K_XROW_FWD, s, "F_u2D x-FFT", [&] { return launch_xrow_fwd<T>(c, Tb, Gb, ns, D, tb, s); });
      if (!rc)
        rc = timed(P, K_GATHER, s, "F_u2D gather", [&] { return launch_gather<T>(c, Gb, o, nullptr, k0, ns, D, tb, s); });
    } else {
      const cpx<T>* r = reinterpret_cast<const cpx<T>*>(in);
      rc = timed(P, K_SCATTER, s, "F*_u2D scatter", [&] { return launch_scatter<T>(c, r, Gb, k0, ns, D, tb, s); });
      if (!rc) rc = timed(P, K_XROW_ADJ, s, "F*_u2D x-FFT", [&] { return launch_xrow_adj<T>(c, Gb, Tb, ns, D, tb, s); });
      if (!rc) rc = timed(P, K_YCOL_ADJ, s, "F*_u2D y-FFT", [&] { return launch_ycol_adj<T>(c, Tb, U1, k0, ns, D, tb, s); });
    }
  }
  return rc;
}

// d^ = W d: centred forward 2D DFT per projection, unnormalised (Algorithm 2's d^)
template <typename T>
int run_data_hat(lam_plan_s* P, const void* d, void* dhat, hipStream_t s) {
  const Tables<T> tb = tables<T>(P);
  const cpx<T>* in = reinterpret_cast<const cpx<T>*>(d);
  cpx<T>* o = reinterpret_cast<cpx<T>*>(dhat);
  const int nt = P->p.ntheta;
  int rc = timed(P, K_ROWFFT, s, "W rows", [&] { return launch_rowfft<T>(P->cfg, in, o, false, nt, P->D, tb, s); });
  if (!rc)
    rc = timed(P, K_COLFFT, s, "W columns", [&] { return launch_colfft<T>(P->cfg, o, o, false, 1.0, nt, P->D, tb, s); });
  return rc;
}

int stream_setup(lam_plan_s* P) {
  if (P->copy) return LAM_OK;
  hipError_t e = hipStreamCreateWithFlags(&P->copy, hipStreamNonBlocking);
  for (hipEvent_t* ev : {&P->ev_ready[0], &P->ev_ready[1], &P->ev_freed[0], &P->ev_freed[1], &P->ev_start, &P->ev_done})
    if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  return hip_status(e, "stream setup");
}

#define LAM_TRY(expr, what)                           \
  do {                                                \
    const int rc_ = hip_status((expr), what);         \
    if (rc_) return rc_;                              \
  } while (0)

// d_host = L u_host with u and d in pinned host memory: y-slabs of u are
// copied in on the plan's copy stream and consumed by the z step as they
// land (two staging buffers); the 2D step runs on the resident stage
// buffers; each theta-slab of d is copied out as soon as its 2D DFT is done.
template <typename T>
int run_fwd_streamed(lam_plan_s* P, const void* u_host, bool real_in, void* d_host, hipStream_t s) {
  int rc = stream_setup(P);
  if (rc) return rc;
  const Tables<T> tb = tables<T>(P);
  const LaunchCfg& c = P->cfg;
  const Dims& D = P->D;
  const lam_params& p = P->p;
  const size_t es = real_in ? P->rsize : P->csize;
  cpx<T>* U1 = reinterpret_cast<cpx<T>*>(P->ws + P->off_u1);
  cpx<T>* Pb = reinterpret_cast<cpx<T>*>(P->ws + P->off_p);
  cpx<T>* Tb = reinterpret_cast<cpx<T>*>(P->ws + P->off_t);
  cpx<T>* Gb = reinterpret_cast<cpx<T>*>(P->ws + P->off_g);
  unsigned char* stage[2] = {P->ws + P->off_stage, P->ws + P->off_stage + P->stage_bytes};
  LAM_TRY(hipEventRecord(P->ev_start, s), "stream start");
  LAM_TRY(hipStreamWaitEvent(P->copy, P->ev_start, 0), "stream start");
  for (int j = 0, y0 = 0; y0 < p.n1; y0 += P->ys, ++j) {
    const int ny = std::min(P->ys, p.n1 - y0), b = j & 1;
    if (j >= 2) LAM_TRY(hipStreamWaitEvent(P->copy, P->ev_freed[b], 0), "stage reuse");
    LAM_TRY(hipMemcpy2DAsync(stage[b], (size_t)ny * p.n2 * es,
                             static_cast<const unsigned char*>(u_host) + (size_t)y0 * p.n2 * es,
                             (size_t)p.n1 * p.n2 * es, (size_t)ny * p.n2 * es, p.n0, hipMemcpyHostToDevice, P->copy),
            "volume slab copy");
    LAM_TRY(hipEventRecord(P->ev_ready[b], P->copy), "slab ready");
    LAM_TRY(hipStreamWaitEvent(s, P->ev_ready[b], 0), "slab ready");
    rc = timed(P, K_ZFWD, s, "F_u1D slab", [&] {
      return launch_zfwd<T>(c, stage[b], real_in, U1, y0, ny, (size_t)ny * p.n2, D, tb, s);
    });
    if (rc) return rc;
    LAM_TRY(hipEventRecord(P->ev_freed[b], s), "slab done");
  }
  for (int k0 = 0; !rc && k0 < p.h; k0 += P->slab) {
    const int ns = std::min(P->slab, p.h - k0);
    rc = timed(P, K_YCOL_FWD, s, "F_u2D y-FFT", [&] { return launch_ycol_fwd<T>(c, U1, Tb, k0, ns, D, tb, s); });
    if (!rc) rc = timed(P, K_XROW_FWD, s, "F_u2D x-FFT", [&] { return launch_xrow_fwd<T>(c, Tb, Gb, ns, D, tb, s); });
    if (!rc) rc = timed(P, K_GATHER, s, "F_u2D gather", [&] { return launch_gather<T>(c, Gb, Pb, nullptr, k0, ns, D, tb, s); });
  }
  const size_t proj = (size_t)p.h * p.w;
  for (int j = 0, t0 = 0; !rc && t0 < p.ntheta; t0 += P->ts, ++j) {
    const int nt = std::min(P->ts, p.ntheta - t0), b = j & 1;
    cpx<T>* base = Pb + (size_t)t0 * proj;
    rc = timed(P, K_ROWFFT, s, "F*_2D rows", [&] { return launch_rowfft<T>(c, base, base, true, nt, D, tb, s); });
    if (!rc)
      rc = timed(P, K_COLFFT, s, "F*_2D columns",
                 [&] { return launch_colfft<T>(c, base, base, true, inv_hw(P), nt, D, tb, s); });
    if (rc) return rc;
    LAM_TRY(hipEventRecord(P->ev_ready[b], s), "projections ready");
    LAM_TRY(hipStreamWaitEvent(P->copy, P->ev_ready[b], 0), "projections ready");
    LAM_TRY(hipMemcpyAsync(static_cast<unsigned char*>(d_host) + (size_t)t0 * proj * P->csize, base,
                           (size_t)nt * proj * P->csize, hipMemcpyDeviceToHost, P->copy),
            "projection copy");
  }
  if (rc) return rc;
  LAM_TRY(hipEventRecord(P->ev_done, P->copy), "stream done");
  LAM_TRY(hipStreamWaitEvent(s, P->ev_done, 0), "stream done");
  return LAM_OK;
}

// u_host = L* d_host (Re for a real volume), both in pinned host memory: theta-slabs
// of d are copied into the resident data buffer and transformed as they land;
// the z adjoint writes y-slabs into the staging buffers, copied out as they finish.
template <typename T>
int run_adj_streamed(lam_plan_s* P, const void* d_host, void* u_host, bool real_out, hipStream_t s) {
  int rc = stream_setup(P);
  if (rc) return rc;
  const Tables<T> tb = tables<T>(P);
  const LaunchCfg& c = P->cfg;
  const Dims& D = P->D;
  const lam_params& p = P->p;
  const size_t es = real_out ? P->rsize : P->csize;
  cpx<T>* U1 = reinterpret_cast<cpx<T>*>(P->ws + P->off_u1);
  cpx<T>* Pb = reinterpret_cast<cpx<T>*>(P->ws + P->off_p);
  cpx<T>* Tb = reinterpret_cast<cpx<T>*>(P->ws + P->off_t);
  cpx<T>* Gb = reinterpret_cast<cpx<T>*>(P->ws + P->off_g);
  unsigned char* stage[2] = {P->ws + P->off_stage, P->ws + P->off_stage + P->stage_bytes};
  LAM_TRY(hipEventRecord(P->ev_start, s), "stream start");
  LAM_TRY(hipStreamWaitEvent(P->copy, P->ev_start, 0), "stream start");
  const size_t proj = (size_t)p.h * p.w;
  for (int j = 0, t0 = 0; t0 < p.ntheta; t0 += P->ts, ++j) {
    const int nt = std::min(P->ts, p.ntheta - t0), b = j & 1;
    cpx<T>* base = Pb + (size_t)t0 * proj;
    LAM_TRY(hipMemcpyAsync(base, static_cast<const unsigned char*>(d_host) + (size_t)t0 * proj * P->csize,
                           (size_t)nt * proj * P->csize, hipMemcpyHostToDevice, P->copy),
            "projection copy");
    LAM_TRY(hipEventRecord(P->ev_ready[b], P->copy), "projections ready");
    LAM_TRY(hipStreamWaitEvent(s, P->ev_ready[b], 0), "projections ready");
    rc = timed(P, K_ROWFFT, s, "F_2D rows", [&] { return launch_rowfft<T>(c, base, base, false, nt, D, tb, s); });
    if (!rc)
      rc = timed(P, K_COLFFT, s, "F_2D columns",
                 [&] { return launch_colfft<T>(c, base, base, false, inv_hw(P), nt, D, tb, s); });
    if (rc) return rc;
  }
  for (int k0 = 0; !rc && k0 < p.h; k0 += P->slab) {
    const int ns = std::min(P->slab, p.h - k0);
    rc = timed(P, K_SCATTER, s, "F*_u2D scatter", [&] { return launch_scatter<T>(c, Pb, Gb, k0, ns, D, tb, s); });
    if (!rc) rc = timed(P, K_XROW_ADJ, s, "F*_u2D x-FFT", [&] { return launch_xrow_adj<T>(c, Gb, Tb, ns, D, tb, s); });
    if (!rc) rc = timed(P, K_YCOL_ADJ, s, "F*_u2D y-FFT", [&] { return launch_ycol_adj<T>(c, Tb, U1, k0, ns, D, tb, s); });
  }
  if (rc) return rc;
  for (int j = 0, y0 = 0; y0 < p.n1; y0 += P->ys, ++j) {
    const int ny = std::min(P->ys, p.n1 - y0), b = j & 1;
    if (j >= 2) LAM_TRY(hipStreamWaitEvent(s, P->ev_freed[b], 0), "stage reuse");
    rc = timed(P, K_ZADJ, s, "F*_u1D slab", [&] {
      return launch_zadj<T>(c, U1, stage[b], real_out, y0, ny, (size_t)ny * p.n2, D, tb, s);
    });
    if (rc) return rc;
    LAM_TRY(hipEventRecord(P->ev_ready[b], s), "slab ready");
    LAM_TRY(hipStreamWaitEvent(P->copy, P->ev_ready[b], 0), "slab ready");
    LAM_TRY(hipMemcpy2DAsync(static_cast<unsigned char*>(u_host) + (size_t)y0 * p.n2 * es, (size_t)p.n1 * p.n2 * es,
                             stage[b], (size_t)ny * p.n2 * es, (size_t)ny * p.n2 * es, p.n0, hipMemcpyDeviceToHost,
                             P->copy),
            "volume slab copy");
    LAM_TRY(hipEventRecord(P->ev_freed[b], P->copy), "slab copied");
  }
  LAM_TRY(hipEventRecord(P->ev_done, P->copy), "stream done");
  LAM_TRY(hipStreamWaitEvent(s, P->ev_done, 0), "stream done");
  return LAM_OK;
}

int fwd_any(lam_plan p, const void* u, bool real_in, const void* dhat, void* out, bool to_space, void* stream) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!u || !out) return fail(LAM_ERR_ARG, "null array pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return p->p.dtype == LAM_C64 ? run_fwd<float>(p, p->ws, u, real_in, dhat, out, to_space, s)
                               : run_fwd<double>(p, p->ws, u, real_in, dhat, out, to_space, s);
}

int adj_any(lam_plan p, const void* in, bool from_space, void* u, bool real_out, void* stream) {
  int rc = check_ready(p);
  if (rc) return rc;
  if (!in || !u) return fail(LAM_ERR_ARG, "null array pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return p->p.dtype == LAM_C64 ? run_adj<float>(p, in, from_space, u, real_out, s)
                               : run_adj<double>(p, in, from_space, u, real_out, s);
}

}  // namespace

// ---------------------------------------------------------------- internal
namespace lam {
// Accessors used by the ADMM step (same library).
void* plan_ws(lam_plan p, size_t* off_p) { *off_p = p->off_p; return p->ws; }
const lam_params& plan_params(lam_plan p) { return p->p; }
int plan_fwd_hat_real(lam_plan p, const void* u, const void* dhat, void* r, hipStream_t s) {
  return fwd_any(p, u, true, dhat, r, false, s);
}
int plan_adj_hat_real(lam_plan p, const void* r, void* u, hipStream_t s) { return adj_any(p, r, false, u, true, s); }
int set_error(int code, const char* msg) { return fail(code, msg); }
void* plan_u1(lam_plan p) { return p->ws + p->off_u1; }
int plan_stage(lam_plan p, int stage, const void* in, void* out, const int* hit, int log2chunk, hipStream_t s) {
  return p->p.dtype == LAM_C64 ? run_stage<float>(p, stage, in, out, hit, log2chunk, s)
                               : run_stage<double>(p, stage, in, out, hit, log2chunk, s);
}
}  // namespace lam

// ---------------------------------------------------------------- static scratch
// Device scratch of lam_fwd_scratch, for callers that cannot allocate: every GPU the library runs
// on holds its own copy until the process ends.  In host code `scratch` is only a stand-in for the
// symbol; its device address comes from hipGetSymbolAddress, once per device, and host code uses
// that address only.  The slot of a device records which plan's tables and lists the array holds.
static __device__ __align__(256) unsigned char scratch[LAM_SCRATCH_BYTES];

namespace {
struct ScratchSlot {
  unsigned char* ptr = nullptr;   // device address of `scratch` on this device
  unsigned long long owner = 0;   // uid of the plan whose tables and lists it holds (0: none)
};
constexpr int kScratchDevices = 64;
ScratchSlot g_scratch_slot[kScratchDevices];
std::mutex g_scratch_mu;
}  // namespace

// ---------------------------------------------------------------- C ABI
extern "C" {

int lam_init(lam_plan* out, const lam_params* p) {
  g_last_error.clear();
  if (!out || !p) return fail(LAM_ERR_ARG, "null argument");
  *out = nullptr;
  const char* bad = nullptr;
  // the caller's dtype field is read as the integer it holds: a C caller may store any int there, and
  // a C++ load of a value outside the enumeration is undefined
  static_assert(sizeof(lam_dtype) == sizeof(int), "lam_dtype is an int-sized enumeration");
  int dtype;
  std::memcpy(&dtype, &p->dtype, sizeof dtype);
  if (!is_len_in(p->n0, 16, 4096) || !is_len_in(p->n1, 16, 4096) || !is_len_in(p->n2, 16, 4096))
    bad = "n0, n1, n2 must be 2^k or 3 2^k in [16, 4096]";
  else if (!is_len_in(p->h, 16, 4096) || !is_len_in(p->w, 16, 4096))
    bad = "h, w must be 2^k or 3 2^k in [16, 4096]";
  else if (p->ntheta < 1 || p->ntheta > 4096) bad = "ntheta must be in [1, 4096]";
  else if (!(p->phi >= 0.0 && p->phi < M_PI / 2)) bad = "phi must be in [0, pi/2)";
  else if (p->oversample != 2) bad = "oversample must be 2";
  else if (p->m < 1 || p->m > 8) bad = "m must be in [1, 8]";
  else if (dtype != LAM_C64 && dtype != LAM_C128) bad = "dtype must be LAM_C64 or LAM_C128";
  else if (p->slab < 0) bad = "slab must be >= 0";
  if (bad) return fail(LAM_ERR_ARG, bad);
  lam_plan_s* P = new (std::nothrow) lam_plan_s();
  if (!P) return fail(LAM_ERR_NOMEM, "plan allocation failed");
  try {
    P->p = *p;
    P->uid = ++g_next_uid;
    P->theta.resize(p->ntheta);
    for (int t = 0; t < p->ntheta; ++t) {
      P->theta[t] = p->theta ? p->theta[t] : 2.0 * M_PI * (double)t / (double)p->ntheta;
      if (!std::isfinite(P->theta[t])) { delete P; return fail(LAM_ERR_ARG, "theta must be finite"); }
    }
    P->p.theta = nullptr;
    const int rc = build(P);
    if (rc) { delete P; return rc; }
  } catch (const std::bad_alloc&) {
    delete P;
    return fail(LAM_ERR_NOMEM, "host table allocation failed");
  }
  *out = P;
  return LAM_OK;
}

size_t lam_workspace_bytes(lam_plan p) { return p ? p->ws_need : 0; }

int lam_set_workspace(lam_plan p, void* dev_ptr, size_t bytes) {
  g_last_error.clear();
  if (!p) return fail(LAM_ERR_ARG, "null plan");
  if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255)) return fail(LAM_ERR_ARG, "workspace must be 256-byte aligned");
  if (bytes < p->ws_need) return fail(LAM_ERR_WORKSPACE, "workspace smaller than lam_workspace_bytes");
  unsigned char* w = static_cast<unsigned char*>(dev_ptr);
  int rc = upload_tables(p, w);
  if (rc) return rc;
  ListHost lh;
  rc = p->p.dtype == LAM_C64 ? build_lists<float>(p, w, lh) : build_lists<double>(p, w, lh);
  if (rc) return rc;
  p->ws = w;
  p->ws_bytes = bytes;
  return LAM_OK;
}

int lam_fwd(lam_plan p, const void* u, void* d, void* s) { g_last_error.clear(); return fwd_any(p, u, false, nullptr, d, true, s); }
int lam_adj(lam_plan p, const void* d, void* u, void* s) { g_last_error.clear(); return adj_any(p, d, true, u, false, s); }
int lam_fwd_real(lam_plan p, const void* u, void* d, void* s) { g_last_error.clear(); return fwd_any(p, u, true, nullptr, d, true, s); }
int lam_adj_real(lam_plan p, const void* d, void* u, void* s) { g_last_error.clear(); return adj_any(p, d, true, u, true, s); }
int lam_fwd_hat(lam_plan p, const void* u, const void* dhat, void* r, void* s) {
  g_last_error.clear();
  return fwd_any(p, u, false, dhat, r, false, s);
}
int lam_adj_hat(lam_plan p, const void* r, void* u, void* s) { g_last_error.clear(); return adj_any(p, r, false, u, false, s); }

int lam_fwd_streamed(lam_plan p, const void* u_host, int u_real, void* d_host, void* stream) {
  g_last_error.clear();
  int rc = check_ready(p);
  if (rc) return rc;
  if (!u_host || !d_host) return fail(LAM_ERR_ARG, "null array pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return p->p.dtype == LAM_C64 ? run_fwd_streamed<float>(p, u_host, u_real != 0, d_host, s)
                               : run_fwd_streamed<double>(p, u_host, u_real != 0, d_host, s);
}

int lam_adj_streamed(lam_plan p, const void* d_host, void* u_host, int u_real, void* stream) {
  g_last_error.clear();
  int rc = check_ready(p);
  if (rc) return rc;
  if (!u_host || !d_host) return fail(LAM_ERR_ARG, "null array pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return p->p.dtype == LAM_C64 ? run_adj_streamed<float>(p, d_host, u_host, u_real != 0, s)
                               : run_adj_streamed<double>(p, d_host, u_host, u_real != 0, s);
}

int lam_stream_slabs(lam_plan p, int y_rows, int theta_proj) {
  if (!p) return fail(LAM_ERR_ARG, "null plan");
  const size_t row = (size_t)p->p.n0 * p->p.n2 * p->csize;
  if (y_rows < 1 || y_rows > p->p.n1 || (size_t)y_rows * row > p->stage_bytes)
    return fail(LAM_ERR_ARG, "y_rows must be in [1, n1] and fit the staging buffers");
  if (theta_proj < 1 || theta_proj > p->p.ntheta) return fail(LAM_ERR_ARG, "theta_proj must be in [1, ntheta]");
  p->ys = y_rows;
  p->ts = theta_proj;
  return LAM_OK;
}

int lam_data_hat(lam_plan p, const void* d, void* dhat, void* stream) {
  g_last_error.clear();
  int rc = check_ready(p);
  if (rc) return rc;
  if (!d || !dhat) return fail(LAM_ERR_ARG, "null array pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return p->p.dtype == LAM_C64 ? run_data_hat<float>(p, d, dhat, s) : run_data_hat<double>(p, d, dhat, s);
}

int lam_fwd_scratch(lam_plan p, const void* u, void* d, void* stream) {
  g_last_error.clear();
  if (!p) return fail(LAM_ERR_ARG, "null plan");
  if (!u || !d) return fail(LAM_ERR_ARG, "null array pointer");
  if (p->off_stage > kScratchBytes)
    return fail(LAM_ERR_WORKSPACE, "the plan needs " + std::to_string(p->off_stage) +
                                       " bytes of scratch, the static scratch holds " + std::to_string(kScratchBytes));
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "device query");
  if (dev < 0 || dev >= kScratchDevices) return fail(LAM_ERR_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  ScratchSlot& sl = g_scratch_slot[dev];
  if (!sl.ptr) {
    // the array's device address on this device (each device holds its own copy)
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_status(e, "scratch address");
    sl.ptr = static_cast<unsigned char*>(ptr);
  }
  if (sl.owner != p->uid) {
    // another plan's tables (or none) are in this device's scratch: let the device's pending work
    // finish, then build this plan's tables and target lists there
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_status(e, "scratch handover");
    sl.owner = 0;
    int rc = upload_tables(p, sl.ptr);
    if (!rc) rc = p->p.dtype == LAM_C64 ? build_lists<float>(p, sl.ptr, p->lh) : build_lists<double>(p, sl.ptr, p->lh);
    if (rc) return rc;
    sl.owner = p->uid;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return p->p.dtype == LAM_C64 ? run_fwd<float>(p, sl.ptr, u, false, nullptr, d, true, s)
                               : run_fwd<double>(p, sl.ptr, u, false, nullptr, d, true, s);
}

int lam_profile(lam_plan p, int on) {
  if (!p) return fail(LAM_ERR_ARG, "null plan");
  p->prof_on = on != 0;
  return LAM_OK;
}

int lam_profile_read(lam_plan p, double* total_ms, long long* launches) {
  if (!p || !total_ms || !launches) return fail(LAM_ERR_ARG, "null argument");
  for (int k = 0; k < LAM_NUM_KERNELS; ++k) { total_ms[k] = 0.0; launches[k] = 0; }
  int rc = LAM_OK;
  for (auto& r : p->recs) {
    float ms = 0.f;
    if (rc == LAM_OK) {
      hipError_t e = hipEventSynchronize(r.b);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
      if (e != hipSuccess) rc = fail(LAM_ERR_HIP, std::string("profile read: ") + hipGetErrorString(e));
    }
    total_ms[r.slot] += ms;
    launches[r.slot] += 1;
    p->ev_pool.push_back(r.a);
    p->ev_pool.push_back(r.b);
  }
  p->recs.clear();
  return rc;
}

const char* lam_kernel_name(int k) { return (k >= 0 && k < LAM_NUM_KERNELS) ? kKernelNames[k] : ""; }

void lam_destroy(lam_plan p) { delete p; }

const char* lam_error_string(int code) {
  switch (code) {
    case LAM_OK: return "success";
    case LAM_ERR_ARG: return "invalid argument";
    case LAM_ERR_NOMEM: return "out of host memory";
    case LAM_ERR_HIP: return "HIP runtime error";
    case LAM_ERR_WORKSPACE: return "workspace missing or too small";
    case LAM_ERR_STATE: return "invalid state";
    default: return "unknown status";
  }
}

const char* lam_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
