// One ADMM-TV iteration on the device (Section 2, Equation 1, Algorithm 2).
//
// LSP: n_inner conjugate-gradient steps on
//     f(u) = 1/2 |L^ u - d^|^2 / (h w) + rho/2 |grad u - g|^2,  g = psi - lambda/rho,
// in the cancelled frequency domain: the residual r = L^ u - d^ comes from
// F_u2D's gather with the subtraction fused, and is then updated as
// r += gamma L^ p, so each step costs one L^ and one L^*.  Directions are
// Fletcher-Reeves, the step is the exact line search of the quadratic.  All
// inner products are accumulated in FP64 and every scalar (beta, gamma, rho)
// stays in device memory: the host never synchronises.
// RSP: isotropic TV shrink of grad u + lambda/rho, multiplier update, and
// residual-balanced penalty update (factor 2 when one residual exceeds ten
// times the other).
// grad is the forward difference along z, y, x with the last difference on
// each axis set to 0; grad^T is its exact adjoint.
#include <algorithm>

#include "lam_admm.hpp"
#include "lam_internal.hpp"
#include "lam_memo.hpp"

namespace lam {
namespace {

constexpr int NB = 1024;   // blocks of every reduction kernel
constexpr int NT = 256;    // threads per block

// device scalars in the work buffer
enum { S_GG = 0, S_GGPREV, S_GP, S_BETA, S_GAMMA, S_COUNT = 16 };
// user scalars (lam_admm_state::scal)
enum { U_RHO = 0, U_ALPHA, U_GAMMA, U_PRIMAL, U_DUAL, U_GNORM, U_RHO_USED, U_SPARE };

struct Vol {
  int n0, n1, n2;
  size_t V, plane;
};

__device__ __forceinline__ void block_sum_to(double v, double* out) {
  __shared__ double sh[NT / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int w = 0; w < NT / 64; ++w) s += sh[w];
    *out = s;
  }
}

__device__ __forceinline__ void coords(const Vol& v, size_t i, int& z, int& y, int& x) {
  z = (int)(i / v.plane);
  const size_t r = i - (size_t)z * v.plane;
  y = (int)(r / v.n2);
  x = (int)(r - (size_t)y * v.n2);
}

// G = G / (h w) + rho grad^T(grad u - psi + lambda/rho);  part <- sum G^2
template <typename T>
__global__ __launch_bounds__(NT) void k_tv_grad(T* __restrict__ G, const T* __restrict__ u, const T* __restrict__ psi,
                                                const T* __restrict__ mult, const double* __restrict__ user,
                                                double inv_hw, Vol v, double* __restrict__ part) {
  const double rho = user[U_RHO];
  const T r = (T)rho, ir = (T)(1.0 / rho);
  const size_t st[3] = {v.plane, (size_t)v.n2, 1};
  const int nn[3] = {v.n0, v.n1, v.n2};
  double acc = 0;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < v.V; i += (size_t)NB * NT) {
    int c[3];
    coords(v, i, c[0], c[1], c[2]);
    const T ui = u[i];
    T div = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T* pa = psi + a * v.V;
      const T* la = mult + a * v.V;
      if (c[a] <= nn[a] - 2) div -= (u[i + st[a]] - ui) - pa[i] + la[i] * ir;
      if (c[a] >= 1) {
        const size_t j = i - st[a];
        div += (ui - u[j]) - pa[j] + la[j] * ir;
      }
    }
    const T g = (T)((double)G[i] * inv_hw) + r * div;
    G[i] = g;
    acc += (double)g * (double)g;
  }
  block_sum_to(acc, part + blockIdx.x);
}

// p = -G + beta p (beta = 0 on the first step);  part <- sum G p
template <typename T>
__global__ __launch_bounds__(NT) void k_cg_dir(const T* __restrict__ G, T* __restrict__ p, const double* __restrict__ sc,
                                               size_t V, double* __restrict__ part) {
  const double beta = sc[S_BETA];
  const T b = (T)beta;
  double acc = 0;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < V; i += (size_t)NB * NT) {
    const T g = G[i];
    const T pn = beta == 0.0 ? -g : -g + b * p[i];
    p[i] = pn;
    acc += (double)g * (double)pn;
  }
  block_sum_to(acc, part + blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_norm2_c(const cpx<T>* __restrict__ x, size_t n, double* __restrict__ part) {
  double acc = 0;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < n; i += (size_t)NB * NT) {
    const cpx<T> q = x[i];
    acc += (double)q.x * (double)q.x + (double)q.y * (double)q.y;
  }
  block_sum_to(acc, part + blockIdx.x);
}

// part <- |grad p|^2
template <typename T>
__global__ __launch_bounds__(NT) void k_gradnorm(const T* __restrict__ p, Vol v, double* __restrict__ part) {
  const size_t st[3] = {v.plane, (size_t)v.n2, 1};
  const int nn[3] = {v.n0, v.n1, v.n2};
  double acc = 0;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < v.V; i += (size_t)NB * NT) {
    int c[3];
    coords(v, i, c[0], c[1], c[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (c[a] <= nn[a] - 2) {
        const double d = (double)p[i + st[a]] - (double)p[i];
        acc += d * d;
      }
  }
  block_sum_to(acc, part + blockIdx.x);
}

// u += gamma p ; r += gamma Lp
template <typename T>
__global__ __launch_bounds__(NT) void k_cg_update(T* __restrict__ u, const T* __restrict__ p, cpx<T>* __restrict__ r,
                                                  const cpx<T>* __restrict__ Lp, const double* __restrict__ sc,
                                                  size_t V, size_t P) {
  const T g = (T)sc[S_GAMMA];
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < V; i += (size_t)NB * NT) u[i] += g * p[i];
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < P; i += (size_t)NB * NT) {
    const cpx<T> a = r[i], b = Lp[i];
    r[i] = mk(a.x + g * b.x, a.y + g * b.y);
  }
}

// RSP + multiplier: psi_new = shrink(grad u + lambda/rho, alpha/rho);
// D = psi_new - psi; lambda += rho (grad u - psi_new); part <- |grad u - psi_new|^2
template <typename T>
__global__ __launch_bounds__(NT) void k_rsp(const T* __restrict__ u, T* __restrict__ psi, T* __restrict__ mult,
                                            T* __restrict__ D, const double* __restrict__ user, Vol v,
                                            double* __restrict__ part) {
  const double rho = user[U_RHO], alpha = user[U_ALPHA];
  const T r = (T)rho, ir = (T)(1.0 / rho), th = (T)(alpha / rho);
  const size_t st[3] = {v.plane, (size_t)v.n2, 1};
  const int nn[3] = {v.n0, v.n1, v.n2};
  double acc = 0;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < v.V; i += (size_t)NB * NT) {
    int c[3];
    coords(v, i, c[0], c[1], c[2]);
    T gu[3], z[3];
    T nrm2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      gu[a] = c[a] <= nn[a] - 2 ? u[i + st[a]] - u[i] : (T)0;
      z[a] = gu[a] + mult[a * v.V + i] * ir;
      nrm2 += z[a] * z[a];
    }
    const T nrm = sqrt(nrm2);
    const T scale = nrm > (T)0 ? (T)fmax(0.0, 1.0 - (double)th / (double)nrm) : (T)0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T pn = z[a] * scale;
      const size_t j = a * v.V + i;
      D[j] = pn - psi[j];
      psi[j] = pn;
      const T res = gu[a] - pn;
      mult[j] += r * res;
      acc += (double)res * (double)res;
    }
  }
  block_sum_to(acc, part + blockIdx.x);
}

// part <- |grad^T D|^2
template <typename T>
__global__ __launch_bounds__(NT) void k_divnorm(const T* __restrict__ D, Vol v, double* __restrict__ part) {
  const size_t st[3] = {v.plane, (size_t)v.n2, 1};
  const int nn[3] = {v.n0, v.n1, v.n2};
  double acc = 0;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < v.V; i += (size_t)NB * NT) {
    int c[3];
    coords(v, i, c[0], c[1], c[2]);
    double div = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T* da = D + a * v.V;
      if (c[a] <= nn[a] - 2) div -= (double)da[i];
      if (c[a] >= 1) div += (double)da[i - st[a]];
    }
    acc += div * div;
  }
  block_sum_to(acc, part + blockIdx.x);
}

enum { F_GG, F_GP, F_GAMMA, F_RHO };

// One block: reduce the partial sums and derive the step scalars.
__global__ __launch_bounds__(NT) void k_finish(int mode, int first, const double* __restrict__ part, double* sc,
                                               double* user, double inv_hw) {
  __shared__ double sh[2][NT];
  double a = 0, b = 0;
  for (int i = threadIdx.x; i < NB; i += NT) {
    a += part[i];
    b += part[NB + i];
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double A = 0, B = 0;
  for (int i = 0; i < NT; ++i) { A += sh[0][i]; B += sh[1][i]; }
  const double rho = user[U_RHO];
  if (mode == F_GG) {
    sc[S_BETA] = (first || sc[S_GGPREV] == 0.0) ? 0.0 : A / sc[S_GGPREV];
    sc[S_GG] = A;
    user[U_GNORM] = sqrt(A);
  } else if (mode == F_GP) {
    sc[S_GP] = A;
  } else if (mode == F_GAMMA) {
    const double den = A * inv_hw + rho * B;
    sc[S_GAMMA] = den > 0.0 ? -sc[S_GP] / den : 0.0;
    sc[S_GGPREV] = sc[S_GG];
    user[U_GAMMA] = sc[S_GAMMA];
  } else {
    const double r = sqrt(A), s = rho * sqrt(B);
    user[U_PRIMAL] = r;
    user[U_DUAL] = s;
    user[U_RHO_USED] = rho;
    double nr = rho;
    if (r > 10.0 * s) nr = 2.0 * rho;
    else if (s > 10.0 * r) nr = 0.5 * rho;
    user[U_RHO] = nr;
  }
}

size_t al(size_t v) { return (v + 255) / 256 * 256; }

struct WorkLayout {
  size_t r, lp, g, p, d, part, sc, total;
};

WorkLayout layout(const lam_params& q) {
  const size_t cs = q.dtype == LAM_C64 ? 8 : 16, rs = cs / 2;
  const size_t V = (size_t)q.n0 * q.n1 * q.n2, P = (size_t)q.ntheta * q.h * q.w;
  WorkLayout L{};
  size_t o = 0;
  L.r = o; o += al(P * cs);
  L.lp = o; o += al(P * cs);
  L.g = o; o += al(V * rs);
  L.p = o; o += al(V * rs);
  L.d = o; o += al(3 * V * rs);
  L.part = o; o += al(2 * NB * sizeof(double));
  L.sc = o; o += al(S_COUNT * sizeof(double));
  L.total = o;
  return L;
}

int hip_ok(hipError_t e) { return e == hipSuccess ? LAM_OK : set_error(LAM_ERR_HIP, hipGetErrorString(e)); }

template <typename T>
int step(lam_plan pl, const lam_admm_state* s, const void* dhat, int n_inner, hipStream_t st) {
  const lam_params& q = plan_params(pl);
  const WorkLayout W = layout(q);
  unsigned char* w = static_cast<unsigned char*>(s->work);
  cpx<T>* r = reinterpret_cast<cpx<T>*>(w + W.r);
  cpx<T>* Lp = reinterpret_cast<cpx<T>*>(w + W.lp);
  T* G = reinterpret_cast<T*>(w + W.g);
  T* p = reinterpret_cast<T*>(w + W.p);
  T* D = reinterpret_cast<T*>(w + W.d);
  double* part = reinterpret_cast<double*>(w + W.part);
  double* sc = reinterpret_cast<double*>(w + W.sc);
  T* u = static_cast<T*>(s->u);
  T* psi = static_cast<T*>(s->psi);
  T* mult = static_cast<T*>(s->lam);
  double* user = s->scal;
  Vol v{q.n0, q.n1, q.n2, (size_t)q.n0 * q.n1 * q.n2, (size_t)q.n1 * q.n2};
  const size_t P = (size_t)q.ntheta * q.h * q.w;
  const double inv_hw = 1.0 / ((double)q.h * (double)q.w);
  const dim3 g(NB), b(NT);
  int rc = plan_fwd_hat_real(pl, u, dhat, r, st);                    // r = L^ u - d^ (fused)
  for (int it = 0; !rc && it < n_inner; ++it) {
    rc = plan_adj_hat_real(pl, r, G, st);                            // G = Re L^* r
    if (rc) break;
    hipLaunchKernelGGL(k_tv_grad<T>, g, b, 0, st, G, u, psi, mult, user, inv_hw, v, part);
    hipLaunchKernelGGL(k_finish, dim3(1), b, 0, st, (int)F_GG, it == 0 ? 1 : 0, part, sc, user, inv_hw);
    hipLaunchKernelGGL(k_cg_dir<T>, g, b, 0, st, G, p, sc, v.V, part);
    hipLaunchKernelGGL(k_finish, dim3(1), b, 0, st, (int)F_GP, 0, part, sc, user, inv_hw);
    if ((rc = hip_ok(hipGetLastError()))) break;
    rc = plan_fwd_hat_real(pl, p, nullptr, Lp, st);                  // L^ p
    if (rc) break;
    hipLaunchKernelGGL(k_norm2_c<T>, g, b, 0, st, Lp, P, part);
    hipLaunchKernelGGL(k_gradnorm<T>, g, b, 0, st, p, v, part + NB);
    hipLaunchKernelGGL(k_finish, dim3(1), b, 0, st, (int)F_GAMMA, 0, part, sc, user, inv_hw);
    hipLaunchKernelGGL(k_cg_update<T>, g, b, 0, st, u, p, r, Lp, sc, v.V, P);
    rc = hip_ok(hipGetLastError());
  }
  if (rc) return rc;
  hipLaunchKernelGGL(k_rsp<T>, g, b, 0, st, u, psi, mult, D, user, v, part);
  hipLaunchKernelGGL(k_divnorm<T>, g, b, 0, st, D, v, part + NB);
  hipLaunchKernelGGL(k_finish, dim3(1), b, 0, st, (int)F_RHO, 0, part, sc, user, inv_hw);
  return hip_ok(hipGetLastError());
}

// One ADMM-TV iteration with the LSP's forward and adjoint passes memoized (Section 4.4): every inner
// iteration recomputes the residual r = M_u2D(M_u1D u) - d^ and the gradient
// G = Re M*_u1D(M*_u2D r) / (h w) + rho grad^T(grad u - g) through the memoized operators (Algorithm 2's
// forward and adjoint passes), then takes the Fletcher-Reeves direction p and the exact line search,
// which applies the plain L^ to p.  The RSP, multiplier and penalty updates are those of step().
template <typename T>
int step_memo(lam_plan pl, const lam_admm_state* s, const void* dhat, int n_inner, const lam_memo& m, hipStream_t st) {
  const lam_params& q = plan_params(pl);
  const WorkLayout W = layout(q);
  unsigned char* w = static_cast<unsigned char*>(s->work);
  cpx<T>* r = reinterpret_cast<cpx<T>*>(w + W.r);
  cpx<T>* Lp = reinterpret_cast<cpx<T>*>(w + W.lp);
  T* G = reinterpret_cast<T*>(w + W.g);
  T* p = reinterpret_cast<T*>(w + W.p);
  T* D = reinterpret_cast<T*>(w + W.d);
  double* part = reinterpret_cast<double*>(w + W.part);
  double* sc = reinterpret_cast<double*>(w + W.sc);
  T* u = static_cast<T*>(s->u);
  T* psi = static_cast<T*>(s->psi);
  T* mult = static_cast<T*>(s->lam);
  double* user = s->scal;
  void* U1 = plan_u1(pl);
  Vol v{q.n0, q.n1, q.n2, (size_t)q.n0 * q.n1 * q.n2, (size_t)q.n1 * q.n2};
  const size_t P = (size_t)q.ntheta * q.h * q.w;
  const double inv_hw = 1.0 / ((double)q.h * (double)q.w);
  const dim3 g(NB), b(NT);
  int rc = memo_prepare(pl, m, st);
  for (int it = 0; !rc && it < n_inner; ++it) {
    rc = memo_apply<T>(pl, m, 0, u, U1, nullptr, st);                 // forward pass: F_u1D u
    if (!rc) rc = memo_apply<T>(pl, m, 1, U1, r, dhat, st);           //   r = F_u2D u1 - d^
    if (!rc) rc = memo_apply<T>(pl, m, 2, r, U1, nullptr, st);        // adjoint pass: F*_u2D r
    if (!rc) rc = memo_apply<T>(pl, m, 3, U1, G, nullptr, st);        //   G = Re F*_u1D u1
    if (rc) break;
    hipLaunchKernelGGL(k_tv_grad<T>, g, b, 0, st, G, u, psi, mult, user, inv_hw, v, part);
    hipLaunchKernelGGL(k_finish, dim3(1), b, 0, st, (int)F_GG, it == 0 ? 1 : 0, part, sc, user, inv_hw);
    hipLaunchKernelGGL(k_cg_dir<T>, g, b, 0, st, G, p, sc, v.V, part);
    hipLaunchKernelGGL(k_finish, dim3(1), b, 0, st, (int)F_GP, 0, part, sc, user, inv_hw);
    if ((rc = hip_ok(hipGetLastError()))) break;
    rc = plan_fwd_hat_real(pl, p, nullptr, Lp, st);                  // L^ p (exact line search)
    if (rc) break;
    hipLaunchKernelGGL(k_norm2_c<T>, g, b, 0, st, Lp, P, part);
    hipLaunchKernelGGL(k_gradnorm<T>, g, b, 0, st, p, v, part + NB);
    hipLaunchKernelGGL(k_finish, dim3(1), b, 0, st, (int)F_GAMMA, 0, part, sc, user, inv_hw);
    hipLaunchKernelGGL(k_cg_update<T>, g, b, 0, st, u, p, r, Lp, sc, v.V, (size_t)0);   // u += gamma p
    rc = hip_ok(hipGetLastError());
  }
  if (rc) return rc;
  hipLaunchKernelGGL(k_rsp<T>, g, b, 0, st, u, psi, mult, D, user, v, part);
  hipLaunchKernelGGL(k_divnorm<T>, g, b, 0, st, D, v, part + NB);
  hipLaunchKernelGGL(k_finish, dim3(1), b, 0, st, (int)F_RHO, 0, part, sc, user, inv_hw);
  return hip_ok(hipGetLastError());
}

}  // namespace
}  // namespace lam

extern "C" size_t lam_admm_work_bytes(lam_plan p) { return p ? lam::layout(lam::plan_params(p)).total : 0; }

extern "C" int lam_admm_step(lam_plan p, const lam_admm_state* s, const void* dhat, int n_inner, void* stream) {
  if (!p || !s || !dhat) return lam::set_error(LAM_ERR_ARG, "null argument");
  if (!s->u || !s->psi || !s->lam || !s->work || !s->scal) return lam::set_error(LAM_ERR_ARG, "null state pointer");
  if (n_inner < 1 || n_inner > 1000) return lam::set_error(LAM_ERR_ARG, "n_inner must be in [1, 1000]");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  return lam::plan_params(p).dtype == LAM_C64 ? lam::step<float>(p, s, dhat, n_inner, st)
                                                : lam::step<double>(p, s, dhat, n_inner, st);
}

extern "C" int lam_admm_step_memo(lam_plan p, const lam_admm_state* s, const void* dhat, int n_inner,
                                  const lam_memo* m, void* stream) {
  if (!p || !s || !dhat) return lam::set_error(LAM_ERR_ARG, "null argument");
  if (!s->u || !s->psi || !s->lam || !s->work || !s->scal) return lam::set_error(LAM_ERR_ARG, "null state pointer");
  if (n_inner < 1 || n_inner > 1000) return lam::set_error(LAM_ERR_ARG, "n_inner must be in [1, 1000]");
  int rc = lam::memo_check(p, m, true);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  return lam::plan_params(p).dtype == LAM_C64 ? lam::step_memo<float>(p, s, dhat, n_inner, *m, st)
                                                : lam::step_memo<double>(p, s, dhat, n_inner, *m, st);
}
