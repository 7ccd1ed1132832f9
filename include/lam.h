/*
 * lam.h - C ABI of the MI355X laminography operator library (liblam.so).
 *
 * The library computes the forward laminography operator of ADMM-FFT
 * laminography, L = F*_2D F_u2D F_u1D, and its adjoint
 * L* = F*_u1D F*_u2D F_2D (Section 2, Algorithm 1, forward and adjoint
 * passes), the frequency-domain pair L^ = F_u2D F_u1D / L^* used after the
 * cancellation F_2D F*_2D = I (Section 4.2, Algorithm 2), with the data
 * subtraction fused into F_u2D, and one ADMM-TV iteration built on them
 * (Section 2, Equation 1 and Algorithm 2).
 *
 * Conventions (the paper gives the factorisation and array shapes; the
 * geometry and the unequally-spaced FFT follow the Fourier-slice theorem
 * and Gaussian gridding, Dutt & Rokhlin 1993 / Greengard & Lee 2004):
 *   - u: volume (n0, n1, n2) = (z, y, x), C order, z = rotation axis.  The
 *     paper writes u[n1, n0, n2]; this is the same array with the rotation
 *     axis stored slowest.  Centred indices j in [-n/2, n/2).
 *   - d: projections (ntheta, h, w) = (angle, detector row v, column p).
 *   - theta_t = 2 pi t / ntheta unless an explicit angle list is given.
 *   - Frequency of detector bin (k_v, k_u):
 *       nu = (k_u/w) (cos t, sin t, 0) + (k_v/h) (sin phi sin t, -sin phi cos t, cos phi)
 *     as (x, y, z), cycles per voxel; forward exponent exp(-2 pi i nu.j).
 *   - F*_2D is the centred inverse DFT with 1/(h w); the adjoint's F_2D is
 *     the centred forward DFT with 1/(h w).  L^ carries no normalisation, so
 *     L = W^H L^ / (h w) with W the unnormalised centred 2D DFT.
 *   - USFFT: oversampling R, half-width m (2m taps per axis), M = R n,
 *     tau = pi m / (n^2 R (R - 1/2)), beta = pi (R - 1/2)/(R m),
 *     deconvolution c(j) = sqrt(pi/tau) exp(tau j^2) / M.
 *
 * Memory.  Every array argument is a DEVICE pointer to a contiguous C-order
 * buffer owned by the caller (the host-streamed pair takes host pointers).  Complex arrays are interleaved (re, im):
 * float pairs for LAM_C64, double pairs for LAM_C128.  Real arrays (the
 * *_real entry points and the ADMM state) are float for LAM_C64 and double
 * for LAM_C128.  The library never allocates device memory: scratch space is
 * the caller's workspace (lam_workspace_bytes / lam_set_workspace).
 *
 * Execution.  Every compute call only enqueues kernels on the given HIP
 * stream (a hipStream_t passed as void*, NULL = default stream) and returns;
 * no call synchronises the host.  One call at a time per plan: calls on one
 * plan share its workspace, so calls that overlap in time (different
 * streams, different threads) race.
 *
 * Errors.  Every call returns a lam_status.  Argument errors are reported
 * before anything is enqueued and leave all outputs untouched.  LAM_ERR_HIP
 * means a HIP runtime call failed (no device, launch failure); asynchronous
 * device faults surface at a later call or stream synchronisation.
 * lam_last_error() gives a thread-local text for the last failing call.
 * NaN or Inf inputs are not checked: they propagate to the outputs.
 */
#ifndef LAM_H
#define LAM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lam_plan_s* lam_plan;

typedef enum { LAM_C64 = 0, LAM_C128 = 1 } lam_dtype;

typedef enum {
  LAM_OK = 0,
  LAM_ERR_ARG = 1,        /* invalid argument or unsupported size           */
  LAM_ERR_NOMEM = 2,      /* host allocation failed                          */
  LAM_ERR_HIP = 3,        /* a HIP runtime call failed                       */
  LAM_ERR_WORKSPACE = 4,  /* no workspace set, or the one given is too small */
  LAM_ERR_STATE = 5       /* call not valid in the plan's current state      */
} lam_status;

/* Problem statement (Section 2: volume n0 x n1 x n2, ntheta projection
 * angles, detector h x w; plus tilt, oversampling and kernel half-width). */
typedef struct {
  int n0, n1, n2;        /* volume (z, y, x); each 2^k or 3 2^k, 16 .. 4096 (the
                            transforms of 3 2^k points take a radix-3 stage)        */
  int ntheta;            /* number of projection angles, 1 .. 4096                  */
  const double* theta;   /* host array [ntheta] in radians, or NULL: 2 pi t/ntheta  */
  double phi;            /* tilt of the rotation axis from the tomographic
                            position, radians, 0 <= phi < pi/2 (phi = 0: tomography) */
  int h, w;              /* detector rows (k_v) and columns (k_u); each 2^k or
                            3 2^k, 16 .. 4096                                       */
  int oversample;        /* R; must be 2                                            */
  int m;                 /* Gaussian half-width, 1 .. 8 (2m taps per axis)          */
  lam_dtype dtype;       /* LAM_C64: complex64 data, FP32 arithmetic, FP64
                            coordinates, FP64 tables, 2D stencil weights as FP32
                            exponentials; LAM_C128: complex128 throughout          */
  int slab;              /* k_v slices per internal slab of the 2D step; 0 = auto.
                            Bounds the oversampled-grid scratch to slab slices.     */
} lam_params;

/* Validate the parameters and build the plan's FP64 tables on the host
 * (angles, deconvolution factors, z-gather bases and weights, twiddles).
 * Touches no device.  *out receives the plan; lam_destroy releases it.
 * Errors: LAM_ERR_ARG (null pointers, sizes outside the ranges above, R != 2,
 * m outside 1..8, phi outside [0, pi/2), theta non-finite), LAM_ERR_NOMEM. */
int lam_init(lam_plan* out, const lam_params* p);

/* Bytes of device workspace the plan needs (tables + stage buffers). */
size_t lam_workspace_bytes(lam_plan p);

/* Hand the plan a device workspace of at least lam_workspace_bytes(p) bytes
 * (256-byte aligned), owned by the caller for the plan's lifetime, and copy
 * the plan's tables into it (a synchronous host-to-device copy).  Must be
 * called once before any compute call; calling it again moves the plan to
 * the new workspace.  Errors: LAM_ERR_ARG (null/misaligned pointer),
 * LAM_ERR_WORKSPACE (too small), LAM_ERR_HIP (copy failed or no device). */
int lam_set_workspace(lam_plan p, void* dev_ptr, size_t bytes);

/* d = L u: forward laminography operator (Algorithm 1, forward pass).
 * u: complex (n0, n1, n2); d: complex (ntheta, h, w).  u and d must not
 * overlap.  d is also used as scratch for F_u2D's output. */
int lam_fwd(lam_plan p, const void* u, void* d, void* hip_stream);

/* u = L* d: adjoint (Algorithm 1, adjoint pass).  d: complex (ntheta, h, w),
 * read only; u: complex (n0, n1, n2). */
int lam_adj(lam_plan p, const void* d, void* u, void* hip_stream);

/* As lam_fwd / lam_adj with a real volume u (float or double per dtype):
 * d = L u for real u, and u = Re(L* d). */
int lam_fwd_real(lam_plan p, const void* u, void* d, void* hip_stream);
int lam_adj_real(lam_plan p, const void* d, void* u, void* hip_stream);

/* r = L^ u - dhat (Algorithm 2 forward pass; the subtraction is fused into
 * F_u2D's gather, Section 4.2 "Operation Cancellation and Fusion").
 * u: complex volume; dhat: complex (ntheta, h, w) or NULL (then r = L^ u);
 * r: complex (ntheta, h, w).  r may alias dhat. */
int lam_fwd_hat(lam_plan p, const void* u, const void* dhat, void* r, void* hip_stream);

/* u = L^* r, the exact adjoint of lam_fwd_hat's linear part (no 1/(h w)).
 * r: complex (ntheta, h, w), read only; u: complex volume. */
int lam_adj_hat(lam_plan p, const void* r, void* u, void* hip_stream);

/* Host-streamed forward and adjoint for volumes and data that live in host
 * memory (the chunk pipeline the Background section describes for LSP, where
 * host-to-device chunk transfers overlap the FFT work).
 *   u_host  host array (n0, n1, n2): real (u_real != 0; float or double per
 *           dtype) or complex
 *   d_host  host complex array (ntheta, h, w)
 * Pinned memory lets the copies overlap the kernels; pageable memory is
 * accepted (HIP stages those copies, which then do not overlap).  The volume
 * moves in y-slabs through two staging buffers of the workspace (F_u1D needs
 * whole z columns), the data in theta-slabs through the workspace's resident
 * data buffer (F_2D needs whole projections); the intermediate stage arrays
 * stay in device memory.  Copies run on a stream the plan owns, ordered
 * against the caller's stream with events; the call returns at once and the
 * host arrays are complete when the caller's stream is.  lam_stream_slabs
 * sets the slab sizes (volume rows per y-slab, at most the staging capacity
 * chosen at lam_init, about 64 MiB; projections per theta-slab).  Errors as
 * for lam_fwd; LAM_ERR_ARG for null host pointers or slab sizes out of range. */
int lam_fwd_streamed(lam_plan p, const void* u_host, int u_real, void* d_host, void* hip_stream);
int lam_adj_streamed(lam_plan p, const void* d_host, void* u_host, int u_real, void* hip_stream);
int lam_stream_slabs(lam_plan p, int y_rows, int theta_proj);

/* dhat = W d: the unnormalised centred 2D DFT of every projection, computed
 * once before the LSP loop (Algorithm 2, "d^ <- F_2D d"); with this scaling
 * |L u - d|^2 = |L^ u - d^|^2 / (h w).  d, dhat: complex (ntheta, h, w);
 * they may be the same buffer. */
int lam_data_hat(lam_plan p, const void* d, void* dhat, void* hip_stream);

/* ADMM-TV state for lam_admm_step: all device pointers, caller-owned, real
 * arrays of the plan's real type (float for LAM_C64, double for LAM_C128).
 *   u      [n0 n1 n2]        reconstruction (updated)
 *   psi    [3][n0 n1 n2]     auxiliary variable psi ~ grad u (updated)
 *   lam    [3][n0 n1 n2]     multiplier lambda (updated)
 *   work   lam_admm_work_bytes(p) bytes of device scratch
 *   scal   device array of 8 doubles: scal[0] = rho (read, then updated by the
 *          penalty rule), scal[1] = alpha (read); written with diagnostics:
 *          scal[2] last CG step gamma, scal[3] primal residual |grad u - psi|,
 *          scal[4] dual residual rho |grad^T(psi - psi_prev)|, scal[5] |G| of
 *          the last CG step, scal[6] the rho this step used.  FP64 throughout.
 * u, psi and lam are updated in place; start from zeros for a fresh solve. */
typedef struct {
  void* u;
  void* psi;
  void* lam;
  void* work;
  double* scal;
} lam_admm_state;

/* Bytes of ADMM scratch lam_admm_step needs beyond the plan workspace. */
size_t lam_admm_work_bytes(lam_plan p);

/* One ADMM-TV iteration for min_u 1/2 |L u - d|^2 + alpha |u|_TV (Equation 1):
 * LSP by n_inner conjugate-gradient steps in the cancelled frequency domain
 * (Algorithm 2: one L^ and one L^* per step, the subtraction of dhat fused,
 * Fletcher-Reeves directions, exact line search, FP64 scalars kept on the
 * device), then the TV subproblem (isotropic shrink), the multiplier update
 * and residual-balanced penalty update.  dhat = W d, complex (ntheta, h, w).
 * Enqueues work only; no host synchronisation. */
int lam_admm_step(lam_plan p, const lam_admm_state* s, const void* dhat, int n_inner, void* hip_stream);

/* d = L u as lam_fwd, with no workspace and no allocation: for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The plan's tables, target lists
 * and stage buffers live in a static device array of LAM_SCRATCH_BYTES that
 * the library holds on every GPU it runs on until the process ends; the plan
 * needs no lam_set_workspace for this call.  The caller passes u (complex
 * (n0, n1, n2)) and d (complex (ntheta, h, w)) as for lam_fwd; the result is
 * the same as lam_fwd's.
 * The array of a GPU is shared by every call on it and keeps the last call's
 * contents: the first call of a plan on a GPU (and the first after another
 * plan's call there) synchronises the device and rebuilds the plan's tables
 * and target lists in it (host-to-device copies and list kernels on the null
 * stream); later calls of the same plan only enqueue on hip_stream.  Calls
 * that overlap in time on one GPU (other threads, other streams, other plans)
 * race on the array.  No hipMalloc, hipFree or allocating library call is
 * made.  Errors: as lam_fwd; LAM_ERR_WORKSPACE when the plan needs more than
 * LAM_SCRATCH_BYTES (lam_workspace_bytes less the host-streaming buffers;
 * about 64^3 volumes, or larger ones with a small slab). */
#define LAM_SCRATCH_BYTES ((size_t)64 << 20)
int lam_fwd_scratch(lam_plan p, const void* u, void* d, void* hip_stream);

/* Memoization of the LSP's operator applications (Section 4.4 "Memoization Cache", Section 4.5
 * Equation (cs)).  Each of F_u1D, F_u2D, F*_u2D and F*_u1D keeps a private cache per chunk location
 * (chunk_y volume rows for the z steps, chunk_kv k_v slices for the 2D steps): one (key, value) item,
 * replaced first-in-first-out.  The key of an input chunk is a signed random projection of length
 * key_dim (count sketch: value q of the chunk, C order, complex values as (re, im), adds to bucket
 * q mod key_dim with the sign of the top bit of SplitMix64 output number chunk * 2^40 + q from state
 * seed + operator index 0..3), standing in for the paper's CNN encoder.  A query whose key has cosine
 * similarity above tau with the chunk's cached key takes the cached output; otherwise the chunk is
 * computed and its (key, output) replaces the item.
 *   tau        similarity threshold; tau >= 1 never hits (the plain step), the paper uses 0.92
 *   chunk_y    power of two in [1, n1]; chunk_kv power of two in [1, h]; the plan's n0, n1, n2, h
 *              and w must be powers of two (LAM_ERR_ARG otherwise)
 *   key_dim    power of two in [64, 4096]
 *   work       device memory of lam_memo_bytes bytes holding the caches (outputs of the four
 *              operators), keys, flags and the sign tables; caller-owned, ZERO-FILLED before the
 *              first step of a solve (empty caches); keep it across the steps of one solve
 *   counters   device array of 8 int64: hits and misses of F_u1D, F_u2D, F*_u2D, F*_u1D, accumulated
 *              by every step (the caller clears them) */
typedef struct {
  double tau;
  int chunk_y;
  int chunk_kv;
  int key_dim;
  unsigned long long seed;
  void* work;
  long long* counters;
} lam_memo;

/* Bytes of memoization work for the plan and the parameters in *m (0 for invalid parameters). */
size_t lam_memo_bytes(lam_plan p, const lam_memo* m);

/* lam_admm_step with memoized operators: every inner iteration recomputes the residual
 * r = M_u2D(M_u1D u) - d^ and the data gradient Re M*_u1D(M*_u2D r) / (h w) through the memoized
 * operators (Algorithm 2's forward and adjoint passes; F_u2D's cached outputs exclude d^, so dhat may
 * change between steps), then takes the Fletcher-Reeves direction p and the exact line search, which
 * applies the plain L^ to p.  RSP, multiplier and penalty updates as lam_admm_step.  With tau >= 1 it
 * computes what lam_admm_step does (up to rounding: the residual is recomputed, not updated).  Enqueues
 * work only.  Errors: as lam_admm_step; LAM_ERR_ARG for parameters outside the ranges above. */
int lam_admm_step_memo(lam_plan p, const lam_admm_state* s, const void* dhat, int n_inner, const lam_memo* m,
                       void* hip_stream);

/* ADMM-Offload planning (Section 5.1).  One ADMM iteration is nphases phases run back to back and
 * repeated (phase_s: durations in seconds, e.g. LSP, RSP, multiplier update, penalty update, from a
 * profile of one iteration).  Each variable has a size, whether it is an offloading candidate, and
 * per phase whether the phase accesses it, the offsets (seconds from the phase's start) of its first
 * and last access there, and whether the phase overwrites it before reading it (its old value is then
 * dead before the phase).  The planner evaluates every set of candidates: after each access phase k,
 * up to the variable's next access phase k', a dead gap leaves it absent with no transfer; otherwise
 * it is offloaded after its last access in k unless the offload cannot end before its first access in
 * k' (the maximum prefetch distance, constraint 3), and prefetched after the offload (constraint 1),
 * as late as lets it end when k' starts (constraint 4), unless no prefetch distance is left
 * (constraint 2).  One link of link_bps bytes/s carries one transfer at a time: offloads in the order
 * of their last accesses, then prefetches in the order of their planned starts.  M = the bytes of
 * all variables less the plan's peak of resident bytes over the iteration; T = the sum of the delays
 * of prefetches that end after the first access they serve; MT = M / max(T, 1 us).  The plan with
 * the largest MT wins (the empty plan has M = 0, MT = 0; ties keep the plan whose candidate bitmask is
 * smaller).  With budget > 0 only plans whose peak (resident + variables - M) fits the budget
 * compete; if none does, out->MT = -1.  Host computation only; no device is touched.
 * Errors: LAM_ERR_ARG for null pointers, counts outside [1, 8] phases / [1, 16] variables, durations
 * not positive, offsets outside [0, duration] or first > last, a variable with no access. */
#define LAM_OFFLOAD_MAX_PHASES 8
#define LAM_OFFLOAD_MAX_VARS 16
typedef struct {
  double bytes;
  int candidate;
  int accessed[LAM_OFFLOAD_MAX_PHASES];
  double first[LAM_OFFLOAD_MAX_PHASES];
  double last[LAM_OFFLOAD_MAX_PHASES];
  int writes_first[LAM_OFFLOAD_MAX_PHASES];
} lam_offload_var;
typedef struct {
  unsigned mask;   /* bit v set: variable v is offloaded */
  double M;        /* memory saving, bytes */
  double T;        /* performance loss, seconds per iteration */
  double MT;       /* M / max(T, 1e-6), or -1 when no plan fits the budget */
  double peak;     /* resident + variables - M, bytes */
} lam_offload_result;
int lam_offload_plan(const double* phase_s, int nphases, const lam_offload_var* vars, int nvars, double resident,
                     double link_bps, double budget, lam_offload_result* out);

/* M, T, MT and peak of one plan (bit v of mask: variable v offloaded, candidate or not), by the rules
 * of lam_offload_plan.  Errors as lam_offload_plan; LAM_ERR_ARG for mask bits at or beyond nvars. */
int lam_offload_evaluate(const double* phase_s, int nphases, const lam_offload_var* vars, int nvars, double resident,
                         double link_bps, unsigned mask, lam_offload_result* out);

/* Per-kernel timing, for measurement.  With profiling on, every kernel the
 * plan launches is bracketed by a pair of HIP events recorded on its stream
 * (this adds a small gap between kernels).  lam_profile_read waits for the
 * recorded events, returns per-kernel totals in milliseconds and launch
 * counts in arrays of LAM_NUM_KERNELS entries indexed as lam_kernel_name
 * lists them, and clears the record.  Kernels: 0 zfwd (F_u1D), 1 ycol_fwd,
 * 2 xrow_fwd, 3 gather (F_u2D), 4 rowfft, 5 colfft (F*_2D / F_2D),
 * 6 scatter, 7 xrow_adj, 8 ycol_adj (F*_u2D), 9 zadj (F*_u1D). */
#define LAM_NUM_KERNELS 10
int lam_profile(lam_plan p, int on);
int lam_profile_read(lam_plan p, double* total_ms, long long* launches);
const char* lam_kernel_name(int k);

/* Release the plan (host memory only; the workspace stays the caller's).  Waits
 * for the copies of host-streamed calls still in flight on the plan's copy
 * stream; kernels already enqueued on the caller's streams keep reading the
 * workspace, so the caller must not free it before those streams finish. */
void lam_destroy(lam_plan p);

/* Static text for a status code. */
const char* lam_error_string(int code);

/* Thread-local detail text for the last failing call ("" if none). */
const char* lam_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LAM_H */
