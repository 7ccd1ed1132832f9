"""Python binding of liblam.so: argument marshalling only.

Every step of the operator runs in the HIP kernels of liblam.so; PyTorch only
supplies device memory (the workspace and the arrays) and the stream.  If
the library is not built, or no GPU is present, these calls raise: there is
no CPU fallback.

    plan = Plan(512, ntheta=512, phi=math.radians(30), h=512, w=512)
    d = plan.fwd(u)              # L u          (u complex or real)
    v = plan.adj(d)              # L* d         (complex; plan.adj(d, real=True) -> Re)
    r = plan.fwd_hat(u, dhat)    # L^ u - d^    (Algorithm 2, fused subtraction)
    w = plan.adj_hat(r)          # L^* r
    y = LamOp.apply(u, plan)     # autograd: backward is the adjoint kernel
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, byref, c_double, c_int, c_size_t, c_void_p

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblam.so")

LAM_C64, LAM_C128 = 0, 1
STATUS = {0: "LAM_OK", 1: "LAM_ERR_ARG", 2: "LAM_ERR_NOMEM", 3: "LAM_ERR_HIP", 4: "LAM_ERR_WORKSPACE",
          5: "LAM_ERR_STATE"}


class LamError(RuntimeError):
    def __init__(self, code: int, detail: str):
        super().__init__(f"{STATUS.get(code, code)}: {detail}")
        self.code = code


class LamParams(ctypes.Structure):
    _fields_ = [
        ("n0", c_int), ("n1", c_int), ("n2", c_int),
        ("ntheta", c_int),
        ("theta", POINTER(c_double)),
        ("phi", c_double),
        ("h", c_int), ("w", c_int),
        ("oversample", c_int),
        ("m", c_int),
        ("dtype", c_int),
        ("slab", c_int),
    ]


class AdmmState(ctypes.Structure):
    _fields_ = [("u", c_void_p), ("psi", c_void_p), ("lam", c_void_p), ("work", c_void_p),
                ("scal", POINTER(c_double))]


class LamMemo(ctypes.Structure):
    _fields_ = [("tau", c_double), ("chunk_y", c_int), ("chunk_kv", c_int), ("key_dim", c_int),
                ("seed", ctypes.c_ulonglong), ("work", c_void_p), ("counters", POINTER(ctypes.c_longlong))]


class OffloadVar(ctypes.Structure):
    _fields_ = [("bytes", c_double), ("candidate", c_int), ("accessed", c_int * 8), ("first", c_double * 8),
                ("last", c_double * 8), ("writes_first", c_int * 8)]


class OffloadResult(ctypes.Structure):
    _fields_ = [("mask", ctypes.c_uint), ("M", c_double), ("T", c_double), ("MT", c_double), ("peak", c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load liblam.so (built in-tree by paper_2511_01893_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2511_01893_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.lam_init.argtypes = [POINTER(c_void_p), POINTER(LamParams)]
        L.lam_workspace_bytes.argtypes = [c_void_p]
        L.lam_workspace_bytes.restype = c_size_t
        L.lam_set_workspace.argtypes = [c_void_p, c_void_p, c_size_t]
        for name in ("lam_fwd", "lam_adj", "lam_fwd_real", "lam_adj_real", "lam_adj_hat"):
            getattr(L, name).argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        L.lam_fwd_hat.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
        L.lam_fwd_scratch.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        L.lam_data_hat.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
        L.lam_fwd_streamed.argtypes = [c_void_p, c_void_p, c_int, c_void_p, c_void_p]
        L.lam_adj_streamed.argtypes = [c_void_p, c_void_p, c_void_p, c_int, c_void_p]
        L.lam_stream_slabs.argtypes = [c_void_p, c_int, c_int]
        L.lam_admm_work_bytes.argtypes = [c_void_p]
        L.lam_admm_work_bytes.restype = c_size_t
        L.lam_admm_step.argtypes = [c_void_p, POINTER(AdmmState), c_void_p, c_int, c_void_p]
        L.lam_memo_bytes.argtypes = [c_void_p, POINTER(LamMemo)]
        L.lam_memo_bytes.restype = c_size_t
        L.lam_admm_step_memo.argtypes = [c_void_p, POINTER(AdmmState), c_void_p, c_int, POINTER(LamMemo), c_void_p]
        L.lam_offload_plan.argtypes = [POINTER(c_double), c_int, POINTER(OffloadVar), c_int, c_double, c_double,
                                       c_double, POINTER(OffloadResult)]
        L.lam_offload_evaluate.argtypes = [POINTER(c_double), c_int, POINTER(OffloadVar), c_int, c_double, c_double,
                                           ctypes.c_uint, POINTER(OffloadResult)]
        L.lam_profile.argtypes = [c_void_p, c_int]
        L.lam_profile_read.argtypes = [c_void_p, POINTER(c_double), POINTER(ctypes.c_longlong)]
        L.lam_kernel_name.argtypes = [c_int]
        L.lam_kernel_name.restype = ctypes.c_char_p
        L.lam_destroy.argtypes = [c_void_p]
        L.lam_destroy.restype = None
        L.lam_error_string.argtypes = [c_int]
        L.lam_error_string.restype = ctypes.c_char_p
        L.lam_last_error.argtypes = []
        L.lam_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise LamError(rc, lib().lam_last_error().decode())


class Plan:
    """Operator plan: problem statement + device workspace (owned by torch)."""

    def __init__(self, n0: int, n1: int | None = None, n2: int | None = None, *, ntheta: int, phi: float,
                 h: int | None = None, w: int | None = None, m: int = 4, oversample: int = 2,
                 dtype: torch.dtype = torch.complex64, slab: int = 0, theta=None, device="cuda",
                 workspace: bool = True):
        n1 = n0 if n1 is None else n1
        n2 = n0 if n2 is None else n2
        h = n0 if h is None else h
        w = n2 if w is None else w
        if dtype not in (torch.complex64, torch.complex128):
            raise ValueError("dtype must be torch.complex64 or torch.complex128")
        self.n0, self.n1, self.n2, self.ntheta, self.phi, self.h, self.w = n0, n1, n2, ntheta, phi, h, w
        self.m, self.oversample, self.dtype = m, oversample, dtype
        self.rdtype = torch.float32 if dtype == torch.complex64 else torch.float64
        self.device = torch.device(device)
        self._theta = None
        p = LamParams(n0, n1, n2, ntheta, None, float(phi), h, w, oversample, m,
                      LAM_C64 if dtype == torch.complex64 else LAM_C128, slab)
        if theta is not None:
            self._theta = (c_double * ntheta)(*[float(t) for t in theta])
            p.theta = ctypes.cast(self._theta, POINTER(c_double))
        self._h = c_void_p()
        _check(lib().lam_init(byref(self._h), byref(p)))
        self._home = torch.cuda.current_stream(self.device)
        self.workspace = None
        if workspace:   # workspace=False: a plan for fwd_scratch only (the library's static scratch)
            nbytes = lib().lam_workspace_bytes(self._h)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            _check(lib().lam_set_workspace(self._h, c_void_p(self.workspace.data_ptr()), nbytes))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lam_destroy(h)
            self._h = None

    # ---------------------------------------------------------------- shapes
    @property
    def vol_shape(self):
        return (self.n0, self.n1, self.n2)

    @property
    def data_shape(self):
        return (self.ntheta, self.h, self.w)

    def _stream(self, *tensors):
        """The calling stream; the workspace (and `tensors`, device scratch of the caller) are
        marked as used on it, so the caching allocator does not hand their memory out again
        while work of this call is pending on a stream other than the one they came from."""
        s = torch.cuda.current_stream(self.device)
        if s != self._home:
            if self.workspace is not None:
                self.workspace.record_stream(s)
            for t in tensors:
                t.record_stream(s)
        return c_void_p(s.cuda_stream)

    def _arr(self, x: torch.Tensor, shape, what: str, allow_real=False) -> torch.Tensor:
        if tuple(x.shape) != tuple(shape):
            raise ValueError(f"{what}: expected shape {tuple(shape)}, got {tuple(x.shape)}")
        if x.device != self.device and not (x.device.type == "cuda" and self.device.type == "cuda"
                                            and (x.device.index or 0) == (self.device.index or 0)):
            raise ValueError(f"{what}: expected a tensor on {self.device}, got {x.device}")
        ok = (self.dtype,) + ((self.rdtype,) if allow_real else ())
        if x.dtype not in ok:
            raise ValueError(f"{what}: expected dtype in {ok}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError(f"{what}: tensor must be contiguous")
        return x

    # ---------------------------------------------------------------- operators
    def fwd(self, u: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """d = L u (F*_2D F_u2D F_u1D); u complex or real."""
        self._arr(u, self.vol_shape, "u", allow_real=True)
        out = torch.empty(self.data_shape, dtype=self.dtype, device=self.device) if out is None else out
        self._arr(out, self.data_shape, "d")
        f = lib().lam_fwd if u.is_complex() else lib().lam_fwd_real
        _check(f(self._h, c_void_p(u.data_ptr()), c_void_p(out.data_ptr()), self._stream()))
        return out

    def fwd_scratch(self, u: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """d = L u for complex u through lam_fwd_scratch: no workspace, nothing allocated (out is the
        caller's); the plan's tables live in the library's static device scratch."""
        self._arr(u, self.vol_shape, "u")
        self._arr(out, self.data_shape, "d")
        _check(lib().lam_fwd_scratch(self._h, c_void_p(u.data_ptr()), c_void_p(out.data_ptr()),
                                     c_void_p(torch.cuda.current_stream(self.device).cuda_stream)))
        return out

    def adj(self, d: torch.Tensor, real: bool = False, out: torch.Tensor | None = None) -> torch.Tensor:
        """u = L* d (F*_u1D F*_u2D F_2D); real=True returns Re(L* d)."""
        self._arr(d, self.data_shape, "d")
        dt = self.rdtype if real else self.dtype
        out = torch.empty(self.vol_shape, dtype=dt, device=self.device) if out is None else out
        f = lib().lam_adj_real if real else lib().lam_adj
        _check(f(self._h, c_void_p(d.data_ptr()), c_void_p(out.data_ptr()), self._stream()))
        return out

    def fwd_hat(self, u: torch.Tensor, dhat: torch.Tensor | None = None,
                out: torch.Tensor | None = None) -> torch.Tensor:
        """r = L^ u - d^ (Algorithm 2, subtraction fused into F_u2D)."""
        self._arr(u, self.vol_shape, "u")
        if dhat is not None:
            self._arr(dhat, self.data_shape, "dhat")
        out = torch.empty(self.data_shape, dtype=self.dtype, device=self.device) if out is None else out
        _check(lib().lam_fwd_hat(self._h, c_void_p(u.data_ptr()),
                                 c_void_p(dhat.data_ptr() if dhat is not None else None),
                                 c_void_p(out.data_ptr()), self._stream()))
        return out

    def adj_hat(self, r: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """u = L^* r (exact adjoint of fwd_hat's linear part)."""
        self._arr(r, self.data_shape, "r")
        out = torch.empty(self.vol_shape, dtype=self.dtype, device=self.device) if out is None else out
        _check(lib().lam_adj_hat(self._h, c_void_p(r.data_ptr()), c_void_p(out.data_ptr()), self._stream()))
        return out


    def data_hat(self, d: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """d^ = W d: unnormalised centred 2D DFT of every projection (Algorithm 2's d^)."""
        self._arr(d, self.data_shape, "d")
        out = torch.empty(self.data_shape, dtype=self.dtype, device=self.device) if out is None else out
        _check(lib().lam_data_hat(self._h, c_void_p(d.data_ptr()), c_void_p(out.data_ptr()), self._stream()))
        return out

    # ---------------------------------------------------------------- host-streamed
    def _host(self, x: torch.Tensor, shape, what: str, allow_real=False) -> torch.Tensor:
        # pinned memory lets the slab copies overlap the kernels; pageable memory works too (HIP stages the
        # copies), for arrays too large to pin
        if x.device.type != "cpu":
            raise ValueError(f"{what}: expected a host tensor")
        if tuple(x.shape) != tuple(shape):
            raise ValueError(f"{what}: expected shape {tuple(shape)}, got {tuple(x.shape)}")
        ok = (self.dtype,) + ((self.rdtype,) if allow_real else ())
        if x.dtype not in ok:
            raise ValueError(f"{what}: expected dtype in {ok}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError(f"{what}: tensor must be contiguous")
        return x

    def stream_slabs(self, y_rows: int, theta_proj: int):
        """Slab sizes of the host-streamed calls: volume rows per y-slab, projections per theta-slab."""
        _check(lib().lam_stream_slabs(self._h, int(y_rows), int(theta_proj)))

    def fwd_streamed(self, u: torch.Tensor, out: torch.Tensor | None = None, wait: bool = True) -> torch.Tensor:
        """d = L u with u and d in host memory (pinned: slab copies overlapped with the kernels)."""
        self._host(u, self.vol_shape, "u", allow_real=True)
        out = torch.empty(self.data_shape, dtype=self.dtype, pin_memory=True) if out is None else out
        self._host(out, self.data_shape, "d")
        _check(lib().lam_fwd_streamed(self._h, c_void_p(u.data_ptr()), 0 if u.is_complex() else 1,
                                      c_void_p(out.data_ptr()), self._stream()))
        if wait:
            torch.cuda.current_stream(self.device).synchronize()
        return out

    def adj_streamed(self, d: torch.Tensor, real: bool = False, out: torch.Tensor | None = None,
                     wait: bool = True) -> torch.Tensor:
        """u = L* d (Re if real) with d and u in host memory (pinned: copies overlapped with the kernels)."""
        self._host(d, self.data_shape, "d")
        dt = self.rdtype if real else self.dtype
        out = torch.empty(self.vol_shape, dtype=dt, pin_memory=True) if out is None else out
        self._host(out, self.vol_shape, "u", allow_real=True)
        if out.dtype != dt:
            raise ValueError(f"u: expected dtype {dt}")
        _check(lib().lam_adj_streamed(self._h, c_void_p(d.data_ptr()), c_void_p(out.data_ptr()),
                                      1 if real else 0, self._stream()))
        if wait:
            torch.cuda.current_stream(self.device).synchronize()
        return out

    # ---------------------------------------------------------------- timing
    def profile(self, on: bool = True):
        """Bracket every kernel of this plan with HIP events (for measurement)."""
        _check(lib().lam_profile(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        """{kernel name: (total ms, launches)} since the last read; waits for the events."""
        n = NUM_KERNELS
        ms = (c_double * n)()
        cnt = (ctypes.c_longlong * n)()
        _check(lib().lam_profile_read(self._h, ms, cnt))
        return {lib().lam_kernel_name(k).decode(): (ms[k], cnt[k]) for k in range(n)}


NUM_KERNELS = 10


class LamOp(torch.autograd.Function):
    """d = L u with backward = the hand-written adjoint kernel.

    Complex u: PyTorch's conjugate-Wirtinger convention gives grad_u = L* g.
    Real u: grad_u = Re(L* g).  L is linear, so nothing is saved."""

    @staticmethod
    def forward(ctx, u, plan: Plan):
        ctx.plan = plan
        ctx.real = not u.is_complex()
        return plan.fwd(u.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.adj(g.contiguous(), real=ctx.real), None


OPS = ("F_u1D", "F_u2D", "F*_u2D", "F*_u1D")


class Memo:
    """Private per-chunk memoization caches of the LSP's four operators for one ADMM solve
    (Section 4.4): chunks of chunk_y volume rows (F_u1D, F*_u1D) and chunk_kv k_v slices (F_u2D,
    F*_u2D), sketch keys of length key_dim, similarity threshold tau (Equation (cs)).  The device
    work (caches, keys, sign tables) starts zeroed, i.e. with empty caches."""

    def __init__(self, plan: Plan, tau: float = 0.92, chunk_y: int = 16, chunk_kv: int = 16,
                 key_dim: int = 1024, seed: int = 0):
        self.params = LamMemo(float(tau), int(chunk_y), int(chunk_kv), int(key_dim), int(seed), None, None)
        nbytes = lib().lam_memo_bytes(plan._h, byref(self.params))
        if nbytes == 0:
            raise ValueError("memoization parameters: chunk_y, chunk_kv powers of two within the volume rows / "
                             "detector rows, key_dim a power of two in [64, 4096], tau not NaN")
        self.tau = float(tau)
        self.work = torch.zeros(nbytes, dtype=torch.uint8, device=plan.device)
        self.counters = torch.zeros(8, dtype=torch.int64, device=plan.device)
        self.params.work = c_void_p(self.work.data_ptr())
        self.params.counters = ctypes.cast(c_void_p(self.counters.data_ptr()), POINTER(ctypes.c_longlong))

    def stats(self) -> dict:
        """{operator: (hits, misses)} accumulated over the steps so far (synchronises)."""
        c = self.counters.tolist()
        return {name: (c[2 * i], c[2 * i + 1]) for i, name in enumerate(OPS)}

    def hit_rate(self) -> float:
        c = self.counters.tolist()
        return sum(c[0::2]) / max(1, sum(c))


class AdmmTV:
    """ADMM-TV state on the device for min_u 1/2 |L u - d|^2 + alpha |u|_TV (Equation 1).

    u (real), psi and lam (3 x volume) start at zero; rho starts at rho0.
    step() runs one ADMM iteration (LSP with n_inner CG steps, RSP, multiplier
    and penalty updates) entirely in liblam.so's kernels; with a Memo, the
    LSP's operator applications go through its caches (lam_admm_step_memo)."""

    def __init__(self, plan: Plan, alpha: float, rho0: float = 0.5, memo: Memo | None = None):
        self.plan = plan
        self.memo = memo
        dev, rdt = plan.device, plan.rdtype
        self.u = torch.zeros(plan.vol_shape, dtype=rdt, device=dev)
        self.psi = torch.zeros((3,) + plan.vol_shape, dtype=rdt, device=dev)
        self.lam = torch.zeros((3,) + plan.vol_shape, dtype=rdt, device=dev)
        self.work = torch.empty(lib().lam_admm_work_bytes(plan._h), dtype=torch.uint8, device=dev)
        self.scal = torch.zeros(8, dtype=torch.float64, device=dev)
        self.scal[0] = rho0
        self.scal[1] = alpha

    @property
    def rho(self) -> float:
        return float(self.scal[0].item())

    def diagnostics(self) -> dict:
        s = self.scal.tolist()
        return {"rho": s[0], "alpha": s[1], "gamma": s[2], "primal": s[3], "dual": s[4], "grad_norm": s[5],
                "rho_used": s[6]}

    def step(self, dhat: torch.Tensor, n_inner: int = 4):
        self.plan._arr(dhat, self.plan.data_shape, "dhat")
        st = AdmmState(c_void_p(self.u.data_ptr()), c_void_p(self.psi.data_ptr()), c_void_p(self.lam.data_ptr()),
                       c_void_p(self.work.data_ptr()),
                       ctypes.cast(c_void_p(self.scal.data_ptr()), POINTER(c_double)))
        if self.memo is None:
            _check(lib().lam_admm_step(self.plan._h, byref(st), c_void_p(dhat.data_ptr()), n_inner,
                                       self.plan._stream(self.work)))
        else:
            _check(lib().lam_admm_step_memo(self.plan._h, byref(st), c_void_p(dhat.data_ptr()), n_inner,
                                            byref(self.memo.params),
                                            self.plan._stream(self.work, self.memo.work, self.memo.counters)))


def admm_tv(plan: Plan, d: torch.Tensor, alpha: float, n_outer: int = 4, n_inner: int = 4,
            rho0: float = 0.5) -> AdmmTV:
    """Run n_outer ADMM-TV iterations on projections d (complex, (ntheta, h, w))."""
    dhat = plan.data_hat(d)
    s = AdmmTV(plan, alpha, rho0)
    for _ in range(n_outer):
        s.step(dhat, n_inner)
    return s


def _offload_args(phase_s, variables):
    names = list(variables)
    arr = (OffloadVar * len(names))()
    for i, n in enumerate(names):
        v = variables[n]
        arr[i].bytes = float(v["bytes"])
        arr[i].candidate = 1 if v.get("candidate", True) else 0
        for k, (first, last, wf) in v["access"].items():
            arr[i].accessed[k] = 1
            arr[i].first[k] = float(first)
            arr[i].last[k] = float(last)
            arr[i].writes_first[k] = 1 if wf else 0
    ph = (c_double * len(phase_s))(*[float(t) for t in phase_s])
    return names, arr, ph


def offload_plan(phase_s, variables: dict, resident: float, link_bps: float, budget: float | None = None) -> dict:
    """ADMM-Offload plan (Section 5.1) by lam_offload_plan: phase durations (s), variables
    {name: {"bytes", "access": {phase: (first, last, writes_first)}, "candidate"}}, never-offloaded
    bytes, link bandwidth (bytes/s), optional device-memory budget (bytes)."""
    names, arr, ph = _offload_args(phase_s, variables)
    out = OffloadResult()
    _check(lib().lam_offload_plan(ph, len(phase_s), arr, len(names), float(resident), float(link_bps),
                                  float(budget) if budget else 0.0, byref(out)))
    return {"offload": [n for i, n in enumerate(names) if out.mask >> i & 1], "M": out.M, "T": out.T, "MT": out.MT,
            "peak": out.peak}


def offload_evaluate(phase_s, variables: dict, resident: float, link_bps: float, offload) -> dict:
    """M, T, MT and peak of the plan that offloads the named variables (lam_offload_evaluate)."""
    names, arr, ph = _offload_args(phase_s, variables)
    mask = sum(1 << names.index(n) for n in offload)
    out = OffloadResult()
    _check(lib().lam_offload_evaluate(ph, len(phase_s), arr, len(names), float(resident), float(link_bps), mask,
                                      byref(out)))
    return {"M": out.M, "T": out.T, "MT": out.MT, "peak": out.peak}


def plan_for(name: str, dtype=torch.complex64, device="cuda", slab: int = 0) -> Plan:
    """Plan for one of the named workloads (see paper_2511_01893_amd.inputs.WORKLOADS)."""
    from .inputs import WORKLOADS

    w = WORKLOADS[name]
    return Plan(w["n"], ntheta=w["ntheta"], phi=math.radians(w["phi_deg"]), h=w["det"], w=w["det"], dtype=dtype,
                device=device, slab=slab)
