"""Benchmark: laminography forward + adjoint pairs per second on one MI355X.

One step = one pair lam_fwd (u -> d, F*_2D F_u2D F_u1D) + lam_adj
(d -> u, F*_u1D F*_u2D F_2D) on complex64 device arrays, inputs resident in
HBM before timing starts.  Workload (default): 512^3 volume, 512 angles
uniform in [0, 2 pi), tilt 30 deg, 512 x 512 detector, R = 2, m = 4; u is the
seeded blob + cube phantom, d seeded complex N(0,1).

Prints one JSON line.  Besides the contract fields it reports:
  roofline       dominant kernel's algorithmic rate against its bound,
                 from per-kernel HIP events in a second pass of the same steps
  pair_hbm_frac  the whole pair's algorithmic bytes (u, u1, u2, d traffic) / time / 8 TB/s
                 (also with the oversampled grid's traffic, and for the frequency-domain pair)
  alu            flops of the pair (FFTs 5 N log2 N, 5 per stencil tap) against the FP32 peaks
  memo           memoized ADMM-TV (private per-chunk caches): accuracy and hit rate against tau,
                 time per step
  offload        ADMM-Offload plan for one ADMM-TV iteration (profiled phases, host link bandwidth)
  fp64_*         the same kernels instantiated in complex128 (the plain FP64 operator)
  accuracy       c64 vs c128 GPU (whole arrays) and c64 vs the FP64 oracle on sampled slices
  cpu_baseline   the FP64 oracle timed on a bounded sample on this host
"""
from __future__ import annotations

import argparse
import csv
import json
import math
import os
import re
import sys
import time
from collections import defaultdict

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VALU_TFLOPS = 78.6        # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, packed FP32 disabled
TFLOPS_FP64 = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(n0, n1, n2, ntheta, h, w, s, su):
    """Bytes one operator must move (u read, u1 written + read, u2 written + read, d written)."""
    V, H1, P = n0 * n1 * n2, h * n1 * n2, ntheta * h * w
    return su * V + 2 * s * H1 + 3 * s * P


def pair_flops(n0, n1, n2, ntheta, h, w, m=4):
    """Flops of one pair: 5 N log2 N per FFT of length N (padded lengths, no pruning), 5 per
    stencil tap of the gathers and spreads; each operator: z FFTs of 2 n0 on n1 n2 columns and h x 2m
    taps per column, y FFTs of 2 n1 on n2 columns and x FFTs of 2 n2 on 2 n1 rows per slice,
    (2m)^2 taps per target, and the h x w 2D DFT of every projection."""
    def fft(N):
        return 5.0 * N * math.log2(N)
    op = (n1 * n2 * (fft(2 * n0) + 5.0 * h * 2 * m)
          + h * (n2 * fft(2 * n1) + 2 * n1 * fft(2 * n2)) + 5.0 * ntheta * h * w * (2 * m) ** 2
          + ntheta * (h * fft(w) + w * fft(h)))
    return 2.0 * op


def kernel_units(name, plan, s, su, slab):
    """Algorithmic bytes per launch and taps per launch for each kernel.

    Per unit (one column of F_u1D, one k_v slice of F_u2D, one projection of
    the 2D DFT) the kernel's share of the operator's algorithmic traffic:
    zfwd / zadj: s_u*V + s*H1 for the volume; F_u2D kernels: s*(n1 n2 + ntheta w)
    per slice; rowfft / colfft: 2 s P per pass."""
    n0, n1, n2, nt, h, w = plan.n0, plan.n1, plan.n2, plan.ntheta, plan.h, plan.w
    if name in ("zfwd", "zadj"):
        return su * n0 * n1 * n2 + s * h * n1 * n2
    if name in ("rowfft", "colfft"):
        return 2 * s * nt * h * w
    return s * (n1 * n2 + nt * w) * slab


def time_pairs(plan, u, d, steps, warmup):
    import torch

    out_d = torch.empty_like(d)
    out_u = torch.empty_like(u)
    for _ in range(warmup):
        plan.fwd(u, out=out_d)
        plan.adj(d, out=out_u)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        plan.fwd(u, out=out_d)
        plan.adj(d, out=out_u)
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return e0.elapsed_time(e1) / steps, wall, out_d, out_u


def cpu_baseline(wl, budget_slices=16, col_fraction=16, nproj=32):
    """Time the FP64 oracle on a bounded sample of one pair and scale to pairs/s.

    Sample (about 10 s of CPU work at 512^3): F_u1D / F*_u1D on 1/col_fraction
    of the (y, x) columns, F_u2D / F*_u2D on `budget_slices` k_v slices, F*_2D /
    F_2D on `nproj` projections; each part is scaled by (total units / sampled
    units)."""
    import numpy as np

    from oracle import lam_oracle as O

    n, nt, h = wl["n"], wl["ntheta"], wl["det"]
    g = O.Geometry(n, n, n, nt, math.radians(wl["phi_deg"]), h, h, 2, 4)
    rng = np.random.default_rng(0)

    def cplx(*shape):
        return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)

    ncol = n * n // col_fraction
    _, _, nu_z = O.frequencies(g)
    x = cplx(n, ncol)
    t = time.perf_counter(); f = O.usfft1d_fwd(x, n * nu_z, 2, 4); t_z = time.perf_counter() - t
    t = time.perf_counter(); O.usfft1d_adj(f, n * nu_z, n, 2, 4); t_za = time.perf_counter() - t
    sl = list(range(h // 2 - budget_slices // 2, h // 2 + budget_slices // 2))
    u1 = np.zeros((h, n, n), complex)
    for k in sl:
        u1[k] = cplx(n, n)
    t = time.perf_counter(); r = O.fu2d(u1, g, kv_list=sl); t_2 = time.perf_counter() - t
    t = time.perf_counter(); O.fu2d_adj(r, g, kv_list=sl); t_2a = time.perf_counter() - t
    pp = cplx(nproj, h, h)
    t = time.perf_counter(); O.f2d_inv(pp); t_f = time.perf_counter() - t
    t = time.perf_counter(); O.f2d(pp); t_fa = time.perf_counter() - t
    per_pair = ((t_z + t_za) * col_fraction + (t_2 + t_2a) * h / len(sl) + (t_f + t_fa) * nt / nproj)
    sample_s = t_z + t_za + t_2 + t_2a + t_f + t_fa
    return {
        "value": 1.0 / per_pair,
        "unit": "pairs/s",
        "cores": O.WORKERS,
        "kind": "oracle",
        "sample": (f"F_u1D+adj on {ncol} of {n * n} columns, F_u2D+adj on {len(sl)} of {h} slices, "
                   f"F*_2D+F_2D on {nproj} of {nt} projections; {sample_s:.1f} s of CPU time, scaled"),
        "seconds_per_pair": per_pair,
    }


def host_info() -> dict:
    """CPU model, logical CPUs this process may use, and RAM of the host."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram = 0
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = int(line.split()[1]) * 1024
                break
    except OSError:
        pass
    return {"cpu_model": model, "cpus": len(os.sched_getaffinity(0)), "ram_gb": round(ram / 1e9, 1)}


def oracle_pair_c2(reps=3):
    """One full FP64 oracle pair (L u, L* d) at the 256^3 workload, timed reps times (median): the
    oracle as it stands, F_u2D slices split over the host's threads (the tests' harness)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    from oracle import lam_oracle as O
    from paper_2511_01893_amd import inputs as I

    w = I.WORKLOADS["lam256"]
    n = w["n"]
    g = O.Geometry(n, n, n, w["ntheta"], math.radians(w["phi_deg"]), w["det"], w["det"], 2, 4)
    u = I.blob_phantom(g.vol_shape, I.draw_blobs(w["seed"], w["nblobs"]))
    d = I.random_detector_data(g.data_shape, w["seed"])
    nw = len(os.sched_getaffinity(0))
    sets = [list(range(i, g.h, nw)) for i in range(nw)]
    times = []
    for _ in range(reps):
        t = time.perf_counter()
        u1 = O.fu1d(u, g)
        with ThreadPoolExecutor(nw) as ex:
            u2 = sum(ex.map(lambda ks: O.fu2d(u1, g, kv_list=ks), sets))
        O.f2d_inv(u2)
        r = O.f2d(d)
        with ThreadPoolExecutor(nw) as ex:
            a1 = sum(ex.map(lambda ks: O.fu2d_adj(r, g, kv_list=ks), sets))
        O.fu1d_adj(a1, g)
        times.append(time.perf_counter() - t)
    return {"seconds_per_pair": float(np.median(times)), "runs": times, "workload": "lam256", "threads": nw}


def sampled_oracle_check(plan, u_host, kv_list):
    """c64 GPU L^ u vs the FP64 oracle on a few k_v slices (full F_u1D on the host)."""
    import numpy as np
    import torch

    from oracle import lam_oracle as O

    g = O.Geometry(plan.n0, plan.n1, plan.n2, plan.ntheta, plan.phi, plan.h, plan.w, 2, plan.m)
    u1 = O.fu1d(u_host, g)
    ref = O.fu2d(u1, g, kv_list=kv_list)[:, kv_list, :]
    got = plan.fwd_hat(torch.from_numpy(u_host).to(plan.dtype).cuda())[:, kv_list, :].cpu().numpy()
    return O.relerr(got.astype(np.complex128), ref)


def memo_study(lam, I, dev, wl_name="lam256", n_outer=20, n_inner=4,
               taus=(0.86, 0.88, 0.90, 0.92, 0.94, 0.96, 0.99, 0.999, 0.9999)):
    """Memoized ADMM-TV (Section 4.4) against the plain one on a synthetic workload: the plain
    device step gives R_comp, the memoized step at each tau gives R_LB; accuracy = 1 - |R_comp -
    R_LB|_F / |R_comp|_F (the evaluation section's metric), hit rates of the four operators' private
    caches (chunks of 16 rows / slices, sketch keys of 1024), and the time per ADMM step with the
    caches, without any hit (tau = 2: the same recomputing LSP) and for the plain step."""
    import torch

    wl = I.WORKLOADS[wl_name]
    n, nt, h = wl["n"], wl["ntheta"], wl["det"]
    phi = math.radians(wl["phi_deg"])
    plan = lam.Plan(n, ntheta=nt, phi=phi, h=h, w=h, dtype=torch.complex64, device=dev)
    u_true = I.blob_phantom_torch((n, n, n), I.draw_blobs(wl["seed"], wl["nblobs"], cube_layer=wl["cubes"], n=n),
                                  dev, torch.float32)
    dre = plan.fwd(u_true).real
    noise = torch.from_numpy(I.gaussian_noise(tuple(dre.shape), wl["seed"], 0.01 * dre.abs().max().item())).to(dev)
    dhat = plan.data_hat(torch.complex(dre + noise.float(), torch.zeros_like(dre)))
    del dre, noise, u_true

    def run(tau):
        memo = None if tau is None else lam.Memo(plan, tau=tau, chunk_y=16, chunk_kv=16, key_dim=1024, seed=1)
        s = lam.AdmmTV(plan, 1e-3, rho0=0.5, memo=memo)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(n_outer):
            s.step(dhat, n_inner)
        e1.record()
        torch.cuda.synchronize()
        return s, memo, e0.elapsed_time(e1) / n_outer

    ref, _, ms_plain = run(None)
    _, m2, ms_nohit = run(2.0)
    rows = []
    for tau in taus:
        s, m, ms = run(tau)
        acc = 1.0 - ((s.u - ref.u).norm() / ref.u.norm()).item()
        rows.append({"tau": tau, "accuracy": acc, "hit_rate": m.hit_rate(), "ms_per_step": ms,
                     "hits_misses": m.stats()})
        log(f"[bench] memo tau {tau}: accuracy {acc:.4f}, hit rate {m.hit_rate():.3f}, {ms:.2f} ms per step")
    return {"workload": f"{wl_name} (tilt {wl['phi_deg']:g} deg) phantom + 1 % noise, alpha 1e-3, "
                        f"{n_outer} outer x {n_inner} inner, chunks of 16, sketch keys of 1024",
            "ms_per_step_plain": ms_plain, "ms_per_step_no_hits": ms_nohit, "table": rows}


def offload_study(lam, I, dev, wl_name="lam512", n_inner=4):
    """ADMM-Offload planning (Section 5.1) for one ADMM-TV iteration of the given workload on this
    GPU: phase durations from timings of the device step (t(n) = a + n b for n inner iterations,
    L^ timed alone, the remainder split between the RSP with the multiplier update and the penalty
    update by their bytes), the host link's bandwidth from pinned 1 GiB copies each way, and the
    ADMM variables of the paper's formulation with their accesses: g = psi - lambda/rho formed at the
    LSP's start and read through it, psi and lambda read there and updated in the RSP, D = psi -
    psi_prev written in the RSP and read by the penalty update, the CG work written and used in the
    LSP; u stays resident.  Reports the planner's choice, and M and T of the paper's choice
    (psi, lambda, g), with and without a memory budget of half the variables."""
    import torch

    wl = I.WORKLOADS[wl_name]
    n, nt, h = wl["n"], wl["ntheta"], wl["det"]
    plan = lam.Plan(n, ntheta=nt, phi=math.radians(wl["phi_deg"]), h=h, w=h, dtype=torch.complex64, device=dev)
    d = I.random_complex_torch(plan.data_shape, wl["seed"] + 200, dev, torch.complex64)
    dhat = plan.data_hat(d)
    u0 = torch.zeros(plan.vol_shape, dtype=torch.complex64, device=dev)
    r = torch.empty_like(d)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    s = lam.AdmmTV(plan, 1e-3, rho0=0.5)
    t1 = timed(lambda: s.step(dhat, 1))
    tn = timed(lambda: s.step(dhat, n_inner))
    b = (tn - t1) / (n_inner - 1)
    a = t1 - b
    t_fwd = timed(lambda: plan.fwd_hat(u0, dhat, out=r))
    V = n * n * n
    rest = max(a - t_fwd, 1e-6)
    t_rsp, t_pen = rest * 16.0 / 19.0, rest * 3.0 / 19.0          # bytes: RSP 16 V floats, penalty 3 V
    t_lsp = t_fwd + n_inner * b
    t_g = 9.0 * V * 4 / 4.5e12                                      # forming g: read psi, lambda, write g
    host = torch.empty(1 << 30, dtype=torch.uint8, pin_memory=True)
    devb = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    h2d = timed(lambda: devb.copy_(host, non_blocking=True))
    d2h = timed(lambda: host.copy_(devb, non_blocking=True))
    link = (1 << 30) / max(h2d, d2h)
    del host, devb
    f4 = 4.0 * V
    P = nt * h * h
    variables = {
        "psi": {"bytes": 3 * f4, "access": {0: (0.0, t_g, False), 1: (0.0, t_rsp, False)}},
        "lambda": {"bytes": 3 * f4, "access": {0: (0.0, t_g, False), 1: (0.0, t_rsp, False)}},
        "g": {"bytes": 3 * f4, "access": {0: (0.0, t_lsp, True)}},
        "D": {"bytes": 3 * f4, "access": {1: (0.0, t_rsp, True), 2: (0.0, t_pen, False)}},
        "cg_work": {"bytes": 2 * f4 + 4 * 4.0 * P, "access": {0: (0.0, t_lsp, True)}},
    }
    phases = [t_lsp, t_rsp, t_pen]
    resident = f4                                                    # u
    total = resident + sum(v["bytes"] for v in variables.values())
    out = {"workload": f"{wl_name}, complex64, {n_inner} inner", "phase_s": phases, "link_GBps": link / 1e9,
           "bytes_total": total, "plan": lam.offload_plan(phases, variables, resident, link),
           "paper_choice": lam.offload_evaluate(phases, variables, resident, link, ["psi", "lambda", "g"]),
           "plan_budget_half": lam.offload_plan(phases, variables, resident, link, budget=0.5 * total)}
    log(f"[bench] offload: phases {[round(x * 1e3, 2) for x in phases]} ms, link {link / 1e9:.1f} GB/s; plan "
        f"{out['plan']['offload']} M {out['plan']['M'] / 1e9:.2f} GB T {out['plan']['T'] * 1e3:.2f} ms; "
        f"psi/lambda/g: M {out['paper_choice']['M'] / 1e9:.2f} GB T {out['paper_choice']['T'] * 1e3:.2f} ms")
    return out


def source_digest() -> str:
    """SHA-256 over the HIP sources: counter-derived figures are valid only for the kernels they were taken on."""
    import hashlib
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2511_01893_amd", "csrc")
    hsh = hashlib.sha256()
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            hsh.update(f.encode())
            hsh.update(open(os.path.join(csrc, f), "rb").read())
    return hsh.hexdigest()


def measured_traffic(workload: str, kernel: str, slab: int):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading),
    from the committed counter summary of this workload; None if there is none, it was taken with
    another slab, or the kernels have changed since."""
    f = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", f"traffic_{workload}.json")
    if not os.path.exists(f):
        return None
    t = json.load(open(f))
    if t.get("source_sha256") != source_digest() or t.get("slab") != slab or kernel not in t.get("kernels", {}):
        return None
    return t["kernels"][kernel]["hbm_bytes_per_launch"]


# ---------------------------------------------------------------- profile summaries (profiles/)
PROF_SHORT = {"k_zfwd": "zfwd", "k_ycol_fwd": "ycol_fwd", "k_xrow_fwd": "xrow_fwd", "k_gather": "gather",
         "k_rowfft": "rowfft", "k_colfft": "colfft", "k_scatter_fx": "scatter", "k_scatter": "scatter",
         "k_xrow_adj": "xrow_adj", "k_ycol_adj": "ycol_adj", "k_zadj": "zadj"}
PROF_ORDER = ["zfwd", "ycol_fwd", "xrow_fwd", "gather", "rowfft", "colfft", "scatter", "xrow_adj", "ycol_adj", "zadj"]
PROF_COPY = "__amd_rocclr_copyBuffer"


def prof_short(name):
    m = re.search(r"lam::(k_[a-z_]+)<", name)
    return PROF_SHORT.get(m.group(1)) if m else None


def prof_stats(path):
    out, total = {}, 0.0
    for r in csv.DictReader(open(path)):
        total += float(r["TotalDurationNs"])
        k = prof_short(r["Name"])
        if k:
            c, t = out.get(k, (0, 0.0))
            out[k] = (c + int(r["Calls"]), t + float(r["TotalDurationNs"]))
    return out, total


def prof_counters(path):
    per = defaultdict(lambda: defaultdict(list))
    copies = defaultdict(list)
    for r in csv.DictReader(open(path)):
        v = float(r["Counter_Value"])
        if r["Kernel_Name"] == PROF_COPY:
            copies[(r["Dispatch_Id"], r["Counter_Name"])].append(v)
            continue
        k = prof_short(r["Kernel_Name"])
        if k:
            per[k][(r["Dispatch_Id"], r["Counter_Name"])].append(v)
    # a dispatch's counter summed over its instances (XCDs / shader engines), then averaged over dispatches
    avg = {}
    for k, d in per.items():
        by = defaultdict(list)
        for (disp, c), vals in d.items():
            by[c].append(sum(vals))
        avg[k] = {c: sum(v) / len(v) for c, v in by.items()}
    cp = defaultdict(list)
    for (disp, c), vals in copies.items():
        cp[c].append(sum(vals))
    return avg, cp


def prof_bench_json(log):
    for line in open(log):
        if line.startswith("{"):
            return json.loads(line)
    raise RuntimeError(f"no JSON line in {log}")


def summarize_profiles(d):
    """Writes profiles/kernels_lam512.md, profiles/traffic_lam512.json and profiles/kernels_lam1536.md
    from the rocprofv3 output under d (kt512/, fetch/, write/, sq1/, sq2/, kt1536/ and the logs of
    the profiled bench runs, kt512.log and kt1536.log)."""
    HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
    kt, total = prof_stats(os.path.join(d, "kt512", "kt_kernel_stats.csv"))
    res = prof_bench_json(os.path.join(d, "kt512.log"))
    cfg = res["config"]
    n, nt, h, slab = cfg["n"], cfg["ntheta"], cfg["det"], cfg["slab"]

    class P:
        n0 = n1 = n2 = n
        ntheta, w = nt, h
    P.h = h
    fetch, fcp = prof_counters(os.path.join(d, "fetch", "fetch_counter_collection.csv"))
    write, wcp = prof_counters(os.path.join(d, "write", "write_counter_collection.csv"))
    # calibration: the 1 GiB copy (the largest copy dispatch) moves 1 GiB each way
    wmax = max(wcp["WRITE_SIZE"])
    fmax = max(fcp["FETCH_SIZE"])
    sf, sw = (1 << 20) / fmax, (1 << 20) / wmax
    sq1, _ = prof_counters(os.path.join(d, "sq1", "sq1_counter_collection.csv"))
    sq2, _ = prof_counters(os.path.join(d, "sq2", "sq2_counter_collection.csv"))
    traffic = {"workload": "lam512", "slab": slab, "source_sha256": source_digest(), "scale_fetch": sf,
               "scale_write": sw,
               "calibration": f"1 GiB device-to-device copy ({PROF_COPY}): FETCH_SIZE {fmax:.0f} KiB, WRITE_SIZE {wmax:.0f} KiB",
               "kernels": {}}
    rows = []
    for k in PROF_ORDER:
        calls, tns = kt[k]
        avg_us = tns / calls / 1e3
        alg = kernel_units(k, P, 8, 8, slab)
        fk, wk = fetch[k]["FETCH_SIZE"], write[k]["WRITE_SIZE"]
        hbm = (fk * sf + wk * sw) * 1024
        traffic["kernels"][k] = {"fetch_kib_per_launch": fk, "write_kib_per_launch": wk, "hbm_bytes_per_launch": int(hbm)}
        rows.append((k, calls, avg_us, 100 * tns / total, alg, alg / (avg_us * 1e3), hbm, hbm / (avg_us * 1e3)))
    json.dump(traffic, open(os.path.join(HERE, "traffic_lam512.json"), "w"), indent=1)
    dom = res["roofline"]
    pair_kernel_ms = sum(kern["ms_total_per_step"] for kern in res["kernels"].values())
    L = []
    L.append("# Kernel profile: lam512 forward + adjoint pair (complex64)\n")
    L.append("Workload: 512^3 volume, 512 angles, tilt 30 deg, 512 x 512 detector, R = 2, m = 4, "
             f"k_v slabs of {slab}.\n")
    L.append("Commands (from a directory outside the tree, `TMPDIR=/tmp`; `R` = the repository):\n")
    L.append("```")
    b5 = "--steps 5 --warmup 2 --no-cpu --no-check --no-fp64 --no-memo --no-offload --no-1536 --calib-copy"
    b1 = "--steps 1 --warmup 1 --no-cpu --no-check --no-fp64 --no-memo --no-offload --no-1536 --calib-copy"
    L.append(f"rocprofv3 --kernel-trace --stats --output-format csv -d prof/kt512 -o kt -- python3 $R/bench.py {b5}")
    L.append(f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d prof/fetch -o fetch -- python3 $R/bench.py {b1}")
    L.append(f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d prof/write -o write -- python3 $R/bench.py {b1}")
    L.append("rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAVE_CYCLES SQ_BUSY_CYCLES "
             f"SQ_WAIT_INST_LDS SQ_INSTS_VMEM_RD --output-format csv -d prof/sq1 -o sq1 -- python3 $R/bench.py {b1}")
    L.append("rocprofv3 --pmc SQ_LDS_BANK_CONFLICT SQ_LDS_ADDR_CONFLICT SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_VALU "
             "SQ_INSTS_LDS_ATOMIC SQ_WAIT_ANY SQ_INSTS_SMEM SQ_INSTS_VMEM_WR --output-format csv -d prof/sq2 -o sq2 "
             f"-- python3 $R/bench.py {b1}")
    L.append("python3 $R/bench.py --summarize-profiles prof")
    L.append("```\n")
    L.append(f"Kernel trace ({kt['zfwd'][0]} pairs: warm-up, timed, and bench's per-kernel event pass; the gather and "
             "spread also run in the frequency-domain pair):\n")
    L.append("| kernel | calls | avg us | % of GPU time | algorithmic bytes / launch | algorithmic GB/s | "
             "HBM bytes / launch (counters) | HBM GB/s |")
    L.append("|---|---|---|---|---|---|---|---|")
    for k, calls, avg_us, pct, alg, ag, hbm, hg in rows:
        L.append(f"| {k} | {calls} | {avg_us:.1f} | {pct:.1f} | {alg / 1e6:.1f} MB | {ag:.0f} | {hbm / 1e6:.1f} MB | {hg:.0f} |")
    L.append("")
    L.append(f"The bench line of the traced run: pair {res['ms_per_step']:.3f} ms ({res['value']:.2f} pairs/s); "
             f"kernel time per pair from its HIP events {pair_kernel_ms:.2f} ms. Dominant kernel "
             f"`{dom['kernel']}`: {dom['avg_launch_ms'] * 1e3:.1f} us per launch by the bench's HIP events, "
             f"{dict((r[0], r[2]) for r in rows)[dom['kernel']]:.1f} us by the trace above "
             "(the trace's average also holds the frequency-domain pair's launches).\n")
    L.append(f"HBM byte counters are scaled by a plain 1 GiB copy measured in the same runs: FETCH_SIZE reads "
             f"{fmax:.0f} KiB for the copy's 1048576 KiB (factor {sf:.3f}), WRITE_SIZE {wmax:.0f} KiB (factor {sw:.3f}).\n")
    L.append("SQ counters, per dispatch (summed over the counter instances, averaged over dispatches):\n")
    cols = [("WAVES", sq1, "SQ_WAVES"), ("INSTS_VALU", sq1, "SQ_INSTS_VALU"), ("INSTS_SALU", sq1, "SQ_INSTS_SALU"),
            ("INSTS_LDS", sq1, "SQ_INSTS_LDS"), ("INSTS_LDS_ATOMIC", sq2, "SQ_INSTS_LDS_ATOMIC"),
            ("ACTIVE_INST_LDS", sq2, "SQ_ACTIVE_INST_LDS"), ("ACTIVE_INST_VALU", sq2, "SQ_ACTIVE_INST_VALU"),
            ("LDS_BANK_CONFLICT", sq2, "SQ_LDS_BANK_CONFLICT"), ("WAIT_INST_LDS", sq1, "SQ_WAIT_INST_LDS"),
            ("WAVE_CYCLES", sq1, "SQ_WAVE_CYCLES"), ("WAIT_ANY", sq2, "SQ_WAIT_ANY"), ("BUSY_CYCLES", sq1, "SQ_BUSY_CYCLES")]
    L.append("| kernel | " + " | ".join(c[0] for c in cols) + " |")
    L.append("|---|" + "---|" * len(cols))
    for k in PROF_ORDER:
        L.append(f"| {k} | " + " | ".join(f"{src[k].get(cn, float('nan')):.3g}" for _, src, cn in cols) + " |")
    open(os.path.join(HERE, "kernels_lam512.md"), "w").write("\n".join(L) + "\n")

    kt15, total15 = prof_stats(os.path.join(d, "kt1536", "kt_kernel_stats.csv"))
    r15 = prof_bench_json(os.path.join(d, "kt1536.log"))
    c15 = r15["config"]
    M = ["# Kernel profile: lam1536 forward + adjoint pair (complex64)\n",
         f"Workload: 1536^3 volume, 1536 angles, tilt 20 deg, 1536 x 1536 detector, R = 2, m = 4, k_v slabs of {c15['slab']} "
         "(transforms of 3072 = 3·2^10 and 1536 = 3·2^9 points).\n",
         "```",
         "rocprofv3 --kernel-trace --stats --output-format csv -d prof/kt1536 -o kt -- python3 $R/bench.py --workload lam1536 "
         "--steps 2 --warmup 1 --no-cpu --no-check --no-fp64 --no-memo --no-offload",
         "python3 $R/bench.py --summarize-profiles prof",
         "```\n",
         "| kernel | calls | avg us | % of GPU time |", "|---|---|---|---|"]
    for k in PROF_ORDER:
        calls, tns = kt15[k]
        M.append(f"| {k} | {calls} | {tns / calls / 1e3:.1f} | {100 * tns / total15:.1f} |")
    M.append("")
    M.append(f"The bench line of the traced run: pair {r15['ms_per_step']:.1f} ms ({r15['value']:.3f} pairs/s); dominant "
             f"kernel `{r15['roofline']['kernel']}` {r15['roofline']['avg_launch_ms'] * 1e3:.1f} us per launch by the "
             "bench's HIP events.")
    open(os.path.join(HERE, "kernels_lam1536.md"), "w").write("\n".join(M) + "\n")



def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lam512")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the complex128 comparison")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled oracle accuracy check")
    ap.add_argument("--slab", type=int, default=0, help="k_v slices per 2D-step slab (0: automatic)")
    ap.add_argument("--no-memo", action="store_true", help="skip the memoized ADMM-TV study")
    ap.add_argument("--no-offload", action="store_true", help="skip the ADMM-Offload planning study")
    ap.add_argument("--no-1536", action="store_true",
                    help="skip the pair at the 1.5K^3 shape (1536^3, 1536 angles, 1536^2 detector)")
    ap.add_argument("--oracle-c2", action="store_true",
                    help="also time three full FP64 oracle pairs at 256^3 (several minutes of host time)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (reference kernel for HBM byte counters)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write the summaries in profiles/ from the rocprofv3 output under DIR, then exit")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the operator runs on one GPU: --gpus must be 1 (the sharded design is described, not built)", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2511_01893_amd import inputs as I
    from paper_2511_01893_amd import lam

    wl = I.WORKLOADS[args.workload]
    n, nt, h = wl["n"], wl["ntheta"], wl["det"]
    phi = math.radians(wl["phi_deg"])
    dev = torch.device("cuda:0")
    log(f"[bench] workload {args.workload}: n={n} ntheta={nt} det={h} phi={wl['phi_deg']} c64")

    plan = lam.Plan(n, ntheta=nt, phi=phi, h=h, w=h, dtype=torch.complex64, device=dev, slab=args.slab)
    blobs = I.draw_blobs(wl["seed"], wl["nblobs"], cube_layer=wl["cubes"], n=n)
    u = I.blob_phantom_torch((n, n, n), blobs, dev, torch.float32).to(torch.complex64)
    d = I.random_complex_torch((nt, h, h), wl["seed"] + 200, dev, torch.complex64)
    torch.cuda.synchronize()

    if args.calib_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ms, wall_ms, d64, u64 = time_pairs(plan, u, d, args.steps, args.warmup)
    log(f"[bench] c64 pair {ms:.3f} ms (host wall {wall_ms:.3f} ms)")
    B_pair = 2 * algorithmic_bytes(n, n, n, nt, h, h, 8, 8)

    # per-kernel durations: second pass of the same steps with events around every kernel
    plan.profile(True)
    for _ in range(args.steps):
        plan.fwd(u)
        plan.adj(d)
    prof = plan.profile_read()
    plan.profile(False)
    kern = {}
    for name, (tot, cnt) in prof.items():
        if cnt:
            kern[name] = {"ms_total_per_step": tot / args.steps, "launches_per_step": cnt / args.steps,
                          "avg_launch_ms": tot / cnt}
    dom = max(kern, key=lambda k: kern[k]["ms_total_per_step"])
    log("[bench] kernels: " + ", ".join(f"{k} {v['ms_total_per_step']:.3f} ms/step x{v['launches_per_step']:.0f}"
                                        for k, v in kern.items()))
    # slab of this plan = h / launches of gather per op
    plan_slab = int(round(h / kern["gather"]["launches_per_step"])) if "gather" in kern else h
    bytes_launch = kernel_units(dom, plan, 8, 8, plan_slab)
    ach = bytes_launch / (kern[dom]["avg_launch_ms"] * 1e-3) / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(args.workload, dom, plan_slab),
            "bytes_per_launch": bytes_launch, "avg_launch_ms": kern[dom]["avg_launch_ms"]}

    # the frequency-domain pair that the CG loop runs (Algorithm 2): L^ u - d^ and L^* r
    r = torch.empty_like(d)
    uh = torch.empty_like(u)
    for _ in range(args.warmup):
        plan.fwd_hat(u, d, out=r)
        plan.adj_hat(r, out=uh)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        plan.fwd_hat(u, d, out=r)
        plan.adj_hat(r, out=uh)
    e1.record()
    torch.cuda.synchronize()
    ms_hat = e0.elapsed_time(e1) / args.steps
    log(f"[bench] frequency-domain pair (L^, L^*) {ms_hat:.3f} ms")
    del r, uh
    flops = pair_flops(n, n, n, nt, h, h)
    G_bytes = 2 * 2 * (4 * n * n * h * 8)          # per operator the oversampled grid written and read
    alu = {"flops_per_pair": flops, "achieved_tflops": flops / (ms * 1e-3) / 1e12,
           "frac_fp32_78.6": flops / (ms * 1e-3) / (FP32_VALU_TFLOPS * 1e12),
           "frac_fp32_157.3": flops / (ms * 1e-3) / (157.3e12),
           "note": "78.6 TFLOP/s: 256 CU x 64 lanes x FMA x 2.4 GHz, packed FP32 disabled; 157.3 with packing"}

    result = {
        "metric": f"lam fwd+adj pairs/s at {n}^3 (c64 vs FP64, rel err <=1e-4); % HBM roofline",
        "value": 1000.0 / ms,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n}^3 volume, {nt} angles, tilt {wl['phi_deg']:g} deg, "
                               f"{h}x{h} detector, R=2, m=4, blob phantom seed {wl['seed']}",
                   "n": n, "ntheta": nt, "det": h, "phi_deg": wl["phi_deg"], "oversample": 2, "m": 4,
                   "slab": plan_slab},
        "pair_algorithmic_bytes": B_pair,
        "pair_hbm_frac": B_pair / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "pair_hbm_frac_with_grid": (B_pair + G_bytes) / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "hat_pair_ms": ms_hat,
        # L^ u - d^: u read, u1 written and read, d^ read, r written; L^* r: r read, u1 written and read, u written
        "hat_pair_hbm_frac": (B_pair - 3 * 8 * nt * h * h) / (ms_hat * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "alu": alu,
        "roofline": roof,
        "kernels": kern,
    }

    if not args.no_fp64:
        plan128 = lam.Plan(n, ntheta=nt, phi=phi, h=h, w=h, dtype=torch.complex128, device=dev)
        u128, d128 = u.to(torch.complex128), d.to(torch.complex128)
        ms128, _, dd, uu = time_pairs(plan128, u128, d128, max(3, args.steps // 2), 1)
        result["fp64_ms_per_step"] = ms128
        result["fp64_pairs_per_s"] = 1000.0 / ms128
        result["speedup_vs_fp64"] = ms128 / ms
        e_f = ((d64.to(torch.complex128) - dd).norm() / dd.norm()).item()
        e_a = ((u64.to(torch.complex128) - uu).norm() / uu.norm()).item()
        result["accuracy"] = {"c64_vs_c128_fwd": e_f, "c64_vs_c128_adj": e_a}
        log(f"[bench] c128 pair {ms128:.3f} ms; c64 vs c128 fwd {e_f:.2e} adj {e_a:.2e}")
        del plan128, u128, d128, dd, uu
        torch.cuda.empty_cache()

    if not args.no_check:
        t = time.perf_counter()
        kvs = [h // 2 - h // 4, h // 2 + 3]
        err = sampled_oracle_check(plan, u.real.double().cpu().numpy().astype(np.complex128), kvs)
        result.setdefault("accuracy", {})["c64_vs_oracle_fwd_hat_sampled"] = err
        result["accuracy"]["oracle_sample"] = f"L^ u on k_v slices {kvs} (all angles, all k_u)"
        log(f"[bench] c64 vs oracle (slices {kvs}) {err:.2e} in {time.perf_counter() - t:.1f} s")

    if not args.no_memo:
        t = time.perf_counter()
        result["memo"] = memo_study(lam, I, dev)
        log(f"[bench] memo study in {time.perf_counter() - t:.1f} s")
        torch.cuda.empty_cache()

    if not args.no_offload:
        t = time.perf_counter()
        result["offload"] = offload_study(lam, I, dev, args.workload)
        log(f"[bench] offload study in {time.perf_counter() - t:.1f} s")
        torch.cuda.empty_cache()

    if not args.no_1536 and args.workload == "lam512":
        # the paper's second default dataset shape: transforms of 3 2^k points; measured after the
        # 512^3 objects are freed (its plan, volume and data take ~130 GB)
        t = time.perf_counter()
        del plan, u, d, d64, u64
        torch.cuda.empty_cache()
        w15 = I.WORKLOADS["lam1536"]
        n15 = w15["n"]
        p15 = lam.Plan(n15, ntheta=w15["ntheta"], phi=math.radians(w15["phi_deg"]), h=w15["det"], w=w15["det"],
                       dtype=torch.complex64, device=dev)
        u15 = I.blob_phantom_torch((n15, n15, n15), I.draw_blobs(w15["seed"], 64), dev, torch.float32)
        d15 = I.random_complex_torch(p15.data_shape, w15["seed"] + 200, dev, torch.complex64)
        ms15, _, _, _ = time_pairs(p15, u15.to(torch.complex64), d15, 3, 1)
        result["lam1536"] = {"workload": "1536^3 volume, 1536 angles, tilt 20 deg, 1536x1536 detector, R=2, m=4, "
                                         "c64 (transforms of 3072 = 3 2^10 and 1536 = 3 2^9 points)",
                             "ms_per_pair": ms15, "pairs_per_s": 1000.0 / ms15, "steps": 3,
                             "pair_hbm_frac": 2 * algorithmic_bytes(n15, n15, n15, w15["ntheta"], n15, n15, 8, 8)
                             / (ms15 * 1e-3) / (HBM_PEAK_GBS * 1e9)}
        log(f"[bench] 1536^3 pair {ms15:.1f} ms in {time.perf_counter() - t:.1f} s")
        del p15, u15, d15
        torch.cuda.empty_cache()

    if not args.no_cpu:
        t = time.perf_counter()
        result["cpu_baseline"] = cpu_baseline(wl)
        result["cpu_baseline"].update(host_info())
        log(f"[bench] cpu baseline {result['cpu_baseline']['value']:.3e} pairs/s in {time.perf_counter() - t:.1f} s")

    if args.oracle_c2:
        t = time.perf_counter()
        result["oracle_pair_lam256"] = oracle_pair_c2()
        log(f"[bench] oracle 256^3 pair {result['oracle_pair_lam256']['seconds_per_pair']:.1f} s (median of 3)")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
