"""GPU parity at the study's configurations and on the compile-time-size kernels.

* 256^3 (256 angles, tilt 20 deg, 256^2 detector): the full forward L u and
  adjoint L* d, complex64 and complex128, each against the FP64 oracle on the
  whole arrays (the relative L2 error of each is printed).
* Compile-time FFT sizes (transform lengths 512, 1024, 2048; 2D DFTs of 512^2
  and 1024^2): rectangular geometries with one axis or the detector at those
  sizes, full L and L* against the oracle; at 512^3 the centred 2D DFT passes
  of L and L* against numpy on every projection.
* ADMM-TV: 128^3 (4 x 4 tiles of the oversampled grid, row-pair spread),
  3 outer x 4 inner iterations against the oracle's admm_step per iterate;
  the 512^3 workload (64 blobs + cubes, tilt 30 deg, 1 % noise, alpha = 1e-3,
  4 outer x 4 inner), complex64 against complex128 per iterate.

The oracle calls at 256^3 run one k_v slice set per thread (the oracle's
slice-restricted entry points, summed); nothing of the HIP path enters them.
"""
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

from oracle import lam_oracle as O
from paper_2511_01893_amd import inputs as I

pytestmark = pytest.mark.gpu

NW = len(os.sched_getaffinity(0))


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01893_amd import lam
    lam.lib()
    return lam


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


def report(name, err, tol):
    print(f"{name}: rel err {err:.3e} (bar {tol:.0e})", flush=True)
    assert err <= tol, (name, err, tol)


def oracle_fwd_adj(u, d, g):
    """O.lam_fwd(u), O.lam_adj(d) with F_u2D / F*_u2D split over k_v slice sets on threads."""
    sets = [list(range(i, g.h, NW)) for i in range(NW)]
    u1 = O.fu1d(u, g)
    with ThreadPoolExecutor(NW) as ex:
        u2 = sum(ex.map(lambda ks: O.fu2d(u1, g, kv_list=ks), sets))
    fwd = O.f2d_inv(u2)
    r = O.f2d(d)
    with ThreadPoolExecutor(NW) as ex:
        a1 = sum(ex.map(lambda ks: O.fu2d_adj(r, g, kv_list=ks), sets))
    return fwd, O.fu1d_adj(a1, g)


# ---------------------------------------------------------------- 256^3
@pytest.fixture(scope="module")
def c2_ref():
    w = I.WORKLOADS["lam256"]
    n = w["n"]
    g = O.Geometry(n, n, n, w["ntheta"], math.radians(w["phi_deg"]), w["det"], w["det"], 2, 4)
    u = I.blob_phantom(g.vol_shape, I.draw_blobs(w["seed"], w["nblobs"]))
    d = I.random_detector_data(g.data_shape, w["seed"])
    fwd, adj = oracle_fwd_adj(u, d, g)
    return g, u, d, fwd, adj


@pytest.mark.parametrize("dtype,tol", [(torch.complex64, 1e-4), (torch.complex128, 1e-12)], ids=["c64", "c128"])
def test_lam256_full_pair_vs_oracle(L, c2_ref, dtype, tol):
    g, u, d, fwd, adj = c2_ref
    plan = L.Plan(g.n0, ntheta=g.ntheta, phi=g.phi, h=g.h, w=g.w, dtype=dtype)
    rdt = torch.float32 if dtype == torch.complex64 else torch.float64
    got_f = plan.fwd(torch.from_numpy(u).to(rdt).cuda())
    got_a = plan.adj(torch.from_numpy(d).to(dtype).cuda())
    tag = "c64" if dtype == torch.complex64 else "c128"
    report(f"256^3 {tag} L u vs oracle", O.relerr(host(got_f), fwd), tol)
    report(f"256^3 {tag} L* d vs oracle", O.relerr(host(got_a), adj), tol)


# ---------------------------------------------------------------- compile-time sizes
@pytest.mark.parametrize("dtype,tol", [(torch.complex64, 1e-4), (torch.complex128, 1e-12)], ids=["c64", "c128"])
@pytest.mark.parametrize("case", [
    dict(n0=1024, n1=32, n2=32, ntheta=6, phi=25.0, h=64, w=32),      # z transforms of 2048 points
    dict(n0=512, n1=16, n2=16, ntheta=2, phi=30.0, h=768, w=16),      # z of 1024, more rows than threads
    dict(n0=16, n1=1024, n2=32, ntheta=5, phi=30.0, h=16, w=32),      # y transforms of 2048 points
    dict(n0=16, n1=32, n2=1024, ntheta=3, phi=30.0, h=16, w=64),      # x transforms of 2048 points
    dict(n0=16, n1=512, n2=512, ntheta=3, phi=20.0, h=16, w=512),     # y, x of 1024; 2D DFT rows of 512
    dict(n0=32, n1=32, n2=32, ntheta=2, phi=20.0, h=1024, w=1024),    # 2D DFT of 1024^2
    dict(n0=32, n1=32, n2=32, ntheta=3, phi=35.0, h=512, w=512),      # 2D DFT of 512^2
], ids=["z2048", "zrows768", "y2048", "x2048", "yx1024", "dft1024", "dft512"])
def test_compile_time_sizes_vs_oracle(L, dtype, tol, case):
    c = dict(case)
    phi = math.radians(c["phi"])
    plan = L.Plan(c["n0"], c["n1"], c["n2"], ntheta=c["ntheta"], phi=phi, h=c["h"], w=c["w"], dtype=dtype)
    g = O.Geometry(c["n0"], c["n1"], c["n2"], c["ntheta"], phi, c["h"], c["w"], 2, 4)
    u = I.random_complex(g.vol_shape, 41)
    d = I.random_detector_data(g.data_shape, 41)
    report("fwd", O.relerr(host(plan.fwd(torch.from_numpy(u).to(dtype).cuda())), O.lam_fwd(u, g)), tol)
    report("adj", O.relerr(host(plan.adj(torch.from_numpy(d).to(dtype).cuda())), O.lam_adj(d, g)), tol)
    report("data_hat", O.relerr(host(plan.data_hat(torch.from_numpy(d).to(dtype).cuda())), O.f2d_unnorm(d)),
           1e-5 if dtype == torch.complex64 else 1e-12)


def test_lam512_2d_dft_passes_vs_numpy(L):
    """At the benchmark's size the centred 2D DFT passes of L (F*_2D) and L* (F_2D)
    against numpy on every projection: L u = F*_2D(L^ u) and L* d = L^*(F_2D d)."""
    w = I.WORKLOADS["lam512"]
    n = w["n"]
    plan = L.Plan(n, ntheta=w["ntheta"], phi=math.radians(w["phi_deg"]), h=w["det"], w=w["det"])
    u = I.blob_phantom_torch((n, n, n), I.draw_blobs(w["seed"], w["nblobs"], cube_layer=True, n=n), "cuda",
                             torch.float32).to(torch.complex64)
    uh = host(plan.fwd_hat(u))
    report("512^3 L u vs F*_2D(L^ u) (numpy)", O.relerr(host(plan.fwd(u)), O.f2d_inv(uh)), 1e-5)
    del uh
    d = I.random_complex_torch(plan.data_shape, w["seed"] + 200, "cuda", torch.complex64)
    rh = torch.from_numpy(O.f2d(host(d))).to(torch.complex64).cuda()
    report("512^3 L* d vs L^*(F_2D d) (numpy)", O.relerr(host(plan.adj(d)), host(plan.adj_hat(rh))), 1e-5)
    report("512^2 data_hat vs numpy", O.relerr(host(plan.data_hat(d)), O.f2d_unnorm(host(d))), 1e-5)


# ---------------------------------------------------------------- ADMM-TV
@pytest.fixture(scope="module")
def admm128_ref():
    n, nt = 128, 32
    g = O.Geometry(n, n, n, nt, math.radians(30.0), n, n, 2, 4)
    u_true = I.blob_phantom(g.vol_shape, I.draw_blobs(6, 8))
    d = O.lam_fwd(u_true, g).real.astype(np.complex128)
    dhat = O.f2d_unnorm(d)
    alpha = 1e-3
    u = np.zeros(g.vol_shape)
    psi = np.zeros((3,) + g.vol_shape)
    lam = np.zeros_like(psi)
    rho = 0.5
    its = []
    for it in range(3):
        u, psi, lam, rho = O.admm_step(u, psi, lam, rho, dhat, g, alpha, 4)
        its.append((u, psi, lam, rho))
        print(f"oracle ADMM 128^3 iteration {it} done", flush=True)
    return g, d, alpha, its


@pytest.mark.parametrize("dtype,tol", [(torch.complex64, 1e-4), (torch.complex128, 1e-9)], ids=["c64", "c128"])
def test_admm_128_vs_oracle(L, admm128_ref, dtype, tol):
    g, d, alpha, its = admm128_ref
    plan = L.Plan(g.n0, ntheta=g.ntheta, phi=g.phi, h=g.h, w=g.w, dtype=dtype)
    s = L.AdmmTV(plan, alpha, rho0=0.5)
    dh = plan.data_hat(torch.from_numpy(d).to(dtype).cuda())
    for it, (uo, po, lo, rho) in enumerate(its):
        s.step(dh, 4)
        eu, ep, el = O.relerr(host(s.u), uo), O.relerr(host(s.psi), po), O.relerr(host(s.lam), lo)
        print(f"128^3 iteration {it}: u {eu:.2e} psi {ep:.2e} lambda {el:.2e} rho {s.rho} (oracle {rho})", flush=True)
        assert eu < tol and ep < 10 * tol and el < 10 * tol
        assert s.rho == rho


def test_admm_lam512_c64_vs_c128(L):
    """The 512^3 ADMM-TV run: simulated Re(L u) + 1 % Gaussian noise, alpha = 1e-3,
    4 outer x 4 inner; complex64 against complex128 per iterate; the data misfit falls."""
    w = I.WORKLOADS["lam512"]
    n = w["n"]
    phi = math.radians(w["phi_deg"])
    kw = dict(ntheta=w["ntheta"], phi=phi, h=w["det"], w=w["det"])
    p64 = L.Plan(n, dtype=torch.complex64, **kw)
    p128 = L.Plan(n, dtype=torch.complex128, **kw)
    u_true = I.blob_phantom_torch((n, n, n), I.draw_blobs(w["seed"], w["nblobs"], cube_layer=True, n=n), "cuda",
                                  torch.float64)
    dre = p128.fwd(u_true).real
    sigma = 0.01 * dre.abs().max().item()
    noise = torch.from_numpy(I.gaussian_noise(tuple(dre.shape), w["seed"], sigma)).cuda()
    d = torch.complex(dre + noise, torch.zeros_like(dre))
    del dre, noise
    s64 = L.AdmmTV(p64, 1e-3, rho0=0.5)
    s128 = L.AdmmTV(p128, 1e-3, rho0=0.5)
    dh64 = p64.data_hat(d.to(torch.complex64))
    dh128 = p128.data_hat(d)
    mis0 = d.norm().item()
    worst = 0.0
    for it in range(4):
        s64.step(dh64, 4)
        s128.step(dh128, 4)
        eu = ((s64.u.double() - s128.u).norm() / s128.u.norm()).item()
        ep = ((s64.psi.double() - s128.psi).norm() / s128.psi.norm()).item()
        mis = ((p128.fwd(s128.u) - d).norm() / mis0).item()
        dg = s64.diagnostics()
        print(f"512^3 ADMM iteration {it}: c64 vs c128 u {eu:.2e} psi {ep:.2e}; misfit {mis:.3e}; "
              f"primal {dg['primal']:.3e} dual {dg['dual']:.3e} rho {dg['rho']}", flush=True)
        worst = max(worst, eu)
        assert s64.rho == s128.rho
    assert worst < 1e-3
    assert mis < 0.2
