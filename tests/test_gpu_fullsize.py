"""GPU checks at the benchmark's full size (512^3, 512 angles, 30 deg, 512^2
detector) and at 1024^3 with slabs of 128 slices.

At 512^3 the FP64 oracle evaluates sampled outputs: L^ u on two whole k_v
slices (it needs F_u1D of the whole volume, then F_u2D of those slices only),
and L^* r for data that is non-zero on two slices only (then only those
slices' F*_u2D is needed).  Properties that hold at any size are checked on
the whole arrays: the adjoint identity, complex64 against complex128 (the
same kernels in FP64, pinned to the oracle at smaller sizes).  At 1024^3 the
oracle does not fit this box's test budget; the complex128 instantiation is
the reference there, plus the finite-difference gradient check.
"""
import math

import numpy as np
import pytest
import torch

from oracle import lam_oracle as O
from paper_2511_01893_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01893_amd import lam
    lam.lib()
    return lam


def rel(a, b):
    return ((a - b).norm() / b.norm()).item()


@pytest.fixture(scope="module")
def c3(L):
    w = I.WORKLOADS["lam512"]
    n = w["n"]
    phi = math.radians(w["phi_deg"])
    plan = L.Plan(n, ntheta=w["ntheta"], phi=phi, h=w["det"], w=w["det"], dtype=torch.complex64)
    geo = O.Geometry(n, n, n, w["ntheta"], phi, w["det"], w["det"], 2, 4)
    blobs = I.draw_blobs(w["seed"], w["nblobs"], cube_layer=True, n=n)
    u = I.blob_phantom_torch((n, n, n), blobs, "cuda", torch.float32)
    return plan, geo, u


def test_lam512_fwd_hat_sampled_slices(c3):
    plan, geo, u = c3
    kvs = [100, 256, 401]
    got = plan.fwd_hat(u.to(torch.complex64))[:, kvs, :].cpu().numpy().astype(np.complex128)
    uh = u.double().cpu().numpy()
    ref = O.fu2d(O.fu1d(uh, geo), geo, kv_list=kvs)[:, kvs, :]
    err = O.relerr(got, ref)
    print(f"512^3 L^ u on slices {kvs}: rel err {err:.2e}")
    assert err < 1e-4


def test_lam512_adj_hat_sparse_data(c3):
    plan, geo, _ = c3
    kvs = [37, 300]
    r = torch.zeros(geo.data_shape, dtype=torch.complex64, device="cuda")
    vals = I.random_complex_torch((geo.ntheta, len(kvs), geo.w), 31, "cuda", torch.complex64)
    r[:, kvs, :] = vals
    got = plan.adj_hat(r).cpu().numpy().astype(np.complex128)
    rh = r.cpu().numpy().astype(np.complex128)
    ref = O.fu1d_adj(O.fu2d_adj(rh, geo, kv_list=kvs), geo)
    err = O.relerr(got, ref)
    print(f"512^3 L^* r (r on slices {kvs}): rel err {err:.2e}")
    assert err < 1e-4


def test_lam512_adjoint_and_c128(L, c3):
    plan, geo, u = c3
    uc = u.to(torch.complex64)
    d = I.random_complex_torch(geo.data_shape, 203, "cuda", torch.complex64)
    Lu, Lsd = plan.fwd(uc), plan.adj(d)
    a = torch.vdot(d.reshape(-1).to(torch.complex128), Lu.reshape(-1).to(torch.complex128))
    b = torch.vdot(Lsd.reshape(-1).to(torch.complex128), uc.reshape(-1).to(torch.complex128))
    err = (abs(a - b) / (Lu.to(torch.complex128).norm() * d.to(torch.complex128).norm())).item()
    print(f"512^3 adjoint identity {err:.2e}")
    assert err < 1e-5
    p128 = L.Plan(geo.n0, ntheta=geo.ntheta, phi=geo.phi, h=geo.h, w=geo.w, dtype=torch.complex128)
    e_f = rel(Lu.to(torch.complex128), p128.fwd(uc.to(torch.complex128)))
    e_a = rel(Lsd.to(torch.complex128), p128.adj(d.to(torch.complex128)))
    print(f"512^3 c64 vs c128: fwd {e_f:.2e} adj {e_a:.2e}")
    assert e_f < 1e-4 and e_a < 1e-4


def test_lam1024_slabs_of_128(L):
    """The 1024^3 workload in slabs of 128 slices: complex64 against complex128,
    slabbed against the automatic slab size, and directional finite differences
    of the data term."""
    w = I.WORKLOADS["lam1024"]
    n = w["n"]
    phi = math.radians(w["phi_deg"])
    kw = dict(ntheta=w["ntheta"], phi=phi, h=w["det"], w=w["det"])
    p64 = L.Plan(n, dtype=torch.complex64, slab=128, **kw)
    u = I.blob_phantom_torch((n, n, n), I.draw_blobs(w["seed"], w["nblobs"]), "cuda", torch.float32)
    d = I.random_complex_torch((w["ntheta"], n, n), w["seed"] + 200, "cuda", torch.complex64)
    Lu = p64.fwd(u)
    Lsd = p64.adj(d, real=True)
    torch.cuda.synchronize()
    pauto = L.Plan(n, dtype=torch.complex64, **kw)
    assert torch.equal(pauto.fwd(u), Lu)
    assert rel(pauto.adj(d, real=True), Lsd) < 1e-6
    del pauto
    torch.cuda.empty_cache()
    p128 = L.Plan(n, dtype=torch.complex128, slab=128, **kw)
    e_f = rel(Lu.to(torch.complex128), p128.fwd(u.double()))
    e_a = rel(Lsd.double(), p128.adj(d.to(torch.complex128), real=True))
    print(f"1024^3 c64 vs c128: fwd {e_f:.2e} adj {e_a:.2e}")
    assert e_f < 1e-4 and e_a < 1e-4
    # central differences at 16 random voxels (seed 304) of 1/2 |L u - d|^2 evaluated through the
    # complex128 plan (a complex64 loss at this size cannot resolve one voxel), against the complex64
    # autograd gradient (backward = the adjoint kernel); the loss is quadratic, so the central
    # difference is the directional derivative up to FP64 rounding
    ug = u.clone().requires_grad_(True)
    (0.5 * (L.LamOp.apply(ug, p64) - d).abs().pow(2).sum()).backward()
    g64 = ug.grad.detach()
    d128 = d.to(torch.complex128)
    ud = u.double()

    def loss128(x):
        r = p128.fwd(x) - d128
        return 0.5 * float((r.real ** 2 + r.imag ** 2).sum())

    idx = np.random.default_rng(304).integers(0, u.numel(), 16)
    eps, gmax, worst = 0.5, g64.abs().max().item(), 0.0
    for i in idx:
        e = torch.zeros(u.numel(), dtype=torch.float64, device="cuda")
        e[int(i)] = eps
        e = e.view_as(ud)
        fd = (loss128(ud + e) - loss128(ud - e)) / (2 * eps)
        worst = max(worst, abs(fd - g64.view(-1)[int(i)].item()) / gmax)
    print(f"1024^3 finite differences at 16 voxels (complex128 loss): worst error / max |grad| {worst:.2e}")
    assert worst < 1e-3
    del p128, d128, ud, e
    torch.cuda.empty_cache()
    # directional finite differences of 1/2 |L u - d|^2 along whole-volume directions (one voxel
    # moves a 1024^3 loss by less than its complex64 rounding): the loss is quadratic, so the central
    # difference equals <grad, v> up to rounding; the step moves the loss by at most about 1 %
    ug = u.clone().requires_grad_(True)
    (0.5 * (L.LamOp.apply(ug, p64) - d).abs().pow(2).sum()).backward()
    g = ug.grad.detach()

    def loss_of(x):
        r = (p64.fwd(x) - d).to(torch.complex128)
        return 0.5 * float((r.real ** 2 + r.imag ** 2).sum())

    loss0 = loss_of(u)
    smooth = I.blob_phantom_torch((n, n, n), I.draw_blobs(w["seed"] + 7, 64), "cuda", torch.float32)
    worst = 0.0
    for v in (g / g.norm(), smooth / smooth.norm()):
        gv = float((g.double() * v.double()).sum())
        q = float(p64.fwd(v).abs().double().pow(2).sum())
        eps = min(0.01 * loss0 / max(abs(gv), 1e-30), math.sqrt(0.02 * loss0 / max(q, 1e-30)))
        fd = (loss_of(u + eps * v) - loss_of(u - eps * v)) / (2 * eps)
        worst = max(worst, abs(fd - gv) / abs(gv))
    print(f"1024^3 directional finite differences: worst relative error {worst:.2e}")
    assert worst < 1e-3


def test_lam1024_streamed_matches_resident(L):
    """The host-streamed pair at 1024^3 (volume and data in pinned host memory) against the resident
    operators: the forward bit-identical, the adjoint equal up to the spread's accumulation order.
    Prints both rates (the streamed one includes the PCIe transfers)."""
    import time
    w = I.WORKLOADS["lam1024"]
    n = w["n"]
    plan = L.Plan(n, ntheta=w["ntheta"], phi=math.radians(w["phi_deg"]), h=w["det"], w=w["det"], slab=128)
    u = I.blob_phantom_torch((n, n, n), I.draw_blobs(w["seed"], w["nblobs"]), "cuda", torch.float32)
    d = I.random_complex_torch(plan.data_shape, w["seed"] + 200, "cuda", torch.complex64)
    uh, dh = u.cpu().pin_memory(), d.cpu().pin_memory()
    fo = torch.empty(plan.data_shape, dtype=torch.complex64, pin_memory=True)
    ao = torch.empty(plan.vol_shape, dtype=torch.float32, pin_memory=True)
    plan.fwd_streamed(uh, out=fo)
    plan.adj_streamed(dh, real=True, out=ao)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.fwd_streamed(uh, out=fo)
    plan.adj_streamed(dh, real=True, out=ao)
    t_str = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref_f = plan.fwd(u)
    ref_a = plan.adj(d, real=True)
    torch.cuda.synchronize()
    t_res = time.perf_counter() - t0
    print(f"1024^3 pair: resident {t_res * 1e3:.1f} ms, host-streamed {t_str * 1e3:.1f} ms")
    assert torch.equal(fo, ref_f.cpu())
    assert rel(ao, ref_a.cpu()) < 1e-6
