"""GPU checks of the autograd form (LamOp: backward = the adjoint kernel) and
of the device ADMM-TV step against the FP64 oracle's admm_step."""
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


def make(L, dtype, n, nt, phi_deg, m=4):
    plan = L.Plan(n, ntheta=nt, phi=math.radians(phi_deg), h=n, w=n, m=m, dtype=dtype)
    geo = O.Geometry(n, n, n, nt, math.radians(phi_deg), n, n, 2, m)
    return plan, geo


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


@pytest.mark.parametrize("dtype,tol", [(torch.complex64, 1e-5), (torch.complex128, 1e-13)], ids=["c64", "c128"])
def test_data_hat(L, dtype, tol):
    plan, geo = make(L, dtype, 32, 16, 30.0)
    d = I.random_detector_data(geo.data_shape, 4)
    got = plan.data_hat(torch.from_numpy(d).to(dtype).cuda())
    err = O.relerr(host(got), O.f2d_unnorm(d))
    print(f"data_hat rel err {err:.2e}")
    assert err < tol


@pytest.mark.parametrize("dtype,tol", [(torch.complex64, 1e-4), (torch.complex128, 1e-12)], ids=["c64", "c128"])
def test_autograd_gradient_matches_oracle(L, dtype, tol):
    plan, geo = make(L, dtype, 32, 24, 30.0)
    u = I.blob_phantom(geo.vol_shape, I.draw_blobs(3, 6))
    d = I.random_detector_data(geo.data_shape, 3)
    rdt = torch.float32 if dtype == torch.complex64 else torch.float64
    ug = torch.from_numpy(u).to(rdt).cuda().requires_grad_(True)
    dg = torch.from_numpy(d).to(dtype).cuda()
    loss = 0.5 * (L.LamOp.apply(ug, plan) - dg).abs().pow(2).sum()
    loss.backward()
    ref = O.lam_adj(O.lam_fwd(u, geo) - d, geo).real       # d/du of 1/2|Lu - d|^2 for real u
    err = O.relerr(host(ug.grad), ref)
    print(f"autograd grad rel err {err:.2e}")
    assert err < tol
    # complex input: conjugate-Wirtinger convention, grad = L*(Lu - d)
    uc = torch.from_numpy(u.astype(np.complex128)).to(dtype).cuda().requires_grad_(True)
    loss = 0.5 * (L.LamOp.apply(uc, plan) - dg).abs().pow(2).sum()
    loss.backward()
    refc = O.lam_adj(O.lam_fwd(u.astype(complex), geo) - d, geo)
    assert O.relerr(host(uc.grad), refc) < tol


def test_autograd_gradcheck_c128(L):
    plan, geo = make(L, torch.complex128, 16, 8, 25.0)
    u = torch.from_numpy(I.random_complex(geo.vol_shape, 2).real).cuda().requires_grad_(True)
    # the adjoint's tile accumulation (FP64 LDS atomics) is order-independent only to rounding,
    # so repeated backward passes may differ in the last bits
    kw = dict(fast_mode=True, atol=1e-8, rtol=1e-6, nondet_tol=1e-12)
    assert torch.autograd.gradcheck(lambda x: L.LamOp.apply(x, plan), (u,), **kw)
    uc = torch.from_numpy(I.random_complex(geo.vol_shape, 3)).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: L.LamOp.apply(x, plan), (uc,), **kw)


def test_autograd_finite_differences_c64(L):
    """Central differences of the FP64-reduced loss at 16 random voxels (the loss is
    quadratic in u, so the central difference is exact up to rounding)."""
    plan, geo = make(L, torch.complex64, 32, 24, 20.0)
    u = torch.from_numpy(I.blob_phantom(geo.vol_shape, I.draw_blobs(4, 6))).float().cuda()
    d = torch.from_numpy(I.random_detector_data(geo.data_shape, 4)).to(torch.complex64).cuda()

    def loss_of(x):
        r = (plan.fwd(x) - d).to(torch.complex128)
        return 0.5 * float((r.real ** 2 + r.imag ** 2).sum())

    ug = u.clone().requires_grad_(True)
    (0.5 * (L.LamOp.apply(ug, plan) - d).abs().pow(2).sum()).backward()
    rng = np.random.default_rng(304)
    idx = rng.integers(0, u.numel(), 16)
    eps = 0.05
    flat = u.view(-1)
    worst = 0.0
    scale = ug.grad.abs().max().item()
    for i in idx:
        up, dn = flat.clone(), flat.clone()
        up[i] += eps
        dn[i] -= eps
        fd = (loss_of(up.view_as(u)) - loss_of(dn.view_as(u))) / (2 * eps)
        worst = max(worst, abs(fd - ug.grad.view(-1)[i].item()) / scale)
    print(f"finite-difference worst error relative to max |grad|: {worst:.2e}")
    assert worst < 1e-2


@pytest.mark.parametrize("dtype,tol", [(torch.complex64, 1e-4), (torch.complex128, 1e-9)], ids=["c64", "c128"])
def test_admm_step_matches_oracle(L, dtype, tol):
    plan, geo = make(L, dtype, 16, 16, 30.0)
    u_true = I.blob_phantom(geo.vol_shape, I.draw_blobs(3, 4))
    d = O.lam_fwd(u_true, geo).real.astype(np.complex128)
    alpha = 1e-3
    # oracle
    dhat = O.f2d_unnorm(d)
    uo = np.zeros(geo.vol_shape)
    po = np.zeros((3,) + geo.vol_shape)
    lo = np.zeros_like(po)
    rho = 0.5
    # device
    s = L.AdmmTV(plan, alpha, rho0=0.5)
    dh = plan.data_hat(torch.from_numpy(d).to(dtype).cuda())
    for it in range(3):
        uo, po, lo, rho = O.admm_step(uo, po, lo, rho, dhat, geo, alpha, 4)
        s.step(dh, 4)
        eu = O.relerr(host(s.u), uo)
        ep = O.relerr(host(s.psi), po)
        el = O.relerr(host(s.lam), lo)
        print(f"iter {it}: u {eu:.2e} psi {ep:.2e} lambda {el:.2e} rho gpu {s.rho} oracle {rho}")
        assert eu < tol and ep < 10 * tol and el < 10 * tol
        assert s.rho == rho
    diag = s.diagnostics()
    assert diag["primal"] >= 0 and diag["dual"] >= 0 and math.isfinite(diag["gamma"])


def test_admm_reduces_data_misfit(L):
    plan, geo = make(L, torch.complex64, 32, 32, 30.0)
    u_true = torch.from_numpy(I.blob_phantom(geo.vol_shape, I.draw_blobs(5, 8))).float().cuda()
    d = plan.fwd(u_true)
    d = torch.complex(d.real, torch.zeros_like(d.real))
    s = L.admm_tv(plan, d, alpha=1e-3, n_outer=4, n_inner=4)
    err = ((s.u - u_true).norm() / u_true.norm()).item()
    mis = ((plan.fwd(s.u) - d).norm() / d.norm()).item()
    print(f"ADMM-TV 4x4 on 32^3: rel err {err:.3f}, data misfit {mis:.3e}")
    assert mis < 0.1 and err < 0.6
