"""GPU checks of the host-streamed entry points (volume and data in pinned
host memory, moved in y-slabs and theta-slabs on the plan's copy stream)
against the resident operators, at sizes with several ragged slabs."""
import math

import pytest
import torch

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


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
@pytest.mark.parametrize("slabs", [(20, 13), (1, 1), None], ids=["ragged", "single", "auto"])
def test_streamed_matches_resident(L, dtype, slabs):
    n, nt = 64, 40
    plan = L.Plan(n, ntheta=nt, phi=math.radians(25), dtype=dtype)
    if slabs is not None:
        plan.stream_slabs(*slabs)
    rdt = plan.rdtype
    u = I.blob_phantom_torch((n, n, n), I.draw_blobs(7, 10), "cuda", rdt)
    d = I.random_complex_torch(plan.data_shape, 71, "cuda", dtype)
    # real volume
    ref_f = plan.fwd(u)
    ref_a = plan.adj(d, real=True)
    uh = u.cpu().pin_memory()
    dh = d.cpu().pin_memory()
    got_f = plan.fwd_streamed(uh)
    got_a = plan.adj_streamed(dh, real=True)
    print(f"{dtype} slabs {slabs}: fwd {rel(got_f, ref_f.cpu()):.1e} adj {rel(got_a, ref_a.cpu()):.1e}")
    # same kernels on the same values: the forward is bit-identical; the adjoint's tile
    # accumulation order is free, so it agrees to rounding
    assert torch.equal(got_f, ref_f.cpu())
    assert rel(got_a, ref_a.cpu()) < (1e-6 if dtype == torch.complex64 else 1e-14)
    # complex volume
    uc = (u + 0.5j * u.flip(0)).to(dtype)
    assert torch.equal(plan.fwd_streamed(uc.cpu().pin_memory()), plan.fwd(uc).cpu())
    got_ac = plan.adj_streamed(dh)
    assert rel(got_ac, plan.adj(d).cpu()) < (1e-6 if dtype == torch.complex64 else 1e-14)


def test_streamed_ordering_on_a_side_stream(L):
    """Calls are asynchronous on the caller's stream: back-to-back calls on a side stream,
    one wait at the end, each output checked."""
    n, nt = 64, 24
    plan = L.Plan(n, ntheta=nt, phi=math.radians(30))
    plan.stream_slabs(7, 5)
    us = [I.blob_phantom_torch((n, n, n), I.draw_blobs(s, 5), "cuda", torch.float32) for s in (11, 12, 13)]
    refs = [plan.fwd(u).cpu() for u in us]
    hosts = [u.cpu().pin_memory() for u in us]
    outs = [torch.empty(plan.data_shape, dtype=torch.complex64, pin_memory=True) for _ in us]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for h, o in zip(hosts, outs):
            plan.fwd_streamed(h, out=o, wait=False)
    side.synchronize()
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)


def test_streamed_pageable_and_argument_errors(L):
    plan = L.Plan(32, ntheta=16, phi=math.radians(20))
    u = I.blob_phantom_torch(plan.vol_shape, I.draw_blobs(9, 4), "cpu", torch.float32)
    # pageable host memory is accepted (the copies are staged by HIP and do not overlap)
    assert torch.equal(plan.fwd_streamed(u), plan.fwd(u.cuda()).cpu())
    with pytest.raises(ValueError):
        plan.fwd_streamed(u.cuda())                           # device tensor
    with pytest.raises(ValueError):
        plan.fwd_streamed(u.double())                         # wrong dtype
    with pytest.raises(L.LamError):
        plan.stream_slabs(0, 4)
    with pytest.raises(L.LamError):
        plan.stream_slabs(4, 17)
