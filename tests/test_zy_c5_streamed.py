"""The 2048^3 workload (2048 angles, 2048^2 detector, 20 deg) with the volume and the data in host
memory, streamed through the device in slabs (about two minutes; set LAM_TEST_SKIP_C5=1 to skip).

The FP64 oracle cannot evaluate any output at this size in a test's time (one k_v slice needs F_u1D
of the whole volume), so the forward is checked against the closed-form line integrals of the
Gaussian-blob phantom at 3000 sampled detector points (tests/blob_closed_form.py, pinned to the
oracle on the CPU; its residual falls as 1/N, about 1e-5 here), and the adjoint through the
identity <L u, L u> = <u, Re L* L u> for the real volume u.  This file sorts after the other GPU
files and before the no-allocation test, so that a host-memory shortfall here hides nothing else.
"""
import math
import os
import time

import numpy as np
import pytest
import torch

from oracle import lam_oracle as O
from paper_2511_01893_amd import inputs as I
from tests.blob_closed_form import blob_data

pytestmark = pytest.mark.gpu


@pytest.mark.skipif(os.environ.get("LAM_TEST_SKIP_C5") == "1", reason="LAM_TEST_SKIP_C5=1")
def test_lam2048_streamed(capsys):
    """The volume pinned (34 GB), the data (69 GB) and the adjoint's output pageable: L u streamed out,
    sampled against the closed form; then Re L* (L u) streamed back, and the adjoint identity.  The
    phase lines bypass pytest's output capture, so that a long run shows progress as it goes."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")

    def say(msg):
        with capsys.disabled():
            print(msg, flush=True)

    from paper_2511_01893_amd import lam as L
    w = I.WORKLOADS["lam2048"]
    n = w["n"]
    phi = math.radians(w["phi_deg"])
    say("2048^3 streamed: building the plan")
    plan = L.Plan(n, ntheta=w["ntheta"], phi=phi, h=w["det"], w=w["det"])
    say("2048^3 streamed: plan built")
    blobs = I.draw_blobs(w["seed"], w["nblobs"])
    uh = torch.empty((n, n, n), dtype=torch.float32, pin_memory=True)
    for z0 in range(0, n, 128):               # the phantom, generated on the device a z-slab at a time
        uh[z0:z0 + 128] = I.blob_phantom_torch((n, n, n), blobs, "cuda", torch.float32, z_range=(z0, z0 + 128)).cpu()
    say("2048^3 phantom in pinned host memory")
    fo = torch.empty(plan.data_shape, dtype=torch.complex64)
    t0 = time.perf_counter()
    plan.fwd_streamed(uh, out=fo)
    t_f = time.perf_counter() - t0
    say(f"2048^3 streamed forward {t_f:.2f} s")
    # sampled detector points against the closed-form data of the blobs
    rng = np.random.default_rng(7)
    ti = rng.integers(0, w["ntheta"], 3000)
    vi = rng.integers(0, w["det"], 3000)
    ui = rng.integers(0, w["det"], 3000)
    got = fo[torch.from_numpy(ti), torch.from_numpy(vi), torch.from_numpy(ui)].numpy().astype(np.complex128)
    thetas = 2 * np.pi * ti / w["ntheta"]
    ref = blob_data(blobs, n, thetas, phi, O.centred(w["det"])[ui] / n, O.centred(w["det"])[vi] / n)
    err_cf = np.linalg.norm(got.real - ref) / np.linalg.norm(ref)
    say(f"2048^3 forward at 3000 sampled points vs closed form: {err_cf:.2e}")
    assert err_cf < 1e-4
    ao = torch.empty((n, n, n), dtype=torch.float32)
    t0 = time.perf_counter()
    plan.adj_streamed(fo, real=True, out=ao)
    t_a = time.perf_counter() - t0
    say(f"2048^3 streamed adjoint {t_a:.2f} s")
    lhs = rhs = 0.0
    for a in range(0, n, 64):                 # FP64 sums on the device, 64 planes at a time
        lhs += float(torch.view_as_real(fo[a:a + 64].cuda()).double().pow(2).sum())
        rhs += float((uh[a:a + 64].cuda().double() * ao[a:a + 64].cuda().double()).sum())
    err = abs(lhs - rhs) / lhs
    say(f"2048^3 streamed: forward {t_f:.2f} s, adjoint {t_a:.2f} s; adjoint identity {err:.2e}")
    assert err < 1e-4
