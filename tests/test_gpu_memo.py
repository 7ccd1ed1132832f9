"""GPU checks of the memoized ADMM step (lam_admm_step_memo; Section 4.4 "Memoization Cache",
Equation (cs)) against the oracle's admm_step_memo: the same iterates and the same hit and miss
counts of the four operators' private per-chunk caches, in complex128 (similarities agree to
rounding, so every hit decision is the oracle's) and complex64; without hits (tau above 1) the
step equals the plain lam_admm_step; below tau = -1 every query after the first hits."""
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


N, NT, PHI, ALPHA, INNER = 32, 24, math.radians(30.0), 1e-3, 3
MEMO = dict(chunk_y=8, chunk_kv=4, key_dim=256, seed=5)


def problem():
    g = O.Geometry(N, N, N, NT, PHI, N, N, 2, 4)
    u_true = I.blob_phantom(g.vol_shape, I.draw_blobs(21, 6))
    d = O.lam_fwd(u_true, g).real.astype(np.complex128)
    d = d + I.gaussian_noise(d.shape, 121, 0.01 * np.abs(d).max())
    return g, d


@pytest.fixture(scope="module")
def oracle_run():
    g, d = problem()
    dhat = O.f2d_unnorm(d)
    memo = O.Memo(g, 0.995, MEMO["chunk_y"], MEMO["chunk_kv"], MEMO["key_dim"], MEMO["seed"])
    st = (np.zeros(g.vol_shape), np.zeros((3,) + g.vol_shape), np.zeros((3,) + g.vol_shape), 0.5)
    its = []
    for it in range(4):
        st = O.admm_step_memo(*st[:3], st[3], dhat, g, ALPHA, INNER, memo)
        its.append((st, [tuple(c) for c in memo.counts()]))
        print(f"oracle memo ADMM iteration {it}: counts {memo.counts()}", flush=True)
    return g, d, its


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-9), (torch.complex64, 1e-4)], ids=["c128", "c64"])
def test_memo_admm_vs_oracle(L, oracle_run, dtype, tol):
    g, d, its = oracle_run
    plan = L.Plan(N, ntheta=NT, phi=PHI, dtype=dtype)
    memo = L.Memo(plan, tau=0.995, **MEMO)
    s = L.AdmmTV(plan, ALPHA, rho0=0.5, memo=memo)
    dh = plan.data_hat(torch.from_numpy(d).to(dtype).cuda())
    host = lambda t: t.double().cpu().numpy()
    for it, ((uo, po, lo, rho), counts) in enumerate(its):
        s.step(dh, INNER)
        st = memo.stats()
        got = [st[k] for k in L.OPS]
        eu, ep = O.relerr(host(s.u), uo), O.relerr(host(s.psi), po)
        print(f"memo ADMM iteration {it}: u {eu:.2e} psi {ep:.2e}; counts {got} (oracle {counts})", flush=True)
        assert got == counts
        assert eu < tol and ep < 10 * tol
        assert s.rho == rho
    assert sum(h for h, _ in got) > 0          # the later iterations do find similar chunks


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-10), (torch.complex64, 2e-5)], ids=["c128", "c64"])
def test_memo_without_hits_is_the_plain_step(L, dtype, tol):
    g, d = problem()
    plan = L.Plan(N, ntheta=NT, phi=PHI, dtype=dtype)
    dh = plan.data_hat(torch.from_numpy(d).to(dtype).cuda())
    a = L.AdmmTV(plan, ALPHA, rho0=0.5)
    memo = L.Memo(plan, tau=2.0, **MEMO)
    b = L.AdmmTV(plan, ALPHA, rho0=0.5, memo=memo)
    for _ in range(3):
        a.step(dh, INNER)
        b.step(dh, INNER)
    e = ((a.u - b.u).norm() / a.u.norm()).item()
    print(f"memo (no hits) vs plain step: u {e:.2e}", flush=True)
    assert e < tol and a.rho == b.rho
    st = memo.stats()
    assert all(h == 0 for h, _ in st.values())
    assert st["F_u1D"][1] == 3 * INNER * (N // MEMO["chunk_y"]) and st["F_u2D"][1] == 3 * INNER * (N // MEMO["chunk_kv"])


def test_memo_always_hits_below_minus_one(L):
    g, d = problem()
    plan = L.Plan(N, ntheta=NT, phi=PHI)
    dh = plan.data_hat(torch.from_numpy(d).to(torch.complex64).cuda())
    memo = L.Memo(plan, tau=-2.0, **MEMO)
    s = L.AdmmTV(plan, ALPHA, rho0=0.5, memo=memo)
    s.step(dh, INNER)
    st = memo.stats()
    ny, nk = N // MEMO["chunk_y"], N // MEMO["chunk_kv"]
    # the first application of each operator fills its caches, every later query hits
    assert st == {"F_u1D": ((INNER - 1) * ny, ny), "F_u2D": ((INNER - 1) * nk, nk),
                  "F*_u2D": ((INNER - 1) * nk, nk), "F*_u1D": ((INNER - 1) * ny, ny)}
    assert torch.isfinite(s.u).all()


def test_memo_argument_errors(L):
    plan = L.Plan(N, ntheta=NT, phi=PHI)
    with pytest.raises(ValueError):
        L.Memo(plan, chunk_y=3)
    with pytest.raises(ValueError):
        L.Memo(plan, key_dim=100)
