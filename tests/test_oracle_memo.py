"""Pins of the oracle's memoization (Section 4.4 "Memoization Cache", Equation (cs)):
the SplitMix64 generator against its published first outputs, the sketch key
against the plain cosine similarity it estimates, and the private per-chunk
FIFO cache against the behaviour the paper specifies (never hit above tau = 1,
always hit below tau = -1 once filled, replacement on a miss, chunks
independent), and the memoized ADMM step against the plain one."""
import math

import numpy as np
import pytest

from oracle import lam_oracle as O


def test_splitmix64_published_outputs():
    # the first three outputs of SplitMix64 from state 0 (Vigna's reference implementation)
    z = O.splitmix64(0, np.arange(3))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_splitmix64_signs_balanced():
    n = 1 << 20
    z = O.splitmix64(17, np.arange(n, dtype=np.uint64) + (np.uint64(3) << np.uint64(40)))
    s = 1.0 - 2.0 * (z >> np.uint64(63)).astype(np.float64)
    assert abs(s.mean()) < 5.0 / math.sqrt(n)
    assert abs((s[1:] * s[:-1]).mean()) < 5.0 / math.sqrt(n)     # neighbours uncorrelated


def test_sketch_exact_when_every_value_has_its_bucket():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 4, 5)) + 1j * rng.standard_normal((3, 4, 5))
    y = x + 0.3 * (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape))
    kx, ky = O.sketch(x, 120, 9, 2, 5), O.sketch(y, 120, 9, 2, 5)
    xr, yr = x.view(np.float64).ravel(), y.view(np.float64).ravel()
    assert np.linalg.norm(kx) == pytest.approx(np.linalg.norm(xr), rel=1e-14)
    assert O.cosine(kx, ky) == pytest.approx(float(xr @ yr / np.linalg.norm(xr) / np.linalg.norm(yr)), rel=1e-13)


def test_sketch_linear_and_unbiased():
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal((8, 64)), rng.standard_normal((8, 64))
    np.testing.assert_allclose(O.sketch(2 * x - 3 * y, 32, 4, 0, 1),
                               2 * O.sketch(x, 32, 4, 0, 1) - 3 * O.sketch(y, 32, 4, 0, 1), atol=1e-12)
    # over many seeds the key's squared norm is |x|^2 on average and its cosine
    # similarity concentrates on the plain one
    y2 = x + 0.5 * y
    true_cs = float((x * y2).sum() / np.linalg.norm(x) / np.linalg.norm(y2))
    n2, cs = [], []
    for seed in range(400):
        kx, ky = O.sketch(x, 64, seed, 0, 0), O.sketch(y2, 64, seed, 0, 0)
        n2.append(kx @ kx / (x * x).sum())
        cs.append(O.cosine(kx, ky))
    assert abs(np.mean(n2) - 1.0) < 4 * np.std(n2) / math.sqrt(len(n2))
    assert abs(np.mean(cs) - true_cs) < 0.02


def _op(calls):
    def fn(x, chunks):
        calls.append(list(chunks))
        return np.cumsum(x, axis=0) * 2.0          # acts along axis 0 only, so chunks along axis 1 are independent
    return fn


def test_memo_never_hits_above_one():
    calls = []
    op = O.MemoOp(_op(calls), 1, 1, 3, 1.5, 16, 5, 0)
    rng = np.random.default_rng(3)
    for _ in range(3):
        x = rng.standard_normal((4, 8))
        np.testing.assert_array_equal(op(x), np.cumsum(x, axis=0) * 2.0)
    assert (op.hits, op.misses) == (0, 9)
    assert calls == [[0, 1, 2]] * 3


def test_memo_always_hits_below_minus_one_once_filled():
    op = O.MemoOp(_op([]), 1, 1, 3, -2.0, 16, 5, 0)
    rng = np.random.default_rng(4)
    x1, x2 = rng.standard_normal((4, 8)), rng.standard_normal((4, 8))
    first = op(x1)
    np.testing.assert_array_equal(op(x2), first)          # every chunk served from the cache
    assert (op.hits, op.misses) == (3, 3)


def test_memo_fifo_replacement_and_similarity_gate():
    op = O.MemoOp(_op([]), 1, 1, 8, 0.9, 64, 5, 0)
    rng = np.random.default_rng(5)
    x1, x2 = rng.standard_normal((4, 8)), rng.standard_normal((4, 8))
    op(x1)
    np.testing.assert_array_equal(op(x1 * 1.001), np.cumsum(x1, axis=0) * 2.0)   # similar: the cached value
    op(x2)                                                                        # dissimilar: miss, replaces
    np.testing.assert_array_equal(op(x1), np.cumsum(x1, axis=0) * 2.0)            # x1 no longer cached: miss
    assert (op.hits, op.misses) == (1, 3)


def test_memo_chunks_independent_on_fu2d():
    g = O.Geometry(8, 8, 8, 6, math.radians(30.0), 8, 8, 2, 4)
    rng = np.random.default_rng(6)
    u1 = rng.standard_normal((8, 8, 8)) + 1j * rng.standard_normal((8, 8, 8))
    memo = O.Memo(g, 0.9, 4, 2, 32, 7)
    op = memo.ops[1]
    a = op(u1)
    np.testing.assert_allclose(a, O.fu2d(u1, g), rtol=0, atol=0)
    u1b = u1.copy()
    u1b[2:4] = rng.standard_normal((2, 8, 8))                 # only chunk 1 (slices 2, 3) changes
    b = op(u1b)
    assert (op.hits, op.misses) == (3, 5)
    fresh = O.fu2d(u1b, g)
    np.testing.assert_array_equal(b[:, 2:4], fresh[:, 2:4])
    np.testing.assert_array_equal(b[:, :2], a[:, :2])
    np.testing.assert_array_equal(b[:, 4:], a[:, 4:])


def test_admm_step_memo_without_hits_is_admm_step():
    g = O.Geometry(8, 8, 8, 6, math.radians(25.0), 8, 8, 2, 4)
    rng = np.random.default_rng(7)
    u_true = rng.standard_normal(g.vol_shape)
    dhat = O.f2d_unnorm(O.lam_fwd(u_true, g).real.astype(np.complex128))
    st = (np.zeros(g.vol_shape), np.zeros((3,) + g.vol_shape), np.zeros((3,) + g.vol_shape), 0.5)
    memo = O.Memo(g, 1.5, 3, 3, 32, 11)
    a, b = st, st
    for _ in range(2):
        a = O.admm_step(*a[:3], a[3], dhat, g, 1e-3, 3)
        b = O.admm_step_memo(*b[:3], b[3], dhat, g, 1e-3, 3, memo)
        for x, y in zip(a[:3], b[:3]):
            np.testing.assert_array_equal(x, y)
        assert a[3] == b[3]
    assert all(h == 0 for h, _ in memo.counts())


def test_admm_step_memo_hits_later_iterations():
    """Below tau = 1 the later iterations find similar chunks (the paper's observation
    that a chunk location's inputs become similar as ADMM converges) and the result
    stays close to the plain iteration."""
    g = O.Geometry(16, 16, 16, 12, math.radians(30.0), 16, 16, 2, 4)
    rng = np.random.default_rng(8)
    u_true = np.zeros(g.vol_shape)
    u_true[4:12, 5:11, 3:13] = 1.0
    dhat = O.f2d_unnorm(O.lam_fwd(u_true, g).real.astype(np.complex128))
    a = b = (np.zeros(g.vol_shape), np.zeros((3,) + g.vol_shape), np.zeros((3,) + g.vol_shape), 0.5)
    memo = O.Memo(g, 0.99, 4, 4, 64, 3)
    for _ in range(6):
        a = O.admm_step(*a[:3], a[3], dhat, g, 1e-3, 4)
        b = O.admm_step_memo(*b[:3], b[3], dhat, g, 1e-3, 4, memo)
    hits = sum(h for h, _ in memo.counts())
    assert hits > 0
    assert O.relerr(b[0], a[0]) < 0.2
