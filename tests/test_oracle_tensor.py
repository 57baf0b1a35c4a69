"""Pins of the oracle's Sec. 2 tensor algebra against brute force, closed
forms and the identities the paper states (CPU only)."""

import cmath
import itertools

import numpy as np
import pytest

from oracle import tensor as T
import workloads


def rng(seed=0):
    return np.random.default_rng(seed)


# ------------------------------------------------------------------ DFT

def dft_bruteforce(a):
    """Forward DFT along every trailing mode written as the explicit sum."""
    n1, n2 = a.shape[:2]
    dims = a.shape[2:]
    out = np.zeros(a.shape, dtype=complex)
    for k in itertools.product(*[range(n) for n in dims]):
        acc = np.zeros((n1, n2), dtype=complex)
        for t in itertools.product(*[range(n) for n in dims]):
            ph = sum(kk * tt / n for kk, tt, n in zip(k, t, dims))
            acc += a[(slice(None), slice(None)) + t] * cmath.exp(-2j * cmath.pi * ph)
        out[(slice(None), slice(None)) + k] = acc
    return out


@pytest.mark.parametrize("shape", [(2, 3, 5), (3, 2, 4), (2, 2, 3, 4)])
def test_fourier_matches_explicit_sum(shape):
    a = rng(1).normal(size=shape)
    np.testing.assert_allclose(T.fourier(a), dft_bruteforce(a), rtol=0, atol=1e-12)


def test_fourier_impulse_and_constant():
    n3 = 7
    a = np.zeros((1, 1, n3))
    a[0, 0, 0] = 1.0
    np.testing.assert_allclose(T.fourier(a)[0, 0], np.ones(n3), atol=1e-15)
    c = np.full((1, 1, n3), 2.0)
    expect = np.zeros(n3, dtype=complex)
    expect[0] = 2.0 * n3
    np.testing.assert_allclose(T.fourier(c)[0, 0], expect, atol=1e-13)
    # shifted impulse: e^{-2 pi i k / n3}
    s = np.zeros((1, 1, n3))
    s[0, 0, 1] = 1.0
    np.testing.assert_allclose(T.fourier(s)[0, 0], np.exp(-2j * np.pi * np.arange(n3) / n3),
                               atol=1e-14)


@pytest.mark.parametrize("shape", [(4, 3, 8), (3, 5, 7), (2, 3, 3, 6), (2, 2, 4, 5)])
def test_fourier_roundtrip_parseval_half(shape):
    a = rng(2).normal(size=shape)
    ah = T.fourier(a)
    np.testing.assert_allclose(np.real(T.ifourier(ah)), a, atol=1e-13)
    ntr = int(np.prod(shape[2:]))
    assert np.isclose(np.sum(np.abs(ah) ** 2), ntr * np.sum(a ** 2), rtol=1e-12)
    half = T.fourier_half(a)
    q = shape[-1]
    np.testing.assert_allclose(half, ah[..., : q // 2 + 1], atol=1e-12)
    np.testing.assert_allclose(T.ifourier_half(half, shape[2:]), a, atol=1e-13)
    # conjugate symmetry of the spectrum of real data
    mirror = ah
    for ax in range(2, a.ndim):
        mirror = np.roll(np.flip(mirror, axis=ax), 1, axis=ax)
    np.testing.assert_allclose(mirror, np.conj(ah), atol=1e-12)


# ------------------------------------------------------------ t-product

def tprod_loops(a, b):
    """t-product with every sum written as a Python loop (tiny sizes)."""
    n1, n2, n3 = a.shape
    n4 = b.shape[1]
    c = np.zeros((n1, n4, n3))
    for i in range(n1):
        for j in range(n4):
            for k in range(n2):
                for t in range(n3):
                    for s in range(n3):
                        c[i, j, t] += a[i, k, s] * b[k, j, (t - s) % n3]
    return c


def test_tprod_direct_equals_loops():
    g = rng(3)
    a, b = g.normal(size=(3, 4, 5)), g.normal(size=(4, 2, 5))
    np.testing.assert_allclose(T.tprod_direct(a, b), tprod_loops(a, b), atol=1e-12)


@pytest.mark.parametrize("n3", [1, 4, 5, 8])
def test_tprod_fft_route_equals_definition(n3):
    g = rng(4)
    a, b = g.normal(size=(3, 4, n3)), g.normal(size=(4, 6, n3))
    np.testing.assert_allclose(T.tprod_fft(a, b), T.tprod_direct(a, b), atol=1e-12)


def test_tprod_noncommutative_operands_not_swapped():
    g = rng(5)
    a, b = g.normal(size=(3, 3, 4)), g.normal(size=(3, 3, 4))
    assert np.abs(T.tprod_direct(a, b) - T.tprod_direct(b, a)).max() > 1e-3


def test_identity_transpose_associativity():
    g = rng(6)
    a = g.normal(size=(3, 4, 5))
    b = g.normal(size=(4, 2, 5))
    c = g.normal(size=(2, 3, 5))
    np.testing.assert_allclose(T.tprod_direct(T.tidentity(3, 5), a), a, atol=1e-14)
    np.testing.assert_allclose(T.tprod_direct(a, T.tidentity(4, 5)), a, atol=1e-14)
    lhs = T.ttranspose(T.tprod_direct(a, b))
    rhs = T.tprod_direct(T.ttranspose(b), T.ttranspose(a))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)
    np.testing.assert_allclose(T.tprod_direct(T.tprod_direct(a, b), c),
                               T.tprod_direct(a, T.tprod_direct(b, c)), atol=1e-11)
    np.testing.assert_allclose(T.ttranspose(T.ttranspose(a)), a)
    # transpose is the per-slice conjugate transpose in the Fourier domain
    np.testing.assert_allclose(T.fourier(T.ttranspose(a)),
                               np.conj(np.transpose(T.fourier(a), (1, 0, 2))), atol=1e-12)


def test_planting_tprod_matches_oracle():
    g = rng(7)
    a, b = g.normal(size=(5, 2, 6)), g.normal(size=(2, 7, 6))
    np.testing.assert_allclose(workloads.plant_tprod(a, b), T.tprod_direct(a, b), atol=1e-12)
    w = workloads.completion_small(0)
    assert w["X"].shape == (32, 32, 16)
    np.testing.assert_array_equal(T.multirank(w["X"]), np.full(16, 2))


# ---------------------------------------------------------------- t-SVD

@pytest.mark.parametrize("shape", [(4, 3, 5), (3, 5, 4), (4, 4, 1), (3, 4, 6)])
def test_tsvd_reconstruction_and_orthogonality(shape):
    m = rng(8).normal(size=shape)
    u, s, v, *_ = T.tsvd(m)
    n3 = shape[2]
    np.testing.assert_allclose(T.tprod_direct(T.tprod_direct(u, s), T.ttranspose(v)), m,
                               atol=1e-12)
    for q, n in ((u, shape[0]), (v, shape[1])):
        np.testing.assert_allclose(T.tprod_direct(T.ttranspose(q), q), T.tidentity(n, n3),
                                   atol=1e-12)
        np.testing.assert_allclose(T.tprod_direct(q, T.ttranspose(q)), T.tidentity(n, n3),
                                   atol=1e-12)
    assert T.is_fdiagonal(s, atol=1e-13)


def test_tsvd_4d_reconstruction():
    m = rng(9).normal(size=(3, 4, 3, 4))
    u, s, v, uh, sh, vh = T.tsvd(m)
    np.testing.assert_allclose(T.tprod_fft(T.tprod_fft(u, s), _ttranspose_nd(v)), m, atol=1e-12)
    np.testing.assert_allclose(T.tprod_fft(_ttranspose_nd(u), u)[:, :, 0, 0], np.eye(3), atol=1e-12)
    assert T.is_fdiagonal(s, atol=1e-13)


def _ttranspose_nd(v):
    """N-D tensor transpose: per-slice transpose with every trailing index
    negated (mod n), the N-D form of the Sec. 2.1 definition."""
    out = np.transpose(v, (1, 0) + tuple(range(2, v.ndim)))
    for ax in range(2, v.ndim):
        out = np.roll(np.flip(out, axis=ax), 1, axis=ax)
    return out


def test_truncation_theorem_error_and_optimality():
    """Theorem 2.3.1: M_k is the best fit among X * Y with k lateral slices;
    its error is the Parseval sum of the dropped Fourier singular values."""
    g = rng(10)
    m = g.normal(size=(5, 4, 6))
    u, s, v, uh, sh, vh = T.tsvd(m)
    for k in (1, 2, 3):
        mk = T.tsvd_truncate(u, s, v, k)
        err2 = np.sum((m - mk) ** 2)
        sv = np.stack([np.abs(np.diagonal(sh[:, :, t])) for t in range(6)], axis=1)
        expect = np.sum(sv[k:, :] ** 2) / 6.0
        assert np.isclose(err2, expect, rtol=1e-10)
        for _ in range(20):
            x = g.normal(size=(5, k, 6))
            y = g.normal(size=(k, 4, 6))
            assert np.sum((m - T.tprod_direct(x, y)) ** 2) >= err2 - 1e-9
        # the t-SVD truncation has tubal rank k
        assert T.tubal_rank(mk) == k


def test_multirank_tubal_rank_tnn_blkdiag():
    g = rng(11)
    _, _, x = workloads.lowrank(g, 6, 7, 5, 3)
    np.testing.assert_array_equal(T.multirank(x), np.full(5, 3))
    assert T.tubal_rank(x) == 3
    xh = T.fourier(x)
    assert np.isclose(T.tnn(x), np.linalg.svd(T.blkdiag(xh), compute_uv=False).sum(), rtol=1e-12)
    # TNN is a norm: homogeneity and triangle inequality
    y = g.normal(size=x.shape)
    assert np.isclose(T.tnn(-2.5 * x), 2.5 * T.tnn(x), rtol=1e-12)
    assert T.tnn(x + y) <= T.tnn(x) + T.tnn(y) + 1e-9
    # a tensor whose first slice only is non-zero: all Fourier slices equal
    e = np.zeros((3, 3, 4))
    e[:, :, 0] = np.diag([3.0, 2.0, 0.0])
    np.testing.assert_array_equal(T.multirank(e), np.full(4, 2))
    assert np.isclose(T.tnn(e), 4 * 5.0)
