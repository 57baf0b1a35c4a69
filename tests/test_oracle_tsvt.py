"""Pins of the oracle's t-SVT (Sec. 4 Z-update, Sec. 4.1 shrinkage lemma)
against special cases, closed forms, an optimality certificate and brute
force (CPU only)."""

import json
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import tensor as T
from oracle.tsvt import svt_matrix, tsvt, tsvt_objective

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rng(seed=0):
    return np.random.default_rng(seed)


def test_n3_one_is_matrix_svt_via_gesvd():
    """n3 = 1: the transform is the identity and t-SVT is the matrix D_tau of
    the Sec. 4.1 lemma; compared with LAPACK gesvd (a different driver from
    the oracle's gesdd)."""
    g = rng(1)
    for shape in ((7, 5), (5, 7), (6, 6)):
        x = g.normal(size=shape)
        u, s, vt = scipy.linalg.svd(x, full_matrices=False, lapack_driver="gesvd")
        tau = 0.6 * np.median(s)
        expect = u @ np.diag(np.maximum(s - tau, 0)) @ vt
        z, r = tsvt(x[:, :, None], tau)
        np.testing.assert_allclose(z[:, :, 0], expect, atol=1e-12)
        assert r[0] == np.count_nonzero(s > tau)


def test_tau_zero_identity_and_large_tau_zero():
    x = rng(2).normal(size=(5, 4, 6))
    z, r = tsvt(x, 0.0)
    np.testing.assert_allclose(z, x, atol=1e-12)
    smax = max(np.linalg.svd(T.fourier(x)[:, :, k], compute_uv=False).max() for k in range(6))
    z, r = tsvt(x, smax * 1.0001)
    assert np.abs(z).max() == 0.0 and r.sum() == 0


@pytest.mark.parametrize("shape", [(5, 4, 6), (4, 6, 7), (3, 3, 1), (4, 5, 2), (4, 3, 3, 4),
                                   (3, 4, 2, 5)])
def test_half_spectrum_equals_full_spectrum(shape):
    x = rng(3).normal(size=shape)
    tau = 0.8
    zh, _ = tsvt(x, tau, "half")
    zf, _ = tsvt(x, tau, "full")
    np.testing.assert_allclose(zh, zf, atol=1e-12)


def test_prox_certificate_per_slice():
    """Sec. 4.1 lemma optimality: per slice, Xhat - Zhat = tau (U1 V1^H + R)
    with ||R||_2 <= 1, U1^H R = 0, R V1 = 0 (U1, V1 from the SVD of Zhat)."""
    x = rng(4).normal(size=(6, 5, 8))
    tau = 1.5
    z, ranks = tsvt(x, tau)
    xh, zh = T.fourier(x), T.fourier(z)
    for k in range(8):
        u, s, vh = np.linalg.svd(zh[:, :, k], full_matrices=False)
        r = int(np.count_nonzero(s > 1e-9))
        u1, v1 = u[:, :r], np.conj(vh[:r].T)
        g = (xh[:, :, k] - zh[:, :, k]) / tau
        rem = g - u1 @ np.conj(v1.T)
        assert np.linalg.norm(rem, 2) <= 1 + 1e-9
        assert np.abs(np.conj(u1.T) @ rem).max() < 1e-9
        assert np.abs(rem @ v1).max() < 1e-9
        if k <= 4:
            assert r == ranks[k]


def test_bruteforce_objective_never_decreases():
    """Tiny tensor: random real perturbations of tsvt's output never lower
    (tau/n3) TNN(Z) + 1/2 ||Z - X||^2."""
    g = rng(5)
    x = g.normal(size=(3, 4, 5))
    tau = 1.2
    z, _ = tsvt(x, tau)
    f0 = tsvt_objective(z, x, tau)
    for eps in (1e-1, 1e-3, 1e-5):
        for _ in range(200):
            e = g.normal(size=x.shape)
            assert tsvt_objective(z + eps * e / np.linalg.norm(e), x, tau) >= f0 - 1e-12
    # and the oracle beats a generic derivative-free optimiser started at X
    from scipy.optimize import minimize

    x2 = x[:2, :2, :3]
    z2, _ = tsvt(x2, tau)
    res = minimize(lambda v: tsvt_objective(v.reshape(x2.shape), x2, tau), x2.ravel(),
                   method="Powell", options=dict(maxiter=4000, xtol=1e-9, ftol=1e-13))
    assert tsvt_objective(z2, x2, tau) <= res.fun + 1e-9


def test_nonexpansive_and_equivariances():
    g = rng(6)
    x = g.normal(size=(5, 4, 6))
    y = g.normal(size=(5, 4, 6))
    tau = 0.9
    zx, _ = tsvt(x, tau)
    zy, _ = tsvt(y, tau)
    assert np.linalg.norm(zx - zy) <= np.linalg.norm(x - y) + 1e-12
    # scaling
    z2, _ = tsvt(3.0 * x, 3.0 * tau)
    np.testing.assert_allclose(z2, 3.0 * zx, atol=1e-12)
    # circular shift of all tubes
    zs, _ = tsvt(np.roll(x, 2, axis=2), tau)
    np.testing.assert_allclose(zs, np.roll(zx, 2, axis=2), atol=1e-12)
    # real orthogonal P (mode 1) and Q (mode 2) applied to every frontal slice
    p, _ = np.linalg.qr(g.normal(size=(5, 5)))
    q, _ = np.linalg.qr(g.normal(size=(4, 4)))
    xpq = np.einsum("ai,ijt,jb->abt", p, x, q)
    zpq, _ = tsvt(xpq, tau)
    np.testing.assert_allclose(zpq, np.einsum("ai,ijt,jb->abt", p, zx, q), atol=1e-12)
    # tensor transpose commutes
    zt, _ = tsvt(T.ttranspose(x), tau)
    np.testing.assert_allclose(zt, T.ttranspose(zx), atol=1e-12)


def test_closed_form_rank_one_outer_product():
    """X = a o b o c: every Fourier slice is chat_k a b^T with the single
    singular value |chat_k| ||a|| ||b||."""
    g = rng(7)
    a, b, c = g.normal(size=6), g.normal(size=4), g.normal(size=9)
    x = np.einsum("i,j,t->ijt", a, b, c)
    tau = 0.7 * np.linalg.norm(a) * np.linalg.norm(b) * np.abs(np.fft.fft(c)).mean()
    ch = np.fft.fft(c)
    sig = np.abs(ch) * np.linalg.norm(a) * np.linalg.norm(b)
    fac = np.maximum(1 - tau / sig, 0)
    expect = np.real(np.fft.ifft(ch * fac))
    z, r = tsvt(x, tau)
    np.testing.assert_allclose(z, np.einsum("i,j,t->ijt", a, b, expect), atol=1e-12)
    np.testing.assert_array_equal(r, (sig[:5] > tau).astype(int))


def test_closed_form_fdiagonal_tubal_shrinkage():
    """f-diagonal X: every Fourier slice is diagonal, so t-SVT is the
    elementwise complex shrink of the diagonal tube spectra -- the tubal
    shrinkage by convolution of Sec. 4.1."""
    g = rng(8)
    n1, n2, n3 = 4, 6, 8
    x = np.zeros((n1, n2, n3))
    for i in range(n1):
        x[i, i, :] = g.normal(size=n3)
    tau = 2.0
    z, _ = tsvt(x, tau)
    assert T.is_fdiagonal(z, atol=1e-12)
    for i in range(n1):
        xh = np.fft.fft(x[i, i, :])
        expect = np.real(np.fft.ifft(xh * np.maximum(1 - tau / np.abs(xh), 0)))
        np.testing.assert_allclose(z[i, i, :], expect, atol=1e-12)


def test_golden_hand_worked_examples():
    with open(os.path.join(GOLDEN, "tsvt_hand_examples.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        x = np.array(case["X"], dtype=float)
        z, r = tsvt(x, case["tau"])
        np.testing.assert_allclose(z, np.array(case["Z"]), atol=1e-12, err_msg=case["name"])
        np.testing.assert_array_equal(r, case["multirank"], err_msg=case["name"])


def test_svt_matrix_boundary():
    """sigma == tau maps to zero and is not counted."""
    y = np.diag([3.0, 1.0])
    z, r = svt_matrix(y, 1.0)
    np.testing.assert_allclose(z, np.diag([2.0, 0.0]), atol=1e-15)
    assert r == 1
