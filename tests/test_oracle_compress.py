"""Pins of the oracle's compression methods (Sec. 3) against closed forms,
other routes to the same result and entry counts (CPU only)."""

import numpy as np
import pytest
import scipy.linalg

from oracle import compress as C
from oracle import tensor as T


def rng(seed=0):
    return np.random.default_rng(seed)


# ------------------------------------------------------------ ratios

def test_ratios_count_the_stored_entries():
    """Each ratio is numel(M) over the entries a truncation stores; count
    those entries from factors actually built, not from the formulas."""
    n1, n2, n3 = 7, 5, 6
    m = rng(1).standard_normal((n1, n2, n3))
    k1 = 2
    a = np.stack([m[:, :, k].ravel() for k in range(n3)], axis=1)
    u, s, vt = np.linalg.svd(a, full_matrices=False)
    stored = u[:, :k1].size + s[:k1].size + vt[:k1].size
    assert C.ratio_svd(n1, n2, n3, k1) == pytest.approx(m.size / stored, rel=1e-15)
    # Method 1: k2 Fourier-domain triplets, a column of U (n1), a value, a column of V (n2)
    k2 = 9
    stored1 = k2 * (n1 + 1 + n2)
    assert C.ratio_tsvd(n1, n2, n3, k2) == pytest.approx(m.size / stored1, rel=1e-15)
    # Method 2: k3 lateral slices of U (n1 x n3), tubes of S (n3), lateral slices of V (n2 x n3)
    k3 = 3
    uu, ss, vv, _, _, _ = T.tsvd(m)
    stored2 = uu[:, :k3, :].size + ss[:k3, 0, :].size + vv[:, :k3, :].size
    assert C.ratio_tubal(n1, n2, k3) == pytest.approx(m.size / stored2, rel=1e-15)


def test_ratios_hand_values():
    # 130 x 160 x 50 (the size of the first video of Sec. 3), evaluated by hand
    assert C.ratio_svd(130, 160, 50, 5) == pytest.approx(1040000 / 104255, rel=1e-15)   # 9.97554...
    assert C.ratio_tsvd(130, 160, 50, 500) == pytest.approx(1040000 / 145500, rel=1e-15)  # 7.14776...
    assert C.ratio_tubal(130, 160, 10) == pytest.approx(20800 / 2910, rel=1e-15)  # 7.14776...


# ------------------------------------------------------------ Method 1

def test_method1_keeps_everything_exactly():
    m = rng(2).standard_normal((6, 5, 7))
    out = C.method1(m, 5 * 7)
    np.testing.assert_allclose(out, m, atol=1e-12)


def test_method1_n3_1_is_matrix_truncation():
    m = rng(3).standard_normal((9, 6, 1))
    for k in (1, 3, 6):
        u, s, vt = scipy.linalg.svd(m[:, :, 0])
        ref = (u[:, :k] * s[:k]) @ vt[:k]
        np.testing.assert_allclose(C.method1(m, k)[:, :, 0], ref, atol=1e-12)


def _keep_by_threshold(vals, k2):
    # the reading: the largest set {v >= t} with at most k2 members
    order = np.sort(vals.ravel())[::-1]
    for cut in range(len(order), 0, -1):
        t = order[cut - 1]
        if np.count_nonzero(vals >= t) <= k2:
            return vals >= t
    return np.zeros(vals.shape, dtype=bool)


def test_method1_fdiagonal_closed_form():
    """An f-diagonal tensor has diagonal Fourier slices: the singular values
    are the moduli of the transformed diagonal tubes, so Method 1 masks the
    tubes' spectra directly (no SVD involved)."""
    n, n3 = 4, 8
    tubes = rng(4).standard_normal((n, n3))
    m = np.zeros((n, n, n3))
    for i in range(n):
        m[i, i] = tubes[i]
    half = np.fft.rfft(tubes, axis=1)
    full = np.concatenate([half, np.conj(half[:, 1:n3 - n3 // 2][:, ::-1])], axis=1)
    # exact conjugate pairs: take the moduli of the half spectrum and mirror them
    mag = np.concatenate([np.abs(half), np.abs(half[:, 1:n3 - n3 // 2])[:, ::-1]], axis=1)
    for k2 in (3, 8, 13, 20):
        keep = _keep_by_threshold(mag, k2)
        srt = np.sort(mag.ravel())[::-1]
        kept = int(keep.sum())
        if 0 < kept < mag.size:
            assert srt[kept - 1] - srt[kept] > 1e-9   # no near-tie at the cut
        ref = np.zeros_like(m)
        rec = np.real(np.fft.ifft(full * keep, axis=1))
        for i in range(n):
            ref[i, i] = rec[i]
        out, keep_o, _, imag = C.method1(m, k2, return_details=True)
        np.testing.assert_allclose(out, ref, atol=1e-12)
        assert keep_o.sum() == kept
        assert imag < 1e-12


def test_method1_error_is_the_dropped_energy():
    """||M - M_k2||_F^2 = (1/n3) * sum of the dropped sigma^2 over the full
    spectrum (Parseval for the third-mode DFT), and at most k2 are kept."""
    m = rng(5).standard_normal((8, 6, 10))
    _, _, _, _, sh, _ = T.tsvd(m)
    sig = C.fourier_singular_values(sh)
    for k2 in (1, 7, 20, 41):
        out, keep, _, imag = C.method1(m, k2, return_details=True)
        assert keep.sum() <= k2
        dropped = np.sum((sig * ~keep) ** 2) / m.shape[2]
        assert np.sum((m - out) ** 2) == pytest.approx(dropped, rel=1e-10)
        assert imag < 1e-10 * np.linalg.norm(m)


def test_method1_pairs_kept_together():
    m = rng(6).standard_normal((5, 4, 6))
    for k2 in range(1, 24):
        _, keep, _, _ = C.method1(m, k2, return_details=True)
        for k in range(1, 6):
            np.testing.assert_array_equal(keep[:, k], keep[:, (6 - k) % 6])


def test_method1_error_decreases_with_k2():
    m = rng(7).standard_normal((6, 6, 5))
    errs = [np.linalg.norm(m - C.method1(m, k)) for k in range(1, 31)]
    assert all(b <= a + 1e-12 for a, b in zip(errs, errs[1:]))


# ------------------------------------------------------------ Method 2

def test_method2_equals_fourier_slice_truncation():
    """The sum of the first k3 tubal terms equals the rank-k3 truncation of
    every Fourier slice (the Fourier-domain route to Theorem 2.3.1)."""
    m = rng(8).standard_normal((7, 5, 6))
    mh = np.fft.fft(m, axis=2)
    for k3 in (1, 2, 5):
        zh = np.zeros_like(mh)
        for k in range(6):
            u, s, vt = np.linalg.svd(mh[:, :, k], full_matrices=False)
            zh[:, :, k] = (u[:, :k3] * s[:k3]) @ vt[:k3]
        ref = np.real(np.fft.ifft(zh, axis=2))
        np.testing.assert_allclose(C.method2(m, k3), ref, atol=1e-11)


def test_method2_keeps_everything_exactly():
    m = rng(9).standard_normal((4, 6, 5))
    np.testing.assert_allclose(C.method2(m, 4), m, atol=1e-11)


def test_matrix_svd_baseline_full_rank_and_rank_one():
    m = rng(10).standard_normal((3, 4, 5))
    np.testing.assert_allclose(C.matrix_svd(m, 5), m, atol=1e-12)
    # a tensor whose frontal slices are multiples of one slice is rank 1 unfolded
    base = rng(11).standard_normal((3, 4))
    w = rng(12).standard_normal(5)
    r1 = base[:, :, None] * w[None, None, :]
    np.testing.assert_allclose(C.matrix_svd(r1, 1), r1, atol=1e-12)


def test_compression_rejects_4d():
    with pytest.raises(ValueError):
        C.method1(np.zeros((2, 2, 2, 2)), 1)
    with pytest.raises(ValueError):
        C.method2(np.zeros((2, 2, 2, 2)), 1)
