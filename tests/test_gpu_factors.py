"""t-SVD factors and the compression methods on the GPU (C ABI through the
binding) against the FP64 oracle.  The factors are unique only up to the
phase of each Fourier-domain column, so the tests compare the singular tubes
element by element and check the rest through what is unique: the
reconstruction M = sum_i U(:, i, :) * S(i, i, :) * V(:, i, :)^T and the
orthonormality of every Fourier slice of U and V."""

import numpy as np
import pytest

import paper_1407_1785_amd as lib
from oracle import compress as C
from oracle import tensor as T
from tests.gpu_util import announce, rel_fro, to_gpu, torch_cuda

pytestmark = pytest.mark.gpu

TOL = 1e-10      # FP64 path, relative
TOL32 = 1e-4     # FP32 form, relative

FACTOR_SHAPES = [
    (20, 13, 7),      # n1 > n2, odd tube length
    (13, 20, 8),      # n1 < n2 (transposed slices)
    (32, 32, 16),
    (40, 33, 1),      # n3 = 1: the matrix SVD
    (70, 45, 5),      # several Jacobi blocks
    (1, 7, 6),        # one row
    (9, 12, 3, 4),    # 4-D: conjugate pairs inside the half spectrum (k3, 0) / (3 - k3, 0)
    (10, 8, 4, 6),    # 4-D, even mode 3: self-conjugate slices at k3 = 0 and 2
]


def reconstruct(u, s, v):
    """sum_i U(:, i, :) * S(i, i, :) * V(:, i, :)^T through the Fourier
    domain (slice-wise Uhat diag(Shat) Vhat^H)."""
    uh, sh, vh = T.fourier(u), T.fourier(s[None]), T.fourier(v)
    n0 = s.shape[0]
    out = np.zeros((u.shape[0], v.shape[0]) + u.shape[2:], dtype=np.complex128)
    for idx in np.ndindex(*u.shape[2:]):
        sl = (slice(None), slice(None)) + idx
        d = sh[(0, slice(None)) + idx]
        out[sl] = (uh[sl][:, :n0] * d) @ np.conj(vh[sl][:, :n0]).T
    return np.real(T.ifourier(out))


def orth_error(f):
    fh = T.fourier(f)
    err = 0.0
    for idx in np.ndindex(*f.shape[2:]):
        q = fh[(slice(None), slice(None)) + idx]
        err = max(err, np.abs(np.conj(q).T @ q - np.eye(q.shape[1])).max())
    return err


@pytest.mark.parametrize("shape", FACTOR_SHAPES)
def test_factors_match_oracle(shape):
    torch = torch_cuda()
    rng = np.random.default_rng(sum(shape) + 7)
    m = rng.normal(size=shape)
    _, s_ref, _, _, _, _ = T.tsvd(m)
    n0 = min(shape[0], shape[1])
    tubes_ref = np.stack([s_ref[(i, i)] for i in range(n0)])
    announce("tsvd_factors", shape)
    u, s, v = (t.cpu().numpy() for t in lib.tsvd_factors(to_gpu(torch, m)))
    assert u.shape == (shape[0], n0) + shape[2:] and v.shape == (shape[1], n0) + shape[2:]
    assert rel_fro(s, tubes_ref) <= TOL
    assert rel_fro(reconstruct(u, s, v), m) <= TOL
    assert orth_error(u) <= 1e-10 and orth_error(v) <= 1e-10
    if len(shape) == 3:
        # the paper's sum of t-products, by the t-product's definition
        s_full = np.zeros((n0, n0, shape[2]))
        for i in range(n0):
            s_full[i, i] = s[i]
        assert rel_fro(T.tsvd_truncate(u, s_full, v, n0), m) <= TOL


def test_factors_fp32_form():
    torch = torch_cuda()
    rng = np.random.default_rng(3)
    m = rng.normal(size=(48, 40, 12))
    _, s_ref, _, _, _, _ = T.tsvd(m)
    tubes_ref = np.stack([s_ref[(i, i)] for i in range(40)])
    announce("tsvd_factors fp32")
    u, s, v = (t.cpu().numpy().astype(np.float64)
               for t in lib.tsvd_factors(to_gpu(torch, m, torch.float32), precision=lib.PREC_FP32))
    assert rel_fro(s, tubes_ref) <= TOL32
    assert rel_fro(reconstruct(u, s, v), m) <= TOL32
    assert orth_error(u) <= 1e-4 and orth_error(v) <= 1e-4


def test_factors_rank_deficient_slices():
    """A tubal-rank-2 tensor: the singular tubes beyond the second are zero
    and the reconstruction is still exact."""
    torch = torch_cuda()
    rng = np.random.default_rng(4)
    a, b = rng.normal(size=(24, 2, 10)), rng.normal(size=(2, 18, 10))
    m = T.tprod_fft(a, b)
    announce("tsvd_factors rank 2")
    u, s, v = (t.cpu().numpy() for t in lib.tsvd_factors(to_gpu(torch, m)))
    assert np.abs(s[2:]).max() <= 1e-10 * np.abs(s).max()
    assert rel_fro(reconstruct(u, s, v), m) <= TOL


# ------------------------------------------------------------ compression

COMPRESS_SHAPES = [(20, 13, 7), (13, 20, 8), (32, 32, 16), (40, 33, 1), (70, 45, 5)]


def fourier_sigmas(m):
    _, _, _, _, sh, _ = T.tsvd(m)
    return C.fourier_singular_values(sh)


@pytest.mark.parametrize("shape", COMPRESS_SHAPES)
def test_method2_matches_oracle(shape):
    torch = torch_cuda()
    rng = np.random.default_rng(sum(shape) + 11)
    m = rng.normal(size=shape)
    n0 = min(shape[:2])
    sig = np.sort(fourier_sigmas(m), axis=0)[::-1]
    mg = to_gpu(torch, m)
    for k3 in sorted({1, max(1, n0 // 2), n0}):
        if k3 < n0:
            gap = (sig[k3 - 1] - sig[k3]) / sig[0]
            if gap.min() < 1e-8:
                continue   # the per-slice truncation is not well separated here
        announce("compress tubal", shape, k3)
        out, ratio = lib.compress(mg, lib.COMPRESS_TUBAL, k3)
        assert rel_fro(out.cpu().numpy(), C.method2(m, k3)) <= TOL
        assert ratio == pytest.approx(C.ratio_tubal(shape[0], shape[1], k3), rel=1e-14)


@pytest.mark.parametrize("shape", COMPRESS_SHAPES)
def test_method1_matches_oracle(shape):
    torch = torch_cuda()
    rng = np.random.default_rng(sum(shape) + 13)
    m = rng.normal(size=shape)
    n0, n3 = min(shape[:2]), shape[2]
    sig = fourier_sigmas(m)
    srt = np.sort(np.unique(sig))[::-1]
    mg = to_gpu(torch, m)
    tested = 0
    for k2 in sorted({1, 3, n0, n0 * n3 // 3, n0 * n3 // 2 + 1, n0 * n3}):
        out_ref, keep, t, _ = C.method1(m, k2, return_details=True)
        # the cut must be clear of the next value on both sides
        if np.isfinite(t) and 0 < keep.sum() < keep.size:
            below = srt[srt < t]
            if below.size and (t - below[0]) / srt[0] < 1e-8:
                continue
        announce("compress tsvd", shape, k2)
        out, ratio = lib.compress(mg, lib.COMPRESS_TSVD, k2)
        assert rel_fro(out.cpu().numpy(), out_ref) <= TOL
        assert ratio == pytest.approx(C.ratio_tsvd(shape[0], shape[1], n3, k2), rel=1e-14)
        tested += 1
    assert tested >= 3


def test_compression_fp32_form():
    torch = torch_cuda()
    rng = np.random.default_rng(21)
    m = rng.normal(size=(40, 36, 10))
    mg = to_gpu(torch, m, torch.float32)
    for method, k, ref in ((lib.COMPRESS_TUBAL, 9, C.method2(m, 9)),
                           (lib.COMPRESS_TSVD, 101, C.method1(m, 101))):
        announce("compress fp32", method, k)
        out, _ = lib.compress(mg, method, k, precision=lib.PREC_FP32)
        assert rel_fro(out.cpu().numpy().astype(np.float64), ref) <= TOL32


def test_compression_errors():
    torch = torch_cuda()
    m = to_gpu(torch, np.random.default_rng(0).normal(size=(6, 5, 4)))
    m4 = to_gpu(torch, np.random.default_rng(0).normal(size=(6, 5, 2, 2)))
    announce("compress errors")
    with pytest.raises(lib.TsvdError, match="TSVD_E_SHAPE"):
        lib.compress(m4, lib.COMPRESS_TUBAL, 1)
    for method, k in ((lib.COMPRESS_TUBAL, 0), (lib.COMPRESS_TUBAL, 6), (lib.COMPRESS_TSVD, 0),
                      (lib.COMPRESS_TSVD, 21), (7, 1)):
        with pytest.raises(lib.TsvdError, match="TSVD_E_INVALID"):
            lib.compress(m, method, k)


# ------------------------------------------------------------ full size

def test_factors_and_compression_at_video_size():
    """The synthetic 128 x 160 x 64 video the bench compresses (Sec. 3's
    experiment shape), at the bench's launch configuration: singular tubes
    and reconstruction against the oracle's t-SVD, and Methods 1 and 2 at
    compression ratio ~10 element by element."""
    torch = torch_cuda()
    import workloads

    x = np.asarray(workloads.video_completion(0)["X"], dtype=np.float64)
    n1, n2, n3 = x.shape
    _, s_ref, _, _, _, _ = T.tsvd(x)
    n0 = min(n1, n2)
    tubes_ref = np.stack([s_ref[(i, i)] for i in range(n0)])
    xg = to_gpu(torch, x)
    announce("tsvd_factors video", x.shape)
    u, s, v = (t.cpu().numpy() for t in lib.tsvd_factors(xg))
    assert rel_fro(s, tubes_ref) <= TOL
    assert rel_fro(reconstruct(u, s, v), x) <= TOL
    k2 = round(n1 * n2 * n3 / (10 * (n1 + n2 + 1)))
    k3 = round(n1 * n2 / (10 * (n1 + n2 + 1)))
    out_ref, keep, t, _ = C.method1(x, k2, return_details=True)
    srt = np.sort(np.unique(C.fourier_singular_values(T.tsvd(x)[4])))[::-1]
    below = srt[srt < t]
    assert below.size == 0 or (t - below[0]) / srt[0] > 1e-10   # a clear cut
    announce("compress video", k2, k3)
    m1, r1 = lib.compress(xg, lib.COMPRESS_TSVD, k2)
    assert rel_fro(m1.cpu().numpy(), out_ref) <= TOL
    assert r1 == pytest.approx(C.ratio_tsvd(n1, n2, n3, k2), rel=1e-14)
    m2, r2 = lib.compress(xg, lib.COMPRESS_TUBAL, k3)
    assert rel_fro(m2.cpu().numpy(), C.method2(x, k3)) <= TOL
    assert r2 == pytest.approx(C.ratio_tubal(n1, n2, k3), rel=1e-14)
