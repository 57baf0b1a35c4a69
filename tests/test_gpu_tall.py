"""Tall slices (the stacked columns fit no LDS-resident Jacobi kernel: the
unfoldings of Sec. 3's vectorised baselines) against the FP64 oracle."""

import numpy as np
import pytest

import paper_1407_1785_amd as lib
from oracle import admm
from oracle.tsvt import tsvt as tsvt_oracle
from tests.gpu_util import announce, assert_close_fp32, rel_fro, to_gpu, torch_cuda

pytestmark = pytest.mark.gpu

TOL = 1e-10

TALL = [
    (3000, 40, 1),    # FP64 rows beyond every LDS block, n3 = 1: a matrix SVT
    (2700, 33, 4),    # odd column count (a dummy round-robin player), 3 Fourier slices
    (33, 2900, 3),    # n1 < n2: transposed slices
    (6000, 64, 1),    # the size class of a video unfolding
]


def mid_tau(x):
    sv = np.linalg.svd(x.reshape(x.shape[0], -1) if x.shape[2] == 1 else np.fft.rfft(x, axis=2)[:, :, 0],
                       compute_uv=False)
    return float(0.5 * (sv[len(sv) // 2] + sv[len(sv) // 2 - 1]))


@pytest.mark.parametrize("shape", TALL)
def test_tall_tsvt_matches_oracle(shape):
    torch = torch_cuda()
    rng = np.random.default_rng(sum(shape))
    x = rng.normal(size=shape)
    tau = mid_tau(x)
    z_ref, r_ref = tsvt_oracle(x, tau)
    announce("tall tsvt", shape, tau)
    z, ranks = lib.tsvt(to_gpu(torch, x), tau)
    assert rel_fro(z.cpu().numpy(), z_ref) <= TOL
    assert ranks == list(r_ref)


def test_tall_tsvt_fp32_form():
    """FP32 form on a low-rank-plus-noise matrix with tau in the spectral gap
    (the regime of the completion and RPCA iterates).  A threshold inside a
    clustered band of singular values is ill-conditioned for any FP32
    orthogonalisation and is not tested here."""
    torch = torch_cuda()
    rng = np.random.default_rng(2)
    x = 3.0 * rng.normal(size=(7000, 4)) @ rng.normal(size=(4, 48)) + 0.1 * rng.normal(size=(7000, 48))
    x = x[:, :, None]
    sv = np.linalg.svd(x[:, :, 0], compute_uv=False)
    tau = float(0.5 * (sv[3] + sv[4]))
    z_ref, _ = tsvt_oracle(x, tau)
    announce("tall tsvt fp32")
    z, _ = lib.tsvt(to_gpu(torch, x, torch.float32), tau, precision=lib.PREC_FP32)
    assert_close_fp32(z.cpu().numpy(), z_ref, 1e-4, "tall tsvt")


def test_tall_low_rank_and_zero_columns():
    """Rank 3 with zero columns: the pairs with a zero column are never
    rotated, and the shrink keeps exactly the planted part above tau."""
    torch = torch_cuda()
    rng = np.random.default_rng(3)
    x = rng.normal(size=(4000, 3)) @ rng.normal(size=(3, 30))
    x[:, 5] = 0.0
    x[:, 17] = 0.0
    x = x[:, :, None]
    for tau in (0.0, 1.0, 1e9):
        z_ref, r_ref = tsvt_oracle(x, tau)
        announce("tall low rank", tau)
        z, ranks = lib.tsvt(to_gpu(torch, x), tau)
        z = z.cpu().numpy()
        assert np.abs(z - z_ref).max() <= TOL * max(1.0, np.abs(x).max())
        if tau > 0.0:   # at tau = 0 the count includes rounding-level singular values
            assert ranks == list(r_ref)


def test_tall_completion_of_an_unfolding():
    """Matrix nuclear-norm completion of the n1 n2 x n3 unfolding of a
    low-tubal-rank tensor: the n3 = 1 case of the completion solver."""
    torch = torch_cuda()
    rng = np.random.default_rng(4)
    n1, n2, n3 = 60, 50, 12
    x = rng.normal(size=(n1 * n2, 2)) @ rng.normal(size=(2, n3))
    mask = (rng.random(x.shape) < 0.5).astype(np.uint8)
    x, mask = x[:, :, None], mask[:, :, None]
    kw = dict(rho=1e-2, growth=1.1, rho_max=1e3)
    for iters in (1, 8):
        ref = admm.complete(x * mask, mask, kw["rho"], kw["growth"], kw["rho_max"], max_iter=iters, tol=0.0)
        announce("tall completion", iters)
        out, info = lib.tsvd_complete(to_gpu(torch, x * mask), to_gpu(torch, mask), tol=0.0, max_iter=iters, **kw)
        assert info.iters == iters
        assert rel_fro(out.cpu().numpy(), ref["X"]) <= TOL


@pytest.mark.parametrize("shrink", ["l1", "l112"])
def test_tall_rpca_of_an_unfolding(shrink):
    """Matrix RPCA on an n1 n2 x n3 unfolding (the n3 = 1 case of the RPCA
    solver, tall slice) against the oracle at fixed iteration counts."""
    torch = torch_cuda()
    rng = np.random.default_rng(5)
    lo = rng.normal(size=(3200, 2)) @ rng.normal(size=(2, 24)) / 40.0
    sp = np.where(rng.random(lo.shape) < 0.05, rng.uniform(-1, 1, size=lo.shape), 0.0)
    x = (lo + sp)[:, :, None]
    lam = 1.0 / np.sqrt(3200)
    code = lib.SHRINK_L1 if shrink == "l1" else lib.SHRINK_L112
    for iters in (1, 6):
        ref = admm.trpca(x, lam, 1e-3, 1.2, 1e10, max_iter=iters, tol=0.0, shrink=shrink)
        announce("tall rpca", shrink, iters)
        lg, sg, info = lib.trpca(to_gpu(torch, x), lam, mu=1e-3, tol=0.0, shrink=code, max_iter=iters)
        assert info.iters == iters
        assert rel_fro(lg.cpu().numpy(), ref["L"]) <= TOL
        assert rel_fro(sg.cpu().numpy(), ref["S"]) <= TOL
