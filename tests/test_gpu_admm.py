"""Completion and tensor-RPCA ADMM on the GPU against the FP64 oracle, at a
fixed iteration count (tol = 0) and through convergence."""

import numpy as np
import pytest

import paper_1407_1785_amd as lib
from oracle import admm, metrics
import workloads
from tests.gpu_util import announce, assert_close_fp32, rel_fro, to_gpu, torch_cuda

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.mark.parametrize("iters", [1, 5, 40])
def test_completion_fixed_iterations(iters):
    torch = torch_cuda()
    w = workloads.completion_small(0)
    ref = admm.complete(w["M_obs"], w["mask"], max_iter=iters, tol=0.0)
    announce("complete fixed", iters)
    x, info = lib.tsvd_complete(to_gpu(torch, w["M_obs"]), to_gpu(torch, w["mask"]), 1e-2, 0.0,
                                max_iter=iters)
    assert info.iters == iters and info.converged == 0
    assert rel_fro(x.cpu().numpy(), ref["X"]) <= TOL
    assert np.isclose(info.rho_final, ref["rho"], rtol=1e-15)


def test_completion_converges_like_oracle():
    torch = torch_cuda()
    w = workloads.completion_small(0)
    ref = admm.complete(w["M_obs"], w["mask"], w["rho"], w["growth"], w["rho_max"], w["max_iter"],
                        w["tol"])
    announce("complete converge")
    x, info = lib.tsvd_complete(to_gpu(torch, w["M_obs"]), to_gpu(torch, w["mask"]), w["rho"],
                                w["tol"])
    x = x.cpu().numpy()
    assert info.converged == 1
    assert abs(info.iters - ref["iters"]) <= 1
    assert metrics.rse(x, w["X"]) <= 1e-6
    omega = w["mask"].astype(bool)
    np.testing.assert_array_equal(x[omega], w["X"][omega])


@pytest.mark.parametrize("shape", [(24, 17, 9), (15, 26, 4, 3)])
def test_completion_ragged_and_4d(shape):
    torch = torch_cuda()
    rng = np.random.default_rng(11)
    x_true = rng.normal(size=shape)
    mask = (rng.random(shape) < 0.6).astype(np.uint8)
    ref = admm.complete(x_true * mask, mask, max_iter=12, tol=0.0)
    announce("complete ragged", shape)
    x, info = lib.tsvd_complete(to_gpu(torch, x_true * mask), to_gpu(torch, mask), 1e-2, 0.0,
                                max_iter=12)
    assert rel_fro(x.cpu().numpy(), ref["X"]) <= TOL


@pytest.mark.parametrize("shrink", ["l1", "l112"])
def test_trpca_fixed_iterations(shrink):
    torch = torch_cuda()
    p = workloads.trpca_problem(0, shape=(48, 40, 16), rank=3)
    ref = admm.trpca(p["M"], p["lam"], max_iter=30, tol=0.0, shrink=shrink)
    announce("trpca fixed", shrink)
    code = lib.SHRINK_L1 if shrink == "l1" else lib.SHRINK_L112
    lo, sp, info = lib.trpca(to_gpu(torch, p["M"]), p["lam"], 1e-3, 0.0, shrink=code, max_iter=30)
    assert info.iters == 30
    assert rel_fro(lo.cpu().numpy(), ref["L"]) <= TOL
    assert rel_fro(sp.cpu().numpy(), ref["S"]) <= 1e-9


def test_trpca_recovers_planted():
    torch = torch_cuda()
    p = workloads.trpca_problem(0, shape=(48, 48, 16), rank=3)
    ref = admm.trpca(p["M"], p["lam"], p["mu"], p["growth"], p["mu_max"], p["max_iter"], p["tol"])
    announce("trpca converge")
    lo, sp, info = lib.trpca(to_gpu(torch, p["M"]), p["lam"], p["mu"], p["tol"])
    assert info.converged == 1 and abs(info.iters - ref["iters"]) <= 1
    assert metrics.rse(lo.cpu().numpy(), p["L"]) <= 1e-5
    assert metrics.support_f1(sp.cpu().numpy(), p["S"], p["M"]) >= 0.99


@pytest.mark.parametrize("fp32", [False, True])
def test_trpca_full_size_prefix(fp32):
    """The 256 x 256 x 64 RPCA workload (rank 5, 10% sparse corruption,
    entrywise l1) at its full size: the first 15 iterations against the
    oracle.  mu grows by 1.2 from 1e-3, so the shrink threshold lambda / mu
    drops below the corruption's magnitude after ~12 iterations: S is nonzero
    by the end of the prefix."""
    torch = torch_cuda()
    p = workloads.trpca_problem(0)
    ref = admm.trpca(p["M"], p["lam"], max_iter=15, tol=0.0, shrink="l1")
    assert np.count_nonzero(ref["S"]) > 0
    dt = torch.float32 if fp32 else torch.float64
    prec = lib.PREC_FP32 if fp32 else lib.PREC_FP64
    announce("trpca full size", "fp32" if fp32 else "fp64")
    lo, sp, info = lib.trpca(to_gpu(torch, p["M"], dt), p["lam"], 1e-3, 0.0, shrink=lib.SHRINK_L1, max_iter=15,
                             precision=prec)
    assert info.iters == 15
    lo, sp = lo.cpu().numpy().astype(np.float64), sp.cpu().numpy().astype(np.float64)
    if fp32:
        assert_close_fp32(lo, ref["L"], 1e-4, "rpca 256 prefix L")
        assert np.linalg.norm(sp - ref["S"]) <= 1e-4 * np.linalg.norm(p["M"])
    else:
        assert rel_fro(lo, ref["L"]) <= TOL
        assert rel_fro(sp, ref["S"]) <= 1e-9


def test_completion_random_shapes():
    """Seeded random shapes (either orientation, ragged Jacobi blocks, 3-D
    and 4-D), random sampling rates, 6 warm-started iterations each against
    the oracle."""
    torch = torch_cuda()
    rng = np.random.default_rng(4071)
    for case in range(8):
        n1, n2 = (int(v) for v in rng.integers(2, 150, size=2))
        trail = (int(rng.integers(1, 17)),) if case % 3 else (int(rng.integers(1, 4)), int(rng.integers(2, 7)))
        shape = (n1, n2) + trail
        x = rng.normal(size=shape)
        mask = (rng.random(shape) < rng.uniform(0.2, 0.8)).astype(np.uint8)
        ref = admm.complete(x * mask, mask, 1e-2, 1.1, 1e3, max_iter=6, tol=0.0)
        announce("completion random", shape)
        out, info = lib.tsvd_complete(to_gpu(torch, x * mask), to_gpu(torch, mask), 1e-2, 0.0, max_iter=6)
        assert info.iters == 6
        assert rel_fro(out.cpu().numpy(), ref["X"]) <= TOL, shape


def test_completion_large_slices():
    """256 x 200 slices, 33 of them: the warm-start and rebuild products have
    528 tiles of 64 x 64 and take the tiled form (smaller products take the
    split-K form), 4 warm-started iterations against the oracle."""
    torch = torch_cuda()
    rng = np.random.default_rng(256200)
    a, b = rng.normal(size=(256, 6, 64)), rng.normal(size=(6, 200, 64))
    x = np.fft.irfft(np.einsum("ikt,kjt->ijt", np.fft.rfft(a, axis=2), np.fft.rfft(b, axis=2)), n=64, axis=2)
    x += 0.01 * rng.normal(size=x.shape)
    mask = (rng.random(x.shape) < 0.4).astype(np.uint8)
    ref = admm.complete(x * mask, mask, 1e-2, 1.1, 1e3, max_iter=4, tol=0.0)
    announce("completion large slices", x.shape)
    out, info = lib.tsvd_complete(to_gpu(torch, x * mask), to_gpu(torch, mask), 1e-2, 0.0, max_iter=4)
    assert info.iters == 4
    assert rel_fro(out.cpu().numpy(), ref["X"]) <= TOL


def test_fp64_unchanged_by_the_sweep_floor(monkeypatch):
    """The stopping rule's rounding floor in FP64 lies far below every
    coupling that moves the video-shaped completion: 60 iterations with and
    without it run the same sweeps and return the same tensor, bit for bit,
    and both meet the oracle."""
    torch = torch_cuda()
    w = workloads.video_completion(0)
    kw = dict(rho=w["rho"], tol=0.0, growth=w["growth"], rho_max=w["rho_max"], max_iter=60)
    ref = admm.complete(w["M_obs"].astype(np.float64), w["mask"], w["rho"], w["growth"], w["rho_max"],
                        max_iter=60, tol=0.0)
    obs, mask = to_gpu(torch, w["M_obs"].astype(np.float64)), to_gpu(torch, w["mask"])
    out = {}
    for floor in ("1", "0"):
        monkeypatch.setenv("TSVD_SWEEP_FLOOR", floor)
        announce("complete fp64 video 60 floor", floor)
        x, info = lib.tsvd_complete(obs, mask, **kw)
        out[floor] = (x.cpu().numpy(), info.sweeps_total)
        assert rel_fro(out[floor][0], ref["X"]) <= TOL
    assert out["1"][1] == out["0"][1]
    np.testing.assert_array_equal(out["1"][0], out["0"][0])
