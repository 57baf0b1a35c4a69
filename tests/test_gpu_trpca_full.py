"""The full-size tensor-RPCA workload of Sec. 5 (256 x 256 x 64, tubal rank
5, 10% entrywise corruption U[-1, 1], lambda = 1/sqrt(256 * 64), mu0 = 1e-3
grown by 1.2, tol 1e-7, entrywise l1) against the FP64 oracle's run stored
in tests/golden/trpca_256.npz (written by make_trpca_256.py beside it, which
calls only the oracle and the input generators): the stop iteration, the
planted-recovery bars (RSE of L <= 1e-5, support F1 >= 0.99), and L and S at
8192 seeded positions plus the norms of L, S and every Fourier slice of L,
at the stop and at a fixed 60 iterations."""

import os

import numpy as np
import pytest

import paper_1407_1785_amd as lib
from oracle import metrics
import workloads
from tests.gpu_util import announce, to_gpu, torch_cuda

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "trpca_256.npz")


@pytest.fixture(scope="module")
def golden():
    return dict(np.load(GOLDEN, allow_pickle=False))


@pytest.fixture(scope="module")
def problem():
    return workloads.trpca_problem(0)


def _slice_norms(x):
    return np.sqrt(np.sum(np.abs(np.fft.fft(x, axis=2)) ** 2, axis=(0, 1)))


def _compare(lo, sp, g, tag, bar):
    """L and S against the stored oracle values: the sampled entries (relative
    to the sample's norm), the tensor norms and every Fourier-slice norm of L."""
    pos = g["positions"]
    e_l = np.linalg.norm(lo.ravel()[pos] - g[tag + "_l"]) / np.linalg.norm(g[tag + "_l"])
    e_s = np.linalg.norm(sp.ravel()[pos] - g[tag + "_s"]) / max(np.linalg.norm(g[tag + "_s"]), 1e-300)
    e_nl = abs(np.linalg.norm(lo) - g[tag + "_norm_l"]) / g[tag + "_norm_l"]
    e_ns = abs(np.linalg.norm(sp) - g[tag + "_norm_s"]) / g[tag + "_norm_s"]
    sl = _slice_norms(lo)
    e_sl = np.max(np.abs(sl - g[tag + "_slice_norms_l"]) / np.max(g[tag + "_slice_norms_l"]))
    print(f"[trpca-256 {tag}] samples L {e_l:.2e} S {e_s:.2e}, norms L {e_nl:.2e} S {e_ns:.2e}, "
          f"slice norms {e_sl:.2e} (bar {bar:.0e})", flush=True)
    for v in (e_l, e_s, e_nl, e_ns, e_sl):
        assert v <= bar


def _run(torch, p, fp32, tol, max_iter):
    dt = torch.float32 if fp32 else torch.float64
    prec = lib.PREC_FP32 if fp32 else lib.PREC_FP64
    lo, sp, info = lib.trpca(to_gpu(torch, p["M"], dt), p["lam"], p["mu"], tol, shrink=lib.SHRINK_L1,
                             growth=p["growth"], mu_max=p["mu_max"], max_iter=max_iter, precision=prec)
    return lo.cpu().numpy().astype(np.float64), sp.cpu().numpy().astype(np.float64), info


def test_fp64_to_the_stop(golden, problem):
    torch = torch_cuda()
    announce("trpca 256 fp64 to tol 1e-7")
    lo, sp, info = _run(torch, problem, False, problem["tol"], problem["max_iter"])
    assert golden["stop_converged"] == 1
    assert info.converged == 1 and abs(info.iters - int(golden["stop_iters"])) <= 1
    assert metrics.rse(lo, problem["L"]) <= 1e-5
    assert metrics.support_f1(sp, problem["S"], problem["M"]) >= 0.99
    if info.iters == int(golden["stop_iters"]):
        _compare(lo, sp, golden, "stop", 1e-10)


def test_fp64_fixed_iterations(golden, problem):
    torch = torch_cuda()
    n = int(golden["fixed_iters"])
    announce("trpca 256 fp64 fixed", n)
    lo, sp, info = _run(torch, problem, False, 0.0, n)
    assert info.iters == n
    _compare(lo, sp, golden, "fixed", 1e-10)


def test_fp32_form_at_the_oracle_stop(golden, problem):
    """The FP32 form run for the oracle's iteration count: within the form's
    1e-4 of the oracle, and the planted parts recovered."""
    torch = torch_cuda()
    n = int(golden["stop_iters"])
    announce("trpca 256 fp32 at the oracle stop", n)
    lo, sp, info = _run(torch, problem, True, 0.0, n)
    assert info.iters == n
    _compare(lo, sp, golden, "stop", 1e-4)
    assert metrics.rse(lo, problem["L"]) <= 1e-5
    assert metrics.support_f1(sp, problem["S"], problem["M"]) >= 0.99


FP32_TOL = 1e-6


def test_fp32_form_with_its_stopping_rule(golden, problem):
    """The FP32 form stops by its own rule at tol 1e-6: the workload's 1e-7
    lies below the FP32 iterates' rounding floor (a relative change of 1e-7 is
    under one FP32 unit), so the FP32 form takes the next decade.  It stops
    within the iteration cap, near the oracle's stop, with the planted parts
    recovered."""
    torch = torch_cuda()
    announce("trpca 256 fp32 to tol 1e-6")
    lo, sp, info = _run(torch, problem, True, FP32_TOL, problem["max_iter"])
    print(f"[trpca-256 fp32] converged {info.converged} after {info.iters} iterations "
          f"(oracle at 1e-7: {int(golden['stop_iters'])}); primal {info.primal:.3e} change {info.change:.3e}",
          flush=True)
    assert info.converged == 1 and info.iters <= int(golden["stop_iters"]) + 1
    assert metrics.rse(lo, problem["L"]) <= 1e-5
    assert metrics.support_f1(sp, problem["S"], problem["M"]) >= 0.99
