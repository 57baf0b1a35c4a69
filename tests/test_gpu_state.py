"""Checkpoint and resume of the single-problem solvers (tsvd_state): the
completion ADMM of Sec. 4 (X/Z/Q recursion) and the tensor-RPCA ADMM of
Sec. 5 (L/S/W recursion) run for k iterations, saved, and resumed for N - k
more give bit for bit the N-iteration result when the Jacobi warm start (the
right singular vectors of the last prox) is part of the state, and agree to
rounding without it."""

import numpy as np
import pytest

import paper_1407_1785_amd as lib
from oracle import admm
import workloads
from tests.gpu_util import announce, rel_fro, to_gpu, torch_cuda

pytestmark = pytest.mark.gpu

N, K = 14, 5


def _completion_data(torch, fp32, shape=(40, 34, 12)):
    rng = np.random.default_rng(31)
    _, _, x = workloads.lowrank(rng, *shape, 3)
    mask = (rng.random(shape) < 0.5).astype(np.uint8)
    dt = torch.float32 if fp32 else torch.float64
    return to_gpu(torch, x * mask, dt), to_gpu(torch, mask), x * mask, mask


@pytest.mark.parametrize("fp32", [False, True])
def test_completion_resume_is_bit_exact(fp32):
    torch = torch_cuda()
    y, m, _, _ = _completion_data(torch, fp32)
    prec = lib.PREC_FP32 if fp32 else lib.PREC_FP64
    announce("resume completion", "fp32" if fp32 else "fp64")
    whole, info_w = lib.tsvd_complete(y, m, 1e-2, 0.0, max_iter=N, precision=prec)
    st = lib.SolverState(y)
    _, info_a = lib.tsvd_complete(y, m, 1e-2, 0.0, max_iter=K, precision=prec, state=st, save=True)
    assert info_a.iters == K and st.iter == K
    assert np.isclose(st.penalty, 1e-2 * 1.1 ** K, rtol=1e-12)
    part, info_b = lib.tsvd_complete(y, m, 1e-2, 0.0, max_iter=N - K, precision=prec, state=st, load=True,
                                     save=True)
    assert info_b.iters == N - K and st.iter == N
    np.testing.assert_array_equal(part.cpu().numpy(), whole.cpu().numpy())
    assert info_b.rho_final == info_w.rho_final


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("shrink", ["l1", "l112"])
def test_trpca_resume_is_bit_exact(fp32, shrink):
    torch = torch_cuda()
    p = workloads.trpca_problem(0, shape=(36, 30, 10), rank=3)
    dt = torch.float32 if fp32 else torch.float64
    prec = lib.PREC_FP32 if fp32 else lib.PREC_FP64
    code = lib.SHRINK_L1 if shrink == "l1" else lib.SHRINK_L112
    x = to_gpu(torch, p["M"], dt)
    announce("resume trpca", shrink, "fp32" if fp32 else "fp64")
    Lw, Sw, _ = lib.trpca(x, p["lam"], 1e-3, 0.0, shrink=code, max_iter=N, precision=prec)
    st = lib.SolverState(x, rpca=True)
    lib.trpca(x, p["lam"], 1e-3, 0.0, shrink=code, max_iter=K, precision=prec, state=st, save=True)
    Lr, Sr, _ = lib.trpca(x, p["lam"], 1e-3, 0.0, shrink=code, max_iter=N - K, precision=prec, state=st,
                          load=True)
    np.testing.assert_array_equal(Lr.cpu().numpy(), Lw.cpu().numpy())
    np.testing.assert_array_equal(Sr.cpu().numpy(), Sw.cpu().numpy())


def test_resume_without_singular_vectors_matches_oracle():
    """Without the Jacobi warm start the first resumed SVDs start cold: the
    iterates change by rounding only, so the resumed solve still matches the
    oracle's N iterations."""
    torch = torch_cuda()
    y, m, y_np, m_np = _completion_data(torch, False)
    ref = admm.complete(y_np, m_np, 1e-2, 1.1, 1e3, max_iter=N, tol=0.0)
    st = lib.SolverState(y, with_v=False)
    announce("resume without V")
    lib.tsvd_complete(y, m, 1e-2, 0.0, max_iter=K, state=st, save=True)
    x, _ = lib.tsvd_complete(y, m, 1e-2, 0.0, max_iter=N - K, state=st, load=True)
    assert rel_fro(x.cpu().numpy(), ref["X"]) <= 1e-10


def test_state_from_the_oracle_iterates():
    """A state written from the oracle's own iterates after K iterations (Z,
    the scaled dual Q and the next penalty) continues the recursion: K + (N -
    K) GPU iterations equal the oracle's N."""
    torch = torch_cuda()
    y, m, y_np, m_np = _completion_data(torch, False)
    ref_k = admm.complete(y_np, m_np, 1e-2, 1.1, 1e3, max_iter=K, tol=0.0)
    ref_n = admm.complete(y_np, m_np, 1e-2, 1.1, 1e3, max_iter=N, tol=0.0)
    st = lib.SolverState(y, with_v=False)
    st.z.copy_(to_gpu(torch, ref_k["Z"]))
    st.dual.copy_(to_gpu(torch, ref_k["Q"]))   # already rescaled: dual_scale 1
    st.record.penalty = 1e-2 * 1.1 ** K
    st.record.dual_scale = 1.0
    st.record.iter = K
    announce("state from oracle")
    x, _ = lib.tsvd_complete(y, m, 1e-2, 0.0, max_iter=N - K, state=st, load=True, save=False)
    assert rel_fro(x.cpu().numpy(), ref_n["X"]) <= 1e-10


def test_invalid_state_is_rejected():
    torch = torch_cuda()
    y, m, _, _ = _completion_data(torch, False)
    st = lib.SolverState(y)
    st.record.penalty = -1.0
    announce("invalid state")
    with pytest.raises(lib.TsvdError) as e:
        lib.tsvd_complete(y, m, 1e-2, 0.0, max_iter=2, state=st, load=True)
    assert e.value.status == -1
    st2 = lib.SolverState(y)
    st2.record.dual = None
    with pytest.raises(lib.TsvdError) as e:
        lib.tsvd_complete(y, m, 1e-2, 0.0, max_iter=2, state=st2, save=True)
    assert e.value.status == -1
    # the batched and served forms take no state
    p = lib.complete_problem(y, m, max_iter=2)
    p.record.opts.state = lib.ctypes.pointer(st.record)
    with pytest.raises(lib.TsvdError) as e:
        lib.batch_run([p])
    assert e.value.status == -6
