"""Edge cases through the C ABI: every shape the library rejects, the
largest accepted sizes (tube length 512, 258 Fourier slices, 2^18 rows)
against the FP64 oracle, the zero tensor, and completion with every entry
observed."""

import ctypes

import numpy as np
import pytest

import paper_1407_1785_amd as lib
from oracle import admm
from oracle.tsvt import tsvt as tsvt_oracle
import workloads
from tests.gpu_util import announce, rel_fro, to_gpu, torch_cuda

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _raw_tsvt(torch, dims, buf_elems=64):
    """tsvt on a shape record with non-null device buffers of buf_elems
    doubles (the shape is rejected before any access)."""
    x = torch.zeros(buf_elems, dtype=torch.float64, device="cuda")
    z = torch.zeros_like(x)
    s = lib.Shape()
    s.ndim = len(dims)
    for k, v in enumerate(dims[:4]):
        s.n[k] = int(v)
    ranks = (ctypes.c_int32 * 1024)()
    h = lib.Handle()
    try:
        return lib.load_library().tsvt(h.ptr, ctypes.c_void_p(x.data_ptr()), s, lib.DTYPE_F64, 1.0,
                                       lib.PREC_FP64, ctypes.c_void_p(z.data_ptr()), ranks)
    finally:
        h.close()


@pytest.mark.parametrize("dims", [
    (0, 5, 6),            # a dimension below 1
    (4, 5, -1),
    (4, 5),               # two modes
    (2, 2, 2, 2, 2),      # five modes
    (4, 5, 513),          # tube length above 512
    (4, 5, 4, 129),       # 4-D tube of 516 entries
    (4, 5, 64, 8),        # 4-D: 64 x 5 = 320 Fourier slices (above 300)
    (262145, 2, 1),       # longer matrix mode above 2^18
])
def test_rejected_shapes(dims):
    torch = torch_cuda()
    announce("rejected shape", dims)
    assert _raw_tsvt(torch, dims) == -2   # TSVD_E_SHAPE


def test_empty_tensor_is_rejected():
    torch = torch_cuda()
    announce("empty tensor")
    with pytest.raises(lib.TsvdError):
        lib.tsvt(torch.zeros((0, 5, 6), dtype=torch.float64, device="cuda"), 1.0)


@pytest.mark.parametrize("shape", [(6, 5, 512), (5, 4, 2, 256)])
def test_longest_tubes_and_most_slices(shape):
    """Tube length 512 (257 slices), and 4-D 2 x 256 (258 slices)."""
    torch = torch_cuda()
    rng = np.random.default_rng(sum(shape))
    x = rng.normal(size=shape)
    tau = 1.5
    z_ref, r_ref = tsvt_oracle(x, tau)
    announce("max tube", shape)
    z, ranks = lib.tsvt(to_gpu(torch, x), tau)
    assert rel_fro(z.cpu().numpy(), z_ref) <= TOL
    assert ranks == list(r_ref)


def test_longest_matrix_mode():
    """2^18 rows (the largest accepted), two columns, n3 = 2: tall slices."""
    torch = torch_cuda()
    rng = np.random.default_rng(18)
    x = rng.normal(size=(1 << 18, 2, 2))
    tau = 700.0   # below both singular values of each slice (~724)
    z_ref, r_ref = tsvt_oracle(x, tau)
    announce("max rows", x.shape)
    z, ranks = lib.tsvt(to_gpu(torch, x), tau)
    assert rel_fro(z.cpu().numpy(), z_ref) <= TOL
    assert ranks == list(r_ref)


def test_zero_tensor():
    torch = torch_cuda()
    for shape in [(7, 5, 4), (40, 33, 1), (9, 12, 3, 4)]:
        announce("zero tensor", shape)
        z, ranks = lib.tsvt(torch.zeros(shape, dtype=torch.float64, device="cuda"), 0.5)
        assert torch.count_nonzero(z).item() == 0
        assert all(r == 0 for r in ranks)


def test_completion_with_everything_observed():
    """Omega = 1: the iterate X = Omega.M + (1 - Omega).(Z - Q) is M itself,
    and the solver returns it exactly; the oracle agrees."""
    torch = torch_cuda()
    rng = np.random.default_rng(8)
    m = rng.normal(size=(20, 16, 6))
    mask = np.ones(m.shape, dtype=np.uint8)
    announce("completion all observed")
    out, info = lib.tsvd_complete(to_gpu(torch, m), to_gpu(torch, mask), tol=0.0, max_iter=5)
    np.testing.assert_array_equal(out.cpu().numpy(), m)
    ref = admm.complete(m, mask, 1e-2, 1.1, 1e3, max_iter=5, tol=0.0)
    np.testing.assert_array_equal(ref["X"], m)


def test_persistent_jacobi_fallback(monkeypatch):
    """Every wait between the workgroups of the persistent Jacobi gives up at
    its first poll (spin limit 0 from the host): the workgroups write their
    blocks home and stop, and the one-workgroup-per-slice kernel finishes the
    SVDs from there.  Results still match the oracle."""
    torch = torch_cuda()
    monkeypatch.setenv("TSVD_PERSIST_SPIN", "0")
    rng = np.random.default_rng(77)
    x = rng.normal(size=(96, 80, 12))
    z_ref, r_ref = tsvt_oracle(x, 4.0)
    announce("persistent fallback tsvt")
    z, ranks = lib.tsvt(to_gpu(torch, x), 4.0)
    assert rel_fro(z.cpu().numpy(), z_ref) <= 1e-10 and ranks == list(r_ref)
    w = workloads.completion_small(0)
    ref = admm.complete(w["M_obs"], w["mask"], max_iter=6, tol=0.0)
    announce("persistent fallback completion")
    xo, _ = lib.tsvd_complete(to_gpu(torch, w["M_obs"]), to_gpu(torch, w["mask"]), 1e-2, 0.0, max_iter=6)
    assert rel_fro(xo.cpu().numpy(), ref["X"]) <= 1e-10


@pytest.mark.parametrize("schedule", ["pairs", "rounds", "pairs-fallback"])
def test_jacobi_schedule_when_persistent_grid_exceeds_cus(schedule, monkeypatch):
    """251 Fourier slices of 40 x 36: the persistent Jacobi would need 502
    co-resident workgroups, more than the CUs, so the single-problem drivers
    take the block-pair kernel (one workgroup per block pair, roles in ticket
    order, all sweeps in one launch); TSVD_PAIRS_SINGLE=0 takes one launch
    per round instead; a spin limit of zero makes every wait between the
    block-pair workgroups give up, and the gated one-workgroup-per-slice
    kernel finishes the SVDs.  Each against the oracle: t-SVT in FP64 and in
    the FP32 form, and 8 completion iterations (warm-started SVDs)."""
    torch = torch_cuda()
    if schedule == "rounds":
        monkeypatch.setenv("TSVD_PAIRS_SINGLE", "0")
    if schedule == "pairs-fallback":
        monkeypatch.setenv("TSVD_PERSIST_SPIN", "0")
    rng = np.random.default_rng(251)
    x = rng.normal(size=(40, 36, 500))
    z_ref, r_ref = tsvt_oracle(x, 6.0)
    announce("many-slice tsvt fp64", schedule)
    z, ranks = lib.tsvt(to_gpu(torch, x), 6.0)
    assert rel_fro(z.cpu().numpy(), z_ref) <= 1e-10 and ranks == list(r_ref)
    announce("many-slice tsvt fp32", schedule)
    z32, _ = lib.tsvt(to_gpu(torch, x.astype(np.float32)), 6.0, precision=lib.PREC_FP32)
    assert rel_fro(z32.cpu().numpy().astype(np.float64), z_ref) <= 1e-4
    a = rng.normal(size=(40, 3, 500))
    b = rng.normal(size=(3, 36, 500))
    m = np.real(np.fft.ifft(np.einsum("ikt,kjt->ijt", np.fft.fft(a, axis=2), np.fft.fft(b, axis=2)), axis=2))
    mask = (rng.random(m.shape) < 0.5).astype(np.uint8)
    ref = admm.complete(m * mask, mask, 1e-2, 1.1, 1e3, max_iter=8, tol=0.0)
    announce("many-slice completion", schedule)
    xo, info = lib.tsvd_complete(to_gpu(torch, m * mask), to_gpu(torch, mask), 1e-2, 0.0, max_iter=8)
    assert info.iters == 8
    assert rel_fro(xo.cpu().numpy(), ref["X"]) <= 1e-10
