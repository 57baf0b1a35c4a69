"""The no-allocation t-SVT entry point (tsvt_noalloc) through the C ABI
against tsvt, the entry point it varies: two calls in a row, the second on a
smaller tensor (the shared scratch keeps the first call's contents), both
precision forms, the multi-rank, a shape over the scratch maximum, and no
workspace-sized device allocation during the calls."""

import numpy as np
import pytest

import paper_1407_1785_amd as lib
import workloads
from tests.gpu_util import announce, rel_fro, to_gpu, torch_cuda

pytestmark = pytest.mark.gpu


def _free_bytes(torch):
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("fp32", [False, True])
def test_noalloc_matches_tsvt_twice(fp32):
    torch = torch_cuda()
    dt = torch.float32 if fp32 else torch.float64
    prec = lib.PREC_FP32 if fp32 else lib.PREC_FP64
    bar = 1e-4 if fp32 else 1e-10
    rng = np.random.default_rng(404)
    big = workloads.video_completion(0)["X"].astype(np.float64)   # 128 x 160 x 64, 33 slices of 160 x 128
    small = rng.normal(size=(40, 36, 10))
    handle = lib.Handle(0)
    try:
        cases = [("video", to_gpu(torch, big, dt), 5.0), ("small", to_gpu(torch, small, dt), 3.0)]
        # the references first (these also load every kernel the path uses)
        refs = [lib.tsvt(x, tau, precision=prec, handle=handle) for _, x, tau in cases]
        outs = [torch.empty_like(x) for _, x, _ in cases]
        free0 = _free_bytes(torch)
        got = []
        for (name, x, tau), z in zip(cases, outs):   # two calls in a row, the second smaller
            announce("tsvt_noalloc", name, "fp32" if fp32 else "fp64")
            got.append(lib.tsvt_noalloc(x, tau, precision=prec, handle=handle, Z=z))
        free1 = _free_bytes(torch)
        assert free0 - free1 < (4 << 20), ("device memory was allocated during the calls", free0 - free1)
        for (name, _, _), (z_na, r_na), (z_ref, r_ref) in zip(cases, got, refs):
            err = rel_fro(z_na.cpu().numpy(), z_ref.cpu().numpy())
            print(f"[noalloc] {name} {'fp32' if fp32 else 'fp64'} rel err vs tsvt {err:.3e}", flush=True)
            assert err <= bar, (name, err)
            assert r_na == r_ref
    finally:
        handle.close()


def test_noalloc_rejects_shapes_over_the_scratch():
    torch = torch_cuda()
    x = torch.zeros((256, 256, 64), dtype=torch.float32, device="cuda")
    announce("tsvt_noalloc over the scratch")
    with pytest.raises(lib.TsvdError) as e:
        lib.tsvt_noalloc(x, 1.0, precision=lib.PREC_FP32)
    assert e.value.status == -3
    # the entry point still works after the refusal
    y = to_gpu(torch, np.random.default_rng(5).normal(size=(20, 24, 6)))
    z, _ = lib.tsvt_noalloc(y, 1.0)
    z_ref, _ = lib.tsvt(y, 1.0)
    assert rel_fro(z.cpu().numpy(), z_ref.cpu().numpy()) <= 1e-10
