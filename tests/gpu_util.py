"""Helpers of the GPU parity tests (no solver arithmetic here)."""

import sys

import numpy as np
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def announce(*parts):
    """Name the case on stdout before a GPU step, so a crash names it."""
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()


def to_gpu(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def rel_fro(got, want):
    want = np.asarray(want, dtype=np.float64)
    den = np.linalg.norm(want.ravel())
    num = np.linalg.norm((np.asarray(got, dtype=np.float64) - want).ravel())
    return num / den if den > 0 else num
