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


def _blocks_rel(diff, ref, axes_keep):
    """Relative Frobenius error of every block of `diff` (blocks = the index
    tuples of the kept axes), each against max(its reference block's norm,
    the reference norm spread evenly over the blocks)."""
    red = tuple(i for i in range(diff.ndim) if i not in axes_keep)
    num = np.sqrt(np.sum(np.abs(diff) ** 2, axis=red))
    den_blocks = np.sqrt(np.sum(np.abs(ref) ** 2, axis=red))
    even = np.linalg.norm(ref.ravel()) / np.sqrt(den_blocks.size)
    return float(np.max(num / np.maximum(den_blocks, even)))


def slice_rel_max(got, want):
    """Largest relative error over the Fourier frontal slices (DFT along every
    trailing mode, numpy.fft as the measuring routine).  Each slice is judged
    against its own norm, floored at an even share of the tensor's norm, so
    one wrong slice shows up at its own scale (a norm over the whole tensor
    dilutes it by the square root of the slice count)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    ax = tuple(range(2, want.ndim))
    fw = np.fft.fftn(want, axes=ax)
    fd = np.fft.fftn(got - want, axes=ax)
    return _blocks_rel(fd, fw, ax)


def tube_rel_max(got, want):
    """Largest relative error over the tubes (i, j, :), each against its own
    norm floored at an even share of the tensor's norm."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return _blocks_rel(got - want, want, (0, 1))


def tube_bar(bar, shape):
    """Bar of tube_rel_max matching `bar` on the whole tensor.  An error spread
    evenly over T = n1 n2 tubes of length L gives tube errors whose largest
    exceeds their root mean square by about sqrt(2 ln T / L) (the maximum of
    T chi variables with L degrees of freedom), so the per-tube bar is
    bar (1 + sqrt(2 ln T / L)); an error held by one tube shows up at sqrt(T)
    times its share of the whole, far above it."""
    t = shape[0] * shape[1]
    length = int(np.prod(shape[2:])) if len(shape) > 2 else 1
    return bar * (1.0 + np.sqrt(2.0 * np.log(max(t, 2)) / length))


def assert_close_fp32(got, want, bar, what=""):
    """The precision form's bar on the whole tensor and on every Fourier slice,
    and its per-tube counterpart on every tube (each printed, so the log keeps
    the margins)."""
    f, s, t = rel_fro(got, want), slice_rel_max(got, want), tube_rel_max(got, want)
    tb = tube_bar(bar, np.shape(want))
    print(f"[fp32-error] {what} fro {f:.3e} slice-max {s:.3e} tube-max {t:.3e} (bar {bar:.0e}, tube bar {tb:.2e})",
          flush=True)
    assert f <= bar, (what, "fro", f)
    assert s <= bar, (what, "slice", s)
    assert t <= tb, (what, "tube", t)
