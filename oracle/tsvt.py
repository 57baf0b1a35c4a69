"""Tensor singular value thresholding (t-SVT), plain NumPy FP64.

Test infrastructure only (see the package docstring).

The Z-update of the completion ADMM (Sec. 4) is the proximal map of
(1/rho) ||blkdiag(Zhat)||_* at the Fourier-domain point Xhat + Qhat.  The
paper splits it into one matrix problem per Fourier frontal slice
(Sec. 4.1, eq. shrink2) and solves each with the singular value shrinkage
lemma of Sec. 4.1: D_tau(Y) = U diag((sigma_i - tau)_+) V^*, the unique
minimiser of 1/2 ||X - Y||_F^2 + tau ||X||_*.

Reading of the threshold scale: tau is applied to the singular values of the
unnormalised DFT slices, exactly as the Z-update is written in the Fourier
domain.  So ``tsvt(X, tau)`` is the unique minimiser over real Z of

    tau * sum_k ||Zhat^(k)||_* + 1/2 sum_k ||Zhat^(k) - Xhat^(k)||_F^2,

equivalently (Parseval) of (tau / n3) TNN(Z) + 1/2 ||Z - X||_F^2 with n3 the
product of the trailing dimensions.
"""

from __future__ import annotations

import numpy as np

from . import tensor as T


def svt_matrix(y: np.ndarray, tau: float):
    """D_tau(Y) of the Sec. 4.1 lemma for one (complex) matrix.

    Returns (D_tau(Y), number of singular values above tau).  A singular
    value equal to tau maps to zero."""
    u, s, vh = np.linalg.svd(y, full_matrices=False)
    d = np.maximum(s - tau, 0.0)
    return (u * d) @ vh, int(np.count_nonzero(s > tau))


def tsvt(x: np.ndarray, tau: float, spectrum: str = "half"):
    """t-SVT of a real tensor with threshold tau (see the module docstring).

    spectrum="half": SVT of the independent half spectrum (last trailing axis
    cut to n//2 + 1), real inverse transform.  The shrinkage commutes with
    conjugation, so the dropped slices are the conjugates of kept ones.
    spectrum="full": SVT of every Fourier slice as Algorithm 1 loops over
    all of them, then the real part of the inverse transform.

    Returns (Z, multirank) where multirank holds, per computed slice (in the
    C order of the transformed trailing axes), the count of singular values
    above tau.
    """
    if tau < 0:
        raise ValueError("tau must be non-negative")
    x = np.asarray(x, dtype=np.float64)
    n1, n2 = x.shape[:2]
    dims = x.shape[2:]
    if spectrum == "half":
        xh = T.fourier_half(x)
    elif spectrum == "full":
        xh = T.fourier(x)
    else:
        raise ValueError("spectrum is 'half' or 'full'")
    hdims = xh.shape[2:]
    flat = xh.reshape((n1, n2, -1))
    zflat = np.empty_like(flat)
    ranks = np.zeros(flat.shape[2], dtype=np.int64)
    for k in range(flat.shape[2]):
        zflat[:, :, k], ranks[k] = svt_matrix(flat[:, :, k], tau)
    zh = zflat.reshape((n1, n2) + hdims)
    if spectrum == "half":
        z = T.ifourier_half(zh, dims)
    else:
        z = np.real(T.ifourier(zh))
    return z, ranks


def tsvt_objective(z: np.ndarray, x: np.ndarray, tau: float) -> float:
    """Objective that tsvt(x, tau) minimises, written in the original domain:
    (tau / n3) TNN(Z) + 1/2 ||Z - X||_F^2 (n3 = product of trailing dims)."""
    n3 = int(np.prod(np.asarray(x).shape[2:]))
    return tau / n3 * T.tnn(z) + 0.5 * float(np.sum((np.asarray(z) - np.asarray(x)) ** 2))
