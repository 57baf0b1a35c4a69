"""Compression by truncated t-SVD, Sec. 3 of arXiv:1407.1785, in plain NumPy FP64.

Test infrastructure only (see the package docstring).

Sec. 3 compares three truncations of a third-order tensor M (n1 x n2 x n3):

* the vectorised matrix SVD: each frontal slice becomes a column of an
  n1 n2 x n3 matrix, truncated to rank k1 (ratio n1 n2 n3 / (k1 (n1 n2 + n3 + 1)));
* Method 1, t-SVD compression: keep the k2 largest f-diagonal entries of the
  Fourier-domain S (over all n0 n3 of them, n0 = min(n1, n2)), zero the rest
  together with their columns of U and V, and transform back
  (ratio n1 n2 n3 / (k2 (n1 + n2 + 1)));
* Method 2, t-SVD-tubal compression: keep the first k3 singular tubes,
  M_k3 = sum_{i<k3} U(:, i, :) * S(i, i, :) * V(:, i, :)^T (the truncation of
  Theorem 2.3.1; ratio n1 n2 / (k3 (n1 + n2 + 1))).

Reading for Method 1 (the paper does not say how conjugate pairs are
counted): the entries of S over the full spectrum come in conjugate pairs of
equal value (slice k and slice n3 - k), and a truncation that keeps one
member of a pair gives a complex tensor.  The kept set is therefore
{sigma >= t} for the smallest threshold t whose number of entries (every
entry of the full spectrum counted once) is at most k2: pairs, and exact ties
at the cut, are kept or dropped together, so fewer than k2 entries can be
kept.
"""

from __future__ import annotations

import numpy as np

from . import tensor


def ratio_svd(n1: int, n2: int, n3: int, k1: int) -> float:
    """Compression ratio of the rank-k1 vectorised matrix SVD (Sec. 3)."""
    return n1 * n2 * n3 / (k1 * (n1 * n2 + n3 + 1))


def ratio_tsvd(n1: int, n2: int, n3: int, k2: int) -> float:
    """Compression ratio of Method 1 (Sec. 3)."""
    return n1 * n2 * n3 / (k2 * (n1 + n2 + 1))


def ratio_tubal(n1: int, n2: int, k3: int) -> float:
    """Compression ratio of Method 2 (Sec. 3)."""
    return n1 * n2 / (k3 * (n1 + n2 + 1))


def fourier_singular_values(shat: np.ndarray) -> np.ndarray:
    """The f-diagonal entries of a Fourier-domain S: shape (n0,) + trailing."""
    n0 = min(shat.shape[0], shat.shape[1])
    return np.real(np.stack([shat[i, i] for i in range(n0)]))


def method1_threshold(sig: np.ndarray, k2: int) -> float:
    """Smallest t with #{sigma >= t} <= k2 over the given values (the reading
    above); +inf when even the largest value occurs more than k2 times."""
    vals = np.sort(np.unique(sig.ravel()))[::-1]
    best = np.inf
    for t in vals:
        if np.count_nonzero(sig >= t) <= k2:
            best = t
        else:
            break
    return float(best)


def method1(m: np.ndarray, k2: int, return_details: bool = False):
    """Method 1 (t-SVD compression) of a real third-order tensor.

    Algorithm 1 gives Uhat, Shat, Vhat (one SVD per conjugate pair of Fourier
    slices, mirrored by conjugation); the entries sigma >= t of Shat are kept
    (threshold of method1_threshold), the others and their columns of Uhat
    and Vhat are zeroed, and the product Uhat_k Shat_k Vhat_k^H is
    transformed back along the third mode.  Returns the real approximation
    (and, with return_details, the kept mask, the threshold and the largest
    imaginary part left by the inverse transform)."""
    m = np.asarray(m, dtype=np.float64)
    if m.ndim != 3:
        raise ValueError("the compression methods are stated for third-order tensors")
    _, _, _, uh, sh, vh = tensor.tsvd(m)
    sig = fourier_singular_values(sh)
    t = method1_threshold(sig, k2)
    keep = sig >= t
    n0 = sig.shape[0]
    zh = np.zeros(m.shape, dtype=np.complex128)
    for k in range(m.shape[2]):
        d = sig[:, k] * keep[:, k]
        zh[:, :, k] = (uh[:, :n0, k] * d) @ np.conj(vh[:, :n0, k]).T
    z = tensor.ifourier(zh)
    out = np.real(z)
    if return_details:
        return out, keep, t, float(np.max(np.abs(np.imag(z))))
    return out


def method2(m: np.ndarray, k3: int) -> np.ndarray:
    """Method 2 (t-SVD-tubal compression): the sum of the first k3 t-products
    U(:, i, :) * S(i, i, :) * V(:, i, :)^T of the t-SVD (Theorem 2.3.1)."""
    m = np.asarray(m, dtype=np.float64)
    if m.ndim != 3:
        raise ValueError("the compression methods are stated for third-order tensors")
    u, s, v, _, _, _ = tensor.tsvd(m)
    return tensor.tsvd_truncate(u, s, v, k3)


def matrix_svd(m: np.ndarray, k1: int) -> np.ndarray:
    """The vectorised matrix-SVD baseline of Sec. 3: frontal slices as the
    columns of an n1 n2 x n3 matrix, truncated to rank k1, folded back."""
    m = np.asarray(m, dtype=np.float64)
    n1, n2, n3 = m.shape
    a = np.stack([m[:, :, k].ravel() for k in range(n3)], axis=1)
    u, s, vt = np.linalg.svd(a, full_matrices=False)
    ak = (u[:, :k1] * s[:k1]) @ vt[:k1]
    return np.stack([ak[:, k].reshape(n1, n2) for k in range(n3)], axis=2)
