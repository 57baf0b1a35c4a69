"""t-SVD tensor algebra, Sec. 2 of arXiv:1407.1785, in plain NumPy FP64.

Test infrastructure only (see the package docstring).

Indexing is 0-based.  A third-order tensor ``A`` has shape (n1, n2, n3); its
frontal slice k is ``A[:, :, k]`` and its (i, j) tube is ``A[i, j, :]``
(Sec. 2.1, MATLAB notation shifted to 0-based).  An N-D tensor keeps modes 1
and 2 as the matrix modes and transforms every trailing mode 3..N.

DFT convention (the MATLAB ``fft`` that Algorithm 1 applies along each
trailing mode): unnormalised forward transform

    Ahat[..., k] = sum_t A[..., t] * exp(-2 pi i k t / n),

inverse with the 1/n factor.  For real data the spectrum is conjugate
symmetric, so only the half spectrum (last trailing axis cut to n//2 + 1) is
independent.
"""

from __future__ import annotations

import itertools

import numpy as np


def _trailing_axes(a: np.ndarray) -> tuple[int, ...]:
    if a.ndim < 3:
        raise ValueError("a t-SVD tensor has at least three modes")
    return tuple(range(2, a.ndim))


def fourier(a: np.ndarray) -> np.ndarray:
    """Full DFT along every trailing mode (Algorithm 1, first loop).

    Algorithm 1 prints the transform as restarting from M at every mode; the
    transforms are chained here (mode 3, then mode 4 of the result, ...),
    which is the N-D DFT the algorithm needs.
    """
    d = np.asarray(a, dtype=np.complex128)
    for ax in _trailing_axes(d):
        d = np.fft.fft(d, axis=ax)
    return d


def ifourier(ahat: np.ndarray) -> np.ndarray:
    """Inverse of :func:`fourier` (Algorithm 1, last loop); complex result."""
    d = np.asarray(ahat, dtype=np.complex128)
    for ax in _trailing_axes(d):
        d = np.fft.ifft(d, axis=ax)
    return d


def fourier_half(a: np.ndarray) -> np.ndarray:
    """Half spectrum of a real tensor: last trailing axis cut to n//2+1."""
    return np.fft.rfftn(np.asarray(a, dtype=np.float64), axes=_trailing_axes(a))


def ifourier_half(ahat: np.ndarray, trailing_shape: tuple[int, ...]) -> np.ndarray:
    """Real inverse of :func:`fourier_half` (imaginary parts of the
    self-conjugate bins are discarded, as a real inverse must)."""
    axes = tuple(range(2, 2 + len(trailing_shape)))
    return np.fft.irfftn(ahat, s=trailing_shape, axes=axes)


# ---------------------------------------------------------------- t-product

def tprod_direct(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """t-product by its definition (Sec. 2.1, Def. t-product).

    C(i, j, :) = sum_k A(i, k, :) (*) B(k, j, :), where (*) is the circular
    convolution of two tubes: (x (*) y)[t] = sum_s x[s] y[(t - s) mod n3].
    Third-order tensors only.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n1, n2, n3 = a.shape
    n2b, n4, n3b = b.shape
    if n2 != n2b or n3 != n3b:
        raise ValueError("t-product shape mismatch")
    c = np.zeros((n1, n4, n3))
    for t in range(n3):
        for s in range(n3):
            # frontal slice s of A times frontal slice (t - s) mod n3 of B
            c[:, :, t] += a[:, :, s] @ b[:, :, (t - s) % n3]
    return c


def tprod_fft(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """t-product through the Fourier domain (Sec. 2.1, the paragraph after
    the f-diagonal definition): transform the tubes, multiply matching
    frontal slices, transform back.  Works for N-D tensors (all trailing
    modes transformed)."""
    ah = fourier(a)
    bh = fourier(b)
    ch = np.einsum("ik...,kj...->ij...", ah, bh)
    return np.real(ifourier(ch))


def ttranspose(a: np.ndarray) -> np.ndarray:
    """Tensor transpose (Sec. 2.1, Def. tensor transpose): transpose every
    frontal slice, then reverse the order of frontal slices 2..n3."""
    a = np.asarray(a)
    if a.ndim != 3:
        raise ValueError("tensor transpose is defined for third-order tensors")
    n3 = a.shape[2]
    out = np.empty((a.shape[1], a.shape[0], n3), dtype=a.dtype)
    out[:, :, 0] = a[:, :, 0].T
    for k in range(1, n3):
        out[:, :, k] = a[:, :, n3 - k].T
    return out


def tidentity(n: int, n3: int) -> np.ndarray:
    """Identity tensor (Sec. 2.1): first frontal slice I, the rest zero."""
    e = np.zeros((n, n, n3))
    e[:, :, 0] = np.eye(n)
    return e


def is_fdiagonal(a: np.ndarray, atol: float = 0.0) -> bool:
    """f-diagonal test (Sec. 2.1): every frontal slice is diagonal."""
    a = np.asarray(a)
    n1, n2 = a.shape[:2]
    off = np.ones((n1, n2), dtype=bool)
    for i in range(min(n1, n2)):
        off[i, i] = False
    return bool(np.all(np.abs(a[off]) <= atol))


# -------------------------------------------------------------------- t-SVD

def _mirror(index: tuple[int, ...], dims: tuple[int, ...]) -> tuple[int, ...]:
    return tuple((-k) % n for k, n in zip(index, dims))


def tsvd(m: np.ndarray):
    """t-SVD M = U * S * V^T (Sec. 2.2, Algorithm 1), N-D.

    Algorithm 1 takes one matrix SVD per Fourier frontal slice.  Independent
    SVDs of a slice and of its conjugate mirror would give inconsistent
    phases and complex factors after the inverse transform, so the SVD is
    taken once per conjugate pair and mirrored by conjugation; the
    self-conjugate slices are real matrices and get a real SVD.  The result
    is real U (n1 x n1 x ...), S (n1 x n2 x ..., f-diagonal) and
    V (n2 x n2 x ...).  Returns (U, S, V, Uhat, Shat, Vhat).
    """
    m = np.asarray(m, dtype=np.float64)
    n1, n2 = m.shape[:2]
    dims = m.shape[2:]
    mh = fourier(m)
    uh = np.zeros((n1, n1) + dims, dtype=np.complex128)
    sh = np.zeros((n1, n2) + dims, dtype=np.complex128)
    vh = np.zeros((n2, n2) + dims, dtype=np.complex128)
    r = min(n1, n2)
    for idx in itertools.product(*[range(n) for n in dims]):
        mir = _mirror(idx, dims)
        sl = (slice(None), slice(None)) + idx
        if mir < idx:
            msl = (slice(None), slice(None)) + mir
            uh[sl] = np.conj(uh[msl])
            sh[sl] = sh[msl]
            vh[sl] = np.conj(vh[msl])
            continue
        d = mh[sl]
        if mir == idx:
            u, s, vt = np.linalg.svd(d.real, full_matrices=True)
        else:
            u, s, vt = np.linalg.svd(d, full_matrices=True)
        uh[sl] = u
        vh[sl] = np.conj(vt.T)
        diag = np.zeros((n1, n2))
        diag[np.arange(r), np.arange(r)] = s
        sh[sl] = diag
    u = np.real(ifourier(uh))
    s = np.real(ifourier(sh))
    v = np.real(ifourier(vh))
    return u, s, v, uh, sh, vh


def tsvd_truncate(u: np.ndarray, s: np.ndarray, v: np.ndarray, k: int) -> np.ndarray:
    """M_k = sum_{i<k} U(:, i, :) * S(i, i, :) * V(:, i, :)^T (Theorem 2.3.1),
    third-order tensors."""
    n3 = u.shape[2]
    out = np.zeros((u.shape[0], v.shape[0], n3))
    for i in range(k):
        ui = u[:, i:i + 1, :]
        si = s[i:i + 1, i:i + 1, :]
        vi = ttranspose(v[:, i:i + 1, :])
        out += tprod_direct(tprod_direct(ui, si), vi)
    return out


# ------------------------------------------------- complexity measures (2.4)

def multirank(a: np.ndarray, rtol: float = 1e-10) -> np.ndarray:
    """Tensor multi-rank (Sec. 2.4): rank of every Fourier frontal slice.

    A singular value counts when it exceeds rtol times the largest singular
    value over all slices.  Returned with the trailing-mode shape."""
    ah = fourier(a)
    dims = ah.shape[2:]
    sv = np.linalg.svd(np.moveaxis(ah.reshape(ah.shape[:2] + (-1,)), 2, 0), compute_uv=False)
    cut = rtol * max(sv.max(), np.finfo(float).tiny)
    return (sv > cut).sum(axis=1).reshape(dims)


def tubal_rank(a: np.ndarray, rtol: float = 1e-10) -> int:
    """Tubal rank (Sec. 2.4): number of non-zero singular tubes of S.  A tube
    S(i, i, :) is non-zero when some Fourier slice has an i-th singular value
    above the cut, so the tubal rank is the largest entry of the multi-rank."""
    return int(multirank(a, rtol).max())


def tnn(a: np.ndarray) -> float:
    """Tensor nuclear norm (Sec. 2.4, TNN theorem): the sum of the singular
    values of all Fourier frontal slices (unnormalised DFT)."""
    ah = fourier(a)
    sl = np.moveaxis(ah.reshape(ah.shape[:2] + (-1,)), 2, 0)
    return float(np.linalg.svd(sl, compute_uv=False).sum())


def blkdiag(ahat: np.ndarray) -> np.ndarray:
    """blkdiag of the Fourier frontal slices (Sec. 2.4): a block-diagonal
    matrix whose diagonal blocks are the slices in order."""
    n1, n2 = ahat.shape[:2]
    sl = np.moveaxis(ahat.reshape((n1, n2, -1)), 2, 0)
    out = np.zeros((n1 * len(sl), n2 * len(sl)), dtype=ahat.dtype)
    for k, blk in enumerate(sl):
        out[k * n1:(k + 1) * n1, k * n2:(k + 1) * n2] = blk
    return out
