"""Completion ADMM (Sec. 4) and tensor-RPCA ADMM (Sec. 5), plain NumPy FP64.

Test infrastructure only (see the package docstring).

Readings of the paper used here (each is a choice where the paper is silent):

* Scaled dual.  The completion X-update carries X(:)^T Q(:) + 1/2||X - Z||^2,
  so Q is the dual scaled by the penalty; the tensor-RPCA recursion carries W
  the same way (the paper writes W = rho Y; a scaled dual is W = Y / rho).
* Penalty schedule.  The paper keeps rho fixed; the workloads grow it,
  rho_{k+1} = min(growth * rho_k, rho_max), and the scaled dual is multiplied
  by rho_k / rho_{k+1} so that the unscaled dual is continuous.
* Start.  Z = Q = 0 (so the first X is P_Omega(M)); L = S = W = 0.
* Stop.  Relative Frobenius residuals tested after every iteration: stop when
  max(primal, change) <= tol * ||data||_F.  tol = 0 runs max_iter iterations.
* Threshold scale.  The TNN prox uses tau = 1/rho on the singular values of
  the unnormalised DFT slices (see ``oracle.tsvt``).
* Returned iterate of the completion: X (it satisfies the constraint exactly).
"""

from __future__ import annotations

import numpy as np

from .tsvt import tsvt


def _fro(a) -> float:
    return float(np.sqrt(np.sum(np.square(a))))


def complete(m_obs, mask, rho=1e-2, growth=1.1, rho_max=1e3, max_iter=300, tol=1e-8,
             history=False):
    """TNN completion: min ||X||_TNN s.t. P_Omega(X) = P_Omega(M) (Sec. 4).

    One iteration, in the paper's order:
      X  = argmin over {P_Omega X = P_Omega M} of ||X - (Z - Q)||_F
         = Omega.M + (1 - Omega).(Z - Q)                  (X-update, Sec. 4)
      Z' = tsvt(X + Q, 1/rho)                             (Z-update, Sec. 4/4.1)
      Q~ = Q + X - Z'                                     (dual update, Sec. 4)
      primal = ||X - Z'||_F, change = ||Z' - Z||_F; stop test
      rho' = min(growth*rho, rho_max);  Q' = (rho/rho') Q~

    Values of ``m_obs`` off the mask are ignored.  Returns a dict with X, Z,
    Q (scaled, after the rescale), iters, converged, rho (the rho used by the
    last Z-update), multirank of the last Z-update and, if ``history``, the
    per-iteration (primal, change) pairs.
    """
    omega = np.asarray(mask).astype(bool)
    y = np.where(omega, np.asarray(m_obs, dtype=np.float64), 0.0)
    z = np.zeros_like(y)
    q = np.zeros_like(y)
    scale = _fro(y)
    hist = []
    x = y.copy()
    ranks = None
    converged = False
    it = 0
    rho_used = rho
    for it in range(1, max_iter + 1):
        x = np.where(omega, y, z - q)
        z_new, ranks = tsvt(x + q, 1.0 / rho)
        q_tilde = q + x - z_new
        primal = _fro(x - z_new)
        change = _fro(z_new - z)
        hist.append((primal, change))
        z = z_new
        rho_used = rho
        if max(primal, change) <= tol * scale:
            converged = True
            q = q_tilde
            break
        rho_next = min(growth * rho, rho_max)
        q = (rho / rho_next) * q_tilde
        rho = rho_next
    out = dict(X=x, Z=z, Q=q, iters=it, converged=converged, rho=rho_used, multirank=ranks)
    if history:
        out["history"] = np.asarray(hist)
    return out


def shrink_l1(d, thresh):
    """Entrywise soft threshold: sign(D) max(|D| - thresh, 0)."""
    return np.sign(d) * np.maximum(np.abs(d) - thresh, 0.0)


def shrink_tube(d, thresh):
    """Tube-group shrink of eq. sparse2 (Sec. 5): every tube D(i, j, :) is
    scaled by (1 - thresh / ||D(i, j, :)||_F)_+, and a zero tube stays zero.
    For an N-D tensor the 'tube' is everything past the first two modes."""
    d = np.asarray(d, dtype=np.float64)
    norms = np.sqrt(np.sum(d.reshape(d.shape[:2] + (-1,)) ** 2, axis=2))
    with np.errstate(divide="ignore", invalid="ignore"):
        factor = np.where(norms > 0, np.maximum(1.0 - thresh / norms, 0.0), 0.0)
    return d * factor.reshape(factor.shape + (1,) * (d.ndim - 2))


def trpca(m, lam, mu=1e-3, growth=1.2, mu_max=1e10, max_iter=500, tol=1e-7, shrink="l1",
          history=False):
    """Tensor RPCA: min ||L||_TNN + lam ||S|| s.t. M = L + S (Sec. 5).

    ``shrink="l112"`` is the paper's tube-group norm ||S||_{1,1,2} (eq.
    sparse2); ``shrink="l1"`` is the entrywise l1 norm.  One iteration:
      L' = tsvt(M - S - W, 1/mu)                          (L-update, Sec. 5)
      D  = M - W - L'
      S' = shrink(D, lam/mu)                              (S-update, eq. sparse2)
      W~ = W + L' + S' - M                                (dual update, Sec. 5)
      primal = ||L' + S' - M||_F, change = max(||L' - L||_F, ||S' - S||_F)
      stop test; mu' = min(growth*mu, mu_max); W' = (mu/mu') W~
    Returns a dict with L, S, W, iters, converged, mu, multirank[, history].
    """
    m = np.asarray(m, dtype=np.float64)
    if shrink == "l1":
        shrink_fn = shrink_l1
    elif shrink == "l112":
        shrink_fn = shrink_tube
    else:
        raise ValueError("shrink is 'l1' or 'l112'")
    lo = np.zeros_like(m)
    sp = np.zeros_like(m)
    w = np.zeros_like(m)
    scale = _fro(m)
    hist = []
    ranks = None
    converged = False
    it = 0
    mu_last = mu
    for it in range(1, max_iter + 1):
        l_new, ranks = tsvt(m - sp - w, 1.0 / mu)
        d = m - w - l_new
        s_new = shrink_fn(d, lam / mu)
        w_tilde = w + l_new + s_new - m
        primal = _fro(l_new + s_new - m)
        change = max(_fro(l_new - lo), _fro(s_new - sp))
        hist.append((primal, change))
        lo, sp = l_new, s_new
        mu_last = mu
        if max(primal, change) <= tol * scale:
            converged = True
            w = w_tilde
            break
        mu_next = min(growth * mu, mu_max)
        w = (mu / mu_next) * w_tilde
        mu = mu_next
    out = dict(L=lo, S=sp, W=w, iters=it, converged=converged, mu=mu_last, multirank=ranks)
    if history:
        out["history"] = np.asarray(hist)
    return out
