"""Recovery metrics, plain NumPy.  Test infrastructure only."""

from __future__ import annotations

import numpy as np


def rse(x_hat, x) -> float:
    """Relative error ||X_rec - X||_F / ||X||_F (linear form of Sec. 3's RSE)."""
    x = np.asarray(x, dtype=np.float64)
    return float(np.linalg.norm((np.asarray(x_hat, dtype=np.float64) - x).ravel())
                 / np.linalg.norm(x.ravel()))


def rse_db(x_hat, x) -> float:
    """RSE in dB as Sec. 3 defines it: 20 log10(||X_rec - X||_F / ||X||_F)."""
    return 20.0 * float(np.log10(rse(x_hat, x)))


def support_f1(s_hat, s_true, m, rel=1e-3) -> float:
    """F1 score of the recovered sparse support: predicted entries are
    |S_hat| > rel * max|M|, true entries are S_true != 0."""
    pred = np.abs(np.asarray(s_hat)) > rel * np.max(np.abs(np.asarray(m)))
    truth = np.asarray(s_true) != 0
    tp = np.count_nonzero(pred & truth)
    fp = np.count_nonzero(pred & ~truth)
    fn = np.count_nonzero(~pred & truth)
    if tp == 0:
        return 0.0
    return 2.0 * tp / (2.0 * tp + fp + fn)
