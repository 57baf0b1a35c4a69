"""Writes tests/golden/trpca_256.npz: the FP64 oracle on the full-size tensor
RPCA workload (256 x 256 x 64, tubal rank 5, 10% entrywise corruption
U[-1, 1], lambda = 1/sqrt(256 * 64), mu0 = 1e-3 grown by 1.2, tol 1e-7,
entrywise l1 shrink; Sec. 5 with the readings stated in oracle/admm.py).

Calls only oracle/ and the input generators of workloads/.  The GPU tests
compare against it without re-running the oracle (each oracle iteration
takes about a second on 8 host cores).  Stored:

* the solve to its stop: iteration count, converged flag, (primal, change)
  history, RSE of L against the planted low-rank part, F1 of the recovered
  support, the Frobenius norms of L and S, the norm of every Fourier frontal
  slice of L, and L and S at 8192 seeded sample positions;
* the first FIXED iterations (tol = 0): the same norms and samples.

Run:  python tests/golden/make_trpca_256.py
"""

from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import admm, metrics  # noqa: E402
import workloads  # noqa: E402

FIXED = 60
SAMPLES = 8192
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "trpca_256.npz")


def slice_norms(x):
    return np.sqrt(np.sum(np.abs(np.fft.fft(x, axis=2)) ** 2, axis=(0, 1)))


def main():
    p = workloads.trpca_problem(0)
    rng = np.random.default_rng(20260256)
    pos = rng.choice(p["M"].size, size=SAMPLES, replace=False)
    full = admm.trpca(p["M"], p["lam"], p["mu"], p["growth"], p["mu_max"], p["max_iter"], p["tol"],
                      shrink="l1", history=True)
    print("to the stop:", full["iters"], "iterations, converged", full["converged"], flush=True)
    fixed = admm.trpca(p["M"], p["lam"], p["mu"], p["growth"], p["mu_max"], FIXED, 0.0, shrink="l1")
    np.savez_compressed(
        OUT, positions=pos, fixed_iters=FIXED,
        stop_iters=full["iters"], stop_converged=int(full["converged"]), stop_history=full["history"],
        stop_rse_l=metrics.rse(full["L"], p["L"]), stop_f1=metrics.support_f1(full["S"], p["S"], p["M"]),
        stop_norm_l=np.linalg.norm(full["L"]), stop_norm_s=np.linalg.norm(full["S"]),
        stop_slice_norms_l=slice_norms(full["L"]),
        stop_l=full["L"].ravel()[pos], stop_s=full["S"].ravel()[pos],
        fixed_norm_l=np.linalg.norm(fixed["L"]), fixed_norm_s=np.linalg.norm(fixed["S"]),
        fixed_slice_norms_l=slice_norms(fixed["L"]),
        fixed_l=fixed["L"].ravel()[pos], fixed_s=fixed["S"].ravel()[pos])
    print("wrote", OUT, "RSE(L)", metrics.rse(full["L"], p["L"]), "F1",
          metrics.support_f1(full["S"], p["S"], p["M"]), flush=True)


if __name__ == "__main__":
    main()
