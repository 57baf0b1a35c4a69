"""Plain FP64 CPU oracle for the t-SVD completion and tensor robust-PCA hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_1407_1785_amd``) and imports nothing from it.

What it computes follows Zhang, Ely, Aeron, Hao and Kilmer, "Novel methods for
multilinear data completion and de-noising based on tensor-SVD"
(arXiv:1407.1785):

* ``tensor``  -- Sec. 2 algebra: the mode-3 DFT convention, t-product
  (direct circular convolution and the FFT route), tensor transpose, identity,
  f-diagonal test, Algorithm 1 (t-SVD, N-D), multi-rank, tubal rank, TNN and
  blkdiag.
* ``tsvt``    -- the tensor singular value thresholding step: the Z-update of
  the completion ADMM (Sec. 4, split into one matrix problem per Fourier
  slice) solved with the shrinkage lemma of Sec. 4.1.
* ``admm``    -- the completion ADMM of Sec. 4 and the tensor-RPCA ADMM of
  Sec. 5, iterated in the paper's order with the readings stated in each
  function's docstring.
* ``metrics`` -- RSE (linear and dB, Sec. 3) and the support F1 score.

Everything is NumPy FP64 (``numpy.fft`` = pocketfft, ``numpy.linalg.svd`` =
LAPACK gesdd).  Every function is pinned by ``tests/test_oracle_*.py`` against
brute force, closed forms, textbook special cases and optimality certificates.
"""

from . import tensor, tsvt, admm, metrics  # noqa: F401
