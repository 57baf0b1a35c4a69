/*
 * tsvd.h -- C ABI of the MI355X (gfx950) t-SVT library.
 *
 * Hot path of Zhang, Ely, Aeron, Hao, Kilmer, "Novel methods for multilinear
 * data completion and de-noising based on tensor-SVD" (arXiv:1407.1785):
 * the tensor-nuclear-norm proximal step (t-SVT) and the two ADMM solvers
 * that call it once per iteration.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout.   Tensors are C-order arrays of shape (n1, n2, n3) or
 *           (n1, n2, n3, n4): the trailing modes of one (i, j) "tube" are
 *           contiguous, exactly as a torch/NumPy tensor of that shape.
 * Memory.   Every tensor pointer is a DEVICE pointer on the handle's device,
 *           owned by the caller.  Inputs are read only; outputs are fully
 *           overwritten; inputs and outputs must not overlap.  Host pointers
 *           are named *_host.
 * Streams.  Work is enqueued on the handle's stream (tsvd_set_stream; the
 *           null stream by default) and every call returns after that work
 *           has finished.
 * Errors.   Return codes only; nothing is thrown across the ABI.  On an
 *           error the outputs are unspecified.  tsvd_last_error() gives a
 *           human-readable message for the calling thread's last failure.
 * DFT.      Unnormalised forward DFT along every trailing mode (the MATLAB
 *           fft of Algorithm 1, Sec. 2.2), 1/n on the inverse.  Only the
 *           half spectrum of the real data is processed: for a 3-D tensor
 *           the h = n3/2 + 1 Fourier frontal slices k = 0..n3/2; for a 4-D
 *           tensor h = n3 * (n4/2 + 1) slices ordered k3 * (n4/2 + 1) + k4.
 *           The dropped slices are conjugates of kept ones and the shrinkage
 *           commutes with conjugation, so nothing is lost.
 * Precision. TSVD_PREC_FP64 computes every step in FP64 on FP64 data
 *           (dtype TSVD_F64 only).
 *
 * A handle is not thread safe: calls on one handle must not overlap.
 */
#ifndef TSVD_H
#define TSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tsvd_handle_s* tsvd_handle;

typedef enum {
    TSVD_OK = 0,
    TSVD_E_INVALID = -1,   /* bad scalar argument or null pointer          */
    TSVD_E_SHAPE = -2,     /* ndim not 3 or 4, a dimension < 1, too large   */
    TSVD_E_NOMEM = -3,     /* workspace does not fit the handle's budget    */
    TSVD_E_HIP = -4,       /* a HIP runtime call failed                     */
    TSVD_E_NONFINITE = -5, /* NaN or Inf met in the input or an iterate      */
    TSVD_E_UNSUPPORTED = -6 /* valid request this build does not serve       */
} tsvd_status;

typedef enum { TSVD_F64 = 0, TSVD_F32 = 1 } tsvd_dtype;

typedef enum { TSVD_PREC_FP64 = 0, TSVD_PREC_FP32 = 1 } tsvd_precision;

/* S-update norm of the tensor-RPCA solver (Sec. 5): entrywise l1, or the
 * paper's tube-group norm ||S||_{1,1,2} = sum_ij ||S(i,j,:)||_F (eq. sparse2). */
typedef enum { TSVD_SHRINK_L1 = 0, TSVD_SHRINK_L112 = 1 } tsvd_shrink;

typedef struct {
    int32_t ndim;  /* 3 or 4 */
    int64_t n[4];  /* n1, n2, n3[, n4]; unused entries ignored */
} tsvd_shape;

/* ADMM options.  A NULL pointer means the defaults below. */
typedef struct {
    double growth;        /* penalty growth per iteration (default 1.1 for
                             completion, 1.2 for RPCA)                        */
    double rho_max;       /* penalty cap (default 1e3 completion, 1e10 RPCA)  */
    int32_t max_iter;     /* iteration cap (default 300 completion, 500 RPCA) */
    int32_t precision;    /* tsvd_precision (default TSVD_PREC_FP64)          */
    int32_t max_sweeps;   /* Jacobi sweep cap per SVD (default 30)            */
    int32_t reserved;     /* must be 0                                        */
} tsvd_admm_opts;

/* Per-solve report (host struct filled on return). */
typedef struct {
    int32_t iters;        /* ADMM iterations run                               */
    int32_t converged;    /* 1 if the stopping test passed before max_iter     */
    int32_t sweeps_total; /* Jacobi sweeps summed over iterations (max slice)  */
    int32_t sweeps_last;  /* Jacobi sweeps of the last iteration (max slice)   */
    double primal;        /* last primal residual (Frobenius)                  */
    double change;        /* last iterate-change residual (Frobenius)          */
    double rho_final;     /* penalty used by the last prox                     */
    double seconds;       /* wall time of the solve                            */
} tsvd_info;

/* Create a handle on HIP device `device`.  `hbm_budget_bytes` bounds the
 * workspace the handle may allocate (0 = no bound).  *out receives the
 * handle.  Errors: TSVD_E_INVALID (out NULL), TSVD_E_HIP. */
tsvd_status tsvd_create(int device, size_t hbm_budget_bytes, tsvd_handle* out);

/* Release a handle and its workspace.  NULL is accepted. */
tsvd_status tsvd_destroy(tsvd_handle h);

/* Use `hip_stream` (a hipStream_t, e.g. torch's current stream) for every
 * later call on this handle.  NULL selects the null stream. */
tsvd_status tsvd_set_stream(tsvd_handle h, void* hip_stream);

/* Tensor singular value thresholding.
 *
 * Z = argmin over real Z of  tau * sum_k ||Zhat^(k)||_* +
 *                            1/2 * sum_k ||Zhat^(k) - Xhat^(k)||_F^2,
 * the Z-update of the completion ADMM (Sec. 4) with 1/rho -> tau, split into
 * one problem per Fourier frontal slice (Sec. 4.1, eq. shrink2) and solved by
 * the singular value shrinkage lemma of Sec. 4.1: every Fourier slice is
 * replaced by U diag((sigma - tau)_+) V^H.
 *
 * X, Z: device arrays of shape `shape` (C order), element type `dtype`.
 * tau >= 0.  precision: see the file header.
 * multirank_host: NULL, or a host array of h int32 that receives, per
 *   processed Fourier slice, the number of singular values above tau (the
 *   tensor multi-rank of Sec. 2.4 of the result, on the half spectrum).
 * Errors: TSVD_E_INVALID (null pointer, tau < 0 or NaN), TSVD_E_SHAPE,
 * TSVD_E_UNSUPPORTED (dtype/precision pair not built), TSVD_E_NONFINITE
 * (non-finite X), TSVD_E_NOMEM, TSVD_E_HIP. */
tsvd_status tsvt(tsvd_handle h, const void* X, tsvd_shape shape, tsvd_dtype dtype, double tau,
                 tsvd_precision precision, void* Z, int32_t* multirank_host);

/* Tensor completion by TNN minimisation (Sec. 4):
 *     min ||X||_TNN  subject to  P_Omega(X) = P_Omega(M),
 * solved by the ADMM of Sec. 4 with a scaled dual Q (X-update = projection
 * onto the constraint, Z-update = tsvt with tau = 1/rho, dual update
 * Q += X - Z).  Start Z = Q = 0.  After every iteration, with
 * primal = ||X - Z'||_F and change = ||Z' - Z||_F, the solve stops when
 * max(primal, change) <= tol * ||P_Omega(M)||_F; otherwise
 * rho <- min(growth * rho, rho_max) and Q is multiplied by rho_old/rho_new.
 *
 * X_obs: observed tensor (values off the mask are ignored).
 * mask:  uint8 device array of the same shape, 1 = observed, 0 = missing.
 * rho > 0 is the initial penalty; tol >= 0 (0 runs max_iter iterations).
 * X_out: the last X iterate, equal to X_obs on the mask.
 * info_host: NULL or a host tsvd_info.
 * Errors: as tsvt, plus TSVD_E_INVALID for rho <= 0, tol < 0, growth < 1,
 * rho_max < rho or max_iter < 1.  Reaching max_iter is not an error. */
tsvd_status tsvd_complete(tsvd_handle h, const void* X_obs, const uint8_t* mask,
                          tsvd_shape shape, tsvd_dtype dtype, double rho, double tol,
                          const tsvd_admm_opts* opts, void* X_out, tsvd_info* info_host);

/* Tensor robust PCA (Sec. 5):
 *     min ||L||_TNN + lambda ||S||  subject to  M = L + S,
 * with ||S|| the entrywise l1 norm or the tube norm ||S||_{1,1,2}, solved by
 * the ADMM of Sec. 5 with a scaled dual W: L-update = tsvt(M - S - W, 1/mu),
 * S-update = shrink(M - W - L, lambda/mu) (eq. sparse2 for the tube norm),
 * W += L + S - M.  Start L = S = W = 0.  Stops when
 * max(||L+S-M||_F, max(||dL||_F, ||dS||_F)) <= tol * ||M||_F; otherwise
 * mu <- min(growth * mu, mu_max) and W is multiplied by mu_old/mu_new.
 *
 * X: the observed tensor M.  lambda > 0, mu > 0 (initial penalty), tol >= 0.
 * L_out, S_out: device arrays of the same shape.
 * Errors: as tsvd_complete. */
tsvd_status trpca(tsvd_handle h, const void* X, tsvd_shape shape, tsvd_dtype dtype,
                  double lambda, double mu, double tol, tsvd_shrink shrink,
                  const tsvd_admm_opts* opts, void* L_out, void* S_out, tsvd_info* info_host);

/* Per-kernel timing of the work a handle runs while profiling is on: a HIP
 * event pair around every launch on the handle's stream.  `work` is the
 * kernel's algorithmic work under the cost model stated in its source file:
 * bytes moved for the DFT, shrink and elementwise kernels (work_is_bytes =
 * 1), floating-point operations for the Jacobi kernels (work_is_bytes = 0).
 * Profiling adds a synchronisation after every launch group; it is for
 * measurement runs, not production runs. */
typedef struct {
    char name[32];        /* kernel family, e.g. "jacobi_cross"            */
    int64_t launches;     /* launches timed                                */
    double total_ms;      /* summed event time                             */
    double work;          /* summed algorithmic bytes or flops             */
    int32_t work_is_bytes;
    int32_t reserved;
} tsvd_kernel_stat;

/* enable = 1 clears the statistics and starts timing; 0 stops timing
 * (statistics are kept until the next enable). */
tsvd_status tsvd_profile(tsvd_handle h, int enable);

/* Copy up to `capacity` kernel statistics into out_host (host array) and
 * their number into *count_host.  Families never launched are omitted. */
tsvd_status tsvd_profile_read(tsvd_handle h, tsvd_kernel_stat* out_host, int capacity,
                              int* count_host);

/* Static string for a status code. */
const char* tsvd_status_string(tsvd_status s);

/* Message of the calling thread's last failed call ("" if none). */
const char* tsvd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TSVD_H */
