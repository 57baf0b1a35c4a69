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
 * A handle is not thread safe: calls on one handle must not overlap, except
 * tsvd_submit / tsvd_poll / tsvd_cancel / tsvd_serve_stats_read, which may be
 * called from any thread while the handle's serving worker runs.
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
    TSVD_E_UNSUPPORTED = -6, /* valid request the library does not serve     */
    TSVD_E_BUSY = -7,      /* tsvd_poll: the problem has not finished yet   */
    TSVD_E_CANCELLED = -8, /* serving: the request was cancelled            */
    TSVD_E_TIMEOUT = -9    /* serving: the request passed its deadline      */
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

/* Solver state, for checkpoint and resume of the single-problem solvers.
 *
 * The state after k iterations of the completion ADMM (Sec. 4) is the
 * iterate pair (Z, Q) with Q the scaled dual, the penalty rho of the next
 * iteration, and the factor by which the stored dual is still to be
 * multiplied (the rescale rho_k / rho_{k+1} of the penalty schedule is
 * applied lazily); for tensor RPCA (Sec. 5) it is (L, S, W) with mu.  The
 * right singular vectors of every Fourier slice of the last prox are the
 * Jacobi warm start of the next one: with them, k iterations plus N - k
 * resumed iterations give bit for bit the N-iteration result; without them
 * the first resumed SVDs start cold, which changes the iterates by rounding
 * only.
 *
 * All pointers are DEVICE arrays owned by the caller.  z, dual, s: the
 * tensor's shape and element type (z = Z or L; dual = Q or W, stored
 * values; s = S, RPCA only, else NULL).  v: NULL, or h slices of n x n
 * complex values (interleaved re, im) of the element type, column-major,
 * n = min(n1, n2), h as in the file header.
 * load = 1: the solve starts from this state (iter, penalty and dual_scale
 *   included); load = 0: it starts from zero iterates, as Sec. 4 / Sec. 5
 *   do, with the penalty argument of the call.
 * save = 1: on return the buffers hold the state after the last iteration
 *   run, penalty the next iteration's, dual_scale the pending dual factor,
 *   iter the iterations run in total (this call's added to iter on load).
 * Errors: TSVD_E_INVALID for a null z or dual (or s in RPCA), a penalty or
 *   dual_scale that is not finite and > 0 on load, or iter < 0. */
typedef struct {
    void* z;
    void* dual;
    void* s;
    void* v;
    double penalty;
    double dual_scale;
    int32_t iter;
    int32_t load;
    int32_t save;
    int32_t pad;
} tsvd_state;

/* ADMM options.  A NULL pointer means the defaults below. */
typedef struct {
    double growth;        /* penalty growth per iteration (default 1.1 for
                             completion, 1.2 for RPCA)                        */
    double rho_max;       /* penalty cap (default 1e3 completion, 1e10 RPCA)  */
    int32_t max_iter;     /* iteration cap (default 300 completion, 500 RPCA) */
    int32_t precision;    /* tsvd_precision (default TSVD_PREC_FP64)          */
    int32_t max_sweeps;   /* Jacobi sweep cap per SVD (default 30)            */
    int32_t pad;          /* must be 0                                        */
    tsvd_state* state;    /* NULL, or warm start / checkpoint of the solver
                             (tsvd_complete and trpca only; the batched and
                             served forms reject a non-NULL state)            */
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

/* tsvt without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and errors as tsvt (up to
 * rounding: the DFT matrices are built on the device here).  No hipMalloc,
 * hipFree or other allocating call is made: the workspace is a fixed array
 * of 64 MiB per GPU (a static device array, held by every GPU the library
 * runs on until the process ends), enough for slices and factors of about
 * 48 MB, e.g. a 128 x 160 x 64 tensor in FP64 or 256 x 200 x 64 in FP32.
 * A shape that needs more fails with TSVD_E_NOMEM before any device work.
 * Every call on a GPU uses that GPU's one array, whatever the handle: calls
 * that overlap on one GPU (from several threads or streams) race and must
 * be serialised by the caller; the array keeps the last call's contents,
 * and each call clears what it needs cleared.  Profiling records nothing
 * for this call. */
tsvd_status tsvt_noalloc(tsvd_handle h, const void* X, tsvd_shape shape, tsvd_dtype dtype, double tau,
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

/* The t-SVD M = U * S * V^T (Sec. 2.2, Algorithm 1): one SVD per Fourier
 * slice (half spectrum; in 4-D the conjugate pairs inside it are solved once
 * and mirrored), singular values of every slice in decreasing order, and the
 * inverse transform of the factors along the trailing modes.  The factors
 * are real; they are returned in economy form (n0 = min(n1, n2)): the
 * columns of the paper's U and V beyond n0 multiply zero rows of S.
 *
 * M: device array of shape `shape` (n1 x n2 x trailing, C order), dtype.
 * U_out: device array n1 x n0 x trailing (lateral slices U(:, i, :)).
 * S_out: device array n0 x trailing: the singular tubes S(i, i, :) (the
 *   f-diagonal of S; the rest of S is zero).
 * V_out: device array n2 x n0 x trailing.  M = sum_i U(:, i, :) * S(i, i, :)
 *   * V(:, i, :)^T.  A Fourier-domain singular value of 0 gets a zero
 *   left singular vector.
 * Errors: as tsvt (no tau). */
tsvd_status tsvd_factors(tsvd_handle h, const void* M, tsvd_shape shape, tsvd_dtype dtype,
                         tsvd_precision precision, void* U_out, void* S_out, void* V_out);

typedef enum {
    TSVD_COMPRESS_TSVD = 1,    /* Method 1: the k largest Fourier-domain singular values */
    TSVD_COMPRESS_TUBAL = 2    /* Method 2: the first k singular tubes (Theorem 2.3.1)  */
} tsvd_compress_method;

/* Compression by truncated t-SVD (Sec. 3) of a third-order tensor M:
 * Method 1 keeps the entries sigma >= t of the Fourier-domain S over the full
 * spectrum, t the smallest threshold for which at most k of them (every
 * entry of the full spectrum counted once) are kept -- conjugate pairs and
 * exact ties at the cut are kept or dropped together, so fewer than k can be
 * kept; 1 <= k <= n0 * n3.  Method 2 keeps the first k singular tubes,
 * 1 <= k <= n0.  M_out receives the approximation; ratio_host (nullable)
 * the compression ratio of Sec. 3: n1 n2 n3 / (k (n1 + n2 + 1)) for Method 1,
 * n1 n2 / (k (n1 + n2 + 1)) for Method 2.
 * Errors: TSVD_E_SHAPE for a tensor that is not third-order, TSVD_E_INVALID
 * for k out of range or an unknown method; otherwise as tsvt. */
tsvd_status tsvd_compress(tsvd_handle h, const void* M, tsvd_shape shape, tsvd_dtype dtype,
                          tsvd_precision precision, int32_t method, int64_t k, void* M_out,
                          double* ratio_host);

/* Per-kernel timing of the work a handle runs while profiling is on: a HIP
 * event pair around every launch on the handle's stream.  `work` is the
 * kernel's algorithmic work under the cost model stated in its source file:
 * bytes moved for the DFT, singular-value and elementwise kernels
 * (work_is_bytes = 1), floating-point operations for the Jacobi kernels and
 * the matrix-core GEMMs of the rebuild and the warm start (work_is_bytes = 0).
 * Profiling adds a synchronisation after every launch group; it is for
 * measurement runs, not production runs. */
typedef struct {
    char name[32];        /* kernel family, e.g. "jacobi_persistent"       */
    int64_t launches;     /* launches timed                                */
    double total_ms;      /* summed event time                             */
    double work;          /* summed algorithmic bytes or flops             */
    int32_t work_is_bytes;
    int32_t reserved;
    /* Jacobi families: summed over launches and slices, the sweeps run,
     * the column pairs visited and the rotations applied (0 elsewhere).
     * Their `work` is n (n - 1) / 2 (28 m + 20 n) flops per slice sweep
     * (one complex dot product of the m slice rows plus two rotated columns
     * of m + n stacked rows, per pair), whatever the rotations applied. */
    double slice_sweeps;
    double pairs_visited;
    double rotations;
    /* svt_rebuild: summed over launches and slices, the kept rank r_k (the
     * singular values above tau, the multi-rank of Sec. 2.4); the product
     * runs over all n columns with the dropped ones weighted by 0, and its
     * `work` counts 8 m n^2 flops per slice (0 elsewhere). */
    double kept_rank;
} tsvd_kernel_stat;

/* enable = 1 clears the statistics and starts timing; 0 stops timing
 * (statistics are kept until the next enable). */
tsvd_status tsvd_profile(tsvd_handle h, int enable);

/* Copy up to `capacity` kernel statistics into out_host (host array) and
 * their number into *count_host.  Families never launched are omitted. */
tsvd_status tsvd_profile_read(tsvd_handle h, tsvd_kernel_stat* out_host, int capacity,
                              int* count_host);

/* ------------------------------------------------------------------------
 * Batched and served solves
 * ------------------------------------------------------------------------
 * Many completion (Sec. 4) or tensor-RPCA (Sec. 5) problems of uneven shapes
 * run together on one device: every phase of an ADMM iteration (forward
 * DFT, warm-start GEMMs, Jacobi SVD, singular values, rebuild, inverse DFT,
 * control) is one launch over all running problems, driven by per-problem
 * argument tables; iterations are replayed from a captured HIP graph; the
 * Jacobi block width of every shape is picked by timing the candidates on
 * the device the first time the shape is seen.  Each problem computes
 * exactly what tsvd_complete / trpca compute for it (same kernels, same
 * order of operations; the Jacobi block width may differ, which changes
 * results only by rounding).
 *
 * Device memory: the state of a running problem (iterates, Fourier slices,
 * V, Gram scratch, residual partials) lives in one arena per handle, sized
 * by the handle's hbm_budget_bytes (0: 90% of the device memory free when
 * the arena is first needed).  A problem is admitted only while its state
 * fits in the free part of the arena; the others wait in arrival order. */

typedef enum { TSVD_KIND_COMPLETE = 0, TSVD_KIND_TRPCA = 1 } tsvd_kind;

/* One problem: the arguments of tsvd_complete or trpca in one record.
 * All tensor pointers are device pointers owned by the caller; inputs are
 * read and outputs written while the problem runs (for tsvd_submit: until
 * tsvd_poll has reported it finished). */
typedef struct {
    int32_t kind;          /* tsvd_kind                                         */
    int32_t dtype;         /* tsvd_dtype                                        */
    int32_t precision;     /* tsvd_precision, paired with dtype as for tsvt     */
    int32_t shrink;        /* RPCA: tsvd_shrink                                 */
    tsvd_shape shape;
    const void* x;         /* completion: X_obs; RPCA: the data M               */
    const uint8_t* mask;   /* completion: observation mask; RPCA: unused        */
    double penalty;        /* initial rho (completion) or mu (RPCA), > 0        */
    double lambda;         /* RPCA weight, > 0                                  */
    double tol;            /* >= 0; 0 runs opts.max_iter iterations             */
    tsvd_admm_opts opts;   /* growth, rho_max, max_iter, max_sweeps; its
                              precision field is ignored                        */
    void* out;             /* completion: X_out; RPCA: L_out                    */
    void* out_s;           /* RPCA: S_out                                       */
    double deadline_s;     /* serving: seconds after tsvd_submit after which an
                              unfinished request stops with TSVD_E_TIMEOUT and
                              leaves its outputs unspecified (0: none); the
                              worker checks it between iterations.  Ignored
                              by tsvd_batch_run.  >= 0                          */
} tsvd_problem;

/* Solve `count` problems together and return when all have stopped.
 * infos_host: NULL or `count` host tsvd_info records (seconds = time from
 * the call to the problem's completion).  status_host: NULL or `count` host
 * int32 per-problem statuses (TSVD_OK, TSVD_E_NONFINITE, ...).  Problems of
 * FP32 and FP64 data may be mixed; each dtype runs as its own batch.
 * Errors: TSVD_E_INVALID / TSVD_E_SHAPE / TSVD_E_UNSUPPORTED for a bad record
 * (nothing runs), TSVD_E_NOMEM if one problem alone does not fit the arena,
 * TSVD_E_HIP; a problem that meets a non-finite value stops with
 * TSVD_E_NONFINITE in status_host and does not fail the call. */
tsvd_status tsvd_batch_run(tsvd_handle h, const tsvd_problem* probs, int32_t count, tsvd_info* infos_host,
                           int32_t* status_host);

/* Serving: queue one problem and return at once with its ticket.  A
 * worker thread of the handle admits queued problems as arena space frees
 * up (continuous batching: problems join and leave the running batch
 * between iterations), runs them on a stream of its own, and writes each
 * problem's outputs when it stops.  The record is copied; the tensors it
 * points to must stay valid until tsvd_poll reports the ticket finished.
 * Errors: as tsvd_batch_run for a bad record; TSVD_E_NOMEM if the problem
 * can never fit the arena. */
tsvd_status tsvd_submit(tsvd_handle h, const tsvd_problem* prob, uint64_t* ticket_host);

/* TSVD_E_BUSY while the ticket is queued or running; otherwise the
 * problem's final status (TSVD_OK, TSVD_E_NONFINITE, TSVD_E_CANCELLED,
 * TSVD_E_TIMEOUT, ...), with *info_host filled (seconds = time from
 * submission to completion) when not NULL.  A finished ticket can be polled
 * again; an unknown ticket is TSVD_E_INVALID.  After a device failure ends
 * the serving worker, every ticket it had not finished (queued or running)
 * reports the failure's status (e.g. TSVD_E_HIP). */
tsvd_status tsvd_poll(tsvd_handle h, uint64_t ticket, tsvd_info* info_host);

/* Cancel a queued or running request.  Its status becomes TSVD_E_CANCELLED
 * (a request that has already finished keeps its status); a running request
 * leaves the batch at the worker's next period boundary, and its outputs are
 * unspecified.  The caller must keep the request's tensors alive until
 * tsvd_poll reports it finished.  Errors: TSVD_E_INVALID for an unknown
 * ticket. */
tsvd_status tsvd_cancel(tsvd_handle h, uint64_t ticket);

/* Serving counters (host struct). */
typedef struct {
    int64_t submitted;     /* tickets issued                                   */
    int64_t finished;      /* tickets finished                                 */
    int64_t queued;        /* waiting for arena space                          */
    int64_t running;       /* in the running batch                             */
    int64_t iterations;    /* batched ADMM iterations run by the worker        */
    int64_t arena_bytes;   /* arena size                                       */
    int64_t arena_used;    /* bytes held by running problems                   */
    int64_t peak_running;  /* largest running batch                            */
} tsvd_serve_stats;

tsvd_status tsvd_serve_stats_read(tsvd_handle h, tsvd_serve_stats* out_host);

/* Static string for a status code. */
const char* tsvd_status_string(tsvd_status s);

/* Message of the calling thread's last failed call ("" if none). */
const char* tsvd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TSVD_H */
