// Kernel argument blocks and launchers of the gfx950 t-SVT library (internal).
#pragma once

#include "common.h"

#include <utility>

namespace tsvd {

// Problem-table launches: workgroup b serves problem p when
// wg_start[p] <= b < wg_start[p + 1] (nprob + 1 ascending entries).
__device__ __forceinline__ int batch_find(const int* wg_start, int nprob, int b) {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (wg_start[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Fused prologues of the forward DFT: what tensor is transformed.
enum Prologue : int {
    PRO_COPY = 0,      // A = X                                   (t-SVT)
    PRO_COMPLETE = 1,  // A = X + Q, X = Omega.Y + (1-Omega).(Z - Q) (completion)
    PRO_RPCA = 2,      // A = M - S - W                           (RPCA)
};

// Fused epilogues of the inverse DFT: what is done with the prox output.
enum Epilogue : int {
    EPI_STORE = 0,       // Z = prox output
    EPI_COMPLETE = 1,    // completion dual update + residual partial sums
    EPI_RPCA_L1 = 2,     // RPCA entrywise shrink + dual update + residuals
    EPI_RPCA_L112 = 3,   // RPCA tube-group shrink + dual update + residuals
};

// Dimensions of the DFT matrices of one tube shape (dft.hip).  Forward:
// F (Lk x 2hp, k-major): F[t][s] = Re w(s, t) and F[t][hp + s] = Im w(s, t)
// with w(s, t) = exp(-2 pi i u(s, t) / L), u(s, t) = (t3 k3 Q + t4 k4 P)
// mod L for slice s = k3 Qh + k4 and position t = t3 Q + t4; zero outside
// s < h, t < L.  Inverse: S (Kr x Lr, k-major): S[2s + c][t] = (c_s / L)
// (c ? Im : Re) w(s, t), c_s = 1 for the bins k4 = 0 and 2 k4 = Q, else 2;
// zero outside 2s + c < 2h, t < L.  Every dimension is a multiple of 16.
struct DftDims {
    int hp, Lk, Lr, Kr;
    __host__ __device__ static DftDims of(int h, int L) {
        DftDims d;
        d.hp = (h + 15) / 16 * 16;
        d.Lk = (L + 15) / 16 * 16;
        d.Lr = d.Lk;
        d.Kr = (2 * h + 15) / 16 * 16;
        return d;
    }
    __host__ __device__ int64_t fwd_size() const { return (int64_t)Lk * 2 * hp; }
    __host__ __device__ int64_t inv_size() const { return (int64_t)Kr * Lr; }
    __host__ __device__ int64_t total() const { return fwd_size() + inv_size(); }
};

template <typename T>
struct FwdArgs {
    const T* x;              // COPY: X; COMPLETE: observed Y; RPCA: M
    const uint8_t* mask;     // COMPLETE: 1 = observed
    const T* z;              // COMPLETE: Z_k
    const T* dual;           // COMPLETE: Q stored; RPCA: W stored (times ctrl->dscale)
    const T* s;              // RPCA: S_k
    const Ctrl* ctrl;
    const T* mat;            // forward DFT matrix F (DftDims), element type
    cplx<T>* out;            // h slices, m x n column-major each
    int* nonfinite;          // set to 1 if a transformed value is not finite
    Geometry g;
    int tile;                // tubes per workgroup
    int pro;                 // prologue (problem-table launches)
};

template <typename T>
struct InvArgs {
    const cplx<T>* in;       // h slices of the prox output
    const T* mat;            // inverse DFT matrix S (DftDims), element type
    const Ctrl* ctrl;
    Geometry g;
    int tile;
    T* out;                  // Z (STORE/COMPLETE) or L (RPCA), next iterate
    // completion
    const T* y;
    const uint8_t* mask;
    const T* z_old;
    const T* dual_old;       // stored dual of the current iteration
    T* dual_new;             // stored dual of the next iteration (unscaled)
    // RPCA
    const T* m;
    const T* s_old;
    T* s_new;
    const T* l_old;
    double* partials;        // kNumPartials per workgroup
    int epi;                 // epilogue (problem-table launches)
};

// Stopping rule of every Jacobi variant.  A pair (alpha = ||x||^2,
// beta = ||y||^2, gamma = x^H y) is rotated when |gamma|^2 > tol^2 alpha beta.
// A slice runs another sweep only if some rotation of the sweep had
// |gamma|^2 > kSweepMargin tol alpha beta, i.e. a relative off-diagonal
// above sqrt(kSweepMargin tol).  Cyclic Jacobi converges quadratically: after
// a sweep whose rotations all stayed below sqrt(tol), the off-diagonals the
// next sweep would meet are of order tol, the level the rotation test itself
// leaves standing, so that sweep is not run.  (Smaller rotations of the
// sweep are still applied.)  Margins 0.01 / 0.1 / 1 gave 4.75 / 4.34 / 4.13
// sweeps per iteration on the video-shaped FP32 form at the same accuracy.
constexpr double kSweepMargin = 1.0;
//
// Rounding floor.  floor2 = m eps^2 ||A||_F^2 (eps of the element type,
// ||A||_F of the slice, which the rotations leave unchanged) is the squared
// rounding level of length-m inner products of the slice's entries: already
// the product A V of the warm start moves every column by about
// eps ||A||_F.  Leaving the coupling gamma of two columns unresolved moves
// the thresholded result by about |gamma| / max(||x||, ||y||) in norm (the
// rotation angle times the larger column), so a rotation with
// |gamma|^2 <= floor2 max(alpha, beta) does not force another sweep (it is
// still applied): what it leaves is at the slice's own rounding level.  By
// Cauchy-Schwarz this covers every pair with a column under the floor, whose
// direction is set by rounding.  floor2 = 0 keeps the plain rule.
__device__ __forceinline__ bool rot_forces_sweep(double al, double be, double g2, double tol,
                                                 double floor2 = 0.0) {
    return g2 > (kSweepMargin * tol) * al * be && g2 > floor2 * fmax(al, be);
}

template <typename T>
struct JacArgs {
    cplx<T>* A;     // h slices m x n; overwritten by W = A V
    cplx<T>* V;     // h slices n x n
    int m, n, h;
    int nb;         // column blocks (even)
    int round;      // tournament round of jacobi_cross
    int sweep;      // sweep index; rot is a ring of 3 x h flags
    int* rot;       // rot[(sweep % 3) * h + s] = 1 if sweep rotated slice s
    int* sweeps;    // sweeps run per slice
    unsigned long long* rotations;  // running count of applied rotations
    T tol;          // rotate when |a_p^H a_q| > tol ||a_p|| ||a_q||
    int reset_v;    // jacobi_init: 1 = start from V = I, 0 = keep V (warm start)
    // optional ADMM control block: jacobi_init and the persistent kernel do
    // nothing once ctrl->done is set, and the persistent kernel raises
    // ctrl->sweep_max to each slice's sweep count
    Ctrl* ctrl;
    int* clr[2];    // jacobi_init: optional int ranges zeroed before the sweeps
    int nclr[2];
};

// C[s] = alpha * op(A[s]) * diag(d[s]) * op(B[s]) + beta * D[s] over `batch`
// slices, column-major complex, on the matrix cores (zgemm.hip).
// op = 0: as stored; op = 1: conjugate transpose (A stored K x M, B N x K).
// dk: optional per-slice factors d_k (K per slice, stride sdk); else d = 1.
template <typename T>
struct ZGemmArgs {
    const cplx<T>* A;
    const cplx<T>* B;
    const cplx<T>* D;   // may be null (beta ignored)
    cplx<T>* C;         // must not alias A, B or D's other tiles
    int64_t sA, sB, sD, sC;
    int lda, ldb, ldd, ldc;
    int M, N, K, batch;
    int opA, opB;
    T alpha, beta;
    const double* dk;      // optional column factors, K per slice, stride sdk
    int64_t sdk;
    const Ctrl* ctrl;      // optional: the product is skipped once ctrl->done
    int bf16x3;            // float only: 1 = bf16 split products, 0 = FP32 products
    int herm;              // C = A^H A (B == A, opA = H, opB = N, no D): the split-K
                           // form computes the tiles on and above the diagonal and
                           // mirrors them; other forms compute every tile
    int kcompact;          // with dk: the split-K form sums only over the k with
                           // dk[k] > 0 (the kept columns of a thresholded rebuild;
                           // the others contribute exact zeros), K <= kMaxCompactK
};
constexpr int kMaxCompactK = 1024;

template <typename T>
void launch_zgemm(const ZGemmArgs<T>& g, hipStream_t st);
int zgemm_workgroups(int M, int N, int batch);
template <typename T>
void launch_zgemm_batched(const ZGemmArgs<T>* tab, const int* wg_start, int nprob, int nwg, hipStream_t st);
// t-SVD factors and compression (factors.hip)
template <typename T>
void launch_tsvd_mirror(cplx<T>* W, cplx<T>* V, double* sigma, const Geometry& g, hipStream_t st);
void launch_tsvd_rank(const double* sigma, int n, int h, int* rank, hipStream_t st);
template <typename T>
void launch_tsvd_factors(const cplx<T>* W, const cplx<T>* V, const double* sigma, const int* rank, const Geometry& g,
                         cplx<T>* Uh, cplx<T>* Vh, cplx<T>* Sh, hipStream_t st);
void launch_tubal_select(const int* rank, int64_t count, int k3, double* dk, hipStream_t st);
void launch_global_select(const double* sigma, const Geometry& g, int64_t k2, double* dk, hipStream_t st);

void launch_multirank(const double* sigma, int64_t ssig, int K, int h, const Ctrl* ctrl, int* rank,
                      hipStream_t st);
// One problem of a one-workgroup-per-slice Jacobi launch (jacobi_slice.hip).
template <typename T>
struct JacSliceArgs {
    cplx<T>* A;          // h slices m x n, overwritten by W = A V
    cplx<T>* V;          // h slices n x n (rotated in place; start value is the caller's)
    int m, n, h, nb;     // nb: column blocks of width <= the launch's block width (even)
    T tol;
    int* sweeps;         // optional: sweeps run per slice
    Ctrl* ctrl;          // optional: skip the problem once ctrl->done; sweep_max is raised
    unsigned long long* rotations;  // optional running count
    int max_sweeps;      // sweep cap (0: the launch's)
    int* rot;            // round mode: 3 x h ring of per-sweep rotation flags (ring 0 clear before the SVD)
    const int* only_if;  // optional: the problem is skipped unless *only_if != 0
    int* bar;            // pairs-parallel schedule: h barrier counters, then h x nb block-ready
                         // flags, all zero before the launch (as is ring 0 of rot)
    double floor_scale;  // the rounding floor of rot_forces_sweep is floor_scale ||A||_F^2 (0: none)
    double* fro;         // pairs-parallel schedule with a floor: h x (nb / 2) doubles, the
                         // parts of the slices' squared Frobenius norms
};
// Doubles per problem of the pairs-parallel schedule's Frobenius parts (JacSliceArgs::fro).
inline int64_t jacobi_pairs_fro(int h, int n) { return (int64_t)h * (n / 2 + 1); }
// Ints per problem of the pairs-parallel schedule's barrier area (JacSliceArgs::bar).
inline int64_t jacobi_pairs_words(int h, int nb) { return (int64_t)h * (1 + nb); }
int jacobi_slice_rpt(int m, int n);
size_t jacobi_slice_lds(int bw, int rpt, int elem_bytes);
int jacobi_slice_max_rpt();
// Sets the kernel's LDS limit; call once per (bw, rpt) before launches
// (and before any stream capture).
template <typename T>
hipError_t prepare_jacobi_slice(int bw, int rpt);
template <typename T>
hipError_t launch_jacobi_slice(int bw, int rpt, const JacSliceArgs<T>* tab, const int* wg_start, int nprob,
                               int nwg, int max_sweeps, hipStream_t st);
// Pairs-parallel schedule over a problem table: one launch runs every sweep
// of every slice, nb / 2 workgroups per slice (one per block pair of a round)
// exchanging blocks between rounds; workgroups take their roles in order from
// words[0] (zero before the launch), and a wait between workgroups that gives
// up sets words[1] (the SVDs of that launch are then incomplete).
// role_start: nprob + 1 cumulative role counts (h nb / 2 per problem).
template <typename T>
hipError_t launch_jacobi_pairs(int bw, int rpt, const JacSliceArgs<T>* tab, const int* role_start, int nprob,
                               int nroles, int* words, int spin_limit, hipStream_t st);

template <typename T>
struct SigmaArgs {
    const cplx<T>* W;
    int m, n, h;
    double* sigma;
    double* dk;         // shrink factors (1 - tau/sigma)_+, tau = ctrl->tau
    const Ctrl* ctrl;   // tau; skip the problem once done
};
int svt_sigma_workgroups(int n, int h);
template <typename T>
void launch_svt_sigma_batched(const SigmaArgs<T>* tab, const int* wg_start, int nprob, int nwg, hipStream_t st);

template <typename T>
void launch_svt_sigma(const cplx<T>* W, int m, int n, int h, double* sigma, double* dk, const Ctrl* ctrl,
                      hipStream_t st);

template <typename T>
void launch_dft_forward(int prologue, const FwdArgs<T>& a, hipStream_t st);
template <typename T>
void launch_dft_inverse(int epilogue, const InvArgs<T>& a, hipStream_t st);
template <typename T>
size_t dft_forward_lds(const Geometry& g, int tile);
template <typename T>
size_t dft_inverse_lds(const Geometry& g, int tile, int epilogue);
// Raises the LDS limit of the problem-table DFT kernels when needed
// (call outside stream capture).
template <typename T>
void prepare_dft_batched(size_t lds_forward, size_t lds_inverse);
template <typename T>
void launch_dft_forward_batched(const FwdArgs<T>* tab, const int* wg_start, int nprob, int nwg, size_t lds,
                                hipStream_t st);
template <typename T>
void launch_dft_inverse_batched(const InvArgs<T>* tab, const int* wg_start, int nprob, int nwg, size_t lds,
                                hipStream_t st);
// The forward and inverse DFT matrices of g's tube shape, built on the device
// (DftDims::of(g.h, g.L).total() elements).
template <typename T>
void launch_dft_matrices(T* out, const Geometry& g, hipStream_t st);
int dft_forward_tile(const Geometry& g);
int dft_inverse_tile(const Geometry& g, int epilogue);
int64_t dft_grid(const Geometry& g, int tile);

template <typename T>
void launch_jacobi_init(const JacArgs<T>& a, hipStream_t st);
template <typename T>
void launch_jacobi_self(const JacArgs<T>& a, int bw, hipStream_t st);
template <typename T>
void launch_jacobi_cross(const JacArgs<T>& a, int bw, hipStream_t st);
int jacobi_block_width(int m, int n, int elem_bytes, int h);
inline int jacobi_num_blocks(int n, int bw) { int nb = 2 * ((n + 2 * bw - 1) / (2 * bw)); return nb < 2 ? 2 : nb; }
bool jacobi_supported(int m, int n, int elem_bytes);
// Slices whose stacked columns fit no LDS kernel: columns in global memory,
// one column pair per round-robin slot, rows split into chunks (jacobi.hip).
constexpr int kMaxTallCols = 1024;
bool jacobi_tall(int m, int n, int elem_bytes);
struct TallPlan {
    int players = 0, chunks = 0, rows_per = 0;
    int64_t part_doubles = 0;   // partial sums: 4 per (slice, pair, chunk)
};
TallPlan jacobi_tall_plan(int m, int n, int h);
template <typename T>
void launch_jacobi_tall_round(const JacArgs<T>& a, const TallPlan& t, double* part, hipStream_t st);
// LDS bytes one workgroup may use on the current device
void jacobi_set_lds_limit(size_t bytes);

// Persistent Jacobi (jacobi_persist.hip): one launch per SVD.
struct PersistArgs {
    int* pbar;        // int words, zero before the launch except the error word (zero
                      // before the first launch of a call): h barrier counters, 3 x h
                      // sweep flags, the error word (bit 1: a wait between workgroups
                      // gave up; bit 2: a wait inside one ran out), the role ticket,
                      // h x nb block-ready flags
    double* fro;      // h x (nb / 2) doubles: each workgroup's part of its slice's squared
                      // Frobenius norm (written at the start of the launch)
    double floor_scale;   // m eps^2 of the element type: the rounding floor of
                          // rot_forces_sweep is floor_scale ||A||_F^2 (0: plain rule)
    int max_sweeps;
    int spin_limit;   // polls of a wait between workgroups before it gives up
    int spread;       // 1: reserve over half a CU's LDS, so no two workgroups share a CU
};
int jacobi_persistent_blocks(int n);
bool jacobi_persistent_fits(int m, int n, int h, int elem_bytes, int cus, size_t lds_cap);
template <typename T>
hipError_t launch_jacobi_persistent(const JacArgs<T>& a, const PersistArgs& p, int cus, hipStream_t st);

struct CtrlArgs {
    Ctrl* c;
    const double* partials;
    int nparts, rpca;
    int* rot_ring0;    // optional: h flags cleared after the step (pairs-parallel Jacobi)
    int h;
    int* clr;          // optional: nclr ints cleared after the step (the Jacobi barrier area)
    int nclr;
};
void launch_admm_ctrl_batched(const CtrlArgs* tab, int nprob, hipStream_t st);
// mirror (optional): a copy of the control block after the update, e.g. in
// mapped pinned host memory; written also when the problem had already stopped
void launch_admm_ctrl(Ctrl* c, const double* partials, int nparts, int rpca, Ctrl* mirror, hipStream_t st);
template <typename T>
void launch_sumsq(const T* x, const uint8_t* mask, int64_t n, double* partials, int nparts,
                  hipStream_t st);
void launch_set_tol(Ctrl* c, const double* partials, int nparts, double tol, hipStream_t st);
template <typename T>
void launch_complete_output(const T* y, const uint8_t* mask, const T* z, const T* dual,
                            const Ctrl* c, T* out, int64_t n, hipStream_t st);
template <typename T>
void launch_fill(T* p, T v, int64_t n, hipStream_t st);
template <typename T>
void launch_fill_hash(cplx<T>* p, int64_t n, uint32_t seed, hipStream_t st);
template <typename T>
void launch_set_identity(cplx<T>* v, int n, int h, hipStream_t st);

}  // namespace tsvd
