// One-sided (Hestenes) complex Jacobi SVD of every Fourier frontal slice.
//
// The Z-update of the completion ADMM (Sec. 4) splits into one matrix
// problem per Fourier slice (Sec. 4.1, eq. shrink2), each solved by the
// singular value shrinkage lemma of Sec. 4.1, which needs an SVD of the
// slice.  Here every m x n slice (m >= n) is orthogonalised column-wise:
// plane rotations J are applied on the right, A <- A J and V <- V J (V
// starts at the identity), until every column pair satisfies
// |a_p^H a_q| <= tol ||a_p|| ||a_q||.  Then A = W with orthogonal columns,
// sigma_j = ||w_j||, and the slice equals W V^H.
//
// Rotation of a pair (alpha = ||a_p||^2, beta = ||a_q||^2,
// gamma = a_p^H a_q = |gamma| e):
//   zeta = (beta - alpha) / (2 |gamma|),
//   t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1 + t^2), s = c t,
//   a_p <- c a_p - s conj(e) a_q,   a_q <- s e a_p + c a_q,
// which makes the new pair orthogonal.
//
// Parallel ordering (block round-robin).  The n columns are cut into nb
// blocks of at most BW columns.  One sweep visits every column pair once:
//   * jacobi_self: every block orthogonalises its own columns (round-robin
//     over the block, BW/2 pairs at a time), one workgroup per block;
//   * jacobi_cross, rounds 0..nb-2 of a round-robin tournament over the
//     blocks: every workgroup takes one block pair (I, J) and visits the
//     BW x BW cross pairs in BW steps.  Group g of the workgroup keeps
//     column g of I in registers; the J block sits in LDS and column
//     (g + step) mod BW is the partner at each step.
// A column's V entries ride along as extra rows (rows m..m+n-1 of the
// stacked column), so they are rotated with the same coefficients and are
// excluded from the dot products.
//
// Convergence is tracked per slice: sweep k sets rot[k % 3][s] when any
// pair of slice s was rotated; a slice whose previous sweep rotated nothing
// is skipped.  Sweep k also clears ring entry (k+1) % 3, which nobody reads
// or writes during sweep k.

#include "kernels.h"

#include <algorithm>

namespace tsvd {

namespace {

__device__ __forceinline__ int blk_start(int b, int n, int nb) {
    return (int)(((int64_t)b * n) / nb);
}

// round-robin (circle method) partner lists: player at position pos in round r
__device__ __forceinline__ int rr_player(int pos, int r, int nplayers) {
    return pos == 0 ? 0 : 1 + (pos - 1 + r) % (nplayers - 1);
}

template <int TPG, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = TPG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
struct Rot {
    T c, s, er, ei;
};

// Rotation parameters from the reduced pair sums; false when the pair is
// already orthogonal to tolerance (or a column is zero).
template <typename T>
__device__ __forceinline__ bool make_rotation(T al, T be, T gr, T gi, T tol, Rot<T>& r) {
    const T g = sqrt(gr * gr + gi * gi);
    if (!(g > tol * sqrt(al) * sqrt(be))) return false;
    const T zeta = (be - al) / (g + g);
    const T t = (zeta >= (T)0 ? (T)1 : (T)-1) / (fabs(zeta) + sqrt((T)1 + zeta * zeta));
    r.c = (T)1 / sqrt((T)1 + t * t);
    r.s = r.c * t;
    r.er = gr / g;
    r.ei = gi / g;
    return true;
}

// (x, y) <- (c x - s conj(e) y, s e x + c y)
template <typename T>
__device__ __forceinline__ void apply_rotation(const Rot<T>& r, cplx<T>& x, cplx<T>& y) {
    const T ycr = r.er * y.re + r.ei * y.im;   // conj(e) y
    const T yci = r.er * y.im - r.ei * y.re;
    const T exr = r.er * x.re - r.ei * x.im;   // e x
    const T exi = r.er * x.im + r.ei * x.re;
    const cplx<T> xn{r.c * x.re - r.s * ycr, r.c * x.im - r.s * yci};
    const cplx<T> yn{r.s * exr + r.c * y.re, r.s * exi + r.c * y.im};
    x = xn;
    y = yn;
}

template <typename T>
__device__ __forceinline__ void accum_pair(const cplx<T>& x, const cplx<T>& y, T& al, T& be, T& gr,
                                           T& gi) {
    al += x.re * x.re + x.im * x.im;
    be += y.re * y.re + y.im * y.im;
    gr += x.re * y.re + x.im * y.im;   // Re(conj(x) y)
    gi += x.re * y.im - x.im * y.re;   // Im(conj(x) y)
}

template <typename T>
__device__ __forceinline__ cplx<T> load_stacked(const JacArgs<T>& a, int s, int col, int r) {
    if (r < a.m) return a.A[((int64_t)s * a.n + col) * a.m + r];
    return a.V[((int64_t)s * a.n + col) * a.n + (r - a.m)];
}

template <typename T>
__device__ __forceinline__ void store_stacked(const JacArgs<T>& a, int s, int col, int r, cplx<T> v) {
    if (r < a.m)
        a.A[((int64_t)s * a.n + col) * a.m + r] = v;
    else
        a.V[((int64_t)s * a.n + col) * a.n + (r - a.m)] = v;
}

// true when slice s converged in an earlier sweep
template <typename T>
__device__ __forceinline__ bool slice_done(const JacArgs<T>& a, int s) {
    return a.sweep > 0 && a.rot[((a.sweep - 1) % 3) * a.h + s] == 0;
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(kBlock) void jacobi_init_kernel(JacArgs<T> a) {
    const int s = blockIdx.y;
    const int64_t nn = (int64_t)a.n * a.n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nn;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = idx / a.n, r = idx - c * a.n;
        a.V[(int64_t)s * nn + idx] = cplx<T>{r == c ? (T)1 : (T)0, (T)0};
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.rot[s] = 0;   // ring entry 0 is written by sweep 0
        a.sweeps[s] = 0;
    }
}

template <typename T, int BW>
__global__ __launch_bounds__(kBlock) void jacobi_self_kernel(JacArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem);
    const int s = blockIdx.y, b = blockIdx.x;
    if (slice_done(a, s)) return;
    if (b == 0 && threadIdx.x == 0) {
        a.rot[((a.sweep + 1) % 3) * a.h + s] = 0;
        a.sweeps[s] += 1;
    }
    const int c0 = blk_start(b, a.n, a.nb);
    const int w = blk_start(b + 1, a.n, a.nb) - c0;
    if (w < 2) return;
    const int rows = a.m + a.n;
    for (int idx = threadIdx.x; idx < w * rows; idx += blockDim.x) {
        const int c = idx / rows, r = idx - c * rows;
        lds[c * rows + r] = load_stacked(a, s, c0 + c, r);
    }
    __syncthreads();

    // threads per pair; a pair's lanes stay inside one wavefront
    constexpr int TPP = (kBlock / (BW / 2)) > 64 ? 64 : (kBlock / (BW / 2));
    const int grp = threadIdx.x / TPP, lane = threadIdx.x - grp * TPP;
    const int wp = w + (w & 1);
    bool any = false;
    unsigned nrot = 0;
    for (int st = 0; st < wp - 1; ++st) {
        if (grp < wp / 2 && grp < kBlock / TPP) {
            const int p = rr_player(grp, st, wp);
            const int q = rr_player(wp - 1 - grp, st, wp);
            if (p < w && q < w) {
                cplx<T>* cp = lds + p * rows;
                cplx<T>* cq = lds + q * rows;
                T al = 0, be = 0, gr = 0, gi = 0;
                for (int r = lane; r < a.m; r += TPP) accum_pair(cp[r], cq[r], al, be, gr, gi);
                al = group_sum<TPP>(al);
                be = group_sum<TPP>(be);
                gr = group_sum<TPP>(gr);
                gi = group_sum<TPP>(gi);
                Rot<T> rt;
                if (make_rotation(al, be, gr, gi, a.tol, rt)) {
                    any = true;
                    nrot += lane == 0;
                    for (int r = lane; r < rows; r += TPP) {
                        cplx<T> x = cp[r], y = cq[r];
                        apply_rotation(rt, x, y);
                        cp[r] = x;
                        cq[r] = y;
                    }
                }
            }
        }
        __syncthreads();
    }
    if (any) a.rot[(a.sweep % 3) * a.h + s] = 1;
    if (nrot) atomicAdd(a.rotations, (unsigned long long)nrot);
    for (int idx = threadIdx.x; idx < w * rows; idx += blockDim.x) {
        const int c = idx / rows, r = idx - c * rows;
        store_stacked(a, s, c0 + c, r, lds[c * rows + r]);
    }
}

template <typename T, int BW, int RPT>
__global__ __launch_bounds__(kBlock) void jacobi_cross_kernel(JacArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem);
    const int s = blockIdx.y, pr = blockIdx.x;
    if (slice_done(a, s)) return;
    const int bi = rr_player(pr, a.round, a.nb);
    const int bj = rr_player(a.nb - 1 - pr, a.round, a.nb);
    const int ci0 = blk_start(bi, a.n, a.nb), wi = blk_start(bi + 1, a.n, a.nb) - ci0;
    const int cj0 = blk_start(bj, a.n, a.nb), wj = blk_start(bj + 1, a.n, a.nb) - cj0;
    if (wi == 0 || wj == 0) return;
    const int rows = a.m + a.n;

    constexpr int TPG = kBlock / BW;   // threads per I column
    const int g = threadIdx.x / TPG, lane = threadIdx.x - g * TPG;
    for (int idx = threadIdx.x; idx < wj * rows; idx += blockDim.x) {
        const int c = idx / rows, r = idx - c * rows;
        lds[c * rows + r] = load_stacked(a, s, cj0 + c, r);
    }
    cplx<T> xi[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int r = lane + k * TPG;
        xi[k] = (g < wi && r < rows) ? load_stacked(a, s, ci0 + g, r) : cplx<T>{(T)0, (T)0};
    }
    __syncthreads();

    bool any = false;
    unsigned nrot = 0;
    for (int st = 0; st < BW; ++st) {
        const int jc = (g + st) % BW;
        if (g < wi && jc < wj) {
            cplx<T>* cq = lds + jc * rows;
            cplx<T> yq[RPT];
            T al = 0, be = 0, gr = 0, gi = 0;
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const int r = lane + k * TPG;
                yq[k] = r < rows ? cq[r] : cplx<T>{(T)0, (T)0};
                if (r < a.m) accum_pair(xi[k], yq[k], al, be, gr, gi);
            }
            al = group_sum<TPG>(al);
            be = group_sum<TPG>(be);
            gr = group_sum<TPG>(gr);
            gi = group_sum<TPG>(gi);
            Rot<T> rt;
            if (make_rotation(al, be, gr, gi, a.tol, rt)) {
                any = true;
                nrot += lane == 0;
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const int r = lane + k * TPG;
                    apply_rotation(rt, xi[k], yq[k]);
                    if (r < rows) cq[r] = yq[k];
                }
            }
        }
        __syncthreads();
    }
    if (any) a.rot[(a.sweep % 3) * a.h + s] = 1;
    if (nrot) atomicAdd(a.rotations, (unsigned long long)nrot);
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int r = lane + k * TPG;
        if (g < wi && r < rows) store_stacked(a, s, ci0 + g, r, xi[k]);
    }
    for (int idx = threadIdx.x; idx < wj * rows; idx += blockDim.x) {
        const int c = idx / rows, r = idx - c * rows;
        store_stacked(a, s, cj0 + c, r, lds[c * rows + r]);
    }
}

// ------------------------------------------------------------------ host

namespace {

constexpr int kRptSizes[] = {2, 4, 6, 8, 10, 12, 14, 16, 18, 20, 24, 28, 32, 40};
constexpr size_t kLdsCap = 64 * 1024;

int pick_rpt(int rows, int bw) {
    const int tpg = kBlock / bw;
    const int need = (rows + tpg - 1) / tpg;
    for (int r : kRptSizes)
        if (r >= need) return r;
    return -1;
}

}  // namespace

int jacobi_block_width(int m, int n, int elem_bytes, int h) {
    // Largest block width whose cross phase still gives about one workgroup
    // per CU; smaller blocks mean more launches per sweep.
    const int rows = m + n;
    int fallback = -1;
    for (int bw : {16, 8, 4}) {
        if ((size_t)bw * rows * 2 * elem_bytes > kLdsCap) continue;
        const int rpt = pick_rpt(rows, bw);
        if (rpt < 0) continue;
        fallback = bw;
        const int nb = std::max(2, 2 * ((n + 2 * bw - 1) / (2 * bw)));
        if ((int64_t)(nb / 2) * h >= 240 && rpt <= 24) return bw;
    }
    return fallback;
}

bool jacobi_supported(int m, int n, int elem_bytes) { return jacobi_block_width(m, n, elem_bytes, 1) > 0; }

template <typename T>
void launch_jacobi_init(const JacArgs<T>& a, hipStream_t st) {
    const int64_t nn = (int64_t)a.n * a.n;
    const int gx = (int)std::min<int64_t>((nn + kBlock - 1) / kBlock, 64);
    hipLaunchKernelGGL((jacobi_init_kernel<T>), dim3(gx, a.h), dim3(kBlock), 0, st, a);
}

template <typename T, int BW, int RPT>
static void launch_cross(const JacArgs<T>& a, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL((jacobi_cross_kernel<T, BW, RPT>), dim3(a.nb / 2, a.h), dim3(kBlock), lds, st, a);
}

template <typename T, int BW>
static void dispatch_cross(const JacArgs<T>& a, int rpt, size_t lds, hipStream_t st) {
    switch (rpt) {
        case 2: launch_cross<T, BW, 2>(a, lds, st); break;
        case 4: launch_cross<T, BW, 4>(a, lds, st); break;
        case 6: launch_cross<T, BW, 6>(a, lds, st); break;
        case 8: launch_cross<T, BW, 8>(a, lds, st); break;
        case 10: launch_cross<T, BW, 10>(a, lds, st); break;
        case 12: launch_cross<T, BW, 12>(a, lds, st); break;
        case 14: launch_cross<T, BW, 14>(a, lds, st); break;
        case 16: launch_cross<T, BW, 16>(a, lds, st); break;
        case 18: launch_cross<T, BW, 18>(a, lds, st); break;
        case 20: launch_cross<T, BW, 20>(a, lds, st); break;
        case 24: launch_cross<T, BW, 24>(a, lds, st); break;
        case 28: launch_cross<T, BW, 28>(a, lds, st); break;
        case 32: launch_cross<T, BW, 32>(a, lds, st); break;
        default: launch_cross<T, BW, 40>(a, lds, st); break;
    }
}

template <typename T>
void launch_jacobi_self(const JacArgs<T>& a, int bw, hipStream_t st) {
    const size_t lds = (size_t)bw * (a.m + a.n) * sizeof(cplx<T>);
    switch (bw) {
        case 16: hipLaunchKernelGGL((jacobi_self_kernel<T, 16>), dim3(a.nb, a.h), dim3(kBlock), lds, st, a); break;
        case 8: hipLaunchKernelGGL((jacobi_self_kernel<T, 8>), dim3(a.nb, a.h), dim3(kBlock), lds, st, a); break;
        default: hipLaunchKernelGGL((jacobi_self_kernel<T, 4>), dim3(a.nb, a.h), dim3(kBlock), lds, st, a); break;
    }
}

// One cross round (a.round) of the block tournament.
template <typename T>
void launch_jacobi_cross(const JacArgs<T>& a, int bw, hipStream_t st) {
    const int rows = a.m + a.n;
    const size_t lds = (size_t)bw * rows * sizeof(cplx<T>);
    const int rpt = pick_rpt(rows, bw);
    switch (bw) {
        case 16: dispatch_cross<T, 16>(a, rpt, lds, st); break;
        case 8: dispatch_cross<T, 8>(a, rpt, lds, st); break;
        default: dispatch_cross<T, 4>(a, rpt, lds, st); break;
    }
}

template void launch_jacobi_init<double>(const JacArgs<double>&, hipStream_t);
template void launch_jacobi_self<double>(const JacArgs<double>&, int, hipStream_t);
template void launch_jacobi_cross<double>(const JacArgs<double>&, int, hipStream_t);

}  // namespace tsvd
