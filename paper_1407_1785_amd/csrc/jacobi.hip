// One-sided (Hestenes) complex Jacobi SVD of every Fourier frontal slice.
//
// The Z-update of the completion ADMM (Sec. 4) splits into one matrix
// problem per Fourier slice (Sec. 4.1, eq. shrink2), each solved by the
// singular value shrinkage lemma of Sec. 4.1, which needs an SVD of the
// slice.  Here every m x n slice (m >= n) is orthogonalised column-wise:
// plane rotations J are applied on the right, A <- A J and V <- V J, until
// every column pair satisfies |a_p^H a_q| <= tol ||a_p|| ||a_q||.  Then
// A = W with orthogonal columns, sigma_j = ||w_j||, and the slice is W V^H.
// V starts at the identity (cold start) or at the previous ADMM iteration's
// V with A pre-rotated to A V (warm start, see gemm.hip).
//
// Rotation of a pair (alpha = ||a_p||^2, beta = ||a_q||^2,
// gamma = a_p^H a_q = |gamma| e):
//   zeta = (beta - alpha) / (2 |gamma|),
//   t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1 + t^2), s = c t,
//   a_p <- c a_p - s conj(e) a_q,   a_q <- s e a_p + c a_q,
// which makes the new pair orthogonal.  The rotation is unitary whatever
// the rounding of t, because c is computed from t (to full precision) and
// |e| = 1 (to full precision); t itself only has to be close.
//
// Parallel ordering (block round-robin).  The n columns are cut into nb
// blocks of at most BW columns.  One sweep visits every column pair once:
//   * jacobi_self: every block orthogonalises its own columns (round-robin
//     over the block), one workgroup per block;
//   * jacobi_cross, rounds 0..nb-2 of a round-robin tournament over the
//     blocks: every workgroup takes one block pair (I, J) and visits the
//     BW x BW cross pairs in BW steps.  Wavefront g keeps column g of I in
//     registers; the J block sits in LDS and column (g + step) mod BW is its
//     partner at each step.
// One column pair = one wavefront: each lane holds rows lane + 64 k of the
// stacked column (the m slice rows, then the n rows of V, which are rotated
// with the same coefficients but excluded from the dot products).  The
// three dot products are reduced across the wavefront with DPP row
// operations and readlane, so the rotation parameters are wave-uniform.
//
// Convergence is tracked per slice: sweep k sets rot[k % 3][s] when a
// rotation of slice s forces another sweep (rot_forces_sweep); a slice whose
// previous sweep set nothing is skipped.  Sweep k also clears ring entry (k+1) % 3 of every slice,
// skipped or not, which nobody reads or writes during sweep k.
//
// Work model (floating-point operations): a visited pair costs 16 m for the
// three dot products; an applied rotation another 16 (m + n).

#include "kernels.h"

#include <algorithm>

namespace tsvd {

namespace {

__device__ __forceinline__ int blk_start(int b, int n, int nb) {
    return (int)(((int64_t)b * n) / nb);
}

// round-robin (circle method): player at position pos in round r
__device__ __forceinline__ int rr_player(int pos, int r, int nplayers) {
    return pos == 0 ? 0 : 1 + (pos - 1 + r) % (nplayers - 1);
}

// ---- wave-wide FP64 sum: DPP within 16-lane rows, readlane across rows

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// every lane receives the same sum (rows summed in a fixed order)
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_f64<0x141>(v);   // row_half_mirror: the other quad of the half row
    v += dpp_f64<0x140>(v);   // row_mirror: the other half of the row
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// ---- rotation parameters (FP64, wave-uniform)

__device__ __forceinline__ double rsqrt_acc(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * (1.5 - 0.5 * x * y * y);
    y = y * (1.5 - 0.5 * x * y * y);
    return y;
}

__device__ __forceinline__ double rcp_close(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = y * (2.0 - x * y);
    return y;
}

struct Rot {
    double c, s, er, ei;
    bool big;   // the rotation forces another sweep
};

// False when the pair is already orthogonal to tolerance (or a column is 0).
__device__ __forceinline__ bool make_rotation(double al, double be, double gr, double gi, double tol,
                                              Rot& r) {
    const double g2 = gr * gr + gi * gi;
    if (!(g2 > (tol * tol) * al * be) || !(g2 > 0.0)) return false;
    r.big = rot_forces_sweep(al, be, g2, tol);
    const double rg = rsqrt_acc(g2);
    const double zeta = (be - al) * 0.5 * rg;
    const double az = fabs(zeta);
    const double q = 1.0 + zeta * zeta;
    const double t = rcp_close(az + q * rsqrt_acc(q));
    const double ts = zeta >= 0.0 ? t : -t;
    r.c = rsqrt_acc(1.0 + ts * ts);
    r.s = r.c * ts;
    r.er = gr * rg;
    r.ei = gi * rg;
    return true;
}

// (x, y) <- (c x - s conj(e) y, s e x + c y)
template <typename T>
__device__ __forceinline__ void apply_rotation(const Rot& rd, cplx<T>& x, cplx<T>& y) {
    const T c = (T)rd.c, s = (T)rd.s, er = (T)rd.er, ei = (T)rd.ei;
    const T ycr = er * y.re + ei * y.im;   // conj(e) y
    const T yci = er * y.im - ei * y.re;
    const T exr = er * x.re - ei * x.im;   // e x
    const T exi = er * x.im + ei * x.re;
    const cplx<T> xn{c * x.re - s * ycr, c * x.im - s * yci};
    const cplx<T> yn{s * exr + c * y.re, s * exi + c * y.im};
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

// pointer to row r of stacked column `col` of slice s (A rows, then V rows)
template <typename T>
__device__ __forceinline__ cplx<T>* stacked(const JacArgs<T>& a, int s, int col, int r) {
    return r < a.m ? a.A + ((int64_t)s * a.n + col) * a.m + r
                   : a.V + ((int64_t)s * a.n + col) * a.n + (r - a.m);
}

// Copy w stacked columns of slice s from global memory to LDS (column-major,
// `rows` per column), four independent loads in flight per thread.
template <typename T>
__device__ __forceinline__ void block_to_lds(const JacArgs<T>& a, int s, int c0, int w, int rows,
                                             cplx<T>* lds) {
    const int total = w * rows;
    for (int base = threadIdx.x; base < total; base += 4 * blockDim.x) {
        cplx<T> v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int idx = base + u * blockDim.x;
            if (idx < total) {
                const int c = idx / rows, r = idx - c * rows;
                v[u] = *stacked(a, s, c0 + c, r);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int idx = base + u * blockDim.x;
            if (idx < total) lds[idx] = v[u];
        }
    }
}

template <typename T>
__device__ __forceinline__ void lds_to_block(const JacArgs<T>& a, int s, int c0, int w, int rows,
                                             const cplx<T>* lds) {
    const int total = w * rows;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int c = idx / rows, r = idx - c * rows;
        *stacked(a, s, c0 + c, r) = lds[idx];
    }
}

// true when slice s converged in an earlier sweep
template <typename T>
__device__ __forceinline__ bool slice_done(const JacArgs<T>& a, int s) {
    return a.sweep > 0 && a.rot[((a.sweep - 1) % 3) * a.h + s] == 0;
}

// One pair step for a wavefront: x (registers) against column y in LDS.
// Returns 0 (not rotated), 1 (rotated) or 2 (rotated, forcing another sweep).
template <typename T, int RPT>
__device__ __forceinline__ unsigned pair_step(cplx<T> (&x)[RPT], cplx<T>* y_lds, int rows, int m, int lane,
                                          double tol) {
    cplx<T> y[RPT];
    T al = 0, be = 0, gr = 0, gi = 0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int r = lane + 64 * k;
        y[k] = r < rows ? y_lds[r] : cplx<T>{(T)0, (T)0};
        if (r < m) accum_pair(x[k], y[k], al, be, gr, gi);
    }
    const double sal = wave_sum((double)al), sbe = wave_sum((double)be);
    const double sgr = wave_sum((double)gr), sgi = wave_sum((double)gi);
    Rot rt;
    if (!make_rotation(sal, sbe, sgr, sgi, tol, rt)) return 0u;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int r = lane + 64 * k;
        apply_rotation(rt, x[k], y[k]);
        if (r < rows) y_lds[r] = y[k];
    }
    return rt.big ? 2u : 1u;
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(kBlock) void jacobi_init_kernel(JacArgs<T> a) {
    if (a.ctrl && a.ctrl->done) return;
    const int s = blockIdx.y;
    const int64_t nn = (int64_t)a.n * a.n;
    {
        const int64_t t = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
        const int64_t nt = (int64_t)gridDim.x * gridDim.y * blockDim.x;
        for (int c = 0; c < 2; ++c)
            if (a.clr[c])
                for (int64_t i = t; i < a.nclr[c]; i += nt) a.clr[c][i] = 0;
    }
    if (a.reset_v) {
        for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nn;
             idx += (int64_t)gridDim.x * blockDim.x) {
            const int64_t c = idx / a.n, r = idx - c * a.n;
            a.V[(int64_t)s * nn + idx] = cplx<T>{r == c ? (T)1 : (T)0, (T)0};
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.rot[s] = 0;   // ring entry 0 is written by sweep 0
        a.sweeps[s] = 0;
    }
}

// Intra-block pairs: BW/2 wavefronts, one column pair each per step.
template <typename T, int BW, int RPT>
__global__ __launch_bounds__(32 * BW) void jacobi_self_kernel(JacArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem);
    __shared__ int any_rot;
    const int s = blockIdx.y, b = blockIdx.x;
    // the ring entry of the next sweep is cleared for every slice, converged or not
    if (b == 0 && threadIdx.x == 0) a.rot[((a.sweep + 1) % 3) * a.h + s] = 0;
    if (slice_done(a, s)) return;
    if (b == 0 && threadIdx.x == 0) a.sweeps[s] += 1;
    const int c0 = blk_start(b, a.n, a.nb);
    const int w = blk_start(b + 1, a.n, a.nb) - c0;
    if (w < 2) return;
    const int rows = a.m + a.n;
    if (threadIdx.x == 0) any_rot = 0;
    block_to_lds(a, s, c0, w, rows, lds);
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wp = w + (w & 1);
    unsigned nrot = 0, nbig = 0;
    for (int st = 0; st < wp - 1; ++st) {
        if (wave < wp / 2) {
            const int p = rr_player(wave, st, wp);
            const int q = rr_player(wp - 1 - wave, st, wp);
            if (p < w && q < w) {
                cplx<T>* cp = lds + p * rows;
                cplx<T> x[RPT];
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const int r = lane + 64 * k;
                    x[k] = r < rows ? cp[r] : cplx<T>{(T)0, (T)0};
                }
                if (const unsigned code = pair_step<T, RPT>(x, lds + q * rows, rows, a.m, lane, (double)a.tol)) {
                    ++nrot;
                    nbig += code >> 1;
#pragma unroll
                    for (int k = 0; k < RPT; ++k) {
                        const int r = lane + 64 * k;
                        if (r < rows) cp[r] = x[k];
                    }
                }
            }
        }
        __syncthreads();
    }
    if (lane == 0) {
        if (nbig) any_rot = 1;
        if (nrot) atomicAdd(a.rotations, (unsigned long long)nrot);
    }
    __syncthreads();
    if (threadIdx.x == 0 && any_rot) a.rot[(a.sweep % 3) * a.h + s] = 1;
    lds_to_block(a, s, c0, w, rows, lds);
}

// Cross pairs of one tournament round: BW wavefronts, wave g owns column g
// of block I and meets every column of block J once.
template <typename T, int BW, int RPT>
__global__ __launch_bounds__(64 * BW) void jacobi_cross_kernel(JacArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem);
    __shared__ int any_rot;
    const int s = blockIdx.y, pr = blockIdx.x;
    if (slice_done(a, s)) return;
    const int bi = rr_player(pr, a.round, a.nb);
    const int bj = rr_player(a.nb - 1 - pr, a.round, a.nb);
    const int ci0 = blk_start(bi, a.n, a.nb), wi = blk_start(bi + 1, a.n, a.nb) - ci0;
    const int cj0 = blk_start(bj, a.n, a.nb), wj = blk_start(bj + 1, a.n, a.nb) - cj0;
    if (wi == 0 || wj == 0) return;
    const int rows = a.m + a.n;
    const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x == 0) any_rot = 0;

    cplx<T> xi[RPT];
    if (g < wi) {
        const cplx<T>* colA = a.A + ((int64_t)s * a.n + ci0 + g) * a.m;
        const cplx<T>* colV = a.V + ((int64_t)s * a.n + ci0 + g) * a.n;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int r = lane + 64 * k;
            xi[k] = r < a.m ? colA[r] : (r < rows ? colV[r - a.m] : cplx<T>{(T)0, (T)0});
        }
    }
    block_to_lds(a, s, cj0, wj, rows, lds);
    __syncthreads();

    unsigned nrot = 0, nbig = 0;
    for (int st = 0; st < BW; ++st) {
        const int jc = (g + st) % BW;
        if (g < wi && jc < wj) {
            const unsigned code = pair_step<T, RPT>(xi, lds + jc * rows, rows, a.m, lane, (double)a.tol);
            nrot += code != 0;
            nbig += code >> 1;
        }
        __syncthreads();
    }
    if (lane == 0) {
        if (nbig) any_rot = 1;
        if (nrot) atomicAdd(a.rotations, (unsigned long long)nrot);
    }
    if (g < wi) {
        cplx<T>* colA = a.A + ((int64_t)s * a.n + ci0 + g) * a.m;
        cplx<T>* colV = a.V + ((int64_t)s * a.n + ci0 + g) * a.n;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int r = lane + 64 * k;
            if (r < a.m)
                colA[r] = xi[k];
            else if (r < rows)
                colV[r - a.m] = xi[k];
        }
    }
    lds_to_block(a, s, cj0, wj, rows, lds);
    __syncthreads();
    if (threadIdx.x == 0 && any_rot) a.rot[(a.sweep % 3) * a.h + s] = 1;
}

// ---- tall slices
// Slices whose stacked columns do not fit the LDS kernels (the unfoldings
// of Sec. 3's vectorised baselines: n1 n2 rows) keep their columns in global
// memory.  The rotations are the ones above and the pairs of a round are the
// round-robin over single columns.  One round is two launches over
// (column pairs x row chunks x slices):
//   dots:   FP64 sums of ||a_p||^2, ||a_q||^2 and a_p^H a_q over the slice
//           rows of one chunk of the stacked column;
//   rotate: each workgroup adds its pair's chunk sums in chunk order (the
//           same order in every workgroup, so all of them derive the same
//           rotation) and applies the rotation to its chunk (slice rows and
//           V rows).
// part holds 4 doubles per (slice, pair, chunk).

template <typename T>
__global__ __launch_bounds__(kBlock) void jacobi_tall_dots_kernel(JacArgs<T> a, double* part, int chunks,
                                                                 int rows_per) {
    const int pair = blockIdx.x, c = blockIdx.y, s = blockIdx.z;
    if (slice_done(a, s)) return;
    const int p = rr_player(pair, a.round, a.nb), q = rr_player(a.nb - 1 - pair, a.round, a.nb);
    if (p >= a.n || q >= a.n) return;
    const cplx<T>* ap = a.A + ((int64_t)s * a.n + p) * a.m;
    const cplx<T>* aq = a.A + ((int64_t)s * a.n + q) * a.m;
    const int r0 = c * rows_per, r1 = min(r0 + rows_per, a.m);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = r0 + (int)threadIdx.x; r < r1; r += blockDim.x) {
        const cplx<T> x = ap[r], y = aq[r];
        const double xr = x.re, xi = x.im, yr = y.re, yi = y.im;
        v[0] += xr * xr + xi * xi;
        v[1] += yr * yr + yi * yi;
        v[2] += xr * yr + xi * yi;
        v[3] += xr * yi - xi * yr;
    }
    __shared__ double red[4][kBlock / 64];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double t = v[k];
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = t;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += red[threadIdx.x][w];
        part[(((int64_t)s * (a.nb / 2) + pair) * chunks + c) * 4 + threadIdx.x] = t;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void jacobi_tall_rotate_kernel(JacArgs<T> a, const double* part, int chunks,
                                                                   int rows_per) {
    const int pair = blockIdx.x, c = blockIdx.y, s = blockIdx.z;
    const bool lead = a.round == 0 && pair == 0 && c == 0 && threadIdx.x == 0;
    // the ring entry of the next sweep is cleared for every slice, converged or not
    if (lead) a.rot[((a.sweep + 1) % 3) * a.h + s] = 0;
    if (slice_done(a, s)) return;
    if (lead) a.sweeps[s] += 1;
    const int p = rr_player(pair, a.round, a.nb), q = rr_player(a.nb - 1 - pair, a.round, a.nb);
    if (p >= a.n || q >= a.n) return;
    __shared__ double sum[4];
    if (threadIdx.x < 4) {
        const double* pp = part + ((int64_t)s * (a.nb / 2) + pair) * chunks * 4 + threadIdx.x;
        double t = 0.0;
        for (int k = 0; k < chunks; ++k) t += pp[(int64_t)k * 4];
        sum[threadIdx.x] = t;
    }
    __syncthreads();
    Rot rd;
    if (!make_rotation(sum[0], sum[1], sum[2], sum[3], (double)a.tol, rd)) return;
    if (c == 0 && threadIdx.x == 0) {
        if (rd.big) a.rot[(a.sweep % 3) * a.h + s] = 1;
        if (a.rotations) atomicAdd(a.rotations, 1ull);
    }
    cplx<T>* ap = a.A + ((int64_t)s * a.n + p) * a.m;
    cplx<T>* aq = a.A + ((int64_t)s * a.n + q) * a.m;
    cplx<T>* vp = a.V + ((int64_t)s * a.n + p) * a.n;
    cplx<T>* vq = a.V + ((int64_t)s * a.n + q) * a.n;
    const int r0 = c * rows_per, r1 = min(r0 + rows_per, a.m + a.n);
    for (int r = r0 + (int)threadIdx.x; r < r1; r += blockDim.x) {
        cplx<T>* xp = r < a.m ? ap + r : vp + (r - a.m);
        cplx<T>* xq = r < a.m ? aq + r : vq + (r - a.m);
        cplx<T> x = *xp, y = *xq;
        apply_rotation(rd, x, y);
        *xp = x;
        *xq = y;
    }
}

// ------------------------------------------------------------------ host

namespace {

constexpr int kRpt[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};

int pick_rpt(int rows) {
    const int need = (rows + 63) / 64;
    for (int r : kRpt)
        if (r >= need) return r;
    return -1;
}

size_t g_lds_cap = 64 * 1024;   // set from the device by jacobi_set_lds_limit

template <typename K>
void allow_lds(K kernel, size_t bytes) {
    if (bytes > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

void jacobi_set_lds_limit(size_t bytes) { g_lds_cap = bytes; }

int jacobi_block_width(int m, int n, int elem_bytes, int h) {
    // Widest block (most pairs per workgroup, fewest launches per sweep)
    // whose LDS block fits; narrower if that leaves most CUs idle.
    const int rows = m + n;
    if (pick_rpt(rows) < 0) return -1;
    int best = -1;
    for (int bw : {16, 8, 4}) {
        if ((size_t)bw * rows * 2 * elem_bytes > g_lds_cap) continue;
        if (best < 0) best = bw;
        const int nb = jacobi_num_blocks(n, bw);
        if ((int64_t)(nb / 2) * h >= 128) return bw;
    }
    return best;
}

bool jacobi_tall(int m, int n, int elem_bytes) {
    return jacobi_block_width(m, n, elem_bytes, 1) < 0 && n >= 1 && n <= kMaxTallCols;
}

bool jacobi_supported(int m, int n, int elem_bytes) {
    return jacobi_block_width(m, n, elem_bytes, 1) > 0 || jacobi_tall(m, n, elem_bytes);
}

TallPlan jacobi_tall_plan(int m, int n, int h) {
    TallPlan t;
    t.players = n + (n & 1);
    const int pairs = t.players / 2;
    const int rows = m + n;
    // about a thousand workgroups per launch, chunks of at least 256 rows
    const int64_t want = (1024 + (int64_t)pairs * h - 1) / ((int64_t)pairs * h);
    t.chunks = (int)std::max<int64_t>(1, std::min<int64_t>(want, (rows + 255) / 256));
    t.rows_per = (rows + t.chunks - 1) / t.chunks;
    t.part_doubles = (int64_t)h * pairs * t.chunks * 4;
    return t;
}

template <typename T>
void launch_jacobi_tall_round(const JacArgs<T>& a, const TallPlan& t, double* part, hipStream_t st) {
    const dim3 grid(t.players / 2, t.chunks, a.h);
    hipLaunchKernelGGL((jacobi_tall_dots_kernel<T>), grid, dim3(kBlock), 0, st, a, part, t.chunks, t.rows_per);
    hipLaunchKernelGGL((jacobi_tall_rotate_kernel<T>), grid, dim3(kBlock), 0, st, a, part, t.chunks, t.rows_per);
}

template <typename T>
void launch_jacobi_init(const JacArgs<T>& a, hipStream_t st) {
    const int64_t nn = (int64_t)a.n * a.n;
    const int gx = (int)std::min<int64_t>((nn + kBlock - 1) / kBlock, 64);
    hipLaunchKernelGGL((jacobi_init_kernel<T>), dim3(gx, a.h), dim3(kBlock), 0, st, a);
}

template <typename T, int BW, int RPT>
static void launch_cross_t(const JacArgs<T>& a, size_t lds, hipStream_t st) {
    allow_lds(jacobi_cross_kernel<T, BW, RPT>, lds);
    hipLaunchKernelGGL((jacobi_cross_kernel<T, BW, RPT>), dim3(a.nb / 2, a.h), dim3(64 * BW), lds, st, a);
}

template <typename T, int BW, int RPT>
static void launch_self_t(const JacArgs<T>& a, size_t lds, hipStream_t st) {
    allow_lds(jacobi_self_kernel<T, BW, RPT>, lds);
    hipLaunchKernelGGL((jacobi_self_kernel<T, BW, RPT>), dim3(a.nb, a.h), dim3(32 * BW), lds, st, a);
}

#define TSVD_RPT_SWITCH(FN, BW)                           \
    switch (rpt) {                                        \
        case 1: FN<T, BW, 1>(a, lds, st); break;          \
        case 2: FN<T, BW, 2>(a, lds, st); break;          \
        case 3: FN<T, BW, 3>(a, lds, st); break;          \
        case 4: FN<T, BW, 4>(a, lds, st); break;          \
        case 5: FN<T, BW, 5>(a, lds, st); break;          \
        case 6: FN<T, BW, 6>(a, lds, st); break;          \
        case 8: FN<T, BW, 8>(a, lds, st); break;          \
        case 10: FN<T, BW, 10>(a, lds, st); break;        \
        case 12: FN<T, BW, 12>(a, lds, st); break;        \
        default: FN<T, BW, 16>(a, lds, st); break;        \
    }

template <typename T>
void launch_jacobi_self(const JacArgs<T>& a, int bw, hipStream_t st) {
    const int rows = a.m + a.n;
    const size_t lds = (size_t)bw * rows * sizeof(cplx<T>);
    const int rpt = pick_rpt(rows);
    if (bw == 16) {
        TSVD_RPT_SWITCH(launch_self_t, 16)
    } else if (bw == 8) {
        TSVD_RPT_SWITCH(launch_self_t, 8)
    } else {
        TSVD_RPT_SWITCH(launch_self_t, 4)
    }
}

// One cross round (a.round) of the block tournament.
template <typename T>
void launch_jacobi_cross(const JacArgs<T>& a, int bw, hipStream_t st) {
    const int rows = a.m + a.n;
    const size_t lds = (size_t)bw * rows * sizeof(cplx<T>);
    const int rpt = pick_rpt(rows);
    if (bw == 16) {
        TSVD_RPT_SWITCH(launch_cross_t, 16)
    } else if (bw == 8) {
        TSVD_RPT_SWITCH(launch_cross_t, 8)
    } else {
        TSVD_RPT_SWITCH(launch_cross_t, 4)
    }
}

#undef TSVD_RPT_SWITCH

template void launch_jacobi_init<double>(const JacArgs<double>&, hipStream_t);
template void launch_jacobi_tall_round<double>(const JacArgs<double>&, const TallPlan&, double*, hipStream_t);
template void launch_jacobi_self<double>(const JacArgs<double>&, int, hipStream_t);
template void launch_jacobi_cross<double>(const JacArgs<double>&, int, hipStream_t);

template void launch_jacobi_init<float>(const JacArgs<float>&, hipStream_t);
template void launch_jacobi_tall_round<float>(const JacArgs<float>&, const TallPlan&, double*, hipStream_t);
template void launch_jacobi_self<float>(const JacArgs<float>&, int, hipStream_t);
template void launch_jacobi_cross<float>(const JacArgs<float>&, int, hipStream_t);

}  // namespace tsvd
