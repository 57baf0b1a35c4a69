// Singular value soft-threshold and rebuild of every Fourier frontal slice.
//
// After the Jacobi sweeps a slice is W V^H with orthogonal columns w_j, so
// sigma_j = ||w_j||.  The shrinkage lemma of Sec. 4.1 replaces sigma_j by
// (sigma_j - tau)_+, i.e. it multiplies w_j by d_j = (1 - tau/sigma_j)_+ (the
// tubal-shrinkage factor of Sec. 4.1), and the prox output is
//     Zhat = sum over kept j of d_j w_j v_j^H,
// kept = {j : sigma_j > tau}; their count is the slice's entry of the
// multi-rank (Sec. 2.4).
//
// svt_weights: one workgroup per slice computes sigma, d and the compacted
// kept list (in column order).
// svt_rebuild: a complex GEMM over the kept columns, one workgroup per
// 64 x 32 output tile; W and V panels are staged through LDS in chunks of
// 16 kept columns.

#include "kernels.h"

namespace tsvd {

template <typename T>
__global__ __launch_bounds__(kBlock) void svt_weights_kernel(SvtArgs<T> a) {
    __shared__ T sig[1024];
    __shared__ int cnt;
    const int s = blockIdx.x;
    const double tau = a.ctrl->tau;
    const cplx<T>* W = a.W + (int64_t)s * a.m * a.n;
    // one wavefront per column
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j0 = 0; j0 < a.n; j0 += 1024) {
        const int jn = min(1024, a.n - j0);
        for (int j = wave; j < jn; j += nw) {
            double acc = 0.0;
            for (int r = lane; r < a.m; r += 64) {
                const cplx<T> w = W[(int64_t)(j0 + j) * a.m + r];
                acc += (double)w.re * w.re + (double)w.im * w.im;
            }
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (lane == 0) sig[j] = (T)sqrt(acc);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int c = j0 == 0 ? 0 : cnt;
            for (int j = 0; j < jn; ++j) {
                const T sg = sig[j];
                if ((double)sg > tau) {
                    a.kept[(int64_t)s * a.n + c] = j0 + j;
                    a.d[(int64_t)s * a.n + c] = (T)(1.0 - tau / (double)sg);
                    ++c;
                }
            }
            cnt = c;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) a.rank[s] = cnt;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void svt_rebuild_kernel(SvtArgs<T> a) {
    constexpr int TM = 64, TN = 32, KC = 16;
    __shared__ cplx<T> wt[KC][TM];   // d_j * W(row, j)
    __shared__ cplx<T> vt[KC][TN];   // V(col, j)
    const int s = blockIdx.z;
    const int row0 = blockIdx.x * TM, col0 = blockIdx.y * TN;
    const int r = a.rank[s];
    const cplx<T>* W = a.W + (int64_t)s * a.m * a.n;
    const cplx<T>* V = a.V + (int64_t)s * a.n * a.n;
    const int* kept = a.kept + (int64_t)s * a.n;
    const T* d = a.d + (int64_t)s * a.n;
    const int tr = threadIdx.x & 63, tc = threadIdx.x >> 6;   // 4 column groups of 8
    T accr[8], acci[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) accr[c] = acci[c] = (T)0;

    for (int k0 = 0; k0 < r; k0 += KC) {
        const int kn = min(KC, r - k0);
        for (int idx = threadIdx.x; idx < KC * TM; idx += blockDim.x) {
            const int k = idx / TM, i = idx - k * TM;
            cplx<T> v{(T)0, (T)0};
            if (k < kn && row0 + i < a.m) {
                const int j = kept[k0 + k];
                const T dj = d[k0 + k];
                const cplx<T> w = W[(int64_t)j * a.m + row0 + i];
                v = cplx<T>{dj * w.re, dj * w.im};
            }
            wt[k][i] = v;
        }
        for (int idx = threadIdx.x; idx < KC * TN; idx += blockDim.x) {
            const int k = idx / TN, i = idx - k * TN;
            cplx<T> v{(T)0, (T)0};
            if (k < kn && col0 + i < a.n) v = V[(int64_t)kept[k0 + k] * a.n + col0 + i];
            vt[k][i] = v;
        }
        __syncthreads();
        for (int k = 0; k < kn; ++k) {
            const cplx<T> w = wt[k][tr];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const cplx<T> v = vt[k][tc * 8 + c];
                // w * conj(v)
                accr[c] += w.re * v.re + w.im * v.im;
                acci[c] += w.im * v.re - w.re * v.im;
            }
        }
        __syncthreads();
    }
    if (row0 + tr < a.m) {
        cplx<T>* Z = a.Z + (int64_t)s * a.m * a.n;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int col = col0 + tc * 8 + c;
            if (col < a.n) Z[(int64_t)col * a.m + row0 + tr] = cplx<T>{accr[c], acci[c]};
        }
    }
}

template <typename T>
void launch_svt_weights(const SvtArgs<T>& a, hipStream_t st) {
    hipLaunchKernelGGL((svt_weights_kernel<T>), dim3(a.h), dim3(kBlock), 0, st, a);
}

template <typename T>
void launch_svt_rebuild(const SvtArgs<T>& a, hipStream_t st) {
    dim3 grid((a.m + 63) / 64, (a.n + 31) / 32, a.h);
    hipLaunchKernelGGL((svt_rebuild_kernel<T>), grid, dim3(kBlock), 0, st, a);
}

template void launch_svt_weights<double>(const SvtArgs<double>&, hipStream_t);
template void launch_svt_rebuild<double>(const SvtArgs<double>&, hipStream_t);

template void launch_svt_weights<float>(const SvtArgs<float>&, hipStream_t);
template void launch_svt_rebuild<float>(const SvtArgs<float>&, hipStream_t);

}  // namespace tsvd
