// Singular values of the Jacobi output.
//
// After the Jacobi sweeps a slice is W V^H with orthogonal columns w_j, so
// sigma_j = ||w_j||.  The shrinkage lemma of Sec. 4.1 replaces sigma_j by
// (sigma_j - tau)_+, i.e. it scales w_j by d_j = (1 - tau/sigma_j)_+ (0 for
// sigma_j <= tau).  Both sigma and d are written here; the rebuild
// Zhat = W diag(d) V^H is done by the matrix-core GEMM (zgemm.hip).
//
// One wavefront per column: lanes stride the m rows, FP64 accumulation,
// reduction with cross-lane shuffles.  sigma is FP64 in both precision
// forms (it decides which singular values survive the threshold).

#include "kernels.h"

namespace tsvd {

template <typename T>
__device__ __forceinline__ void svt_sigma_body(const cplx<T>* W, int m, int n, int64_t cols, double* sigma,
                                               double* dk, double tau, int bid) {
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)bid * (kBlock / 64) + (threadIdx.x >> 6);
    if (c >= cols) return;
    const int64_t s = c / n, j = c - s * n;
    const cplx<T>* w = W + (s * n + j) * (int64_t)m;
    double acc = 0.0;
    for (int r = lane; r < m; r += 64) {
        const cplx<T> v = w[r];
        acc += (double)v.re * v.re + (double)v.im * v.im;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) {
        const double sg = sqrt(acc);
        sigma[c] = sg;
        dk[c] = sg > tau ? 1.0 - tau / sg : 0.0;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void svt_sigma_kernel(const cplx<T>* W, int m, int n, int64_t cols,
                                                          double* sigma, double* dk, const Ctrl* ctrl) {
    if (ctrl->done) return;
    svt_sigma_body<T>(W, m, n, cols, sigma, dk, ctrl->tau, (int)blockIdx.x);
}

// Problem-table launch; a problem whose ADMM has stopped is skipped.
template <typename T>
__global__ __launch_bounds__(kBlock) void svt_sigma_batched(const SigmaArgs<T>* tab, const int* wg_start, int nprob) {
    const int p = batch_find(wg_start, nprob, (int)blockIdx.x);
    const SigmaArgs<T>& a = tab[p];
    if (a.ctrl && a.ctrl->done) return;
    svt_sigma_body<T>(a.W, a.m, a.n, (int64_t)a.h * a.n, a.sigma, a.dk, a.ctrl->tau, (int)blockIdx.x - wg_start[p]);
}

int svt_sigma_workgroups(int n, int h) { return (int)(((int64_t)h * n + kBlock / 64 - 1) / (kBlock / 64)); }

template <typename T>
void launch_svt_sigma_batched(const SigmaArgs<T>* tab, const int* wg_start, int nprob, int nwg, hipStream_t st) {
    hipLaunchKernelGGL((svt_sigma_batched<T>), dim3(nwg), dim3(kBlock), 0, st, tab, wg_start, nprob);
}

template void launch_svt_sigma_batched<double>(const SigmaArgs<double>*, const int*, int, int, hipStream_t);
template void launch_svt_sigma_batched<float>(const SigmaArgs<float>*, const int*, int, int, hipStream_t);

template <typename T>
void launch_svt_sigma(const cplx<T>* W, int m, int n, int h, double* sigma, double* dk, const Ctrl* ctrl,
                      hipStream_t st) {
    const int64_t cols = (int64_t)h * n;
    const int64_t grid = (cols + kBlock / 64 - 1) / (kBlock / 64);
    hipLaunchKernelGGL((svt_sigma_kernel<T>), dim3((unsigned)grid), dim3(kBlock), 0, st, W, m, n, cols, sigma, dk, ctrl);
}

template void launch_svt_sigma<double>(const cplx<double>*, int, int, int, double*, double*, const Ctrl*,
                                       hipStream_t);
template void launch_svt_sigma<float>(const cplx<float>*, int, int, int, double*, double*, const Ctrl*, hipStream_t);

}  // namespace tsvd
