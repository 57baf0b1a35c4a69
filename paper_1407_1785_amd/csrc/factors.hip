// Explicit t-SVD factors and the two compression methods (Sec. 2.2,
// Algorithm 1; Sec. 3, Methods 1 and 2), on top of the slice SVDs of the
// t-SVT path.
//
// After the one-sided Jacobi iteration every Fourier slice B (m x n, stored
// as in the t-SVT path) holds W = B V with orthogonal columns, sigma_j =
// ||w_j|| and unitary V.  The kernels here
//   * mirror the conjugate pairs that both lie in the half spectrum (4-D
//     tensors: slices (k3, k4) and (P - k3, k4) for k4 = 0 and, Q even,
//     k4 = Q/2), so that the inverse transforms of the factors are real;
//   * rank the columns of every slice by decreasing sigma (ties by index);
//   * write the Fourier-domain factors Uhat (n1 x n0), Vhat (n2 x n0) and the
//     singular values in that order (n0 = min(n1, n2));
//   * select the kept triplets of a compression as 0/1 factors for the
//     rebuild W diag(d) V^H: Method 2 keeps the first k3 of every slice,
//     Method 1 the k2 largest over the whole spectrum.
// When n1 < n2 a slice is stored transposed (B = Ahat^T), so
// Ahat = conj(V_B) Sigma (W_B / Sigma)^T: Uhat = conj(V_B), Vhat = conj(U_B).

#include "kernels.h"

namespace tsvd {

namespace {

__device__ __forceinline__ int slice_weight(const Geometry& g, int s) {
    // multiplicity of slice s in the full spectrum: 1 when its mirror is
    // itself or also in the half spectrum, 2 when the mirror is implied
    const int k4 = s % g.Qh;
    return (k4 == 0 || 2 * k4 == g.Q) ? 1 : 2;
}

}  // namespace

// One block row per slice (grid.y): slices that are the mirror of a slice
// with a smaller k3 take its conjugate SVD.
template <typename T>
__global__ __launch_bounds__(kBlock) void tsvd_mirror_kernel(cplx<T>* W, cplx<T>* V, double* sigma, Geometry g) {
    const int s = blockIdx.y;
    const int k3 = s / g.Qh, k4 = s - k3 * g.Qh;
    if (g.P < 2 || !(k4 == 0 || 2 * k4 == g.Q) || 2 * k3 <= g.P) return;
    const int src = (g.P - k3) * g.Qh + k4;
    const int64_t mn = (int64_t)g.m * g.n, nn = (int64_t)g.n * g.n;
    const int64_t total = mn + nn + g.n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < mn) {
            const cplx<T> v = W[src * mn + i];
            W[s * mn + i] = cplx<T>{v.re, -v.im};
        } else if (i < mn + nn) {
            const cplx<T> v = V[src * nn + (i - mn)];
            V[s * nn + (i - mn)] = cplx<T>{v.re, -v.im};
        } else {
            sigma[(int64_t)s * g.n + (i - mn - nn)] = sigma[(int64_t)src * g.n + (i - mn - nn)];
        }
    }
}

// rank[s][j] = #{k : sigma_k > sigma_j, or sigma_k == sigma_j and k < j}
// over the n columns of slice s (one workgroup per slice, sigma in LDS).
__global__ __launch_bounds__(kBlock) void tsvd_rank_kernel(const double* sigma, int n, int* rank) {
    extern __shared__ double sl[];
    const int s = blockIdx.x;
    for (int j = threadIdx.x; j < n; j += blockDim.x) sl[j] = sigma[(int64_t)s * n + j];
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double v = sl[j];
        int r = 0;
        for (int k = 0; k < n; ++k) r += (sl[k] > v || (sl[k] == v && k < j)) ? 1 : 0;
        rank[(int64_t)s * n + j] = r;
    }
}

// Uhat, Vhat, Shat of every slice, columns in rank order; a column with
// sigma = 0 gets a zero left singular vector.
template <typename T>
__global__ __launch_bounds__(kBlock) void tsvd_factor_kernel(const cplx<T>* W, const cplx<T>* V, const double* sigma,
                                                            const int* rank, Geometry g, cplx<T>* Uh, cplx<T>* Vh,
                                                            cplx<T>* Sh) {
    const int s = blockIdx.y;
    const int m = g.m, n = g.n;
    const int64_t mn = (int64_t)m * n, nn = (int64_t)n * n;
    const int64_t total = mn + nn + n;
    const int n1 = g.trans ? n : m, n2 = g.trans ? m : n;   // Uhat n1 x n, Vhat n2 x n
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < mn) {
            // a W entry: row of the left vectors of B
            const int j = (int)(i / m), row = (int)(i - (int64_t)j * m);
            const double sg = sigma[(int64_t)s * n + j];
            const int r = rank[(int64_t)s * n + j];
            const cplx<T> w = W[s * mn + i];
            const T f = sg > 0.0 ? (T)(1.0 / sg) : (T)0;
            if (g.trans)
                Vh[(int64_t)s * n2 * n + (int64_t)r * n2 + row] = cplx<T>{w.re * f, -w.im * f};
            else
                Uh[(int64_t)s * n1 * n + (int64_t)r * n1 + row] = cplx<T>{w.re * f, w.im * f};
        } else if (i < mn + nn) {
            const int64_t q = i - mn;
            const int j = (int)(q / n), row = (int)(q - (int64_t)j * n);
            const int r = rank[(int64_t)s * n + j];
            const cplx<T> v = V[s * nn + q];
            if (g.trans)
                Uh[(int64_t)s * n1 * n + (int64_t)r * n1 + row] = cplx<T>{v.re, -v.im};
            else
                Vh[(int64_t)s * n2 * n + (int64_t)r * n2 + row] = v;
        } else {
            const int j = (int)(i - mn - nn);
            Sh[(int64_t)s * n + rank[(int64_t)s * n + j]] = cplx<T>{(T)sigma[(int64_t)s * n + j], (T)0};
        }
    }
}

// Method 2: d = 1 for the first k3 columns of every slice (rank order).
__global__ __launch_bounds__(kBlock) void tubal_select_kernel(const int* rank, int64_t count, int k3, double* dk) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dk[i] = rank[i] < k3 ? 1.0 : 0.0;
}

// Method 1: the kept set is {sigma >= t} for the smallest t whose count over
// the full spectrum (slice multiplicities) is at most k2.  Non-negative
// doubles order like their bit patterns, so t is found by bisection on the
// patterns: the smallest pattern b with count(bits >= b) <= k2 keeps the same
// set.  One workgroup.
__global__ __launch_bounds__(1024) void global_select_kernel(const double* sigma, Geometry g, int64_t k2, double* dk) {
    __shared__ long long part[1024 / 64];
    __shared__ unsigned long long pick;
    const int64_t count = (int64_t)g.h * g.n;
    auto weight_ge = [&](unsigned long long b) -> long long {
        long long c = 0;
        for (int64_t i = threadIdx.x; i < count; i += blockDim.x) {
            const unsigned long long bits = (unsigned long long)__double_as_longlong(sigma[i]);
            if (bits >= b) c += slice_weight(g, (int)(i / g.n));
        }
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
        __syncthreads();
        long long tot = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += part[w];
        __syncthreads();
        return tot;
    };
    // invariant: count(>= hi) <= k2; count(>= lo) > k2 unless lo = 0
    unsigned long long lo = 0, hi = 0x7FF0000000000000ull;   // +inf keeps nothing
    if (weight_ge(0) <= k2) {
        hi = 0;
    } else {
        while (hi - lo > 1) {
            const unsigned long long mid = lo + (hi - lo) / 2;
            if (weight_ge(mid) <= k2) hi = mid;
            else lo = mid;
        }
    }
    if (threadIdx.x == 0) pick = hi;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < count; i += blockDim.x)
        dk[i] = (unsigned long long)__double_as_longlong(sigma[i]) >= pick ? 1.0 : 0.0;
}

template <typename T>
void launch_tsvd_mirror(cplx<T>* W, cplx<T>* V, double* sigma, const Geometry& g, hipStream_t st) {
    if (g.P < 2) return;
    hipLaunchKernelGGL((tsvd_mirror_kernel<T>), dim3(32, g.h), dim3(kBlock), 0, st, W, V, sigma, g);
}

void launch_tsvd_rank(const double* sigma, int n, int h, int* rank, hipStream_t st) {
    const size_t lds = (size_t)n * sizeof(double);
    if (lds > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(tsvd_rank_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(tsvd_rank_kernel, dim3(h), dim3(kBlock), lds, st, sigma, n, rank);
}

template <typename T>
void launch_tsvd_factors(const cplx<T>* W, const cplx<T>* V, const double* sigma, const int* rank, const Geometry& g,
                         cplx<T>* Uh, cplx<T>* Vh, cplx<T>* Sh, hipStream_t st) {
    const int64_t per = (int64_t)g.m * g.n + (int64_t)g.n * g.n + g.n;
    const int gx = (int)std::min<int64_t>((per + kBlock - 1) / kBlock, 256);
    hipLaunchKernelGGL((tsvd_factor_kernel<T>), dim3(gx, g.h), dim3(kBlock), 0, st, W, V, sigma, rank, g, Uh, Vh, Sh);
}

void launch_tubal_select(const int* rank, int64_t count, int k3, double* dk, hipStream_t st) {
    const int grid = (int)std::min<int64_t>((count + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(tubal_select_kernel, dim3(std::max(grid, 1)), dim3(kBlock), 0, st, rank, count, k3, dk);
}

void launch_global_select(const double* sigma, const Geometry& g, int64_t k2, double* dk, hipStream_t st) {
    hipLaunchKernelGGL(global_select_kernel, dim3(1), dim3(1024), 0, st, sigma, g, k2, dk);
}

template void launch_tsvd_mirror<double>(cplx<double>*, cplx<double>*, double*, const Geometry&, hipStream_t);
template void launch_tsvd_mirror<float>(cplx<float>*, cplx<float>*, double*, const Geometry&, hipStream_t);
template void launch_tsvd_factors<double>(const cplx<double>*, const cplx<double>*, const double*, const int*,
                                          const Geometry&, cplx<double>*, cplx<double>*, cplx<double>*, hipStream_t);
template void launch_tsvd_factors<float>(const cplx<float>*, const cplx<float>*, const double*, const int*,
                                         const Geometry&, cplx<float>*, cplx<float>*, cplx<float>*, hipStream_t);

}  // namespace tsvd
