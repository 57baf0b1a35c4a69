// Batched complex GEMM over the Fourier slices (column-major):
//     C[s] = alpha * op(A[s]) * B[s] + beta * D[s],   op(A) = A or A^H.
//
// Used by the warm start of the Jacobi SVD: the slice is pre-rotated by the
// previous iteration's right singular vectors (A V_prev), and V_prev is
// re-orthonormalised by one Newton-Schulz step, V <- 1.5 V - 0.5 V (V^H V),
// which squares its distance from unitarity.
//
// One workgroup per 64 x 64 tile of C, K staged through LDS in chunks of
// 16; every thread accumulates a 4 x 4 block of C in registers.

#include "kernels.h"

namespace tsvd {

template <typename T, bool AH>
__global__ __launch_bounds__(kBlock) void cgemm_kernel(GemmArgs<T> g) {
    constexpr int TM = 64, TN = 64, TK = 16;
    __shared__ cplx<T> As[TK][TM + 1];
    __shared__ cplx<T> Bs[TK][TN + 1];
    const int s = blockIdx.z;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    const cplx<T>* A = g.A + (int64_t)s * g.sA;
    const cplx<T>* B = g.B + (int64_t)s * g.sB;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    T accr[4][4], acci[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) accr[i][j] = acci[i][j] = (T)0;

    for (int k0 = 0; k0 < g.K; k0 += TK) {
        for (int idx = threadIdx.x; idx < TM * TK; idx += blockDim.x) {
            int mm, kk;
            if (AH) {   // A is K x M: walk k fastest for contiguous reads
                kk = idx % TK;
                mm = idx / TK;
            } else {
                mm = idx % TM;
                kk = idx / TM;
            }
            const int m = m0 + mm, k = k0 + kk;
            cplx<T> v{(T)0, (T)0};
            if (m < g.M && k < g.K) {
                if (AH) {
                    const cplx<T> a = A[(int64_t)m * g.lda + k];
                    v = cplx<T>{a.re, -a.im};
                } else {
                    v = A[(int64_t)k * g.lda + m];
                }
            }
            As[kk][mm] = v;
        }
        for (int idx = threadIdx.x; idx < TN * TK; idx += blockDim.x) {
            const int kk = idx % TK, nn = idx / TK;
            const int k = k0 + kk, n = n0 + nn;
            Bs[kk][nn] = (k < g.K && n < g.N) ? B[(int64_t)n * g.ldb + k] : cplx<T>{(T)0, (T)0};
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < TK; ++kk) {
            cplx<T> a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][tx + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][ty + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    accr[i][j] += a[i].re * b[j].re - a[i].im * b[j].im;
                    acci[i][j] += a[i].re * b[j].im + a[i].im * b[j].re;
                }
        }
        __syncthreads();
    }
    cplx<T>* C = g.C + (int64_t)s * g.sC;
    const cplx<T>* D = g.D ? g.D + (int64_t)s * g.sD : nullptr;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int n = n0 + ty + 16 * j;
        if (n >= g.N) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = m0 + tx + 16 * i;
            if (m >= g.M) continue;
            T re = g.alpha * accr[i][j], im = g.alpha * acci[i][j];
            if (D) {
                const cplx<T> d = D[(int64_t)n * g.ldd + m];
                re += g.beta * d.re;
                im += g.beta * d.im;
            }
            C[(int64_t)n * g.ldc + m] = cplx<T>{re, im};
        }
    }
}

template <typename T>
void launch_cgemm(const GemmArgs<T>& g, hipStream_t st) {
    dim3 grid((g.M + 63) / 64, (g.N + 63) / 64, g.batch);
    if (g.opA_h)
        hipLaunchKernelGGL((cgemm_kernel<T, true>), grid, dim3(kBlock), 0, st, g);
    else
        hipLaunchKernelGGL((cgemm_kernel<T, false>), grid, dim3(kBlock), 0, st, g);
}

template void launch_cgemm<double>(const GemmArgs<double>&, hipStream_t);

template void launch_cgemm<float>(const GemmArgs<float>&, hipStream_t);

}  // namespace tsvd
