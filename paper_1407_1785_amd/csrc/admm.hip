// Small kernels of the ADMM drivers: the per-iteration control step, the
// data norm of the stopping rule, the completion output and fills.
//
// Control step (one workgroup per problem), after the fused epilogue has
// written its FP64 residual partial sums:
//   primal = sqrt(sum p0), change = sqrt(sum p1) (completion) or
//   max(sqrt(sum p1), sqrt(sum p2)) (RPCA);
//   stop when max(primal, change) <= tol * ||data||_F;
//   otherwise rho' = min(growth * rho, rho_max) and the stored dual is read
//   as (rho / rho') times its value from then on; a problem-table run also
//   stops at its iteration cap (done = 2) (scaled-dual ADMM with a
//   penalty schedule; the completion recursion of Sec. 4 and the RPCA
//   recursion of Sec. 5 keep rho fixed, the growth is the workloads').
// The partial sums are reduced in a fixed order, so a run is deterministic.

#include "kernels.h"

namespace tsvd {

namespace {

__device__ double block_sum_fixed(const double* p, int nparts, int stride, int c, double* scratch) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += p[(int64_t)i * stride + c];
    scratch[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) scratch[threadIdx.x] += scratch[threadIdx.x + w];
        __syncthreads();
    }
    const double r = scratch[0];
    __syncthreads();
    return r;
}

}  // namespace

__device__ void admm_ctrl_body(Ctrl* c, const double* partials, int nparts, int rpca) {
    __shared__ double scratch[kBlock];
    const double p0 = block_sum_fixed(partials, nparts, kNumPartials, 0, scratch);
    const double p1 = block_sum_fixed(partials, nparts, kNumPartials, 1, scratch);
    const double p2 = block_sum_fixed(partials, nparts, kNumPartials, 2, scratch);
    if (threadIdx.x != 0) return;
    const double primal = sqrt(p0);
    const double change = rpca ? fmax(sqrt(p1), sqrt(p2)) : sqrt(p1);
    c->primal = primal;
    c->change = change;
    c->iter += 1;
    c->sweeps_total += c->sweep_max;
    c->sweeps_last = c->sweep_max;
    c->sweep_max = 0;
    c->rho_used = c->rho;
    c->dscale_used = c->dscale;
    if (!isfinite(primal) || !isfinite(change)) {
        c->nonfinite = 1;
        c->done = 1;
        return;
    }
    if (fmax(primal, change) <= c->tol_abs) {
        c->done = 1;
        c->dscale = 1.0;   // a converged solve keeps the dual unscaled
        return;
    }
    const double rho = c->rho;
    const double next = fmin(c->growth * rho, c->rho_max);
    c->dscale = rho / next;
    c->rho = next;
    c->tau = 1.0 / next;
    c->shrink = c->lambda / next;
    // iteration cap of a problem-table run (0: the host counts iterations)
    if (c->max_iter > 0 && c->iter >= c->max_iter) c->done = 2;
}

// A stopped problem is left alone (iterations queued after the stop do
// nothing); the mirror gets the control block either way.
__global__ __launch_bounds__(kBlock) void admm_ctrl_kernel(Ctrl* c, const double* partials, int nparts,
                                                          int rpca, Ctrl* mirror) {
    if (!c->done) admm_ctrl_body(c, partials, nparts, rpca);
    if (mirror && threadIdx.x == 0) *mirror = *c;
}

// One workgroup per problem; a problem that has stopped is left alone.
__global__ __launch_bounds__(kBlock) void admm_ctrl_batched(const CtrlArgs* tab) {
    const CtrlArgs& a = tab[blockIdx.x];
    if (a.c->done) return;
    // ring 0 of the pairs-parallel Jacobi's sweep flags and its barrier
    // area start clear for the next SVD
    if (a.rot_ring0)
        for (int s = threadIdx.x; s < a.h; s += blockDim.x) a.rot_ring0[s] = 0;
    if (a.clr)
        for (int s = threadIdx.x; s < a.nclr; s += blockDim.x) a.clr[s] = 0;
    admm_ctrl_body(a.c, a.partials, a.nparts, a.rpca);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void sumsq_kernel(const T* x, const uint8_t* mask, int64_t n,
                                                      double* partials) {
    __shared__ double scratch[kBlock];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = (mask == nullptr || mask[i]) ? (double)x[i] : 0.0;
        s += v * v;
    }
    scratch[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) scratch[threadIdx.x] += scratch[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * kNumPartials] = scratch[0];
}

__global__ __launch_bounds__(kBlock) void set_tol_kernel(Ctrl* c, const double* partials, int nparts,
                                                        double tol) {
    __shared__ double scratch[kBlock];
    const double s = block_sum_fixed(partials, nparts, kNumPartials, 0, scratch);
    if (threadIdx.x == 0) c->tol_abs = tol * sqrt(s);
}

// X = Omega.Y + (1 - Omega).(Z - Q) with Q = dscale_used * stored dual
template <typename T>
__global__ __launch_bounds__(kBlock) void complete_output_kernel(const T* y, const uint8_t* mask,
                                                                const T* z, const T* dual,
                                                                const Ctrl* c, T* out, int64_t n) {
    const double ds = c->dscale_used;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T q = (T)(ds * (double)dual[i]);
        out[i] = mask[i] ? y[i] : (T)(z[i] - q);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void fill_kernel(T* p, T v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Deterministic values in [-1, 1) from a 32-bit integer hash of the index
// (test and tuning inputs; no statistical quality is needed).
__device__ __forceinline__ float hash_unit(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return (float)(x >> 8) * (2.0f / 16777216.0f) - 1.0f;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void fill_hash_kernel(cplx<T>* p, int64_t n, uint32_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = (uint32_t)i * 2u + seed * 0x9e3779b9U;
        p[i] = cplx<T>{(T)hash_unit(k), (T)hash_unit(k + 1u)};
    }
}

// h slices of the n x n identity
template <typename T>
__global__ __launch_bounds__(kBlock) void set_identity_kernel(cplx<T>* v, int n, int64_t total) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = i % ((int64_t)n * n);
        const int64_t col = e / n, row = e - col * n;
        v[i] = cplx<T>{row == col ? (T)1 : (T)0, (T)0};
    }
}

static int grid_for(int64_t n) {
    const int64_t g = (n + kBlock - 1) / kBlock;
    return (int)(g < 2048 ? (g < 1 ? 1 : g) : 2048);
}

void launch_admm_ctrl_batched(const CtrlArgs* tab, int nprob, hipStream_t st) {
    hipLaunchKernelGGL(admm_ctrl_batched, dim3(nprob), dim3(kBlock), 0, st, tab);
}

void launch_admm_ctrl(Ctrl* c, const double* partials, int nparts, int rpca, Ctrl* mirror, hipStream_t st) {
    hipLaunchKernelGGL(admm_ctrl_kernel, dim3(1), dim3(kBlock), 0, st, c, partials, nparts, rpca, mirror);
}

template <typename T>
void launch_sumsq(const T* x, const uint8_t* mask, int64_t n, double* partials, int nparts,
                  hipStream_t st) {
    hipLaunchKernelGGL((sumsq_kernel<T>), dim3(nparts), dim3(kBlock), 0, st, x, mask, n, partials);
}

void launch_set_tol(Ctrl* c, const double* partials, int nparts, double tol, hipStream_t st) {
    hipLaunchKernelGGL(set_tol_kernel, dim3(1), dim3(kBlock), 0, st, c, partials, nparts, tol);
}

template <typename T>
void launch_complete_output(const T* y, const uint8_t* mask, const T* z, const T* dual,
                            const Ctrl* c, T* out, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL((complete_output_kernel<T>), dim3(grid_for(n)), dim3(kBlock), 0, st, y, mask, z,
                       dual, c, out, n);
}

template <typename T>
void launch_fill(T* p, T v, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL((fill_kernel<T>), dim3(grid_for(n)), dim3(kBlock), 0, st, p, v, n);
}

template <typename T>
void launch_fill_hash(cplx<T>* p, int64_t n, uint32_t seed, hipStream_t st) {
    hipLaunchKernelGGL((fill_hash_kernel<T>), dim3(grid_for(n)), dim3(kBlock), 0, st, p, n, seed);
}

template <typename T>
void launch_set_identity(cplx<T>* v, int n, int h, hipStream_t st) {
    const int64_t total = (int64_t)h * n * n;
    hipLaunchKernelGGL((set_identity_kernel<T>), dim3(grid_for(total)), dim3(kBlock), 0, st, v, n, total);
}

template void launch_fill_hash<double>(cplx<double>*, int64_t, uint32_t, hipStream_t);
template void launch_fill_hash<float>(cplx<float>*, int64_t, uint32_t, hipStream_t);
template void launch_set_identity<double>(cplx<double>*, int, int, hipStream_t);
template void launch_set_identity<float>(cplx<float>*, int, int, hipStream_t);
template void launch_sumsq<double>(const double*, const uint8_t*, int64_t, double*, int, hipStream_t);
template void launch_complete_output<double>(const double*, const uint8_t*, const double*,
                                             const double*, const Ctrl*, double*, int64_t,
                                             hipStream_t);
template void launch_fill<double>(double*, double, int64_t, hipStream_t);
template void launch_fill<int>(int*, int, int64_t, hipStream_t);
template void launch_fill<long long>(long long*, long long, int64_t, hipStream_t);

template void launch_sumsq<float>(const float*, const uint8_t*, int64_t, double*, int, hipStream_t);
template void launch_complete_output<float>(const float*, const uint8_t*, const float*,
                                            const float*, const Ctrl*, float*, int64_t,
                                            hipStream_t);
template void launch_fill<float>(float*, float, int64_t, hipStream_t);

}  // namespace tsvd
