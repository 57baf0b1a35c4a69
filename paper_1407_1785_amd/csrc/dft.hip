// Tube DFT kernels with the fused ADMM prologue / epilogue.
//
// Forward: the real DFT along the trailing modes of every (i, j) tube
// (Algorithm 1's fft along modes 3..N, unnormalised), half spectrum only,
// written as column-major complex Fourier frontal slices.  The ADMM input of
// the prox (the completion X-update of Sec. 4 plus the dual, or M - S - W
// for the RPCA L-update of Sec. 5) is formed on the fly while the tubes are
// loaded, so it never goes to HBM.
//
// Inverse: the real inverse DFT (1/L normalisation, conjugate-symmetric bins
// counted twice), followed by the rest of the ADMM iteration on the same
// element: the dual update of Sec. 4, or the S-update (entrywise l1 or the
// tube-group shrink of eq. sparse2) and dual update of Sec. 5, plus FP64
// partial sums of the residual norms.
//
// Work unit: one workgroup per tile of `tile` tubes that are consecutive
// along the slice row mode, at one slice column.  The tile's tubes are
// staged through LDS, so tube-contiguous HBM traffic on one side and
// row-contiguous slice traffic on the other are both coalesced.
// Transform: direct DFT against a twiddle table held in LDS (FP64 table,
// rounded to the element type; L is at most a few hundred on this path).

#include "kernels.h"

namespace tsvd {

namespace {

template <typename T>
__device__ __forceinline__ int64_t tube_offset(const Geometry& g, int row, int col) {
    const int64_t i = g.trans ? col : row;
    const int64_t j = g.trans ? row : col;
    return (i * g.n2 + j) * g.L;
}

__device__ __forceinline__ double warp_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sums of kNumPartials values into partials[slot * kNumPartials + c].
__device__ void block_partials(double (&v)[kNumPartials], double* partials, double* scratch, int slot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwave = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int c = 0; c < kNumPartials; ++c) v[c] = warp_sum(v[c]);
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < kNumPartials; ++c) scratch[wave * kNumPartials + c] = v[c];
    }
    __syncthreads();
    if (threadIdx.x < kNumPartials) {
        double s = 0.0;
        for (int w = 0; w < nwave; ++w) s += scratch[w * kNumPartials + threadIdx.x];
        partials[(int64_t)slot * kNumPartials + threadIdx.x] = s;
    }
}

template <typename T>
__device__ __forceinline__ T sq(T v) { return v * v; }

}  // namespace

template <typename T, int PRO>
__device__ __forceinline__ void dft_forward_body(const FwdArgs<T>& a, int bid, unsigned char* smem) {
    const Geometry& g = a.g;
    const int L = g.L, tile = a.tile, ldb = L + 1;
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem);
    T* buf = reinterpret_cast<T*>(tw + L);

    for (int u = threadIdx.x; u < L; u += blockDim.x) tw[u] = cplx<T>{(T)a.tw[u].re, (T)a.tw[u].im};

    const int row_tiles = (g.m + tile - 1) / tile;
    const int col = bid / row_tiles;
    const int row0 = (bid - col * row_tiles) * tile;
    const int nrow = min(tile, g.m - row0);
    const double ds = (PRO == PRO_COPY) ? 1.0 : a.ctrl->dscale;

    // the prox input of U elements per thread per pass: every load is issued
    // (at clamped indices) before any value is used
    constexpr int U = 8;
    const int total = nrow * L;
    bool bad = false;
    for (int base = threadIdx.x; base < total; base += U * (int)blockDim.x) {
        T xv[U], zv[U], qv[U];
        uint8_t mv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = min(base + u * (int)blockDim.x, total - 1);
            const int r = idx / L, t = idx - r * L;
            const int64_t e = tube_offset<T>(g, row0 + r, col) + t;
            xv[u] = a.x[e];
            if (PRO == PRO_COMPLETE) {
                zv[u] = a.z[e];
                qv[u] = a.dual[e];
                mv[u] = a.mask[e];
            } else if (PRO == PRO_RPCA) {
                zv[u] = a.s[e];
                qv[u] = a.dual[e];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * (int)blockDim.x;
            T v;
            if (PRO == PRO_COPY) {
                v = xv[u];
            } else if (PRO == PRO_COMPLETE) {
                const T q = (T)(ds * (double)qv[u]);
                const T x = mv[u] ? xv[u] : (T)(zv[u] - q);
                v = x + q;
            } else {
                const T w = (T)(ds * (double)qv[u]);
                v = (xv[u] - zv[u]) - w;
            }
            if (idx < total) {
                const int r = idx / L, t = idx - r * L;
                bad |= !isfinite(v);
                buf[r * ldb + t] = v;
            }
        }
    }
    if (bad) *a.nonfinite = 1;
    __syncthreads();

    const int P = g.P, Q = g.Q, Qh = g.Qh;
    for (int o = threadIdx.x; o < g.h * tile; o += blockDim.x) {
        const int s = o / tile, r = o - s * tile;
        if (r >= nrow) continue;
        const int k3 = s / Qh, k4 = s - k3 * Qh;
        const int step3 = (k3 * Q) % L, step4 = (k4 * P) % L;
        const T* xb = buf + r * ldb;
        T re = 0, im = 0;
        int u3 = 0;
        for (int t3 = 0; t3 < P; ++t3) {
            int u = u3;
            const T* xr = xb + t3 * Q;
            for (int t4 = 0; t4 < Q; ++t4) {
                const T v = xr[t4];
                re += v * tw[u].re;
                im += v * tw[u].im;
                u += step4;
                if (u >= L) u -= L;
            }
            u3 += step3;
            if (u3 >= L) u3 -= L;
        }
        const int64_t dst = ((int64_t)s * g.n + col) * g.m + row0 + r;
        a.out[dst] = cplx<T>{re, im};
    }
}

template <typename T, int EPI>
__device__ __forceinline__ void dft_inverse_body(const InvArgs<T>& a, int bid, unsigned char* smem) {
    const Geometry& g = a.g;
    const int L = g.L, tile = a.tile, h = g.h;
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* zb = reinterpret_cast<cplx<T>*>(tw + L);               // h x tile
    // L112 only: prox output and D of the tile, tile x L each
    T* lb = reinterpret_cast<T*>(zb + (int64_t)h * tile);
    T* db = lb + (EPI == EPI_RPCA_L112 ? (int64_t)tile * L : 0);
    // reduction scratch (64 doubles) followed by the per-tube shrink factors
    double* red = reinterpret_cast<double*>(db + (EPI == EPI_RPCA_L112 ? (int64_t)tile * L : 0));

    for (int u = threadIdx.x; u < L; u += blockDim.x) tw[u] = cplx<T>{(T)a.tw[u].re, (T)a.tw[u].im};

    const int row_tiles = (g.m + tile - 1) / tile;
    const int col = bid / row_tiles;
    const int row0 = (bid - col * row_tiles) * tile;
    const int nrow = min(tile, g.m - row0);

    // rows past nrow repeat the last row (never read): no branch around the loads
#pragma unroll 4
    for (int idx = threadIdx.x; idx < h * tile; idx += blockDim.x) {
        const int s = idx / tile, r = min(idx - s * tile, nrow - 1);
        zb[idx] = a.in[((int64_t)s * g.n + col) * g.m + row0 + r];
    }
    __syncthreads();

    const int P = g.P, Q = g.Q, Qh = g.Qh;
    const T inv_l = (T)1 / (T)L;
    double part[kNumPartials] = {0.0, 0.0, 0.0, 0.0};
    double ds = 1.0, thr = 0.0;
    if (EPI != EPI_STORE) {
        ds = a.ctrl->dscale;
        thr = a.ctrl->shrink;
    }

    // prox output of element (tube r, position t) of this tile
    auto synth = [&](int r, int t) -> T {
        const int t3 = t / Q, t4 = t - t3 * Q;
        const int step3 = (t3 * Q) % L, step4 = (t4 * P) % L;
        T acc = 0;
        int u3 = 0;
        for (int k3 = 0; k3 < P; ++k3) {
            int u = u3;
            const cplx<T>* zr = zb + (k3 * Qh) * tile + r;
            for (int k4 = 0; k4 < Qh; ++k4) {
                const cplx<T> z = zr[k4 * tile];
                const T wgt = (k4 == 0 || 2 * k4 == Q) ? (T)1 : (T)2;
                acc += wgt * (z.re * tw[u].re + z.im * tw[u].im);
                u += step4;
                if (u >= L) u -= L;
            }
            u3 += step3;
            if (u3 >= L) u3 -= L;
        }
        return acc * inv_l;
    };

    // U elements per thread per pass: the loads of a pass are issued (at
    // clamped indices) before the DFT sums that consume them
    constexpr int U = 4;
    const int total = nrow * L;
    auto elem = [&](int idx, int& r, int& t) -> int64_t {
        r = idx / L;
        t = idx - r * L;
        return tube_offset<T>(g, row0 + r, col) + t;
    };
    if (EPI == EPI_RPCA_L112) {
        // pass 1: prox output and D = M - W - L' into LDS
        for (int base = threadIdx.x; base < total; base += U * (int)blockDim.x) {
            T mv[U], wv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                int r, t;
                const int64_t e = elem(min(base + u * (int)blockDim.x, total - 1), r, t);
                mv[u] = a.m[e];
                wv[u] = a.dual_old[e];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = base + u * (int)blockDim.x;
                if (idx >= total) continue;
                int r, t;
                (void)elem(idx, r, t);
                const T lv = synth(r, t);
                const T w = (T)(ds * (double)wv[u]);
                lb[idx] = lv;
                db[idx] = (mv[u] - w) - lv;
            }
        }
        __syncthreads();
        // pass 2: per-tube shrink factor (1 - thr / ||D(i,j,:)||)_+, 0 for a zero tube
        T* fac = reinterpret_cast<T*>(red + 64);
        for (int r = threadIdx.x; r < nrow; r += blockDim.x) {
            double nrm2 = 0.0;
            for (int t = 0; t < L; ++t) nrm2 += (double)db[r * L + t] * (double)db[r * L + t];
            const T nrm = (T)sqrt(nrm2);
            fac[r] = nrm > (T)0 ? (T)fmax((T)1 - (T)thr / nrm, (T)0) : (T)0;
        }
        __syncthreads();
        for (int base = threadIdx.x; base < total; base += U * (int)blockDim.x) {
            T mv[U], wv[U], lo[U], so[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                int r, t;
                const int64_t e = elem(min(base + u * (int)blockDim.x, total - 1), r, t);
                mv[u] = a.m[e];
                wv[u] = a.dual_old[e];
                lo[u] = a.l_old[e];
                so[u] = a.s_old[e];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = base + u * (int)blockDim.x;
                if (idx >= total) continue;
                int r, t;
                const int64_t e = elem(idx, r, t);
                const T lv = lb[idx];
                const T sn = db[idx] * fac[r];
                const T w = (T)(ds * (double)wv[u]);
                const T wt = ((w + lv) + sn) - mv[u];
                a.out[e] = lv;
                a.s_new[e] = sn;
                a.dual_new[e] = wt;
                part[0] += (double)sq((lv + sn) - mv[u]);
                part[1] += (double)sq(lv - lo[u]);
                part[2] += (double)sq(sn - so[u]);
            }
        }
    } else {
        for (int base = threadIdx.x; base < total; base += U * (int)blockDim.x) {
            T v0[U], v1[U], v2[U], v3[U];
            uint8_t mk[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                int r, t;
                const int64_t e = elem(min(base + u * (int)blockDim.x, total - 1), r, t);
                if (EPI == EPI_COMPLETE) {
                    v0[u] = a.z_old[e];
                    v1[u] = a.dual_old[e];
                    v2[u] = a.y[e];
                    mk[u] = a.mask[e];
                } else if (EPI == EPI_RPCA_L1) {
                    v0[u] = a.m[e];
                    v1[u] = a.dual_old[e];
                    v2[u] = a.l_old[e];
                    v3[u] = a.s_old[e];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = base + u * (int)blockDim.x;
                if (idx >= total) continue;
                int r, t;
                const int64_t e = elem(idx, r, t);
                const T zv = synth(r, t);
                if (EPI == EPI_STORE) {
                    a.out[e] = zv;
                } else if (EPI == EPI_COMPLETE) {
                    const T zo = v0[u];
                    const T q = (T)(ds * (double)v1[u]);
                    const T x = mk[u] ? v2[u] : (T)(zo - q);
                    const T qt = (q + x) - zv;
                    a.out[e] = zv;
                    a.dual_new[e] = qt;
                    part[0] += (double)sq(x - zv);
                    part[1] += (double)sq(zv - zo);
                } else {  // EPI_RPCA_L1
                    const T mv = v0[u];
                    const T w = (T)(ds * (double)v1[u]);
                    const T d = (mv - w) - zv;
                    const T mag = (T)fmax(fabs(d) - (T)thr, (T)0);
                    const T sn = d > (T)0 ? mag : (d < (T)0 ? -mag : (T)0);
                    const T wt = ((w + zv) + sn) - mv;
                    a.out[e] = zv;
                    a.s_new[e] = sn;
                    a.dual_new[e] = wt;
                    part[0] += (double)sq((zv + sn) - mv);
                    part[1] += (double)sq(zv - v2[u]);
                    part[2] += (double)sq(sn - v3[u]);
                }
            }
        }
    }
    if (EPI != EPI_STORE) {
        __syncthreads();
        block_partials(part, a.partials, red, bid);
    }
}

template <typename T, int PRO>
__global__ __launch_bounds__(kBlock) void dft_forward_kernel(FwdArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    dft_forward_body<T, PRO>(a, (int)blockIdx.x, smem);
}

template <typename T, int EPI>
__global__ __launch_bounds__(kBlock) void dft_inverse_kernel(InvArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    dft_inverse_body<T, EPI>(a, (int)blockIdx.x, smem);
}

// Problem-table launches: the prologue / epilogue is a per-problem field;
// a problem whose ADMM has stopped is skipped.
template <typename T>
__global__ __launch_bounds__(kBlock) void dft_forward_batched(const FwdArgs<T>* tab, const int* wg_start, int nprob) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int p = batch_find(wg_start, nprob, (int)blockIdx.x);
    const FwdArgs<T>& a = tab[p];
    if (a.ctrl && a.ctrl->done) return;
    const int bid = (int)blockIdx.x - wg_start[p];
    switch (a.pro) {
        case PRO_COPY: dft_forward_body<T, PRO_COPY>(a, bid, smem); break;
        case PRO_COMPLETE: dft_forward_body<T, PRO_COMPLETE>(a, bid, smem); break;
        default: dft_forward_body<T, PRO_RPCA>(a, bid, smem); break;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void dft_inverse_batched(const InvArgs<T>* tab, const int* wg_start, int nprob) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int p = batch_find(wg_start, nprob, (int)blockIdx.x);
    const InvArgs<T>& a = tab[p];
    if (a.ctrl && a.ctrl->done) return;
    const int bid = (int)blockIdx.x - wg_start[p];
    switch (a.epi) {
        case EPI_STORE: dft_inverse_body<T, EPI_STORE>(a, bid, smem); break;
        case EPI_COMPLETE: dft_inverse_body<T, EPI_COMPLETE>(a, bid, smem); break;
        case EPI_RPCA_L1: dft_inverse_body<T, EPI_RPCA_L1>(a, bid, smem); break;
        default: dft_inverse_body<T, EPI_RPCA_L112>(a, bid, smem); break;
    }
}

int dft_forward_tile(const Geometry& g) {
    // keep the LDS tile near 32 KB so several workgroups share a CU
    int tile = 64;
    while (tile > 8 && (int64_t)tile * (g.L + 1) * 8 > 32768) tile /= 2;
    return tile;
}

int dft_inverse_tile(const Geometry& g, int epilogue) {
    int tile = 64;
    auto bytes = [&](int t) {
        int64_t b = (int64_t)g.h * t * 16;
        if (epilogue == EPI_RPCA_L112) b += 2LL * t * g.L * 8;
        return b;
    };
    while (tile > 8 && bytes(tile) > 40960) tile /= 2;
    return tile;
}

int64_t dft_grid(const Geometry& g, int tile) {
    return (int64_t)g.n * ((g.m + tile - 1) / tile);
}

template <typename T>
size_t dft_forward_lds(const Geometry& g, int tile) {
    return (size_t)g.L * sizeof(cplx<T>) + (size_t)tile * (g.L + 1) * sizeof(T);
}

template <typename T>
size_t dft_inverse_lds(const Geometry& g, int tile, int epilogue) {
    size_t lds = (size_t)g.L * sizeof(cplx<T>) + (size_t)g.h * tile * sizeof(cplx<T>);
    if (epilogue == EPI_RPCA_L112) lds += 2 * (size_t)tile * g.L * sizeof(T);
    return lds + 64 * sizeof(double) + (size_t)tile * sizeof(T) + 16;
}

template <typename T>
void prepare_dft_batched(size_t lds_forward, size_t lds_inverse) {
    if (lds_forward > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(dft_forward_batched<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_forward);
    if (lds_inverse > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(dft_inverse_batched<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_inverse);
}

template <typename T>
void launch_dft_forward_batched(const FwdArgs<T>* tab, const int* wg_start, int nprob, int nwg, size_t lds,
                                hipStream_t st) {
    hipLaunchKernelGGL((dft_forward_batched<T>), dim3(nwg), dim3(kBlock), lds, st, tab, wg_start, nprob);
}

template <typename T>
void launch_dft_inverse_batched(const InvArgs<T>* tab, const int* wg_start, int nprob, int nwg, size_t lds,
                                hipStream_t st) {
    hipLaunchKernelGGL((dft_inverse_batched<T>), dim3(nwg), dim3(kBlock), lds, st, tab, wg_start, nprob);
}

template <typename T>
void launch_dft_forward(int prologue, const FwdArgs<T>& a, hipStream_t st) {
    const int64_t grid = dft_grid(a.g, a.tile);
    const size_t lds = dft_forward_lds<T>(a.g, a.tile);
    switch (prologue) {
        case PRO_COPY:
            hipLaunchKernelGGL((dft_forward_kernel<T, PRO_COPY>), dim3(grid), dim3(kBlock), lds, st, a);
            break;
        case PRO_COMPLETE:
            hipLaunchKernelGGL((dft_forward_kernel<T, PRO_COMPLETE>), dim3(grid), dim3(kBlock), lds, st, a);
            break;
        default:
            hipLaunchKernelGGL((dft_forward_kernel<T, PRO_RPCA>), dim3(grid), dim3(kBlock), lds, st, a);
            break;
    }
}

template <typename T>
void launch_dft_inverse(int epilogue, const InvArgs<T>& a, hipStream_t st) {
    const int64_t grid = dft_grid(a.g, a.tile);
    const size_t lds = dft_inverse_lds<T>(a.g, a.tile, epilogue);
    switch (epilogue) {
        case EPI_STORE:
            hipLaunchKernelGGL((dft_inverse_kernel<T, EPI_STORE>), dim3(grid), dim3(kBlock), lds, st, a);
            break;
        case EPI_COMPLETE:
            hipLaunchKernelGGL((dft_inverse_kernel<T, EPI_COMPLETE>), dim3(grid), dim3(kBlock), lds, st, a);
            break;
        case EPI_RPCA_L1:
            hipLaunchKernelGGL((dft_inverse_kernel<T, EPI_RPCA_L1>), dim3(grid), dim3(kBlock), lds, st, a);
            break;
        default:
            hipLaunchKernelGGL((dft_inverse_kernel<T, EPI_RPCA_L112>), dim3(grid), dim3(kBlock), lds, st, a);
            break;
    }
}

template void prepare_dft_batched<double>(size_t, size_t);
template void prepare_dft_batched<float>(size_t, size_t);
template size_t dft_forward_lds<double>(const Geometry&, int);
template size_t dft_inverse_lds<double>(const Geometry&, int, int);
template size_t dft_forward_lds<float>(const Geometry&, int);
template size_t dft_inverse_lds<float>(const Geometry&, int, int);
template void launch_dft_forward_batched<double>(const FwdArgs<double>*, const int*, int, int, size_t, hipStream_t);
template void launch_dft_inverse_batched<double>(const InvArgs<double>*, const int*, int, int, size_t, hipStream_t);
template void launch_dft_forward_batched<float>(const FwdArgs<float>*, const int*, int, int, size_t, hipStream_t);
template void launch_dft_inverse_batched<float>(const InvArgs<float>*, const int*, int, int, size_t, hipStream_t);
template void launch_dft_forward<double>(int, const FwdArgs<double>&, hipStream_t);
template void launch_dft_inverse<double>(int, const InvArgs<double>&, hipStream_t);
template void launch_dft_forward<float>(int, const FwdArgs<float>&, hipStream_t);
template void launch_dft_inverse<float>(int, const InvArgs<float>&, hipStream_t);

}  // namespace tsvd
