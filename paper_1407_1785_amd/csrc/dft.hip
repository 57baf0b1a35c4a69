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
// Work unit: one workgroup per tile of `tile` tubes (a multiple of 16) that
// are consecutive along the slice row mode, at one slice column.  The tile's
// tubes are staged through LDS, so tube-contiguous HBM traffic on one side
// and row-contiguous slice traffic on the other are both coalesced.
// Transform: both DFTs are small dense products on the matrix cores against
// the DFT matrices of the tube shape (built once in FP64 and rounded to the
// element type; layout in kernels.h, DftDims), 16 x 16 x 4 MFMA steps with
// the element type's own products and accumulation:
//   forward  D (2hp x tile) = F^T X, X the tile's tubes as columns (LDS),
//            rows s and hp + s of D the real and imaginary part of slice s;
//   inverse  L (Lr x tile) = S^T Z, Z the tile's spectra as 2h real rows
//            (real and imaginary part of each slice), L written to LDS and
//            consumed by the epilogue.
// The matrix fragments come from global memory (a few tens of KB, cache
// resident); each wave owns 16-row strips of D and sweeps the 16-column
// blocks of the tile, k in chunks of 16 with the next chunk's fragments in
// flight while the current one is multiplied, four independent accumulator
// chains per block.  The LDS row strides are 4 mod 16 words, so the 64 lanes
// of an operand read (16 columns x 4 k) fall in distinct banks.

#include "kernels.h"

#include <algorithm>

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

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 MFMA in the element type.  Operand lanes: lane l supplies
// row l % 16 of the first operand and column l % 16 of the second, both at
// k = l / 16.  Register v of lane l holds D(row(l, v), l % 16).
template <typename T>
struct Mma;

template <>
struct Mma<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};

template <>
struct Mma<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// LDS row stride for rows of n elements: n rounded up to 16, plus 4.
__host__ __device__ constexpr int lds_stride(int n) { return (n + 15) / 16 * 16 + 4; }

}  // namespace

template <typename T, int PRO>
__device__ __forceinline__ void dft_forward_body(const FwdArgs<T>& a, int bid, unsigned char* smem) {
    const Geometry& g = a.g;
    const DftDims d = DftDims::of(g.h, g.L);
    const int L = g.L, tile = a.tile, ldb = lds_stride(d.Lk);
    T* buf = reinterpret_cast<T*>(smem);   // tile x ldb, tube r at row r

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
    // positions L..Lk-1 meet zero matrix rows but must be finite
    for (int q = threadIdx.x; q < tile * (d.Lk - L); q += blockDim.x) {
        const int r = q / (d.Lk - L);
        buf[r * ldb + L + (q - r * (d.Lk - L))] = (T)0;
    }
    __syncthreads();

    // D = F^T X.  Columns of X past nrow hold stale LDS; they only reach
    // the columns of D that are not stored.
    typedef Mma<T> M;
    typedef typename M::acc_t acc_t;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int c16 = lane & 15, kq = lane >> 4;
    const int nj = (nrow + 15) >> 4;
    const int64_t ldf = 2 * (int64_t)d.hp;
    for (int item = wave; item < (d.hp / 16) * nj; item += nwave) {
        const int i = item / nj, j = item - i * nj;
        const T* fr = a.mat + kq * ldf + i * 16 + c16;
        const T* xb = buf + (j * 16 + c16) * ldb + kq;
        acc_t re0 = {0, 0, 0, 0}, im0 = re0, re1 = re0, im1 = re0;
        T ar[4], ai[4], bx[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ar[u] = fr[4 * u * ldf];
            ai[u] = fr[4 * u * ldf + d.hp];
            bx[u] = xb[4 * u];
        }
        for (int k0 = 0; k0 < d.Lk; k0 += 16) {
            const int kn = k0 + 16 < d.Lk ? k0 + 16 : k0;   // last chunk reloads itself
            T nar[4], nai[4], nbx[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                nar[u] = fr[(kn + 4 * u) * ldf];
                nai[u] = fr[(kn + 4 * u) * ldf + d.hp];
                nbx[u] = xb[kn + 4 * u];
            }
            re0 = M::mma(ar[0], bx[0], re0);
            im0 = M::mma(ai[0], bx[0], im0);
            re1 = M::mma(ar[1], bx[1], re1);
            im1 = M::mma(ai[1], bx[1], im1);
            re0 = M::mma(ar[2], bx[2], re0);
            im0 = M::mma(ai[2], bx[2], im0);
            re1 = M::mma(ar[3], bx[3], re1);
            im1 = M::mma(ai[3], bx[3], im1);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ar[u] = nar[u];
                ai[u] = nai[u];
                bx[u] = nbx[u];
            }
        }
        const int r = j * 16 + c16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int s = i * 16 + M::row(lane, v);
            if (s < g.h && r < nrow)
                a.out[((int64_t)s * g.n + col) * g.m + row0 + r] = cplx<T>{re0[v] + re1[v], im0[v] + im1[v]};
        }
    }
}

template <typename T, int EPI>
__device__ __forceinline__ void dft_inverse_body(const InvArgs<T>& a, int bid, unsigned char* smem) {
    const Geometry& g = a.g;
    const int L = g.L, tile = a.tile, h = g.h;
    const DftDims d = DftDims::of(h, L);
    const int ldl = lds_stride(d.Lr);
    cplx<T>* zb = reinterpret_cast<cplx<T>*>(smem);                  // h x tile spectra
    T* lb = reinterpret_cast<T*>(zb + (int64_t)h * tile);           // tile x ldl prox output
    // L112 only: D of the tile (tile x L), over the spectra once they are used
    T* db = reinterpret_cast<T*>(zb);
    // reduction scratch (64 doubles) followed by the per-tube shrink factors
    double* red = reinterpret_cast<double*>(lb + (int64_t)tile * ldl);

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

    {
        // L = S^T Z: row k of Z is the real (k even) or imaginary part of
        // slice k / 2; rows past 2h meet zero matrix rows (clamped reads).
        // k = k0 + 4u + kq has the parity of kq.
        typedef Mma<T> M;
        typedef typename M::acc_t acc_t;
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
        const int c16 = lane & 15, kq = lane >> 4;
        const bool odd = kq & 1;
        const int nj = (nrow + 15) >> 4;
        for (int item = wave; item < (d.Lr / 16) * nj; item += nwave) {
            const int i = item / nj, j = item - i * nj;
            const T* sr = a.mat + (int64_t)kq * d.Lr + i * 16 + c16;
            const cplx<T>* zr = zb + j * 16 + c16;
            acc_t c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
            T av[4], bz[4];
            auto zval = [&](int k) -> T {
                const cplx<T> z = zr[min(k >> 1, h - 1) * tile];
                return odd ? z.im : z.re;
            };
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                av[u] = sr[(int64_t)(4 * u) * d.Lr];
                bz[u] = zval(4 * u + kq);
            }
            for (int k0 = 0; k0 < d.Kr; k0 += 16) {
                const int kn = k0 + 16 < d.Kr ? k0 + 16 : k0;
                T nav[4], nbz[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    nav[u] = sr[(int64_t)(kn + 4 * u) * d.Lr];
                    nbz[u] = zval(kn + 4 * u + kq);
                }
                c0 = M::mma(av[0], bz[0], c0);
                c1 = M::mma(av[1], bz[1], c1);
                c2 = M::mma(av[2], bz[2], c2);
                c3 = M::mma(av[3], bz[3], c3);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    av[u] = nav[u];
                    bz[u] = nbz[u];
                }
            }
            T* lr = lb + (j * 16 + c16) * ldl + i * 16;
#pragma unroll
            for (int v = 0; v < 4; ++v) lr[M::row(lane, v)] = (c0[v] + c1[v]) + (c2[v] + c3[v]);
        }
    }
    __syncthreads();

    double part[kNumPartials] = {0.0, 0.0, 0.0, 0.0};
    double ds = 1.0, thr = 0.0;
    if (EPI != EPI_STORE) {
        ds = a.ctrl->dscale;
        thr = a.ctrl->shrink;
    }

    // U elements per thread per pass: the loads of a pass are all issued (at
    // clamped indices) before any value is used
    constexpr int U = 4;
    const int total = nrow * L;
    auto elem = [&](int idx, int& r, int& t) -> int64_t {
        r = idx / L;
        t = idx - r * L;
        return tube_offset<T>(g, row0 + r, col) + t;
    };
    if (EPI == EPI_RPCA_L112) {
        // pass 1: D = M - W - L' into LDS
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
                const T lv = lb[r * ldl + t];
                const T w = (T)(ds * (double)wv[u]);
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
                const T lv = lb[r * ldl + t];
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
                const T zv = lb[r * ldl + t];
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
    if (a.ctrl && a.ctrl->done) return;
    dft_forward_body<T, PRO>(a, (int)blockIdx.x, smem);
}

template <typename T, int EPI>
__global__ __launch_bounds__(kBlock) void dft_inverse_kernel(InvArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (a.ctrl && a.ctrl->done) return;
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
    const DftDims d = DftDims::of(g.h, g.L);
    int tile = 64;
    while (tile > 16 && (int64_t)tile * lds_stride(d.Lk) * 8 > 32768) tile /= 2;
    return tile;
}

int dft_inverse_tile(const Geometry& g, int epilogue) {
    (void)epilogue;   // the L112 tile of D reuses the spectra's LDS
    const DftDims d = DftDims::of(g.h, g.L);
    int tile = 64;
    auto bytes = [&](int t) { return (int64_t)g.h * t * 16 + (int64_t)t * lds_stride(d.Lr) * 8; };
    while (tile > 16 && bytes(tile) > 49152) tile /= 2;
    return tile;
}

int64_t dft_grid(const Geometry& g, int tile) {
    return (int64_t)g.n * ((g.m + tile - 1) / tile);
}

template <typename T>
size_t dft_forward_lds(const Geometry& g, int tile) {
    const DftDims d = DftDims::of(g.h, g.L);
    return (size_t)tile * lds_stride(d.Lk) * sizeof(T);
}

template <typename T>
size_t dft_inverse_lds(const Geometry& g, int tile, int epilogue) {
    (void)epilogue;
    const DftDims d = DftDims::of(g.h, g.L);
    const size_t lds = (size_t)g.h * tile * sizeof(cplx<T>) + (size_t)tile * lds_stride(d.Lr) * sizeof(T);
    return lds + 64 * sizeof(double) + (size_t)tile * sizeof(T) + 16;
}

template <typename K>
void allow_lds(K kernel, size_t lds);

template <typename T>
void prepare_dft_batched(size_t lds_forward, size_t lds_inverse) {
    allow_lds(dft_forward_batched<T>, lds_forward);
    allow_lds(dft_inverse_batched<T>, lds_inverse);
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

// Dynamic LDS above the 64 KB default needs the kernel's opt-in (long
// tubes in FP64).
template <typename K>
void allow_lds(K kernel, size_t lds) {
    if (lds > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename T, int PRO>
void launch_forward_as(const FwdArgs<T>& a, hipStream_t st) {
    const size_t lds = dft_forward_lds<T>(a.g, a.tile);
    allow_lds(dft_forward_kernel<T, PRO>, lds);
    hipLaunchKernelGGL((dft_forward_kernel<T, PRO>), dim3(dft_grid(a.g, a.tile)), dim3(kBlock), lds, st, a);
}

template <typename T, int EPI>
void launch_inverse_as(const InvArgs<T>& a, hipStream_t st) {
    const size_t lds = dft_inverse_lds<T>(a.g, a.tile, EPI);
    allow_lds(dft_inverse_kernel<T, EPI>, lds);
    hipLaunchKernelGGL((dft_inverse_kernel<T, EPI>), dim3(dft_grid(a.g, a.tile)), dim3(kBlock), lds, st, a);
}

template <typename T>
void launch_dft_forward(int prologue, const FwdArgs<T>& a, hipStream_t st) {
    switch (prologue) {
        case PRO_COPY: launch_forward_as<T, PRO_COPY>(a, st); break;
        case PRO_COMPLETE: launch_forward_as<T, PRO_COMPLETE>(a, st); break;
        default: launch_forward_as<T, PRO_RPCA>(a, st); break;
    }
}

template <typename T>
void launch_dft_inverse(int epilogue, const InvArgs<T>& a, hipStream_t st) {
    switch (epilogue) {
        case EPI_STORE: launch_inverse_as<T, EPI_STORE>(a, st); break;
        case EPI_COMPLETE: launch_inverse_as<T, EPI_COMPLETE>(a, st); break;
        case EPI_RPCA_L1: launch_inverse_as<T, EPI_RPCA_L1>(a, st); break;
        default: launch_inverse_as<T, EPI_RPCA_L112>(a, st); break;
    }
}

// The DFT matrices of a tube shape (layout in kernels.h, DftDims), built on
// the device: the twiddle exp(-2 pi i u / L) in FP64 (the quarter points
// exact, else sincospi), rounded once to the element type.  One thread per
// entry; entries outside s < h, t < L are zero.
template <typename T>
__global__ __launch_bounds__(kBlock) void dft_matrices_kernel(T* out, Geometry g, DftDims d) {
    const int64_t total = d.total();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int s, t, part;   // part: 0 forward Re, 1 forward Im, 2 inverse Re, 3 inverse Im
        if (i < d.fwd_size()) {
            t = (int)(i / (2 * d.hp));
            const int col = (int)(i - (int64_t)t * 2 * d.hp);
            part = col >= d.hp ? 1 : 0;
            s = col - part * d.hp;
        } else {
            const int64_t j = i - d.fwd_size();
            const int row = (int)(j / d.Lr);
            t = (int)(j - (int64_t)row * d.Lr);
            s = row >> 1;
            part = 2 + (row & 1);
        }
        T v = (T)0;
        if (s < g.h && t < g.L) {
            const int k3 = s / g.Qh, k4 = s - k3 * g.Qh;
            const int t3 = t / g.Q, t4 = t - t3 * g.Q;
            const int64_t u = ((int64_t)t3 * k3 * g.Q + (int64_t)t4 * k4 * g.P) % g.L;
            double re, im;
            if ((4 * u) % g.L == 0) {
                const int q = (int)((4 * u) / g.L);
                re = q == 0 ? 1.0 : (q == 2 ? -1.0 : 0.0);
                im = q == 1 ? -1.0 : (q == 3 ? 1.0 : 0.0);
            } else {
                sincospi(-2.0 * (double)u / (double)g.L, &im, &re);
            }
            if (part < 2) {
                v = (T)(part ? im : re);
            } else {
                const double c = (k4 == 0 || 2 * k4 == g.Q) ? 1.0 : 2.0;
                v = (T)(c / g.L * (part == 3 ? im : re));
            }
        }
        out[i] = v;
    }
}

template <typename T>
void launch_dft_matrices(T* out, const Geometry& g, hipStream_t st) {
    const DftDims d = DftDims::of(g.h, g.L);
    const int64_t blocks = std::min<int64_t>((d.total() + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL((dft_matrices_kernel<T>), dim3((unsigned)blocks), dim3(kBlock), 0, st, out, g, d);
}

template void launch_dft_matrices<double>(double*, const Geometry&, hipStream_t);
template void launch_dft_matrices<float>(float*, const Geometry&, hipStream_t);
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
