// Batched complex GEMM on the matrix cores, one problem per Fourier slice,
// column-major complex operands:
//
//     C[s] = alpha * op(A[s]) * diag(d[s]) * op(B[s]) + beta * D[s],
//     op(X) = X or X^H,  d optional (else 1).
//
// Users:
//   * the rebuild of the shrinkage lemma (Sec. 4.1): Zhat = W diag(d) V^H
//     with the shrink factors d_k = (1 - tau / sigma_k)_+ (written by the
//     singular-value kernel) applied while W is staged, so no compaction
//     pass is needed (dropped columns get d = 0 exactly);
//   * the warm start of the Jacobi SVD: the pre-rotation A V_prev and the
//     Newton-Schulz step V <- 1.5 V - 0.5 V (V^H V).
//
// Arithmetic:
//   double: v_mfma_f64_16x16x4f64, FP64 products and accumulation;
//   float:  v_mfma_f32_16x16x4f32, FP32 products and accumulation (exact
//           FP32 arithmetic), or with bf16x3 set, every FP32 operand x is
//           split into bfloat16 parts hi = bf16(x), lo = bf16(x - hi) and each
//           real product uses the three bf16 products hi*hi + hi*lo + lo*hi
//           (v_mfma_f32_16x16x32_bf16) with FP32 accumulation; the dropped
//           lo*lo term and the split residual leave about 2^-16 relative
//           error per product.
// A complex product takes four real MFMA products (re*re - im*im,
// re*im + im*re).
//
// Tiling: one 256-thread workgroup per 64 x 64 tile of C; wave w owns the
// 32 x 32 quadrant (w & 1, w >> 1), i.e. 2 x 2 MFMA tiles of 16 x 16.  K is
// staged through LDS in chunks of 32, with the real and imaginary parts in
// separate arrays; the next chunk is loaded into registers while the
// current one is multiplied.  The MFMA operands are
// given as (op(B) fragment, op(A) fragment), so the accumulator holds C
// transposed: lane l owns 4 columns at row l % 16 of a 16 x 16 tile, and the
// 16 lanes of a row group store 16 consecutive rows of a column-major C in
// one coalesced access.

#include "kernels.h"

#include <cstdlib>

namespace tsvd {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int TM = 64, TN = 64;

// Operand views: element (r, k) of an R x K view of X is at k * ld + r
// (stored R x K column-major) or at r * ld + k (kcontig: stored K x R),
// conjugated for the op = H operands, zero outside [0,R) x [0,K).  Staging
// clamps the address into the matrix and masks the value afterwards, so all
// loads of a pass are in flight together.
// ---- K = 4 per MFMA (FP64, or exact FP32), stage [k][r] -----------------

constexpr int KC4 = 32, PAD4 = 1;
constexpr int LD4 = TM * KC4 / 256;   // staged elements per thread and operand

template <typename T>
struct Stage4 {
    T ar[KC4][TM + PAD4], ai[KC4][TM + PAD4];
    T br[KC4][TN + PAD4], bi[KC4][TN + PAD4];
};

// Element q of this thread's share of a 64 x KC4 block of an operand view.
__device__ __forceinline__ void slot4(bool kcontig, int q, int& rr, int& kk) {
    const int t = threadIdx.x;
    if (kcontig) {
        kk = t % KC4;
        rr = t / KC4 + (256 / KC4) * q;
    } else {
        rr = t % TM;
        kk = t / TM + 4 * q;
    }
}

// Issue the loads of this thread's share of a 64 x KC4 block (and of the
// column factors d_k when dk is set).  Nothing is done with the values
// here, so the loads of the next chunk stay in flight while the current
// chunk is multiplied; store4 masks, conjugates, scales and writes them.
template <typename T>
__device__ __forceinline__ void load4(const cplx<T>* X, int ld, bool kcontig, int r0, int k0, int R, int K,
                                      const double* dk, cplx<T> (&v)[LD4], double (&dv)[LD4]) {
#pragma unroll
    for (int q = 0; q < LD4; ++q) {
        int rr, kk;
        slot4(kcontig, q, rr, kk);
        const int rc = min(r0 + rr, R - 1), kc = min(k0 + kk, K - 1);
        v[q] = X[kcontig ? (int64_t)rc * ld + kc : (int64_t)kc * ld + rc];
        if (dk) dv[q] = dk[kc];
    }
}

template <typename T>
__device__ __forceinline__ void store4(bool kcontig, bool conj, int r0, int k0, int R, int K, bool scaled,
                                       const cplx<T> (&v)[LD4], const double (&dv)[LD4], T (*re)[TM + PAD4],
                                       T (*im)[TM + PAD4]) {
#pragma unroll
    for (int q = 0; q < LD4; ++q) {
        int rr, kk;
        slot4(kcontig, q, rr, kk);
        const bool in = r0 + rr < R && k0 + kk < K;
        const T f = in ? (scaled ? (T)dv[q] : (T)1) : (T)0;
        re[kk][rr] = f * v[q].re;
        im[kk][rr] = f * (conj ? -v[q].im : v[q].im);
    }
}

template <typename T>
struct Mfma4;

template <>
struct Mfma4<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // register v of lane l holds (row l % 16, column 4 v + l / 16) of the
    // transposed 16 x 16 tile
    static __device__ __forceinline__ int col(int lane, int v) { return 4 * v + (lane >> 4); }
};

template <>
struct Mfma4<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // register v of lane l holds (row l % 16, column 4 (l / 16) + v)
    static __device__ __forceinline__ int col(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <typename T>
__device__ __forceinline__ void zgemm_k4_body(const ZGemmArgs<T>& g, int bx, int by, int s) {
    typedef Mfma4<T> M;
    typedef typename M::acc_t acc_t;
    __shared__ Stage4<T> sm;
    const int row0 = bx * TM, col0 = by * TN;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    const cplx<T>* A = g.A + (int64_t)s * g.sA;
    const cplx<T>* B = g.B + (int64_t)s * g.sB;
    const double* dk = g.dk ? g.dk + (int64_t)s * g.sdk : nullptr;

    acc_t cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) cr[a][b] = ci[a][b] = acc_t{(T)0, (T)0, (T)0, (T)0};

    // op(A): rows M, op N -> stored M x K (r-contiguous); op H -> stored K x M, conj.
    // op(B)^T as an N x K view: op N -> B stored K x N (k-contiguous); op H -> stored N x K, conj.
    const bool akc = g.opA != 0, bkc = g.opB == 0;
    cplx<T> va[LD4], vb[LD4];
    double da[LD4], db[LD4];
    load4<T>(A, g.lda, akc, row0, 0, g.M, g.K, dk, va, da);
    load4<T>(B, g.ldb, bkc, col0, 0, g.N, g.K, nullptr, vb, db);
    for (int k0 = 0; k0 < g.K; k0 += KC4) {
        store4<T>(akc, g.opA != 0, row0, k0, g.M, g.K, dk != nullptr, va, da, sm.ar, sm.ai);
        store4<T>(bkc, g.opB != 0, col0, k0, g.N, g.K, false, vb, db, sm.br, sm.bi);
        __syncthreads();
        if (k0 + KC4 < g.K) {   // prefetch the next chunk while this one is multiplied
            load4<T>(A, g.lda, akc, row0, k0 + KC4, g.M, g.K, dk, va, da);
            load4<T>(B, g.ldb, bkc, col0, k0 + KC4, g.N, g.K, nullptr, vb, db);
        }
#pragma unroll
        for (int kk = 0; kk < KC4; kk += 4) {
            const int kq = kk + (lane >> 4), c16 = lane & 15;
            T a_r[2], a_i[2], b_r[2], b_i[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a_r[x] = sm.ar[kq][wr + 16 * x + c16];
                a_i[x] = sm.ai[kq][wr + 16 * x + c16];
                b_r[x] = sm.br[kq][wc + 16 * x + c16];
                b_i[x] = sm.bi[kq][wc + 16 * x + c16];
            }
            // four passes over the eight accumulators: consecutive MFMAs never
            // depend on each other
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    cr[x][y] = M::mma(b_r[y], a_r[x], cr[x][y]);
                    ci[x][y] = M::mma(b_r[y], a_i[x], ci[x][y]);
                }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    cr[x][y] = M::mma(-b_i[y], a_i[x], cr[x][y]);
                    ci[x][y] = M::mma(b_i[y], a_r[x], ci[x][y]);
                }
        }
        __syncthreads();
    }

    cplx<T>* C = g.C + (int64_t)s * g.sC;
    const cplx<T>* D = g.D ? g.D + (int64_t)s * g.sD : nullptr;
    // beta * D first, from clamped addresses (all loads in flight), then the
    // guarded stores
    cplx<T> dv[2][2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) dv[x][y][v] = cplx<T>{(T)0, (T)0};
    if (D) {
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const int rowc = min(row0 + wr + 16 * x + (lane & 15), g.M - 1);
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int colc = min(col0 + wc + 16 * y + M::col(lane, v), g.N - 1);
                    dv[x][y][v] = D[(int64_t)colc * g.ldd + rowc];
                }
        }
    }
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        const int row = row0 + wr + 16 * x + (lane & 15);
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = col0 + wc + 16 * y + M::col(lane, v);
                const T re = g.alpha * cr[x][y][v] + g.beta * dv[x][y][v].re;
                const T im = g.alpha * ci[x][y][v] + g.beta * dv[x][y][v].im;
                if (row < g.M && col < g.N) C[(int64_t)col * g.ldc + row] = cplx<T>{re, im};
            }
    }
}

// ---- FP32 form: bf16 split, K = 32 per MFMA, stage [r][k] ----------------

constexpr int KC16 = 32, PAD16 = 8;

struct alignas(16) Stage16 {
    // [part][r][k], part: 0 re hi, 1 re lo, 2 im hi, 3 im lo
    __bf16 a[4][TM][KC16 + PAD16];
    __bf16 b[4][TN][KC16 + PAD16];
};

__device__ __forceinline__ void split_store(__bf16 (*dst)[TM][KC16 + PAD16], int rr, int kk, float re, float im) {
    const __bf16 rh = (__bf16)re, ih = (__bf16)im;
    dst[0][rr][kk] = rh;
    dst[1][rr][kk] = (__bf16)(re - (float)rh);
    dst[2][rr][kk] = ih;
    dst[3][rr][kk] = (__bf16)(im - (float)ih);
}

__device__ __forceinline__ void stage16(const cplx<float>* X, int ld, bool kcontig, bool conj, int r0, int k0,
                                        int R, int K, __bf16 (*dst)[TM][KC16 + PAD16], const double* dk) {
    const int t = threadIdx.x;
    cplx<float> v[8];
    double dv[8];
    int rr[8], kk[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if (kcontig) {
            kk[q] = t % KC16;
            rr[q] = t / KC16 + 8 * q;
        } else {
            rr[q] = t % TM;
            kk[q] = t / TM + 4 * q;
        }
        const int rc = min(r0 + rr[q], R - 1), kc = min(k0 + kk[q], K - 1);
        v[q] = X[kcontig ? (int64_t)rc * ld + kc : (int64_t)kc * ld + rc];
        if (dk) dv[q] = dk[kc];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const bool in = r0 + rr[q] < R && k0 + kk[q] < K;
        v[q].re = in ? v[q].re : 0.f;
        v[q].im = in ? (conj ? -v[q].im : v[q].im) : 0.f;
        if (dk) {
            v[q].re *= (float)dv[q];
            v[q].im *= (float)dv[q];
        }
        split_store(dst, rr[q], kk[q], v[q].re, v[q].im);
    }
}

__device__ __forceinline__ v8bf frag16(const __bf16 (*part)[KC16 + PAD16], int r, int k) {
    return *reinterpret_cast<const v8bf*>(&part[r][k]);
}

__device__ __forceinline__ v8bf neg8(v8bf x) {
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    v4u u = __builtin_bit_cast(v4u, x);
    u ^= 0x80008000u;
    return __builtin_bit_cast(v8bf, u);
}

#define MFMA_BF16(acc, x, y) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16((x), (y), (acc), 0, 0, 0)

__device__ __forceinline__ void zgemm_bf16x3_body(const ZGemmArgs<float>& g, int bx, int by, int s) {
    __shared__ Stage16 sm;
    const int row0 = bx * TM, col0 = by * TN;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    const cplx<float>* A = g.A + (int64_t)s * g.sA;
    const cplx<float>* B = g.B + (int64_t)s * g.sB;
    const double* dk = g.dk ? g.dk + (int64_t)s * g.sdk : nullptr;

    v4f cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) cr[a][b] = ci[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < g.K; k0 += KC16) {
        stage16(A, g.lda, g.opA != 0, g.opA != 0, row0, k0, g.M, g.K, sm.a, dk);
        stage16(B, g.ldb, g.opB == 0, g.opB != 0, col0, k0, g.N, g.K, sm.b, nullptr);
        __syncthreads();
        const int kq = 8 * (lane >> 4), c16 = lane & 15;
        v8bf arh[2], arl[2], aih[2], ail[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const int r = wr + 16 * x + c16;
            arh[x] = frag16(sm.a[0], r, kq);
            arl[x] = frag16(sm.a[1], r, kq);
            aih[x] = frag16(sm.a[2], r, kq);
            ail[x] = frag16(sm.a[3], r, kq);
        }
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int r = wc + 16 * y + c16;
            const v8bf brh = frag16(sm.b[0], r, kq), brl = frag16(sm.b[1], r, kq);
            const v8bf bih = frag16(sm.b[2], r, kq), bil = frag16(sm.b[3], r, kq);
            const v8bf nbih = neg8(bih), nbil = neg8(bil);
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                // re: br*ar - bi*ai
                MFMA_BF16(cr[x][y], brh, arh[x]);
                MFMA_BF16(cr[x][y], brh, arl[x]);
                MFMA_BF16(cr[x][y], brl, arh[x]);
                MFMA_BF16(cr[x][y], nbih, aih[x]);
                MFMA_BF16(cr[x][y], nbih, ail[x]);
                MFMA_BF16(cr[x][y], nbil, aih[x]);
                // im: br*ai + bi*ar
                MFMA_BF16(ci[x][y], brh, aih[x]);
                MFMA_BF16(ci[x][y], brh, ail[x]);
                MFMA_BF16(ci[x][y], brl, aih[x]);
                MFMA_BF16(ci[x][y], bih, arh[x]);
                MFMA_BF16(ci[x][y], bih, arl[x]);
                MFMA_BF16(ci[x][y], bil, arh[x]);
            }
        }
        __syncthreads();
    }

    cplx<float>* C = g.C + (int64_t)s * g.sC;
    const cplx<float>* D = g.D ? g.D + (int64_t)s * g.sD : nullptr;
    // beta * D first, from clamped addresses (all loads in flight), then the
    // guarded stores
    cplx<float> dv[2][2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) dv[x][y][v] = cplx<float>{(float)0, (float)0};
    if (D) {
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const int rowc = min(row0 + wr + 16 * x + (lane & 15), g.M - 1);
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int colc = min(col0 + wc + 16 * y + Mfma4<float>::col(lane, v), g.N - 1);
                    dv[x][y][v] = D[(int64_t)colc * g.ldd + rowc];
                }
        }
    }
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        const int row = row0 + wr + 16 * x + (lane & 15);
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = col0 + wc + 16 * y + Mfma4<float>::col(lane, v);
                const float re = g.alpha * cr[x][y][v] + g.beta * dv[x][y][v].re;
                const float im = g.alpha * ci[x][y][v] + g.beta * dv[x][y][v].im;
                if (row < g.M && col < g.N) C[(int64_t)col * g.ldc + row] = cplx<float>{re, im};
            }
    }
}

// ---- split-K form for products with few 64 x 64 tiles -------------------
//
// One 256-thread workgroup per 32 x 32 tile of C.  The four waves split the
// K range into contiguous quarters; each wave computes the whole tile over
// its quarter (2 x 2 MFMA tiles, the same accumulators and operand order as
// the 64 x 64 form) with the fragments loaded straight from memory, no LDS
// staging and no barrier.  The four partial tiles are then summed through LDS
// in a fixed order (quarter 0 first), each wave finishing one 16 x 16 part.
// A 128 x 128 product per slice has 16 such tiles instead of 4, so a batch of
// a few dozen slices spreads over all compute units.

constexpr int SKM = 32, SKN = 32;
// MFMA k-steps (of 4) per load batch: 8 in FP32, 4 in FP64.  With the
// two-pass reduction (16 / 32 KB of LDS) and the launch bound below, both
// fit three workgroups per compute unit, so the 528-660 workgroups of a batch
// of 33 slices of up to 160 x 128 run in one round.
template <typename T>
constexpr int sk_batch() { return sizeof(T) == 8 ? 4 : 8; }

// Raw element (r, k) of an operand view (layout as for the staged form), from
// an address clamped into the matrix, so the load is always in bounds; the
// caller masks, conjugates and scales it.
template <typename T>
__device__ __forceinline__ cplx<T> view_load(const cplx<T>* X, int ld, bool kcontig, int r, int k, int R, int K) {
    const int rc = min(r, R - 1), kc = min(k, K - 1);
    return X[kcontig ? (int64_t)rc * ld + kc : (int64_t)kc * ld + rc];
}

// OPA, OPB: g.opA, g.opB as template arguments, so the operand layouts and
// conjugations are fixed at compile time.
template <typename T, int OPA, int OPB>
__device__ __forceinline__ void zgemm_sk_body(const ZGemmArgs<T>& g, int bx, int by, int s) {
    typedef Mfma4<T> M;
    typedef typename M::acc_t acc_t;
    __shared__ T red[4][2][2][4][64];   // [wave][x][y][register][lane], one part at a time
    const int row0 = bx * SKM, col0 = by * SKN;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int l16 = lane & 15, lk = lane >> 4;
    const cplx<T>* A = g.A + (int64_t)s * g.sA;
    const cplx<T>* B = g.B + (int64_t)s * g.sB;
    const double* dk = g.dk ? g.dk + (int64_t)s * g.sdk : nullptr;
    constexpr bool akc = OPA != 0, bkc = OPB == 0;
    constexpr bool aconj = OPA != 0, bconj = OPB != 0;

    acc_t cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) cr[a][b] = ci[a][b] = acc_t{(T)0, (T)0, (T)0, (T)0};

    // kept-column form: the k with dk[k] > 0 in increasing order, found by
    // wave 0 with ballots (every workgroup of the slice finds the same list)
    __shared__ int klist[kMaxCompactK];
    __shared__ int kcount;
    const bool compact = g.kcompact && dk && g.K <= kMaxCompactK;
    int Kv = g.K;
    if (compact) {
        if (w == 0) {
            int run = 0;
            for (int base = 0; base < g.K; base += 64) {
                const int kk = base + lane;
                const bool keep = kk < g.K && dk[kk] > 0.0;
                const unsigned long long mask = __ballot(keep);
                if (keep) klist[run + __popcll(mask & ((1ull << lane) - 1ull))] = kk;
                run += __popcll(mask);
            }
            if (lane == 0) kcount = run;
        }
        __syncthreads();
        Kv = kcount;
    }
    auto kmap = [&](int k) { return compact ? klist[min(k, Kv - 1)] : k; };
    const int nks = (Kv + 3) / 4, per = (nks + 3) / 4;
    const int ks0 = w * per, ks1 = min(ks0 + per, nks);
    const int kend = min(4 * ks1, Kv);
    constexpr int SKB = sk_batch<T>();
    for (int kb = ks0; kb < ks1; kb += SKB) {
        cplx<T> va[SKB][2], vb[SKB][2];
        double dv[SKB];
#pragma unroll
        for (int j = 0; j < SKB; ++j) {
            const int k = 4 * (kb + j) + lk;
            const int kk = kmap(k);
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                va[j][x] = view_load<T>(A, g.lda, akc, row0 + 16 * x + l16, kk, g.M, g.K);
                vb[j][x] = view_load<T>(B, g.ldb, bkc, col0 + 16 * x + l16, kk, g.N, g.K);
            }
            dv[j] = dk ? dk[min(kk, g.K - 1)] : 1.0;
        }
#pragma unroll
        for (int j = 0; j < SKB; ++j) {
            const int k = 4 * (kb + j) + lk;
            T a_r[2], a_i[2], b_r[2], b_i[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const bool ain = row0 + 16 * x + l16 < g.M && k < kend;
                const bool bin = col0 + 16 * x + l16 < g.N && k < kend;
                const T fa = ain ? (dk ? (T)dv[j] : (T)1) : (T)0;
                const T fb = bin ? (T)1 : (T)0;
                a_r[x] = fa * va[j][x].re;
                a_i[x] = fa * (aconj ? -va[j][x].im : va[j][x].im);
                b_r[x] = fb * vb[j][x].re;
                b_i[x] = fb * (bconj ? -vb[j][x].im : vb[j][x].im);
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    cr[x][y] = M::mma(b_r[y], a_r[x], cr[x][y]);
                    ci[x][y] = M::mma(b_r[y], a_i[x], ci[x][y]);
                }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    cr[x][y] = M::mma(-b_i[y], a_i[x], cr[x][y]);
                    ci[x][y] = M::mma(b_i[y], a_r[x], ci[x][y]);
                }
        }
    }

    // The four partial tiles are summed in a fixed order (quarter 0 first),
    // the real parts first, then the imaginary parts through the same buffer.
    const int x = w & 1, y = w >> 1;
    T sr[4], si[4];
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) red[w][a][b][v][lane] = part ? ci[a][b][v] : cr[a][b][v];
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            T t = red[0][x][y][v][lane];
#pragma unroll
            for (int q = 1; q < 4; ++q) t += red[q][x][y][v][lane];
            (part ? si : sr)[v] = t;
        }
        if (part == 0) __syncthreads();
    }
    const int row = row0 + 16 * x + l16;
    cplx<T>* C = g.C + (int64_t)s * g.sC;
    const cplx<T>* D = g.D ? g.D + (int64_t)s * g.sD : nullptr;
    cplx<T> dd[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        dd[v] = cplx<T>{(T)0, (T)0};
        if (D) {
            const int colc = min(col0 + 16 * y + M::col(lane, v), g.N - 1);
            dd[v] = D[(int64_t)colc * g.ldd + min(row, g.M - 1)];
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int col = col0 + 16 * y + M::col(lane, v);
        const T re = g.alpha * sr[v] + g.beta * dd[v].re;
        const T im = g.alpha * si[v] + g.beta * dd[v].im;
        if (row < g.M && col < g.N) {
            C[(int64_t)col * g.ldc + row] = cplx<T>{re, im};
            if (g.herm && bx != by) C[(int64_t)row * g.ldc + col] = cplx<T>{re, -im};
        }
    }
}

// Tile of this workgroup in a (gx, gy, batch) grid.  The device deals
// workgroups to its 8 XCDs, each with its own L2, in turn by linear index;
// with remap set the tiles are renumbered so that each XCD takes a contiguous
// run of them (tile x fastest, then tile y, then slice), and a slice's
// operands are fetched into one or two L2s instead of into all eight.
__device__ __forceinline__ int xcd_order(int lin, int n) {
    const int q = n / 8, r = n % 8, x = lin % 8;
    return x * q + min(x, r) + lin / 8;
}

__device__ __forceinline__ void grid_tile(int remap, int& bx, int& by, int& s) {
    const int gx = gridDim.x, gy = gridDim.y;
    if (!remap) {
        bx = blockIdx.x;
        by = blockIdx.y;
        s = blockIdx.z;
        return;
    }
    const int id = xcd_order(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * (int)gridDim.z);
    s = id / (gx * gy);
    const int rem = id - s * gx * gy;
    by = rem / gx;
    bx = rem - by * gx;
}

// Tile (ti, tj), ti <= tj, of index t in the column-by-column enumeration of
// the tiles on and above the diagonal: t = tj (tj + 1) / 2 + ti.
__device__ __forceinline__ void upper_tile(int t, int& ti, int& tj) {
    tj = 0;
    while ((tj + 1) * (tj + 2) / 2 <= t) ++tj;
    ti = t - tj * (tj + 1) / 2;
}

template <typename T, int OPA, int OPB>
__global__ __launch_bounds__(256, 3) void zgemm_sk_kernel(ZGemmArgs<T> g, int remap) {
    if (g.ctrl && g.ctrl->done) return;
    int bx, by, s;
    grid_tile(remap, bx, by, s);
    if (g.herm) upper_tile(bx, bx, by);   // grid (tiles on and above the diagonal, 1, batch)
    zgemm_sk_body<T, OPA, OPB>(g, bx, by, s);
}

template <typename T>
__global__ __launch_bounds__(256) void zgemm_k4_kernel(ZGemmArgs<T> g, int remap) {
    if (g.ctrl && g.ctrl->done) return;
    int bx, by, s;
    grid_tile(remap, bx, by, s);
    zgemm_k4_body<T>(g, bx, by, s);
}

__global__ __launch_bounds__(256) void zgemm_bf16x3_kernel(ZGemmArgs<float> g, int remap) {
    if (g.ctrl && g.ctrl->done) return;
    int bx, by, s;
    grid_tile(remap, bx, by, s);
    zgemm_bf16x3_body(g, bx, by, s);
}

// Problem-table launch: problem p owns tiles_m * tiles_n * batch workgroups;
// a problem whose ADMM has stopped (ctrl->done) is skipped.  The XCD
// renumbering of grid_tile is not applied here: on the 64-problem batched
// workload it made the solve 1.6% slower.
template <typename T>
__global__ __launch_bounds__(256) void zgemm_batched_kernel(const ZGemmArgs<T>* tab, const int* wg_start,
                                                            int nprob) {
    const int p = batch_find(wg_start, nprob, (int)blockIdx.x);
    const ZGemmArgs<T>& g = tab[p];
    if (g.ctrl && g.ctrl->done) return;
    const int local = (int)blockIdx.x - wg_start[p];
    const int tm = (g.M + TM - 1) / TM, tn = (g.N + TN - 1) / TN;
    const int s = local / (tm * tn), rem = local - s * (tm * tn);
    const int by = rem / tm, bx = rem - by * tm;
    if constexpr (sizeof(T) == 4) {
        if (g.bf16x3) {
            zgemm_bf16x3_body(g, bx, by, s);
            return;
        }
    }
    zgemm_k4_body<T>(g, bx, by, s);
}

// The multi-rank (Sec. 2.4): rank[s] = #{k < K : sigma_k > tau}, one
// workgroup per slice.
__global__ __launch_bounds__(256) void multirank_kernel(const double* sigma, int64_t ssig, int K, const Ctrl* ctrl,
                                                        int* rank) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const double tau = ctrl->tau;
    const double* sg = sigma + (int64_t)blockIdx.x * ssig;
    int c = 0;
    for (int k = threadIdx.x; k < K; k += blockDim.x) c += sg[k] > tau ? 1 : 0;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(&cnt, c);
    __syncthreads();
    if (threadIdx.x == 0) rank[blockIdx.x] = cnt;
}

}  // namespace

namespace {

// The split-K form when the 64 x 64 grid leaves compute units idle (fewer
// than two tiles per unit of a 256-unit device).  TSVD_GEMM_SPLITK=0 / 1
// forces the 64 x 64 / split-K form.
int env_or(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}

int xcd_remap() {
    static const int on = env_or("TSVD_GEMM_XCD", 1);
    return on;
}

template <typename T>
void launch_split_k(const ZGemmArgs<T>& gin, hipStream_t st) {
    ZGemmArgs<T> g = gin;
    g.herm = g.herm && g.M == g.N && g.A == g.B && g.opA != 0 && g.opB == 0 && !g.D && !g.dk ? 1 : 0;
    const int tm = (g.M + SKM - 1) / SKM;
    const dim3 grid = g.herm ? dim3(tm * (tm + 1) / 2, 1, g.batch) : dim3(tm, (g.N + SKN - 1) / SKN, g.batch);
    const int r = xcd_remap();
    if (g.opA == 0 && g.opB == 0)
        hipLaunchKernelGGL((zgemm_sk_kernel<T, 0, 0>), grid, dim3(256), 0, st, g, r);
    else if (g.opA == 0)
        hipLaunchKernelGGL((zgemm_sk_kernel<T, 0, 1>), grid, dim3(256), 0, st, g, r);
    else if (g.opB == 0)
        hipLaunchKernelGGL((zgemm_sk_kernel<T, 1, 0>), grid, dim3(256), 0, st, g, r);
    else
        hipLaunchKernelGGL((zgemm_sk_kernel<T, 1, 1>), grid, dim3(256), 0, st, g, r);
}

template <typename T>
bool use_split_k_of(const ZGemmArgs<T>& g) {
    static const int forced = env_or("TSVD_GEMM_SPLITK", -1);
    if (forced >= 0) return forced != 0;
    const int64_t tiles = (int64_t)((g.M + TM - 1) / TM) * ((g.N + TN - 1) / TN) * g.batch;
    return tiles < 512;
}

}  // namespace

template <>
void launch_zgemm<double>(const ZGemmArgs<double>& g, hipStream_t st) {
    if (use_split_k_of(g)) {
        launch_split_k(g, st);
        return;
    }
    dim3 grid((g.M + TM - 1) / TM, (g.N + TN - 1) / TN, g.batch);
    hipLaunchKernelGGL(zgemm_k4_kernel<double>, grid, dim3(256), 0, st, g, xcd_remap());
}

template <>
void launch_zgemm<float>(const ZGemmArgs<float>& g, hipStream_t st) {
    if (!g.bf16x3 && use_split_k_of(g)) {
        launch_split_k(g, st);
        return;
    }
    dim3 grid((g.M + TM - 1) / TM, (g.N + TN - 1) / TN, g.batch);
    if (g.bf16x3)
        hipLaunchKernelGGL(zgemm_bf16x3_kernel, grid, dim3(256), 0, st, g, xcd_remap());
    else
        hipLaunchKernelGGL(zgemm_k4_kernel<float>, grid, dim3(256), 0, st, g, xcd_remap());
}

int zgemm_workgroups(int M, int N, int batch) { return ((M + TM - 1) / TM) * ((N + TN - 1) / TN) * batch; }

template <typename T>
void launch_zgemm_batched(const ZGemmArgs<T>* tab, const int* wg_start, int nprob, int nwg, hipStream_t st) {
    hipLaunchKernelGGL((zgemm_batched_kernel<T>), dim3(nwg), dim3(256), 0, st, tab, wg_start, nprob);
}

template void launch_zgemm_batched<double>(const ZGemmArgs<double>*, const int*, int, int, hipStream_t);
template void launch_zgemm_batched<float>(const ZGemmArgs<float>*, const int*, int, int, hipStream_t);

void launch_multirank(const double* sigma, int64_t ssig, int K, int h, const Ctrl* ctrl, int* rank,
                      hipStream_t st) {
    hipLaunchKernelGGL(multirank_kernel, dim3(h), dim3(256), 0, st, sigma, ssig, K, ctrl, rank);
}

}  // namespace tsvd
