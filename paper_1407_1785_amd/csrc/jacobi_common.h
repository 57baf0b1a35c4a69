// Device helpers shared by the Jacobi kernels that keep column blocks in
// LDS (jacobi_persist.hip: several workgroups per slice; jacobi_slice.hip:
// one workgroup per slice).  See jacobi.hip for the rotation and the block
// round-robin ordering.
#pragma once

#include "kernels.h"

namespace tsvd {
namespace jac {

__device__ __forceinline__ int pblk_start(int b, int n, int nb) {
    return (int)(((int64_t)b * n) / nb);
}

__device__ __forceinline__ int ppos_player(int pos, int r, int nb) {
    return pos == 0 ? 0 : 1 + (pos - 1 + r) % (nb - 1);
}

// DPP lane exchange within a 16-lane row.  Every lane reads a valid source
// for the controls used here; with bound_ctrl the exchange folds into the
// consuming add as a DPP source operand.
template <int CTRL>
__device__ __forceinline__ float pdpp(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ double pdpp(double v) {
    return __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true),
                            __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true));
}

// Sum of the two 16-lane rows 2r and 2r + 1, in every lane of both.
// v_permlane16_swap exchanges the odd rows of its first operand with the
// even rows of its second; with both operands holding v, the two registers
// then hold row 2r and row 2r + 1 of v in every lane of the row pair.  The
// instruction is issued from a register-only asm block (no memory access)
// because the compiler's builtin for it returns its first result for both
// results; the s_nop pairs cover the VALU-write / cross-lane-read wait
// states on both sides.
__device__ __forceinline__ float rowpair_sum(float v) {
    unsigned a = __builtin_bit_cast(unsigned, v), b = a;
    asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1\n\ts_nop 1" : "+v"(a), "+v"(b));
    return __builtin_bit_cast(float, a) + __builtin_bit_cast(float, b);
}

__device__ __forceinline__ double rowpair_sum(double v) {
    unsigned al = (unsigned)__double2loint(v), bl = al;
    unsigned ah = (unsigned)__double2hiint(v), bh = ah;
    asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1\n\tv_permlane16_swap_b32 %2, %3\n\ts_nop 1"
                 : "+v"(al), "+v"(bl), "+v"(ah), "+v"(bh));
    return __hiloint2double((int)ah, (int)al) + __hiloint2double((int)bh, (int)bl);
}

// rowpair_sum of several independent values, their swaps in one block.
__device__ __forceinline__ void rowpair_sum2(float& v, float& w) {
    unsigned a = __builtin_bit_cast(unsigned, v), b = a;
    unsigned c = __builtin_bit_cast(unsigned, w), d = c;
    asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1\n\tv_permlane16_swap_b32 %2, %3\n\ts_nop 1"
                 : "+v"(a), "+v"(b), "+v"(c), "+v"(d));
    v = __builtin_bit_cast(float, a) + __builtin_bit_cast(float, b);
    w = __builtin_bit_cast(float, c) + __builtin_bit_cast(float, d);
}

__device__ __forceinline__ void rowpair_sum2(double& v, double& w) {
    v = rowpair_sum(v);
    w = rowpair_sum(w);
}

// Sum over the PG lanes of a pair group, in the element type; every lane of
// the group gets the same bits (each stage adds two equal-shaped partial
// sums, and addition is commutative).  16 lanes = one DPP row; 32 lanes =
// two rows.
template <int PG, typename T>
__device__ __forceinline__ T group_sum(T v) {
    v += pdpp<0xB1>(v);    // lane ^ 1
    v += pdpp<0x4E>(v);    // lane ^ 2
    v += pdpp<0x141>(v);   // other quad of the half row
    v += pdpp<0x140>(v);   // other half of the row
    if (PG == 32) v = rowpair_sum(v);
    return v;
}

// group_sum of two independent values, their exchange stages interleaved
// (each value gets exactly the additions group_sum gives it).
template <int PG, typename T>
__device__ __forceinline__ void group_sum2(T& a, T& b) {
    a += pdpp<0xB1>(a);
    b += pdpp<0xB1>(b);
    a += pdpp<0x4E>(a);
    b += pdpp<0x4E>(b);
    a += pdpp<0x141>(a);
    b += pdpp<0x141>(b);
    a += pdpp<0x140>(a);
    b += pdpp<0x140>(b);
    if (PG == 32) rowpair_sum2(a, b);
}

// 1/sqrt(x) and 1/x from the hardware estimates with Newton steps: NS = 2
// reaches FP64 accuracy, NS = 1 about 2^-44 (enough when the results are
// rounded to FP32).
template <int NS>
__device__ __forceinline__ double prsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int i = 0; i < NS; ++i) y = y * (1.5 - 0.5 * x * y * y);
    return y;
}

__device__ __forceinline__ double prcp(double x) {
    double y = __builtin_amdgcn_rcp(x);
    return y * (2.0 - x * y);
}

// Rotation of a pair from alpha, beta, gamma (FP64): c, and s e = a + i b.
// Also returns t |gamma|, the amount that moves from ||x||^2 to ||y||^2.
struct PRot {
    double c, a, b, tg;
    bool on;
};

// The pair is rotated when |gamma|^2 > tol^2 alpha beta (and gamma != 0).
__device__ __forceinline__ bool prot_needed(double al, double be, double g2, double tol) {
    return g2 > (tol * tol) * al * be && g2 > 0.0;
}

// The rotation through d = beta - alpha and r = sqrt(d^2 + 4 |gamma|^2)
// rather than the cotangent zeta = d / (2 |gamma|): with D = |d| + r,
// t = sgn(d) 2 |gamma| / D, c = 1 / sqrt(1 + t^2) = D / sqrt(D^2 + 4 |gamma|^2)
// = D / sqrt(2 r D), s e = t c gamma / |gamma| = sgn(d) 2 c gamma / D and
// t |gamma| = sgn(d) 2 |gamma|^2 / D (sgn(0) = +1).  Nothing cancels (|d| and
// r are both >= 0), and only two reciprocal square roots and a reciprocal
// are needed, the last two independent of each other: a shorter dependent
// chain than through zeta.
template <typename T>
__device__ __forceinline__ PRot prot_params(double al, double be, double gr, double gi, double g2) {
    constexpr int NS = sizeof(T) == 4 ? 1 : 2;
    PRot r;
    const double d = be - al;
    const double q = d * d + 4.0 * g2;
    const double rq = q * prsqrt<NS>(q);
    const double D = fabs(d) + rq;
    const double iD = prcp(D);
    r.c = D * prsqrt<NS>(2.0 * rq * D);
    const double f = (d >= 0.0 ? 2.0 : -2.0) * iD;
    r.a = f * r.c * gr;
    r.b = f * r.c * gi;
    r.tg = f * g2;
    r.on = true;
    return r;
}

template <typename T>
__device__ __forceinline__ PRot prot(double al, double be, double gr, double gi, double tol) {
    const double g2 = gr * gr + gi * gi;
    if (!prot_needed(al, be, g2, tol)) return PRot{1.0, 0.0, 0.0, 0.0, false};
    return prot_params<T>(al, be, gr, gi, g2);
}

// Partial sums over the first K row groups (the slice rows; the V rows
// below them take part in the rotations only), as chains of fused
// multiply-adds.  The number of slice row
// groups ka is a runtime value: a uniform branch picks the unrolled
// instance, so no per-row select is needed.
template <typename T, int RPT, int K>
__device__ __forceinline__ void dot_first(const cplx<T> (&x)[RPT], const cplx<T> (&y)[RPT], T& gr, T& gi) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        gr = fma(x[k].re, y[k].re, gr);
        gr = fma(x[k].im, y[k].im, gr);
        gi = fma(x[k].re, y[k].im, gi);
        gi = fma(-x[k].im, y[k].re, gi);
    }
}

template <typename T, int RPT, int... K>
__device__ __forceinline__ void dot_rows(const cplx<T> (&x)[RPT], const cplx<T> (&y)[RPT], int ka, T& gr, T& gi,
                                         std::integer_sequence<int, K...>) {
    ((ka == K + 1 ? (dot_first<T, RPT, K + 1>(x, y, gr, gi), 0) : 0), ...);
}

template <typename T, int RPT, int K>
__device__ __forceinline__ T norm_first(const cplx<T> (&x)[RPT]) {
    T acc = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) acc += x[k].re * x[k].re + x[k].im * x[k].im;
    return acc;
}

template <typename T, int RPT, int... K>
__device__ __forceinline__ T norm_rows(const cplx<T> (&x)[RPT], int ka, std::integer_sequence<int, K...>) {
    T acc = 0;
    ((ka == K + 1 ? (acc = norm_first<T, RPT, K + 1>(x), 0) : 0), ...);
    return acc;
}

// Squared norm of the slice rows of a column held in registers (group sum
// in the element type, returned in FP64).
template <typename T, int PG, int RPT>
__device__ __forceinline__ double pnorm2(const cplx<T> (&x)[RPT], int ka) {
    const T acc = norm_rows<T, RPT>(x, ka, std::make_integer_sequence<int, RPT - 1>{});
    return (double)group_sum<PG>(acc);
}

// Device-coherent FP64 store and load (the Frobenius parts of a slice).
__device__ __forceinline__ void coh_store_f64(double* dst, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(dst), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double coh_load_f64(const double* src) {
    return __longlong_as_double((long long)__hip_atomic_load(reinterpret_cast<const unsigned long long*>(src),
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// The part of a slice's squared Frobenius norm (slice rows) held by the
// block pair in LDS (widths w0 and w1): per column slot g the squared norms
// of the two blocks' columns g, added over g in order.  Every thread returns
// the same value.  The Jacobi variants add the parts of a slice's block
// pairs of round 0 in pair order, so all of them derive the same rounding
// floor bit for bit.  Column slots past a block's width are not counted
// (they may hold an earlier block's column); with ZERO_PAST_WIDTH the caller
// guarantees that they hold zeros, and every slot is summed (adding an
// exact 0, so the value is the same).  scratch: BW doubles of LDS.
template <typename T, int PG, int RPT, int BW, bool ZERO_PAST_WIDTH = false>
__device__ __forceinline__ double pair_fro_part(const cplx<T>* blk0, const cplx<T>* blk1, int w0, int w1, int ldc,
                                                int ka, double* scratch) {
    const int g = threadIdx.x / PG, l = threadIdx.x - g * PG;
    cplx<T> c0[RPT], c1[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        c0[k] = blk0[g * ldc + l + PG * k];
        c1[k] = blk1[g * ldc + l + PG * k];
    }
    const double n0 = pnorm2<T, PG, RPT>(c0, ka), n1 = pnorm2<T, PG, RPT>(c1, ka);
    const double part = ZERO_PAST_WIDTH ? n0 + n1 : (g < w0 ? n0 : 0.0) + (g < w1 ? n1 : 0.0);
    if (l == 0) scratch[g] = part;
    __syncthreads();
    double sum = 0.0;
    for (int i = 0; i < BW; ++i) sum += scratch[i];
    __syncthreads();
    return sum;
}

// Orthogonalise column x (registers) against column y in LDS.  Lane l of
// the pair group holds rows l + PG k; the first ka row groups (1 <= ka < RPT)
// are slice rows, the rest V rows, padding rows are zero; only the slice rows
// take part in the test.  al and be are the squared norms of the slice rows,
// exact at the start of a round (or internal level) and tracked through it:
// on a rotation they are updated in place (al -= t|gamma|, be += t|gamma|).
// Returns 0 (not rotated), 1 (rotated) or 2 (rotated, and the rotation
// forces another sweep: rot_forces_sweep with the rounding floor floor2).
template <typename T, int PG, int RPT>
__device__ __forceinline__ unsigned ppair(cplx<T> (&x)[RPT], cplx<T>* y_lds, double& al, double& be, int ka,
                                          int l, double tol, double floor2 = 0.0) {
    cplx<T> y[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) y[k] = y_lds[l + PG * k];
    T gr = 0, gi = 0;
    dot_rows<T, RPT>(x, y, ka, gr, gi, std::make_integer_sequence<int, RPT - 1>{});
    group_sum2<PG>(gr, gi);
    const double dgr = (double)gr, dgi = (double)gi;
    const PRot rt = prot<T>(al, be, dgr, dgi, tol);
    if (!rt.on) return 0u;
    const unsigned code = rot_forces_sweep(al, be, dgr * dgr + dgi * dgi, tol, floor2) ? 2u : 1u;
    // y <- s e x + c y, then x <- c x - s conj(e) y in place (s e = a + i b):
    // the new y is formed and stored while the old x is still there, so the
    // loop-carried x needs no copies
    {
        const T c = (T)rt.c, a = (T)rt.a, b = (T)rt.b;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const cplx<T> yn{c * y[k].re + a * x[k].re - b * x[k].im, c * y[k].im + a * x[k].im + b * x[k].re};
            y_lds[l + PG * k] = yn;
            x[k].re = c * x[k].re - a * y[k].re - b * y[k].im;
            x[k].im = c * x[k].im - a * y[k].im + b * y[k].re;
        }
    }
    al -= rt.tg;
    be += rt.tg;
    return code;
}

// Cross steps wave to wave: a wave finishes step st + 1 only after its
// successor wave (cyclically) has finished step st, whose column it reads
// next; each wave counts its finished steps in LDS (release after its LDS
// writes, acquire before its reads).  Every wave of the workgroup runs every
// step, so the waits end; the bound only guards against a fault.
__device__ __forceinline__ void ring_publish(int* cnt, int value) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if ((threadIdx.x & 63) == 0) __hip_atomic_store(cnt, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void ring_wait(const int* cnt, int value) {
    for (int spins = 0; spins < (1 << 20); ++spins)
        if (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) >= value) return;
}

// LDS column of a block: slice rows 0..m-1 at 0..m-1, V rows at mp..mp+n-1
// (mp = m rounded up to PG), zeros elsewhere.  The NT threads split into
// BW column teams of NT / BW threads; a team copies one column, striding
// over its rows, eight independent loads in flight per thread (addresses
// clamped in range, so loads and stores need no branches), with no integer
// division.
// Complex values move as two-element vectors: a struct copy through a
// generic pointer can be lowered through a stack temporary.
template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));

template <typename T, int NT, int BW>
__device__ __forceinline__ void pcol_in(const cplx<T>* src_c, int len, cplx<T>* dst_c) {
    constexpr int TT = NT / BW;
    const vec2<T>* src = reinterpret_cast<const vec2<T>*>(src_c);
    vec2<T>* dst = reinterpret_cast<vec2<T>*>(dst_c);
    const int t = threadIdx.x % TT;
    for (int base = t; base < len; base += 8 * TT) {
#define TSVD_LD(u) const vec2<T> v##u = src[min(base + (u) * TT, len - 1)]
        TSVD_LD(0); TSVD_LD(1); TSVD_LD(2); TSVD_LD(3); TSVD_LD(4); TSVD_LD(5); TSVD_LD(6); TSVD_LD(7);
#undef TSVD_LD
        // rows past the end rewrite the last row with its own value: no branches
#define TSVD_ST(u) dst[min(base + (u) * TT, len - 1)] = v##u
        TSVD_ST(0); TSVD_ST(1); TSVD_ST(2); TSVD_ST(3); TSVD_ST(4); TSVD_ST(5); TSVD_ST(6); TSVD_ST(7);
#undef TSVD_ST
    }
}

template <typename T, int NT, int BW>
__device__ __forceinline__ void pcol_out(const cplx<T>* src_c, int len, cplx<T>* dst_c) {
    constexpr int TT = NT / BW;
    const vec2<T>* src = reinterpret_cast<const vec2<T>*>(src_c);
    vec2<T>* dst = reinterpret_cast<vec2<T>*>(dst_c);
    for (int r = threadIdx.x % TT; r < len; r += TT) dst[r] = src[r];
}

// Device-coherent copies: relaxed agent-scope atomic loads and stores, which
// the hardware serves at the device's coherence point (never from a stale
// L2 line of another XCD).  Used by workgroups that exchange blocks through
// global memory inside one launch, so that no L2 write-back or invalidation
// is needed around the exchange.
template <typename T>
__device__ __forceinline__ void coh_copy_in(const cplx<T>* src, cplx<T>* dst);

template <>
__device__ __forceinline__ void coh_copy_in<float>(const cplx<float>* src, cplx<float>* dst) {
    const unsigned long long u = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(src),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *reinterpret_cast<unsigned long long*>(dst) = u;
}

template <>
__device__ __forceinline__ void coh_copy_in<double>(const cplx<double>* src, cplx<double>* dst) {
    const unsigned long long* s = reinterpret_cast<const unsigned long long*>(src);
    unsigned long long* d = reinterpret_cast<unsigned long long*>(dst);
    const unsigned long long a = __hip_atomic_load(s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long b = __hip_atomic_load(s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    d[0] = a;
    d[1] = b;
}

template <typename T>
__device__ __forceinline__ void coh_copy_out(const cplx<T>* src, cplx<T>* dst);

template <>
__device__ __forceinline__ void coh_copy_out<float>(const cplx<float>* src, cplx<float>* dst) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(dst), *reinterpret_cast<const unsigned long long*>(src),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <>
__device__ __forceinline__ void coh_copy_out<double>(const cplx<double>* src, cplx<double>* dst) {
    const unsigned long long* s = reinterpret_cast<const unsigned long long*>(src);
    unsigned long long* d = reinterpret_cast<unsigned long long*>(dst);
    __hip_atomic_store(d, s[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(d + 1, s[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ cplx<T> coh_load(const cplx<T>* src) {
    cplx<T> v;
    coh_copy_in<T>(src, &v);
    return v;
}

// Eight coherent loads in flight per thread (addresses clamped in range;
// rows past the end rewrite the last row with its own value).
template <typename T, int NT, int BW>
__device__ __forceinline__ void ccol_in(const cplx<T>* src, int len, cplx<T>* dst_c) {
    constexpr int TT = NT / BW;
    vec2<T>* dst = reinterpret_cast<vec2<T>*>(dst_c);
    const int t = threadIdx.x % TT;
    for (int base = t; base < len; base += 8 * TT) {
#define TSVD_LD(u) const cplx<T> v##u = coh_load<T>(src + min(base + (u) * TT, len - 1))
        TSVD_LD(0); TSVD_LD(1); TSVD_LD(2); TSVD_LD(3); TSVD_LD(4); TSVD_LD(5); TSVD_LD(6); TSVD_LD(7);
#undef TSVD_LD
#define TSVD_ST(u) dst[min(base + (u) * TT, len - 1)] = vec2<T>{v##u.re, v##u.im}
        TSVD_ST(0); TSVD_ST(1); TSVD_ST(2); TSVD_ST(3); TSVD_ST(4); TSVD_ST(5); TSVD_ST(6); TSVD_ST(7);
#undef TSVD_ST
    }
}

template <typename T, int NT, int BW>
__device__ __forceinline__ void ccol_out(const cplx<T>* src, int len, cplx<T>* dst) {
    constexpr int TT = NT / BW;
    for (int r = threadIdx.x % TT; r < len; r += TT) coh_copy_out<T>(src + r, dst + r);
}

// Block blk of a slice (A: m x n, V: n x n, column-major) to / from LDS;
// COH selects the device-coherent copies.
template <typename T, int NT, int BW, bool COH = false>
__device__ __forceinline__ void load_block(const cplx<T>* A, const cplx<T>* V, int m, int n, int nb, int blk,
                                           int mp, int ldc, cplx<T>* lds) {
    const int c0 = pblk_start(blk, n, nb), w = pblk_start(blk + 1, n, nb) - c0;
    const int c = threadIdx.x / (NT / BW);
    if (c < w) {
        if (COH) {
            ccol_in<T, NT, BW>(A + (int64_t)(c0 + c) * m, m, lds + c * ldc);
            ccol_in<T, NT, BW>(V + (int64_t)(c0 + c) * n, n, lds + c * ldc + mp);
        } else {
            pcol_in<T, NT, BW>(A + (int64_t)(c0 + c) * m, m, lds + c * ldc);
            pcol_in<T, NT, BW>(V + (int64_t)(c0 + c) * n, n, lds + c * ldc + mp);
        }
    }
}

// Block blk into LDS with all of a lane's loads in flight before its first
// LDS store (one memory round trip per block): pair group c (PG lanes) takes
// column c, lane t the stacked rows t + PG r (slice rows below m, V rows
// from mp), one address and one predicate per row.  The FP32 block-pair
// kernel takes its incoming blocks with it between rounds (the 64-problem
// batch 3% faster than with the per-segment copies); in FP64 the unrolled
// rows take too many registers, and in the one-workgroup-per-slice kernel
// it brought no clear gain for many more scalar spills.
template <typename T, int PG, int RPT, bool COH>
__device__ __forceinline__ void load_block_rows(const cplx<T>* A, const cplx<T>* V, int m, int n, int nb, int blk,
                                                int mp, int ldc, cplx<T>* lds) {
    const int c = threadIdx.x / PG, t = threadIdx.x - c * PG;
    const int c0 = pblk_start(blk, n, nb);
    const int col = c < pblk_start(blk + 1, n, nb) - c0 ? c0 + c : -1;
    cplx<T> v[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int R = t + PG * r;
        if (col >= 0 && (R < m || (R >= mp && R - mp < n))) {
            const cplx<T>* p = R < m ? A + (int64_t)col * m + R : V + (int64_t)col * n + (R - mp);
            if constexpr (COH) v[r] = coh_load<T>(p);
            else v[r] = *p;
        }
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int R = t + PG * r;
        if (col >= 0 && (R < m || (R >= mp && R - mp < n))) lds[c * ldc + R] = v[r];
    }
}

// Block blk into LDS: load_block_rows in FP32, the per-segment copies
// (load_block) in FP64.
template <typename T, int PG, int RPT, int BW, bool COH = false>
__device__ __forceinline__ void load_block_any(const cplx<T>* A, const cplx<T>* V, int m, int n, int nb, int blk,
                                               int mp, int ldc, cplx<T>* lds) {
    if constexpr (sizeof(T) == 4)
        load_block_rows<T, PG, RPT, COH>(A, V, m, n, nb, blk, mp, ldc, lds);
    else
        load_block<T, BW * PG, BW, COH>(A, V, m, n, nb, blk, mp, ldc, lds);
}

template <typename T, int NT, int BW, bool COH = false>
__device__ __forceinline__ void store_block(cplx<T>* A, cplx<T>* V, int m, int n, int nb, int blk, int mp,
                                            int ldc, const cplx<T>* lds) {
    const int c0 = pblk_start(blk, n, nb), w = pblk_start(blk + 1, n, nb) - c0;
    const int c = threadIdx.x / (NT / BW);
    if (c < w) {
        if (COH) {
            ccol_out<T, NT, BW>(lds + c * ldc, m, A + (int64_t)(c0 + c) * m);
            ccol_out<T, NT, BW>(lds + c * ldc + mp, n, V + (int64_t)(c0 + c) * n);
        } else {
            pcol_out<T, NT, BW>(lds + c * ldc, m, A + (int64_t)(c0 + c) * m);
            pcol_out<T, NT, BW>(lds + c * ldc + mp, n, V + (int64_t)(c0 + c) * n);
        }
    }
}

}  // namespace jac
}  // namespace tsvd
