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

template <int CTRL>
__device__ __forceinline__ double pdpp(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double preadlane(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the PG lanes of a pair group; every lane of the group gets the
// same value.  16 lanes = one DPP row; 32 lanes = two rows combined through
// readlane in a fixed order.
template <int PG>
__device__ __forceinline__ double group_sum(double v) {
    v += pdpp<0xB1>(v);    // lane ^ 1
    v += pdpp<0x4E>(v);    // lane ^ 2
    v += pdpp<0x141>(v);   // other quad of the half row
    v += pdpp<0x140>(v);   // other half of the row
    if (PG == 32) {
        const double lo = preadlane(v, 0) + preadlane(v, 16);
        const double hi = preadlane(v, 32) + preadlane(v, 48);
        v = (__lane_id() < 32) ? lo : hi;
    }
    return v;
}

__device__ __forceinline__ double prsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * (1.5 - 0.5 * x * y * y);
    y = y * (1.5 - 0.5 * x * y * y);
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

__device__ __forceinline__ PRot prot(double al, double be, double gr, double gi, double tol) {
    PRot r{1.0, 0.0, 0.0, 0.0, false};
    const double g2 = gr * gr + gi * gi;
    if (!(g2 > (tol * tol) * al * be) || !(g2 > 0.0)) return r;
    const double rg = prsqrt(g2);
    const double zeta = (be - al) * 0.5 * rg;
    const double q = 1.0 + zeta * zeta;
    const double t = prcp(fabs(zeta) + q * prsqrt(q));
    const double ts = zeta >= 0.0 ? t : -t;
    r.c = prsqrt(1.0 + ts * ts);
    const double s = r.c * ts;
    r.a = s * (gr * rg);
    r.b = s * (gi * rg);
    r.tg = ts * (g2 * rg);
    r.on = true;
    return r;
}

// x <- c x - s conj(e) y,  y <- s e x + c y   with s e = a + i b
template <typename T>
__device__ __forceinline__ void prot_apply(const PRot& rd, cplx<T>& x, cplx<T>& y) {
    const T c = (T)rd.c, a = (T)rd.a, b = (T)rd.b;
    const cplx<T> xn{c * x.re - a * y.re - b * y.im, c * x.im - a * y.im + b * y.re};
    const cplx<T> yn{c * y.re + a * x.re - b * x.im, c * y.im + a * x.im + b * x.re};
    x = xn;
    y = yn;
}

// Squared norm of the slice rows of a column held in registers.
template <typename T, int PG, int RPT>
__device__ __forceinline__ double pnorm2(const cplx<T> (&x)[RPT], int ka) {
    T acc = 0;
#pragma unroll
    for (int k = 0; k < RPT; ++k)
        if (k < ka) acc += x[k].re * x[k].re + x[k].im * x[k].im;
    return group_sum<PG>((double)acc);
}

// Orthogonalise column x (registers, squared norm al) against column y in
// LDS (squared norm be).  Lane l of the pair group holds rows l + PG k; the
// first ka row groups are slice rows, the rest V rows, padding rows are zero.
// On a rotation the norms are updated in place (al -= t|gamma|, be += t|gamma|).
template <typename T, int PG, int RPT>
__device__ __forceinline__ bool ppair(cplx<T> (&x)[RPT], cplx<T>* y_lds, double& al, double& be, int ka,
                                      int l, double tol) {
    cplx<T> y[RPT];
    T gr = 0, gi = 0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        y[k] = y_lds[l + PG * k];
        if (k < ka) {
            gr += x[k].re * y[k].re + x[k].im * y[k].im;
            gi += x[k].re * y[k].im - x[k].im * y[k].re;
        }
    }
    const PRot rt = prot(al, be, group_sum<PG>((double)gr), group_sum<PG>((double)gi), tol);
    if (!rt.on) return false;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        prot_apply(rt, x[k], y[k]);
        y_lds[l + PG * k] = y[k];
    }
    al -= rt.tg;
    be += rt.tg;
    return true;
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

// Block blk of a slice (A: m x n, V: n x n, column-major) to / from LDS.
template <typename T, int NT, int BW>
__device__ __forceinline__ void load_block(const cplx<T>* A, const cplx<T>* V, int m, int n, int nb, int blk,
                                           int mp, int ldc, cplx<T>* lds) {
    const int c0 = pblk_start(blk, n, nb), w = pblk_start(blk + 1, n, nb) - c0;
    const int c = threadIdx.x / (NT / BW);
    if (c < w) {
        pcol_in<T, NT, BW>(A + (int64_t)(c0 + c) * m, m, lds + c * ldc);
        pcol_in<T, NT, BW>(V + (int64_t)(c0 + c) * n, n, lds + c * ldc + mp);
    }
}

template <typename T, int NT, int BW>
__device__ __forceinline__ void store_block(cplx<T>* A, cplx<T>* V, int m, int n, int nb, int blk, int mp,
                                            int ldc, const cplx<T>* lds) {
    const int c0 = pblk_start(blk, n, nb), w = pblk_start(blk + 1, n, nb) - c0;
    const int c = threadIdx.x / (NT / BW);
    if (c < w) {
        pcol_out<T, NT, BW>(lds + c * ldc, m, A + (int64_t)(c0 + c) * m);
        pcol_out<T, NT, BW>(lds + c * ldc + mp, n, V + (int64_t)(c0 + c) * n);
    }
}

}  // namespace jac
}  // namespace tsvd
