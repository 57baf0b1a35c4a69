// Persistent one-sided Jacobi SVD: one launch runs every sweep
// of every Fourier slice (same method, ordering and stopping rule as the
// per-round kernels in jacobi.hip, which remain the path for shapes that do
// not fit this one).
//
// Layout.  Slice s gets G = nb/2 workgroups; workgroup p holds the blocks at
// tournament positions p and nb-1-p in LDS (two BW-column blocks of stacked
// columns: m slice rows, then n rows of V).  A round of the block tournament
// orthogonalises the two resident blocks against each other; between rounds
// every block except the one at position 0 moves to the next position
// (circle method), so a workgroup writes its moving blocks back to their
// home columns in global memory, meets the other workgroups of its slice at
// a barrier, and reads the blocks of its next positions.  The first round of
// every sweep also orthogonalises each block internally.
//
// Work split.  A column pair is handled by a group of PG = 32 lanes (two DPP
// rows), so a 512-thread workgroup (two waves per SIMD) works on BW = 16
// pairs per step; each lane holds rows lane + 32 k of its columns, the
// cross product is reduced with DPP and readlane, and the rotation
// parameters are computed per group in FP64.  Column norms are computed
// exactly at the start of every round and tracked through the rotations of
// the round (a rotation moves t |gamma| from one squared norm to the other).
//
// Synchronisation.  Blocks travel through global memory with device-
// coherent stores and loads.  Within a sweep, a workgroup that has written a
// block waits for the stores to complete and then sets the block's flag to
// the index of the round that takes it next; a workgroup waits only on the
// flags of the two blocks it takes next.  At the end of a sweep all
// workgroups of the slice meet at a counter barrier (the stopping decision
// needs every workgroup's rotation flag).
//
// Residency.  A workgroup takes its role (slice, block pair) from a ticket
// counter when it starts, so the roles of the workgroups running at any time
// are the lowest ones not yet finished: the workgroups of a slice wait only
// for workgroups that are running or will start as soon as others finish.
// The grid holds at most one workgroup per CU, so on an otherwise idle
// device every workgroup is resident at once; under concurrent work the
// slices finish in ticket order.  Every wait between workgroups is bounded
// (PersistArgs.spin_limit polls): a wait that gives up sets bit 1 of the
// error word, and every workgroup that meets the error word at its next wait
// writes its resident blocks home and stops.  Each block is held by one workgroup at a
// time and every rotation is applied to the slice rows and the V rows
// together, so W = A V still holds for the partly rotated slices; the caller
// then finishes the SVD with the one-workgroup-per-slice kernel.
//
// Convergence: workgroups OR a per-slice flag when a rotation of the sweep
// forces another sweep (rot_forces_sweep); after the sweep's last barrier all
// workgroups of the slice read the same flag and stop together when it is
// clear.  The rounding floor of that test needs the slice's Frobenius norm:
// each workgroup writes the part of its two starting blocks, and the
// workgroups of a slice meet once before the first sweep, after which every
// one adds the same parts in the same order.

#include "jacobi_common.h"

#include <algorithm>

namespace tsvd {

namespace {

using namespace jac;

constexpr int PBW = 16;   // columns per block = pairs per step

template <typename T, int NT>
__device__ void pload_block(const JacArgs<T>& a, int s, int blk, int mp, int ldc, cplx<T>* lds) {
    load_block<T, NT, PBW, true>(a.A + (int64_t)s * a.n * a.m, a.V + (int64_t)s * a.n * a.n, a.m, a.n, a.nb, blk,
                                 mp, ldc, lds);
}

// The blocks blk0 and blk1 (-1: none) into LDS.  Up to 10 rows per lane
// every load is in flight before the first LDS store, one memory round trip
// for both blocks, slice and V rows, instead of one per block and row
// segment, with one address and one predicate per row (a select between
// the slice and the V part): +2.9% iterations/s in the FP32 form and +4.5%
// in FP64 on the video shape (9 rows per lane).  Wider columns keep the
// earlier loaders, which hold fewer registers: FP64 the combined loader with
// a branch per row segment, FP32 the per-block loads (the combined loaders
// double the wide FP32 kernels' scalar register spills).  Reading both
// blocks from LDS before the first store of an exchange was 5% slower, so
// the stores stay per block.  Thread team c (PG lanes) takes column c of
// each block, lane t the stacked rows t + PG r: slice rows below m, V rows
// from mp (the padding rows between stay zero).
template <typename T, int PG, int RPT>
__device__ __forceinline__ void pload_pair(const JacArgs<T>& a, int s, int mp, int ldc, int blk0, cplx<T>* lds0,
                                           int blk1, cplx<T>* lds1) {
    if constexpr (sizeof(T) == 4 && RPT > 10) {
        constexpr int NT = PBW * PG;
        if (blk0 >= 0) pload_block<T, NT>(a, s, blk0, mp, ldc, lds0);
        if (blk1 >= 0) pload_block<T, NT>(a, s, blk1, mp, ldc, lds1);
        return;
    }
    const int c = threadIdx.x / PG, t = threadIdx.x - c * PG;
    const cplx<T>* const A = a.A + (int64_t)s * a.n * a.m;
    const cplx<T>* const V = a.V + (int64_t)s * a.n * a.n;
    const int m = a.m, n = a.n;
    auto col = [&](int blk) {
        if (blk < 0) return -1;
        const int c0 = pblk_start(blk, n, a.nb);
        return c < pblk_start(blk + 1, n, a.nb) - c0 ? c0 + c : -1;
    };
    const int col0 = col(blk0), col1 = col(blk1);
    if constexpr (RPT <= 10) {
        auto addr = [&](int cl, int R) {
            return R < m ? A + (int64_t)cl * m + R : V + (int64_t)cl * n + (R - mp);
        };
        auto live = [&](int cl, int R) { return cl >= 0 && (R < m || (R >= mp && R - mp < n)); };
        cplx<T> v0[RPT], v1[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int R = t + PG * r;
            if (live(col0, R)) v0[r] = coh_load<T>(addr(col0, R));
            if (live(col1, R)) v1[r] = coh_load<T>(addr(col1, R));
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int R = t + PG * r;
            if (live(col0, R)) lds0[c * ldc + R] = v0[r];
            if (live(col1, R)) lds1[c * ldc + R] = v1[r];
        }
        return;
    }
    cplx<T> v0[RPT], v1[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int R = t + PG * r;
        if (col0 >= 0) {
            if (R < m)
                v0[r] = coh_load<T>(A + (int64_t)col0 * m + R);
            else if (R >= mp && R - mp < n)
                v0[r] = coh_load<T>(V + (int64_t)col0 * n + (R - mp));
        }
        if (col1 >= 0) {
            if (R < m)
                v1[r] = coh_load<T>(A + (int64_t)col1 * m + R);
            else if (R >= mp && R - mp < n)
                v1[r] = coh_load<T>(V + (int64_t)col1 * n + (R - mp));
        }
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int R = t + PG * r;
        const bool row = R < m || (R >= mp && R - mp < n);
        if (col0 >= 0 && row) lds0[c * ldc + R] = v0[r];
        if (col1 >= 0 && row) lds1[c * ldc + R] = v1[r];
    }
}

template <typename T, int NT>
__device__ void pstore_block(const JacArgs<T>& a, int s, int blk, int mp, int ldc, const cplx<T>* lds) {
    store_block<T, NT, PBW, true>(a.A + (int64_t)s * a.n * a.m, a.V + (int64_t)s * a.n * a.n, a.m, a.n, a.nb, blk,
                                  mp, ldc, lds);
}

// Slice barrier: returns false if the bounded wait ran out.
//
// The blocks travel through global memory with device-coherent (relaxed
// agent-scope atomic) loads and stores, so the barrier needs no L2
// write-back or invalidation: every wave waits until its own stores are
// complete at the coherence point, the workgroup meets at s_barrier, and
// thread 0 counts the arrival and waits for the other workgroups of the
// slice; the next blocks are read only after that (loads are issued in
// program order).
__device__ bool slice_barrier(int* counter, int target, int* err, int spin_limit) {
    __shared__ int ok;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        ok = 1;
        __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            // another workgroup gave up: stop waiting at once
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                ++spins > spin_limit) {
                __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
    }
    __syncthreads();
    return ok != 0;
}

// Bounded wait (thread 0) until a block flag reaches `value`; false if the
// wait ran out or another workgroup gave up.
__device__ bool wait_flag(int* flag, int value, int* err, int spin_limit) {
    int spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < value) {
        __builtin_amdgcn_s_sleep(1);
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > spin_limit) {
            __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

// Cross steps of a round, wave to wave: wave w finishes step st + 1 only
// after reading what wave w + 1 (cyclically) wrote at step st, and nothing
// else.  Each wave counts its finished steps in LDS (release after its LDS
// writes); a wave waits for its successor's count (acquire) instead of a
// workgroup barrier, so a step costs the waves' average rather than the
// slowest pair.  Every wave of the workgroup runs every step of a round
// (giving up happens only between rounds), so a wait lasts at most a few
// steps.  One that runs far longer means a fault: the wave stops waiting
// and sets the error word to 2, which fails the call (the block data can no
// longer be trusted); it checks the error word every 1024 polls, so after
// such a fault no wait spins to its cap again.
__device__ __forceinline__ void lds_publish(int* cnt, int value) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if ((threadIdx.x & 63) == 0) __hip_atomic_store(cnt, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Polls back to back (a sleep between polls cost 0.7% of the iteration);
// 2^18 LDS polls are milliseconds, far beyond any step of a workgroup's own
// waves, and 1024 polls tens of microseconds, tens of steps.
constexpr int kLdsSpinLimit = 1 << 18;

__device__ __forceinline__ void lds_wait(const int* cnt, int value, int* err) {
    int spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < value) {
        ++spins;
        if (spins > kLdsSpinLimit) {
            __hip_atomic_store(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        if ((spins & 1023) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            __hip_atomic_store(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
    }
}

}  // namespace

template <typename T, int PG, int RPT>
__global__ __launch_bounds__(PBW * PG) void jacobi_persistent_kernel(JacArgs<T> a, PersistArgs p) {
    constexpr int NT = PBW * PG;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int rot_any;
    __shared__ int stop;
    __shared__ int ok_flag;
    __shared__ double jnorm[PBW];
    __shared__ double inorm[2 * PBW];   // internal phase: tracked norms of both blocks' columns
    __shared__ int wsteps[NT / 64];   // pair steps finished per wave, over the whole launch
    __shared__ int role;
    if (a.ctrl && a.ctrl->done) return;
    const int G = a.nb / 2;
    // the int words of the launch: h barrier counters, 3h sweep flags, the
    // error word, the role ticket, h x nb block flags
    int* const rotflag = p.pbar + a.h;
    int* const err = p.pbar + 4 * a.h;
    if (threadIdx.x == 0) role = __hip_atomic_fetch_add(err + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    // uniform across the workgroup: keep it (and what derives from it) scalar
    const int rl = __builtin_amdgcn_readfirstlane(role);
    const int s = rl / G, wg = rl - s * G;
    if (s >= a.h) return;
    const int ka = (a.m + PG - 1) / PG;   // row groups holding slice rows
    const int mp = ka * PG;
    // column stride: the padded stacked column plus one element, so the pair
    // groups of a wavefront read different LDS banks
    const int ldc = PG * RPT + 1;
    cplx<T>* const blk0 = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* const blk1 = blk0 + (size_t)PBW * ldc;
    const int pos0 = wg, pos1 = a.nb - 1 - wg;
    const int g = threadIdx.x / PG, l = threadIdx.x - g * PG;
    const double tol = (double)a.tol;
    int* counter = p.pbar + s;
    int arrivals = 0;

    // zero both blocks once: padding rows stay zero under every rotation
    for (int idx = threadIdx.x; idx < 2 * PBW * ldc; idx += NT) blk0[idx] = cplx<T>{(T)0, (T)0};
    const int wave = threadIdx.x >> 6, wave_next = (wave + 1) % (NT / 64);
    if ((threadIdx.x & 63) == 0) wsteps[wave] = 0;
    int steps = 0;   // cross steps finished by every wave before the current round
    __syncthreads();
    int player0 = ppos_player(pos0, 0, a.nb), player1 = ppos_player(pos1, 0, a.nb);
    pload_pair<T, PG, RPT>(a, s, mp, ldc, player0, blk0, player1, blk1);
    if (wg == 0 && threadIdx.x == 0) a.sweeps[s] = 0;
    __syncthreads();

    unsigned nrot_total = 0;
    int swept = 0;   // sweeps started (kept by wg 0, thread 0)
    bool alive = true;
    // resident blocks still to be written home when the sweeps end: both at
    // the sweep cap; after a stop or a give-up, only those that did not move
    // (the moving ones were written before the exchange)
    bool home0 = true, home1 = true;
    double floor2 = 0.0;   // rounding floor of rot_forces_sweep
    if (p.floor_scale > 0.0) {
        // the slots past a block's width were zeroed before the first load
        const double part = pair_fro_part<T, PG, RPT, PBW, true>(blk0, blk1, PBW, PBW, ldc, ka, inorm);
        if (threadIdx.x == 0) coh_store_f64(p.fro + (int64_t)s * G + wg, part);
        arrivals += G;
        if (!slice_barrier(counter, arrivals, err, p.spin_limit)) {
            alive = false;   // giving up before any rotation: both blocks are still home
        } else {
            if (threadIdx.x == 0) {
                double fro2 = 0.0;
                for (int i = 0; i < G; ++i) fro2 += coh_load_f64(p.fro + (int64_t)s * G + i);
                inorm[0] = p.floor_scale * fro2;
            }
            __syncthreads();
            floor2 = inorm[0];
            __syncthreads();
        }
    }
    for (int sweep = 0; sweep < p.max_sweeps && alive; ++sweep) {
        if (threadIdx.x == 0) rot_any = 0;
        if (wg == 0 && threadIdx.x == 0) {
            // read by every workgroup of the slice: a device-coherent store
            __hip_atomic_store(rotflag + ((sweep + 1) % 3) * a.h + s, 0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            a.sweeps[s] = sweep + 1;
            swept = sweep + 1;
        }
        __syncthreads();
        unsigned nrot = 0, nbig = 0;   // rotations of the sweep; those that force another sweep
        {
            // Internal pairs of both resident blocks (groups 0-7 take block 0,
            // groups 8-15 block 1) by halving: the 8 x 8 cross pairs of the
            // block's two halves, then the 4 x 4 cross pairs within each half,
            // then 2 x 2, then the 8 adjacent pairs -- 15 steps, every pair once.
            // Each level runs like a cross round: a group keeps its column of
            // the first half of its subproblem in registers and meets the k
            // columns of the second half, norms exact at the level's start and
            // tracked through it, and a wave waits only for the wave whose
            // previous step wrote the column it takes next.
            const bool second = g >= PBW / 2;
            const int gi = second ? g - PBW / 2 : g;
            const int pl = second ? player1 : player0;
            cplx<T>* const base = second ? blk1 : blk0;
            double* const jn = inorm + (second ? PBW : 0);
            const int w = pblk_start(pl + 1, a.n, a.nb) - pblk_start(pl, a.n, a.nb);
            const int wl = wave & 3, wbase = wave & ~3;   // waves 0-3 hold block 0, 4-7 block 1
            for (int k = PBW / 2; k >= 1; k /= 2) {
                const int sp = gi / k, q = gi - sp * k;
                const int xcol = 2 * k * sp + q, ybase = 2 * k * sp + k;
                // the wave holding group (q + 1) mod k of this subproblem
                const int wnext = k == 8 ? wbase + ((wl + 1) & 3) : (k == 4 ? wave ^ 1 : wave);
                cplx<T> xr[RPT];
#pragma unroll
                for (int r = 0; r < RPT; ++r) xr[r] = base[xcol * ldc + l + PG * r];
                double al = pnorm2<T, PG, RPT>(xr, ka);
                {
                    cplx<T> yr[RPT];
#pragma unroll
                    for (int r = 0; r < RPT; ++r) yr[r] = base[(ybase + q) * ldc + l + PG * r];
                    const double bq = pnorm2<T, PG, RPT>(yr, ka);
                    if (l == 0) jn[ybase + q] = bq;
                }
                __syncthreads();
                for (int st = 0; st < k; ++st) {
                    if (st > 0) lds_wait(wsteps + wnext, steps + st, err);
                    const int ycol = ybase + ((q + st) & (k - 1));
                    if (xcol < w && ycol < w) {
                        double be = jn[ycol];
                        if (const unsigned code = ppair<T, PG, RPT>(xr, base + ycol * ldc, al, be, ka, l, tol, floor2)) {
                            ++nrot;
                            nbig += code >> 1;
                            if (l == 0) jn[ycol] = be;
                        }
                    }
                    lds_publish(wsteps + wave, steps + st + 1);
                }
                steps += k;
                if (xcol < w) {
#pragma unroll
                    for (int r = 0; r < RPT; ++r) base[xcol * ldc + l + PG * r] = xr[r];
                }
                __syncthreads();
            }
        }
        for (int rd = 0; rd < a.nb - 1; ++rd) {
            // cross pairs: column g of block 0 (registers) meets every column of block 1
            const int wi = pblk_start(player0 + 1, a.n, a.nb) - pblk_start(player0, a.n, a.nb);
            const int wj = pblk_start(player1 + 1, a.n, a.nb) - pblk_start(player1, a.n, a.nb);
            cplx<T> xi[RPT];
#pragma unroll
            for (int k = 0; k < RPT; ++k) xi[k] = blk0[g * ldc + l + PG * k];
            // exact squared norms at the start of the round, tracked within it
            double al = pnorm2<T, PG, RPT>(xi, ka);
            {
                cplx<T> yj[RPT];
#pragma unroll
                for (int k = 0; k < RPT; ++k) yj[k] = blk1[g * ldc + l + PG * k];
                const double bj = pnorm2<T, PG, RPT>(yj, ka);
                if (l == 0) jnorm[g] = bj;
            }
            __syncthreads();
            // step st: group g meets column (g + st) mod PBW of block 1, which
            // group g + 1 met at step st - 1
            for (int st = 0; st < PBW; ++st) {
                if (st > 0) lds_wait(wsteps + wave_next, steps + st, err);
                const int jc = (g + st) & (PBW - 1);
                if (g < wi && jc < wj) {
                    double be = jnorm[jc];
                    if (const unsigned code = ppair<T, PG, RPT>(xi, blk1 + jc * ldc, al, be, ka, l, tol, floor2)) {
                        ++nrot;
                        nbig += code >> 1;
                        if (l == 0) jnorm[jc] = be;
                    }
                }
                lds_publish(wsteps + wave, steps + st + 1);
            }
            steps += PBW;
            __syncthreads();
            if (g < wi) {
#pragma unroll
                for (int k = 0; k < RPT; ++k) blk0[g * ldc + l + PG * k] = xi[k];
            }
            // end of the sweep: publish whether this workgroup needs another sweep
            const bool last = rd == a.nb - 2;
            if (last) {
                if (nbig && l == 0) rot_any = 1;
                __syncthreads();
                if (threadIdx.x == 0 && rot_any)
                    __hip_atomic_fetch_or(rotflag + (sweep % 3) * a.h + s, 1, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
            }
            // the next round's players (after the last round: round 0 of the next sweep)
            const int nr = (rd + 1) % (a.nb - 1);
            const int next0 = ppos_player(pos0, nr, a.nb), next1 = ppos_player(pos1, nr, a.nb);
            __syncthreads();
            if (next0 != player0) pstore_block<T, NT>(a, s, player0, mp, ldc, blk0);
            if (next1 != player1) pstore_block<T, NT>(a, s, player1, mp, ldc, blk1);
            if (last) {
                // end of the sweep: every workgroup of the slice meets, then all
                // read the same rotation flag and stop together when it is clear
                arrivals += G;
                if (!slice_barrier(counter, arrivals, err, p.spin_limit)) {
                    home0 = next0 == player0;   // giving up
                    home1 = next1 == player1;
                    alive = false;
                    break;
                }
                if (threadIdx.x == 0) stop = __hip_atomic_load(rotflag + (sweep % 3) * a.h + s,
                                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
                __syncthreads();
                if (stop) {
                    home0 = next0 == player0;   // converged
                    home1 = next1 == player1;
                    alive = false;
                    break;
                }
            } else {
                // within a sweep: publish the blocks written (ready for round R + 1)
                // and wait only for the two blocks this workgroup takes next
                const int R = sweep * (a.nb - 1) + rd;
                int* const bf = err + 2 + s * a.nb;
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (threadIdx.x == 0) {
                    ok_flag = 1;
                    if (next0 != player0) __hip_atomic_store(bf + player0, R + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (next1 != player1) __hip_atomic_store(bf + player1, R + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((next0 != player0 && !wait_flag(bf + next0, R + 1, err, p.spin_limit)) ||
                        (next1 != player1 && !wait_flag(bf + next1, R + 1, err, p.spin_limit)))
                        ok_flag = 0;
                }
                __syncthreads();
                if (!ok_flag) {
                    home0 = next0 == player0;   // giving up
                    home1 = next1 == player1;
                    alive = false;
                    break;
                }
            }
            pload_pair<T, PG, RPT>(a, s, mp, ldc, next0 != player0 ? next0 : -1, blk0,
                                   next1 != player1 ? next1 : -1, blk1);
            player0 = next0;
            player1 = next1;
            __syncthreads();
        }
        nrot_total += nrot;
    }
    __syncthreads();
    if (home0) pstore_block<T, NT>(a, s, player0, mp, ldc, blk0);
    if (home1) pstore_block<T, NT>(a, s, player1, mp, ldc, blk1);
    if (l == 0 && nrot_total) atomicAdd(a.rotations, (unsigned long long)nrot_total);
    if (a.ctrl && swept) atomicMax(&a.ctrl->sweep_max, swept);
}

// ------------------------------------------------------------------ host

namespace {

constexpr int kPG = 32;   // lanes per pair: 512-thread workgroups, two waves per SIMD

// row groups of PG per stacked column: slice rows and V rows each padded to PG
int persist_rpt(int m, int n) {
    const int need = (m + kPG - 1) / kPG + (n + kPG - 1) / kPG;
    for (int r : {2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 14, 16, 20})
        if (r >= need) return r;
    return -1;
}

size_t persist_lds(int rpt, int elem_bytes) { return 2 * (size_t)PBW * (kPG * rpt + 1) * 2 * elem_bytes; }

template <typename T, int RPT>
hipError_t launch_persist_t(const JacArgs<T>& a, const PersistArgs& p, size_t lds, hipStream_t st, int cus) {
    auto* fn = jacobi_persistent_kernel<T, kPG, RPT>;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, PBW * kPG, lds);
    if (e != hipSuccess) return e;
    const int grid = a.h * (a.nb / 2);
    if ((int64_t)per_cu * cus < grid) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(PBW * kPG), lds, st, a, p);
    return hipGetLastError();
}

}  // namespace

int jacobi_persistent_blocks(int n) { return jacobi_num_blocks(n, PBW); }

bool jacobi_persistent_fits(int m, int n, int h, int elem_bytes, int cus, size_t lds_cap) {
    const int rpt = persist_rpt(m, n);
    if (rpt < 0 || n < 2) return false;
    if (persist_lds(rpt, elem_bytes) + 256 > lds_cap) return false;
    const int64_t grid = (int64_t)h * (jacobi_persistent_blocks(n) / 2);
    return grid <= (int64_t)cus;   // one workgroup per CU is always resident
}

template <typename T>
hipError_t launch_jacobi_persistent(const JacArgs<T>& a, const PersistArgs& p, int cus, hipStream_t st) {
    const int rpt = persist_rpt(a.m, a.n);
    size_t lds = persist_lds(rpt, sizeof(T));
    if (p.spread) {
        // more than half of a CU's LDS: the dispatcher cannot pair workgroups on a CU
        int cap = 0, dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
        if ((size_t)cap / 2 + 1024 <= (size_t)cap) lds = std::max(lds, (size_t)cap / 2 + 1024);
    }
    switch (rpt) {
        case 2: return launch_persist_t<T, 2>(a, p, lds, st, cus);
        case 3: return launch_persist_t<T, 3>(a, p, lds, st, cus);
        case 4: return launch_persist_t<T, 4>(a, p, lds, st, cus);
        case 5: return launch_persist_t<T, 5>(a, p, lds, st, cus);
        case 6: return launch_persist_t<T, 6>(a, p, lds, st, cus);
        case 7: return launch_persist_t<T, 7>(a, p, lds, st, cus);
        case 8: return launch_persist_t<T, 8>(a, p, lds, st, cus);
        case 9: return launch_persist_t<T, 9>(a, p, lds, st, cus);
        case 10: return launch_persist_t<T, 10>(a, p, lds, st, cus);
        case 12: return launch_persist_t<T, 12>(a, p, lds, st, cus);
        case 14: return launch_persist_t<T, 14>(a, p, lds, st, cus);
        case 16: return launch_persist_t<T, 16>(a, p, lds, st, cus);
        default: return launch_persist_t<T, 20>(a, p, lds, st, cus);
    }
}

template hipError_t launch_jacobi_persistent<double>(const JacArgs<double>&, const PersistArgs&, int,
                                                     hipStream_t);
template hipError_t launch_jacobi_persistent<float>(const JacArgs<float>&, const PersistArgs&, int,
                                                    hipStream_t);

}  // namespace tsvd
