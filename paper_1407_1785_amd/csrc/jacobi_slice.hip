// One-sided Jacobi SVD with one workgroup per Fourier slice, for batches of
// many problems (same rotation, block round-robin ordering and stopping
// rule as jacobi.hip and jacobi_persist.hip).
//
// A batch of uneven problems has thousands of slices, many more than the
// chip has CUs, so every slice gets a single workgroup and no workgroup
// ever waits for another.  The workgroup runs all sweeps of its slice: in
// every round of the block tournament it visits the round's nb/2 block
// pairs one after the other, each time loading the two blocks (stacked
// columns: m slice rows, then n rows of V) from global memory into LDS,
// orthogonalising them against each other (and, in the first round of a
// sweep, internally) and writing them back.  With nb = 2 the two blocks stay
// in LDS for the whole SVD.  The slice stops after a sweep none of whose
// rotations forces another (rot_forces_sweep), or after max_sweeps.
//
// Work split as in jacobi_persist.hip: a column pair per group of PG = 32
// lanes, BW pairs per step (BW = 4, 8 or 16 columns per block: the block
// width is chosen per problem so that two blocks of its stacked height fit
// in LDS), rotation parameters in FP64, norms exact at the start of a round
// and tracked through it.
//
// Pairs-parallel schedule (jacobi_pairs_kernel) for slices with many
// blocks: one workgroup per block pair of a round, so a large slice is worked
// on by nb/2 workgroups at once, all sweeps in one launch (the blocks travel
// between the workgroups through global memory inside the launch).
//
// Launch: a table of problems; workgroup b serves problem p when
// wg_start[p] <= b < wg_start[p + 1], slice b - wg_start[p].  A problem
// whose ADMM has stopped (ctrl->done) is skipped, and so is one whose
// optional only_if word is zero (the single-problem driver's fallback after
// a persistent launch that gave up); each slice raises ctrl->sweep_max to
// its sweep count.

#include "jacobi_common.h"

namespace tsvd {

namespace {

using namespace jac;

constexpr int kPGs = 32;

// One round of the block tournament on one block pair of a slice, with the
// blocks in LDS (blk0 at tournament position gp, blk1 at nb - 1 - gp):
// optionally the internal pairs of both blocks (first round of a sweep),
// then every cross pair.  Returns the rotations applied (per thread: every
// lane of a pair group counts its group's rotations) and adds those that
// force another sweep to nbig.
template <typename T, int BW, int RPT>
__device__ __forceinline__ unsigned pair_round(cplx<T>* blk0, cplx<T>* blk1, int wi, int wj, bool self_phase,
                                               int ka, int ldc, double tol, double floor2, double* jnorm,
                                               unsigned& nbig) {
    constexpr int PG = kPGs;
    const int g = threadIdx.x / PG, l = threadIdx.x - g * PG;
    unsigned nrot = 0;
    // pair steps finished per wave in this call; a wave waits only for the
    // wave whose previous step wrote the column it takes next
    __shared__ int wsteps[BW * PG / 64];
    __shared__ double inorm[2 * BW];
    const int wave = threadIdx.x >> 6, wave_next = (wave + 1) % (BW * PG / 64);
    if ((threadIdx.x & 63) == 0) wsteps[wave] = 0;
    int steps = 0;
    if (self_phase) {
        // Internal pairs of both blocks (groups 0..BW/2-1 take block 0, the
        // rest block 1) by halving: the cross pairs of the block's two halves,
        // then of the halves of each half, down to adjacent pairs -- BW - 1
        // steps, every pair once.  Each level runs like a cross round: a
        // group keeps its column of the first half of its subproblem in
        // registers and meets the k columns of the second half, norms exact
        // at the level's start and tracked through it.
        const bool second = g >= BW / 2;
        const int gi = second ? g - BW / 2 : g;
        cplx<T>* const base = second ? blk1 : blk0;
        double* const jn = inorm + (second ? BW : 0);
        const int w = second ? wj : wi;
        for (int k = BW / 2; k >= 1; k /= 2) {
            const int sp = gi / k, q = gi - sp * k;
            const int xcol = 2 * k * sp + q, ybase = 2 * k * sp + k;
            // a subproblem of k groups spans k / 2 consecutive waves (one if k <= 2)
            const int span = k >= 4 ? k / 2 : 1, wl = wave % span;
            const int wnext = wave - wl + (wl + 1) % span;
            cplx<T> xr[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) xr[r] = base[xcol * ldc + l + PG * r];
            double ax = pnorm2<T, PG, RPT>(xr, ka);
            {
                cplx<T> yr[RPT];
#pragma unroll
                for (int r = 0; r < RPT; ++r) yr[r] = base[(ybase + q) * ldc + l + PG * r];
                const double bq = pnorm2<T, PG, RPT>(yr, ka);
                if (l == 0) jn[ybase + q] = bq;
            }
            __syncthreads();
            for (int st = 0; st < k; ++st) {
                if (st > 0) ring_wait(wsteps + wnext, steps + st);
                const int ycol = ybase + ((q + st) & (k - 1));
                if (xcol < w && ycol < w) {
                    double be = jn[ycol];
                    if (const unsigned code = ppair<T, PG, RPT>(xr, base + ycol * ldc, ax, be, ka, l, tol, floor2)) {
                        ++nrot;
                        nbig += code >> 1;
                        if (l == 0) jn[ycol] = be;
                    }
                }
                ring_publish(wsteps + wave, steps + st + 1);
            }
            steps += k;
            if (xcol < w) {
#pragma unroll
                for (int r = 0; r < RPT; ++r) base[xcol * ldc + l + PG * r] = xr[r];
            }
            __syncthreads();
        }
    }
    // cross pairs: column g of block 0 (registers) meets every column of block 1
    cplx<T> xi[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) xi[k] = blk0[g * ldc + l + PG * k];
    double al = pnorm2<T, PG, RPT>(xi, ka);
    {
        cplx<T> yj[RPT];
#pragma unroll
        for (int k = 0; k < RPT; ++k) yj[k] = blk1[g * ldc + l + PG * k];
        const double bj = pnorm2<T, PG, RPT>(yj, ka);
        if (l == 0) jnorm[g] = bj;
    }
    __syncthreads();
    for (int st = 0; st < BW; ++st) {
        if (st > 0) ring_wait(wsteps + wave_next, steps + st);
        const int jc = (g + st) & (BW - 1);
        if (g < wi && jc < wj) {
            double be = jnorm[jc];
            if (const unsigned code = ppair<T, PG, RPT>(xi, blk1 + jc * ldc, al, be, ka, l, tol, floor2)) {
                ++nrot;
                nbig += code >> 1;
                if (l == 0) jnorm[jc] = be;
            }
        }
        ring_publish(wsteps + wave, steps + st + 1);
    }
    if (g < wi) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) blk0[g * ldc + l + PG * k] = xi[k];
    }
    return nrot;
}

template <typename T, int BW, int RPT>
__global__ __launch_bounds__(BW * kPGs) void jacobi_slice_kernel(const JacSliceArgs<T>* tab, const int* wg_start,
                                                                  int nprob, int max_sweeps) {
    constexpr int PG = kPGs, NT = BW * PG;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int rot_any;
    __shared__ double jnorm[BW];
    const int p = batch_find(wg_start, nprob, (int)blockIdx.x);
    const JacSliceArgs<T>& a = tab[p];
    if (a.ctrl && a.ctrl->done) return;
    if (a.only_if && *a.only_if == 0) return;
    const int s = (int)blockIdx.x - wg_start[p];
    const int m = a.m, n = a.n, nb = a.nb, G = nb / 2;
    cplx<T>* const A = a.A + (int64_t)s * n * m;
    cplx<T>* const V = a.V + (int64_t)s * n * n;
    const int ka = (m + PG - 1) / PG;
    const int mp = ka * PG;
    const int ldc = PG * RPT + 1;
    cplx<T>* const blk0 = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* const blk1 = blk0 + (size_t)BW * ldc;
    const int l = threadIdx.x % PG;
    const double tol = (double)a.tol;

    for (int idx = threadIdx.x; idx < 2 * BW * ldc; idx += NT) blk0[idx] = cplx<T>{(T)0, (T)0};
    __syncthreads();
    if (G == 1) {
        load_block<T, NT, BW>(A, V, m, n, nb, 0, mp, ldc, blk0);
        load_block<T, NT, BW>(A, V, m, n, nb, 1, mp, ldc, blk1);
    }
    // rounding floor of the stopping rule: the parts of the round-0 block
    // pairs in pair order (as the pairs-parallel and persistent kernels add them)
    double floor2 = 0.0;
    if (a.floor_scale > 0.0) {
        double fro2 = 0.0;
        for (int gp = 0; gp < G; ++gp) {
            const int p0 = ppos_player(gp, 0, nb), p1 = ppos_player(nb - 1 - gp, 0, nb);
            if (G > 1) {
                __syncthreads();
                load_block<T, NT, BW>(A, V, m, n, nb, p0, mp, ldc, blk0);
                load_block<T, NT, BW>(A, V, m, n, nb, p1, mp, ldc, blk1);
            }
            __syncthreads();
            fro2 += pair_fro_part<T, PG, RPT, BW>(blk0, blk1, pblk_start(p0 + 1, n, nb) - pblk_start(p0, n, nb),
                                                  pblk_start(p1 + 1, n, nb) - pblk_start(p1, n, nb), ldc, ka,
                                                  jnorm);
        }
        floor2 = a.floor_scale * fro2;
    }

    unsigned nrot = 0;
    int sweeps = 0;
    const int msw = a.max_sweeps > 0 ? a.max_sweeps : max_sweeps;
    for (int sweep = 0; sweep < msw; ++sweep) {
        if (threadIdx.x == 0) rot_any = 0;
        unsigned nrot_sweep = 0, nbig_sweep = 0;
        for (int rd = 0; rd < nb - 1; ++rd) {
            for (int gp = 0; gp < G; ++gp) {
                const int player0 = ppos_player(gp, rd, nb), player1 = ppos_player(nb - 1 - gp, rd, nb);
                if (G > 1) {
                    __syncthreads();
                    load_block<T, NT, BW>(A, V, m, n, nb, player0, mp, ldc, blk0);
                    load_block<T, NT, BW>(A, V, m, n, nb, player1, mp, ldc, blk1);
                }
                __syncthreads();
                const int wi = pblk_start(player0 + 1, n, nb) - pblk_start(player0, n, nb);
                const int wj = pblk_start(player1 + 1, n, nb) - pblk_start(player1, n, nb);
                nrot_sweep += pair_round<T, BW, RPT>(blk0, blk1, wi, wj, rd == 0, ka, ldc, tol, floor2, jnorm,
                                                     nbig_sweep);
                if (G > 1) {
                    __syncthreads();
                    store_block<T, NT, BW>(A, V, m, n, nb, player0, mp, ldc, blk0);
                    store_block<T, NT, BW>(A, V, m, n, nb, player1, mp, ldc, blk1);
                }
            }
        }
        if (nbig_sweep && l == 0) rot_any = 1;
        __syncthreads();
        nrot += nrot_sweep;
        sweeps = sweep + 1;
        if (!rot_any) break;
        __syncthreads();
    }
    if (G == 1) {
        __syncthreads();
        store_block<T, NT, BW>(A, V, m, n, nb, 0, mp, ldc, blk0);
        store_block<T, NT, BW>(A, V, m, n, nb, 1, mp, ldc, blk1);
    }
    if (threadIdx.x == 0) {
        if (a.sweeps) a.sweeps[s] = sweeps;
        if (a.ctrl) atomicMax(&a.ctrl->sweep_max, sweeps);
    }
    if (l == 0 && nrot && a.rotations) atomicAdd(a.rotations, (unsigned long long)nrot);
}

// Pairs-parallel schedule: nb / 2 workgroups per slice, one per block pair
// of a round, all sweeps in one launch.  Workgroup roles (problem, slice,
// block pair) come in order from words[0], as in jacobi_persist.hip, so the workgroups of a slice wait only
// for workgroups that run or start as soon as others finish; between rounds
// a workgroup writes the blocks that move to their home columns with
// device-coherent stores, sets their ready flags to the round that takes them
// next and waits for the flags of the blocks it takes next; at the end of a
// sweep the slice's workgroups meet at a counter barrier and stop together
// when no rotation of the sweep forces another.  Every wait between
// workgroups is bounded (spin_limit polls); one that gives up sets words[1],
// and every workgroup that meets it writes its resident blocks home and
// stops.  The rotations, their order and the stopping rule are those of the
// one-workgroup-per-slice kernel (pair_round per block pair and round), so
// both schedules give the same results bit for bit.
__device__ bool pairs_barrier(int* counter, int target, int* err, int spin_limit) {
    __shared__ int ok;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        ok = 1;
        __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > spin_limit) {
                __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
    }
    __syncthreads();
    return ok != 0;
}

__device__ bool pairs_wait_flag(int* flag, int value, int* err, int spin_limit) {
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

template <typename T, int BW, int RPT>
__global__ __launch_bounds__(BW * kPGs) void jacobi_pairs_kernel(const JacSliceArgs<T>* tab, const int* role_start,
                                                                  int nprob, int* words, int spin_limit) {
    constexpr int PG = kPGs, NT = BW * PG;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int role_s, rot_any, stop, ok_flag;
    __shared__ double jnorm[BW];
    if (threadIdx.x == 0) role_s = __hip_atomic_fetch_add(words, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int role = __builtin_amdgcn_readfirstlane(role_s);
    const int p = batch_find(role_start, nprob, role);
    const JacSliceArgs<T>& a = tab[p];
    if (a.ctrl && a.ctrl->done) return;   // every workgroup of the problem returns
    const int m = a.m, n = a.n, nb = a.nb, G = nb / 2, h = a.h;
    const int local = role - role_start[p];
    const int s = local / G, gp = local - s * G;
    cplx<T>* const A = a.A + (int64_t)s * n * m;
    cplx<T>* const V = a.V + (int64_t)s * n * n;
    int* const counter = a.bar + s;
    int* const bf = a.bar + h + (int64_t)s * nb;
    int* const rot = a.rot;
    int* const err = words + 1;
    const int ka = (m + PG - 1) / PG;
    const int mp = ka * PG;
    const int ldc = PG * RPT + 1;
    cplx<T>* const blk0 = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* const blk1 = blk0 + (size_t)BW * ldc;
    const int l = threadIdx.x % PG;
    const double tol = (double)a.tol;
    const int msw = a.max_sweeps > 0 ? a.max_sweeps : 30;

    // padding rows stay zero under every rotation
    for (int idx = threadIdx.x; idx < 2 * BW * ldc; idx += NT) blk0[idx] = cplx<T>{(T)0, (T)0};
    __syncthreads();
    const int pos0 = gp, pos1 = nb - 1 - gp;
    int player0 = ppos_player(pos0, 0, nb), player1 = ppos_player(pos1, 0, nb);
    load_block<T, NT, BW, true>(A, V, m, n, nb, player0, mp, ldc, blk0);
    load_block<T, NT, BW, true>(A, V, m, n, nb, player1, mp, ldc, blk1);
    __syncthreads();

    unsigned nrot = 0;
    int sweeps = 0, arrivals = 0;
    bool alive = true, home0 = true, home1 = true;
    // rounding floor of the stopping rule: every workgroup writes the part of
    // its round-0 block pair, the slice's workgroups meet once, and each adds
    // the parts in pair order (as the one-workgroup-per-slice kernel does)
    double floor2 = 0.0;
    if (a.floor_scale > 0.0) {
        __shared__ double fro_s;
        const double part = pair_fro_part<T, PG, RPT, BW>(
            blk0, blk1, pblk_start(player0 + 1, n, nb) - pblk_start(player0, n, nb),
            pblk_start(player1 + 1, n, nb) - pblk_start(player1, n, nb), ldc, ka, jnorm);
        if (threadIdx.x == 0) coh_store_f64(a.fro + (int64_t)s * G + gp, part);
        arrivals += G;
        if (!pairs_barrier(counter, arrivals, err, spin_limit)) {
            alive = false;   // giving up before any rotation: both blocks are still home
        } else {
            if (threadIdx.x == 0) {
                double fro2 = 0.0;
                for (int i = 0; i < G; ++i) fro2 += coh_load_f64(a.fro + (int64_t)s * G + i);
                fro_s = a.floor_scale * fro2;
            }
            __syncthreads();
            floor2 = fro_s;
        }
    }
    for (int sweep = 0; sweep < msw && alive; ++sweep) {
        if (threadIdx.x == 0) rot_any = 0;
        if (gp == 0 && threadIdx.x == 0)
            __hip_atomic_store(rot + ((sweep + 1) % 3) * h + s, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sweeps = sweep + 1;
        __syncthreads();
        unsigned nbig = 0;
        for (int rd = 0; rd < nb - 1; ++rd) {
            const int wi = pblk_start(player0 + 1, n, nb) - pblk_start(player0, n, nb);
            const int wj = pblk_start(player1 + 1, n, nb) - pblk_start(player1, n, nb);
            nrot += pair_round<T, BW, RPT>(blk0, blk1, wi, wj, rd == 0, ka, ldc, tol, floor2, jnorm, nbig);
            const bool last = rd == nb - 2;
            __syncthreads();
            if (last) {
                if (nbig && l == 0) rot_any = 1;
                __syncthreads();
                if (threadIdx.x == 0 && rot_any)
                    __hip_atomic_fetch_or(rot + (sweep % 3) * h + s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            // the next round's players (after the last round: round 0 of the next sweep)
            const int nr = (rd + 1) % (nb - 1);
            const int next0 = ppos_player(pos0, nr, nb), next1 = ppos_player(pos1, nr, nb);
            if (next0 != player0) store_block<T, NT, BW, true>(A, V, m, n, nb, player0, mp, ldc, blk0);
            if (next1 != player1) store_block<T, NT, BW, true>(A, V, m, n, nb, player1, mp, ldc, blk1);
            if (last) {
                arrivals += G;
                if (!pairs_barrier(counter, arrivals, err, spin_limit)) {
                    home0 = next0 == player0;   // giving up
                    home1 = next1 == player1;
                    alive = false;
                    break;
                }
                if (threadIdx.x == 0)
                    stop = __hip_atomic_load(rot + (sweep % 3) * h + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
                __syncthreads();
                if (stop) {
                    home0 = next0 == player0;   // converged
                    home1 = next1 == player1;
                    alive = false;
                    break;
                }
            } else {
                const int R = sweep * (nb - 1) + rd;
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                if (threadIdx.x == 0) {
                    ok_flag = 1;
                    if (next0 != player0) __hip_atomic_store(bf + player0, R + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (next1 != player1) __hip_atomic_store(bf + player1, R + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((next0 != player0 && !pairs_wait_flag(bf + next0, R + 1, err, spin_limit)) ||
                        (next1 != player1 && !pairs_wait_flag(bf + next1, R + 1, err, spin_limit)))
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
            // the incoming blocks: one memory round trip per block in FP32
            if (next0 != player0) load_block_any<T, PG, RPT, BW, true>(A, V, m, n, nb, next0, mp, ldc, blk0);
            if (next1 != player1) load_block_any<T, PG, RPT, BW, true>(A, V, m, n, nb, next1, mp, ldc, blk1);
            player0 = next0;
            player1 = next1;
            __syncthreads();
        }
    }
    __syncthreads();
    if (home0) store_block<T, NT, BW, true>(A, V, m, n, nb, player0, mp, ldc, blk0);
    if (home1) store_block<T, NT, BW, true>(A, V, m, n, nb, player1, mp, ldc, blk1);
    if (threadIdx.x == 0) {
        if (gp == 0 && a.sweeps) a.sweeps[s] = sweeps;
        if (a.ctrl) atomicMax(&a.ctrl->sweep_max, sweeps);
    }
    if (l == 0 && nrot && a.rotations) atomicAdd(a.rotations, (unsigned long long)nrot);
}

// prepare: set the LDS limit of both kernels; else launch the slice kernel
// (x = max_sweeps).
template <typename T, int BW, int RPT>
hipError_t launch_bw_rpt(bool prepare, int mode, const JacSliceArgs<T>* tab, const int* wg_start, int nprob, int nwg,
                         int x, int y, hipStream_t st) {
    auto* fs = jacobi_slice_kernel<T, BW, RPT>;
    const size_t lds = jacobi_slice_lds(BW, RPT, sizeof(T));
    if (prepare) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fs),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        return hipFuncSetAttribute(reinterpret_cast<const void*>(jacobi_pairs_kernel<T, BW, RPT>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    (void)mode;
    (void)y;
    hipLaunchKernelGGL(fs, dim3(nwg), dim3(BW * kPGs), lds, st, tab, wg_start, nprob, x);
    return hipGetLastError();
}

template <typename T, int BW, int... R>
hipError_t dispatch_rpt(int rpt, std::integer_sequence<int, R...>, bool prepare, int mode, const JacSliceArgs<T>* tab,
                        const int* wg_start, int nprob, int nwg, int x, int y, hipStream_t st) {
    hipError_t e = hipErrorInvalidValue;
    ((rpt == R + 2 ? (e = launch_bw_rpt<T, BW, R + 2>(prepare, mode, tab, wg_start, nprob, nwg, x, y, st), 0) : 0),
     ...);
    return e;
}

template <typename T>
hipError_t dispatch(bool prepare, int mode, int bw, int rpt, const JacSliceArgs<T>* tab, const int* wg_start,
                    int nprob, int nwg, int x, int y, hipStream_t st) {
    if (rpt < 2 || rpt > 20) return hipErrorInvalidValue;
    auto seq = std::make_integer_sequence<int, 19>{};
    switch (bw) {
        case 4: return dispatch_rpt<T, 4>(rpt, seq, prepare, mode, tab, wg_start, nprob, nwg, x, y, st);
        case 8: return dispatch_rpt<T, 8>(rpt, seq, prepare, mode, tab, wg_start, nprob, nwg, x, y, st);
        case 16: return dispatch_rpt<T, 16>(rpt, seq, prepare, mode, tab, wg_start, nprob, nwg, x, y, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int BW, int RPT>
hipError_t launch_pairs_bw_rpt(const JacSliceArgs<T>* tab, const int* role_start, int nprob, int nroles, int* words,
                               int spin_limit, hipStream_t st) {
    const size_t lds = jacobi_slice_lds(BW, RPT, sizeof(T));
    hipLaunchKernelGGL((jacobi_pairs_kernel<T, BW, RPT>), dim3(nroles), dim3(BW * kPGs), lds, st, tab, role_start, nprob,
                       words, spin_limit);
    return hipGetLastError();
}

template <typename T, int BW, int... R>
hipError_t dispatch_pairs_rpt(int rpt, std::integer_sequence<int, R...>, const JacSliceArgs<T>* tab,
                              const int* role_start, int nprob, int nroles, int* words, int spin_limit,
                              hipStream_t st) {
    hipError_t e = hipErrorInvalidValue;
    ((rpt == R + 2 ? (e = launch_pairs_bw_rpt<T, BW, R + 2>(tab, role_start, nprob, nroles, words, spin_limit, st), 0)
                   : 0),
     ...);
    return e;
}

}  // namespace

template <typename T>
hipError_t launch_jacobi_pairs(int bw, int rpt, const JacSliceArgs<T>* tab, const int* role_start, int nprob,
                               int nroles, int* words, int spin_limit, hipStream_t st) {
    if (rpt < 2 || rpt > 20) return hipErrorInvalidValue;
    if (nroles <= 0) return hipSuccess;
    auto seq = std::make_integer_sequence<int, 19>{};
    switch (bw) {
        case 4: return dispatch_pairs_rpt<T, 4>(rpt, seq, tab, role_start, nprob, nroles, words, spin_limit, st);
        case 8: return dispatch_pairs_rpt<T, 8>(rpt, seq, tab, role_start, nprob, nroles, words, spin_limit, st);
        case 16: return dispatch_pairs_rpt<T, 16>(rpt, seq, tab, role_start, nprob, nroles, words, spin_limit, st);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_jacobi_pairs<double>(int, int, const JacSliceArgs<double>*, const int*, int, int, int*, int,
                                                hipStream_t);
template hipError_t launch_jacobi_pairs<float>(int, int, const JacSliceArgs<float>*, const int*, int, int, int*, int,
                                               hipStream_t);

int jacobi_slice_rpt(int m, int n) {
    const int need = (m + kPGs - 1) / kPGs + (n + kPGs - 1) / kPGs;
    return need < 2 ? 2 : need;
}

size_t jacobi_slice_lds(int bw, int rpt, int elem_bytes) {
    return 2 * (size_t)bw * (kPGs * rpt + 1) * 2 * elem_bytes;
}

int jacobi_slice_max_rpt() { return 20; }

template <typename T>
hipError_t prepare_jacobi_slice(int bw, int rpt) {
    return dispatch<T>(true, 0, bw, rpt, nullptr, nullptr, 0, 0, 0, 0, nullptr);
}

template <typename T>
hipError_t launch_jacobi_slice(int bw, int rpt, const JacSliceArgs<T>* tab, const int* wg_start, int nprob,
                               int nwg, int max_sweeps, hipStream_t st) {
    return dispatch<T>(false, 0, bw, rpt, tab, wg_start, nprob, nwg, max_sweeps, 0, st);
}

template hipError_t prepare_jacobi_slice<double>(int, int);
template hipError_t prepare_jacobi_slice<float>(int, int);
template hipError_t launch_jacobi_slice<double>(int, int, const JacSliceArgs<double>*, const int*, int, int, int,
                                                hipStream_t);
template hipError_t launch_jacobi_slice<float>(int, int, const JacSliceArgs<float>*, const int*, int, int, int,
                                               hipStream_t);

}  // namespace tsvd
