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
// in LDS for the whole SVD.  The slice stops after a sweep that rotated
// nothing, or after max_sweeps.
//
// Work split as in jacobi_persist.hip: a column pair per group of PG = 32
// lanes, BW pairs per step (BW = 4, 8 or 16 columns per block: the block
// width is chosen per problem so that two blocks of its stacked height fit
// in LDS), rotation parameters in FP64, norms exact at the start of a round
// and tracked through it.
//
// Round mode (jacobi_round_kernel) for slices with many blocks: one launch
// per (sweep, round) and one workgroup per block pair, so a large slice is
// worked on by nb/2 workgroups at once; the launch boundaries order the
// rounds.
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
                                               int ka, int ldc, double tol, double* jnorm, unsigned& nbig) {
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
                    if (const unsigned code = ppair<T, PG, RPT>(xr, base + ycol * ldc, ax, be, ka, l, tol)) {
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
            if (const unsigned code = ppair<T, PG, RPT>(xi, blk1 + jc * ldc, al, be, ka, l, tol)) {
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
                nrot_sweep += pair_round<T, BW, RPT>(blk0, blk1, wi, wj, rd == 0, ka, ldc, tol, jnorm, nbig_sweep);
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

// Round mode: one launch per (sweep, round); workgroup b of problem p takes
// slice (b - wg_start[p]) / G, block pair (b - wg_start[p]) % G.  A slice
// whose previous sweep forced no further sweep (rot_forces_sweep) is
// skipped; sweep k records such rotations in rot[(k % 3) h + s] and clears
// rot[((k + 1) % 3) h + s], the
// entry that nobody reads or writes during sweep k (ring 0 is cleared by the
// control step before every SVD).
template <typename T, int BW, int RPT>
__global__ __launch_bounds__(BW * kPGs) void jacobi_round_kernel(const JacSliceArgs<T>* tab, const int* wg_start,
                                                                  int nprob, int sweep, int rd) {
    constexpr int PG = kPGs, NT = BW * PG;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int rot_any;
    __shared__ double jnorm[BW];
    const int p = batch_find(wg_start, nprob, (int)blockIdx.x);
    const JacSliceArgs<T>& a = tab[p];
    if (a.ctrl && a.ctrl->done) return;
    if (a.only_if && *a.only_if == 0) return;
    const int m = a.m, n = a.n, nb = a.nb, G = nb / 2;
    if (sweep >= (a.max_sweeps > 0 ? a.max_sweeps : 30) || rd >= nb - 1) return;
    const int local = (int)blockIdx.x - wg_start[p];
    const int s = local / G, gp = local - s * G;
    int* const rot = a.rot;
    if (rd == 0 && gp == 0 && threadIdx.x == 0) rot[((sweep + 1) % 3) * a.h + s] = 0;
    if (sweep > 0 && rot[((sweep + 2) % 3) * a.h + s] == 0) return;   // converged in the previous sweep
    cplx<T>* const A = a.A + (int64_t)s * n * m;
    cplx<T>* const V = a.V + (int64_t)s * n * n;
    const int ka = (m + PG - 1) / PG;
    const int mp = ka * PG;
    const int ldc = PG * RPT + 1;
    cplx<T>* const blk0 = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* const blk1 = blk0 + (size_t)BW * ldc;
    const int l = threadIdx.x % PG;
    for (int idx = threadIdx.x; idx < 2 * BW * ldc; idx += NT) blk0[idx] = cplx<T>{(T)0, (T)0};
    if (threadIdx.x == 0) rot_any = 0;
    __syncthreads();
    const int player0 = ppos_player(gp, rd, nb), player1 = ppos_player(nb - 1 - gp, rd, nb);
    load_block<T, NT, BW>(A, V, m, n, nb, player0, mp, ldc, blk0);
    load_block<T, NT, BW>(A, V, m, n, nb, player1, mp, ldc, blk1);
    __syncthreads();
    const int wi = pblk_start(player0 + 1, n, nb) - pblk_start(player0, n, nb);
    const int wj = pblk_start(player1 + 1, n, nb) - pblk_start(player1, n, nb);
    unsigned nbig = 0;
    const unsigned nrot = pair_round<T, BW, RPT>(blk0, blk1, wi, wj, rd == 0, ka, ldc, (double)a.tol, jnorm, nbig);
    if (nbig && l == 0) rot_any = 1;
    __syncthreads();
    store_block<T, NT, BW>(A, V, m, n, nb, player0, mp, ldc, blk0);
    store_block<T, NT, BW>(A, V, m, n, nb, player1, mp, ldc, blk1);
    if (threadIdx.x == 0) {
        if (rot_any) atomicOr(rot + (sweep % 3) * a.h + s, 1);
        if (rd == 0 && gp == 0) {
            if (a.sweeps) a.sweeps[s] = sweep + 1;
            if (a.ctrl) atomicMax(&a.ctrl->sweep_max, sweep + 1);
        }
    }
    if (l == 0 && nrot && a.rotations) atomicAdd(a.rotations, (unsigned long long)nrot);
}

// mode 0: slice kernel (x = max_sweeps); mode 1: round kernel (x = sweep, y = round);
// prepare: set the LDS limit of both kernels.
template <typename T, int BW, int RPT>
hipError_t launch_bw_rpt(bool prepare, int mode, const JacSliceArgs<T>* tab, const int* wg_start, int nprob, int nwg,
                         int x, int y, hipStream_t st) {
    auto* fs = jacobi_slice_kernel<T, BW, RPT>;
    auto* fr = jacobi_round_kernel<T, BW, RPT>;
    const size_t lds = jacobi_slice_lds(BW, RPT, sizeof(T));
    if (prepare) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fs),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        return hipFuncSetAttribute(reinterpret_cast<const void*>(fr), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds);
    }
    if (mode == 0)
        hipLaunchKernelGGL(fs, dim3(nwg), dim3(BW * kPGs), lds, st, tab, wg_start, nprob, x);
    else
        hipLaunchKernelGGL(fr, dim3(nwg), dim3(BW * kPGs), lds, st, tab, wg_start, nprob, x, y);
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

}  // namespace

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

template <typename T>
hipError_t launch_jacobi_round(int bw, int rpt, const JacSliceArgs<T>* tab, const int* wg_start, int nprob,
                               int nwg, int sweep, int round, hipStream_t st) {
    return dispatch<T>(false, 1, bw, rpt, tab, wg_start, nprob, nwg, sweep, round, st);
}

// Round mode: *flag = 1 when a slice of a running problem of the table
// rotated in sweep `sweep` and may run another sweep (below its cap), else 0.
// One workgroup; the flag is written once, after the scan.
template <typename T>
__global__ __launch_bounds__(256) void jacobi_round_active_kernel(const JacSliceArgs<T>* tab, int nprob, int sweep,
                                                                 int* flag) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int p = 0; p < nprob; ++p) {
        const JacSliceArgs<T>& a = tab[p];
        if (a.ctrl && a.ctrl->done) continue;
        if (sweep + 1 >= (a.max_sweeps > 0 ? a.max_sweeps : 30)) continue;
        for (int s = threadIdx.x; s < a.h; s += blockDim.x)
            if (a.rot[(sweep % 3) * a.h + s]) atomicOr(&any, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *flag = any;
}

template <typename T>
void launch_jacobi_round_active(const JacSliceArgs<T>* tab, int nprob, int sweep, int* flag, hipStream_t st) {
    hipLaunchKernelGGL((jacobi_round_active_kernel<T>), dim3(1), dim3(256), 0, st, tab, nprob, sweep, flag);
}

template void launch_jacobi_round_active<double>(const JacSliceArgs<double>*, int, int, int*, hipStream_t);
template void launch_jacobi_round_active<float>(const JacSliceArgs<float>*, int, int, int*, hipStream_t);

template hipError_t launch_jacobi_round<double>(int, int, const JacSliceArgs<double>*, const int*, int, int, int,
                                                int, hipStream_t);
template hipError_t launch_jacobi_round<float>(int, int, const JacSliceArgs<float>*, const int*, int, int, int, int,
                                               hipStream_t);

template hipError_t prepare_jacobi_slice<double>(int, int);
template hipError_t prepare_jacobi_slice<float>(int, int);
template hipError_t launch_jacobi_slice<double>(int, int, const JacSliceArgs<double>*, const int*, int, int, int,
                                                hipStream_t);
template hipError_t launch_jacobi_slice<float>(int, int, const JacSliceArgs<float>*, const int*, int, int, int,
                                               hipStream_t);

}  // namespace tsvd
