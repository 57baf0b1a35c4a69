// C ABI of the gfx950 t-SVT library: handles, workspace, the t-SVT step and
// the completion / RPCA ADMM drivers (declarations and contracts in
// include/tsvd.h).
//
// One ADMM iteration on the device is
//   dft_forward (fused prologue)  ->  Jacobi sweeps  ->  svt weights+rebuild
//   ->  dft_inverse (fused epilogue + residual partials)  ->  admm_ctrl,
// all on the handle's stream, with the control scalars in device memory.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>


#include "host.h"

using namespace tsvd;

namespace {

// Bump allocator over the handle's workspace.
struct Carver {
    char* base;
    size_t off = 0;
    template <typename U>
    U* take(int64_t count) {
        off = (off + 255) & ~size_t(255);
        U* p = reinterpret_cast<U*>(base + off);
        off += (size_t)count * sizeof(U);
        return p;
    }
};

template <typename T>
struct SvtBuffers {
    cplx<T>* A;       // slices in (and Jacobi work array on a cold start)
    cplx<T>* Z;       // second slice buffer
    cplx<T>* V[2];    // right singular vectors, ping-pong for re-orthonormalisation
    cplx<T>* G;       // n x n Gram scratch
    double* sigma;    // h x n singular values (FP64)
    double* dk;       // h x n shrink factors
    int* rank;
    int* rot;
    int* sweeps;
    int* pbar;        // persistent Jacobi: h barrier counters, 3h flags, the error word, the role
                      // ticket, h x nb block flags
    double* fro;      // persistent Jacobi: h x (nb / 2) parts of the slices' Frobenius norms
    double* partials;
    int nparts;
    double* tall;     // tall slices: the Jacobi partial sums (jacobi_tall_plan)
    // after a persistent launch that gave up (error word set): the one-
    // workgroup-per-slice kernel finishes the SVD; entry 2 (work == Z) + vc
    // of the table, and the problem-table start {0, h}
    JacSliceArgs<T>* ftab;
    int* fws;
};

// pbar words of a geometry: barriers, rotation flags, error word, ticket, block flags
inline int64_t pbar_words(const Geometry& g) { return 4 * (int64_t)g.h + 2 + (int64_t)g.h * (g.n + 2); }
// doubles of the per-workgroup Frobenius parts (at most n / 2 block pairs per slice)
inline int64_t fro_doubles(const Geometry& g) { return (int64_t)g.h * (g.n / 2 + 1); }

// Warm-start state carried across the iterations of one solve.
struct WarmState {
    bool enabled = false;   // pre-rotate by the previous V
    bool valid = false;     // V[vcur] holds the previous iteration's V
    int vcur = 0;
    int iter = 0;
    int reorth_every = 4;
};

template <typename T>
size_t svt_bytes(const Geometry& g, int nparts) {
    const int64_t slice = (int64_t)g.h * g.m * g.n;
    const int64_t vv = (int64_t)g.h * g.n * g.n;
    size_t b = 0;
    b += 2 * slice * sizeof(cplx<T>) + 512;
    b += 3 * vv * sizeof(cplx<T>) + 768;
    b += 2 * (int64_t)g.h * g.n * sizeof(double) + 512;
    b += (int64_t)g.h * 5 * sizeof(int) + 768;
    b += pbar_words(g) * sizeof(int) + 256;
    b += fro_doubles(g) * sizeof(double) + 256;
    b += (int64_t)nparts * kNumPartials * sizeof(double) + 256;
    b += 8 * sizeof(JacSliceArgs<T>) + 4 * sizeof(int) + 512;
    if (jacobi_tall(g.m, g.n, sizeof(T))) b += jacobi_tall_plan(g.m, g.n, g.h).part_doubles * sizeof(double) + 256;
    return b;
}

template <typename T>
SvtBuffers<T> carve_svt(Carver& c, const Geometry& g, int nparts) {
    SvtBuffers<T> s{};
    const int64_t slice = (int64_t)g.h * g.m * g.n;
    const int64_t vv = (int64_t)g.h * g.n * g.n;
    s.A = c.take<cplx<T>>(slice);
    s.Z = c.take<cplx<T>>(slice);
    s.V[0] = c.take<cplx<T>>(vv);
    s.V[1] = c.take<cplx<T>>(vv);
    s.G = c.take<cplx<T>>(vv);
    s.sigma = c.take<double>((int64_t)g.h * g.n);
    s.dk = c.take<double>((int64_t)g.h * g.n);
    s.rank = c.take<int>(g.h);
    s.rot = c.take<int>(3 * g.h);
    s.sweeps = c.take<int>(g.h);
    s.pbar = c.take<int>(pbar_words(g));
    s.fro = c.take<double>(fro_doubles(g));
    s.partials = c.take<double>((int64_t)nparts * kNumPartials);
    s.nparts = nparts;
    s.tall = jacobi_tall(g.m, g.n, sizeof(T)) ? c.take<double>(jacobi_tall_plan(g.m, g.n, g.h).part_doubles)
                                              : nullptr;
    s.ftab = c.take<JacSliceArgs<T>>(8);
    s.fws = c.take<int>(4);
    return s;
}

void ensure_workspace(tsvd_handle h, size_t bytes) {
    if (bytes <= h->ws_bytes) return;
    if (h->budget && bytes > h->budget)
        fail(TSVD_E_NOMEM, "workspace of " + std::to_string(bytes) + " bytes exceeds the handle budget");
    if (h->ws) hip_check(hipFree(h->ws), "hipFree");
    h->ws = nullptr;
    h->ws_bytes = 0;
    hipError_t e = hipMalloc(&h->ws, bytes);
    if (e != hipSuccess) fail(TSVD_E_NOMEM, std::string("hipMalloc workspace: ") + hipGetErrorString(e));
    h->ws_bytes = bytes;
}

void ensure_host_ints(tsvd_handle h, int count) {
    if (count <= h->host_ints_len) return;
    if (h->host_ints) hip_check(hipHostFree(h->host_ints), "hipHostFree");
    h->host_ints = nullptr;
    hip_check(hipHostMalloc(reinterpret_cast<void**>(&h->host_ints), sizeof(int) * count, 0),
              "hipHostMalloc");
    h->host_ints_len = count;
}

void* ensure_host_stage(tsvd_handle h, size_t bytes) {
    if (bytes > h->host_stage_len) {
        if (h->host_stage) hip_check(hipHostFree(h->host_stage), "hipHostFree");
        h->host_stage = nullptr;
        hip_check(hipHostMalloc(&h->host_stage, bytes, 0), "hipHostMalloc");
        h->host_stage_len = bytes;
    }
    return h->host_stage;
}

// How the single-problem drivers run the Jacobi sweeps of a geometry:
// PERSIST, the persistent kernel (one workgroup per block pair of 16
// columns, every workgroup resident); PAIRS, the block-pair kernel of the
// batched form when the persistent grid would exceed the CUs or its blocks
// the LDS (one workgroup per block pair of bw columns, all sweeps in one
// launch, roles in ticket order so that more workgroups than CUs are fine);
// ROUNDS, one launch per round (or the tall kernels).  TSVD_PERSIST=0 and
// TSVD_PAIRS_SINGLE=0 turn the first two off.
enum class JacMode { PERSIST, PAIRS, ROUNDS };

struct JacPlan {
    JacMode mode = JacMode::ROUNDS;
    int bw = 16;    // block width of the block-pair kernel and of the fallback
    int rpt = 0;    // rows per lane of the one-workgroup-per-slice / block-pair kernels
    int nb = 0;     // blocks per slice of the block-pair kernel
};

template <typename T>
JacPlan jacobi_plan(tsvd_handle h, const Geometry& g) {
    JacPlan p;
    p.rpt = jacobi_slice_rpt(g.m, g.n);
    if (jacobi_tall(g.m, g.n, sizeof(T))) return p;
    if (env_int("TSVD_PERSIST", 1) != 0 && jacobi_persistent_fits(g.m, g.n, g.h, sizeof(T), h->cus, h->lds_cap)) {
        p.mode = JacMode::PERSIST;
        return p;
    }
    if (env_int("TSVD_PAIRS_SINGLE", 1) == 0 || p.rpt > jacobi_slice_max_rpt()) return p;
    for (int bw : {16, 8, 4}) {
        if (jacobi_slice_lds(bw, p.rpt, sizeof(T)) + 256 > h->lds_cap) continue;
        const int nb = jacobi_num_blocks(g.n, bw);
        if (nb / 2 < 2) break;   // one block pair per slice: nothing to run in parallel
        p.mode = JacMode::PAIRS;
        p.bw = bw;
        p.nb = nb;
        return p;
    }
    return p;
}

// The argument tables of the Jacobi sweeps that run as one launch, uploaded
// once per call (with the kernels' LDS limit):
//  entries 0-3, the fallback after a persistent or block-pair launch that
//  gave up: the one-workgroup-per-slice kernel on the same slices (work
//  buffer A or Z, V buffer 0 or 1), gated on the error word at pbar + 4h;
//  entries 4-7 (PAIRS only), the block-pair kernel on the same buffers.
// In PAIRS mode the persistent kernel's int words hold the block-pair
// kernel's: the rotation-flag ring at pbar, the role ticket at pbar + 4h - 1
// and the error word at pbar + 4h (the fallback's gate), the barrier
// counters and block flags from pbar + 4h + 1.
template <typename T>
void upload_fallback(tsvd_handle h, const Geometry& g, const SvtBuffers<T>& sb, int max_sweeps) {
    const JacPlan plan = jacobi_plan<T>(h, g);
    if (plan.mode == JacMode::ROUNDS) return;
    const bool pairs = plan.mode == JacMode::PAIRS;
    JacSliceArgs<T> tab[8];
    for (int k = 0; k < 8; ++k) {
        JacSliceArgs<T>& a = tab[k];
        a = JacSliceArgs<T>{};
        a.A = (k & 2) ? sb.Z : sb.A;
        a.V = sb.V[k & 1];
        a.m = g.m;
        a.n = g.n;
        a.h = g.h;
        a.nb = pairs ? plan.nb : jacobi_persistent_blocks(g.n);
        a.tol = (T)jacobi_tol(g.m, sizeof(T));
        a.sweeps = sb.sweeps;
        a.ctrl = h->ctrl;
        a.rotations = h->rot_counter + 1;
        a.max_sweeps = max_sweeps;
        a.floor_scale = jacobi_floor_scale(g.m, sizeof(T));
        if (k < 4) {
            a.only_if = sb.pbar + 4 * g.h;
        } else {
            a.rot = sb.pbar;
            a.bar = sb.pbar + 4 * g.h + 1;
            a.fro = sb.fro;
        }
    }
    const int ws[4] = {0, g.h, 0, pairs ? g.h * (plan.nb / 2) : 0};
    char* stage = static_cast<char*>(ensure_host_stage(h, sizeof(tab) + sizeof(ws)));
    std::memcpy(stage, tab, sizeof(tab));
    std::memcpy(stage + sizeof(tab), ws, sizeof(ws));
    hip_check(hipMemcpyAsync(sb.ftab, stage, sizeof(tab), hipMemcpyHostToDevice, h->stream), "hipMemcpyAsync");
    hip_check(hipMemcpyAsync(sb.fws, stage + sizeof(tab), sizeof(ws), hipMemcpyHostToDevice, h->stream),
              "hipMemcpyAsync");
    hip_check(prepare_jacobi_slice<T>(plan.bw, plan.rpt), "jacobi fallback attribute");
    hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
}

// The DFT matrices of the tube shape of g in the element type, cached on
// the handle for consecutive calls on the same shape.
template <typename T>
const T* ensure_dft_matrices(tsvd_handle h, const Geometry& g) {
    const int64_t key = ((int64_t)g.P << 32) | ((int64_t)g.Q << 8) | (int64_t)sizeof(T);
    if (h->dmat_key == key) return static_cast<const T*>(h->dmat);
    hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    if (h->dmat) hip_check(hipFree(h->dmat), "hipFree");
    h->dmat = nullptr;
    h->dmat_key = -1;
    const std::vector<T> m = dft_matrices_host<T>(g);
    hip_check(hipMalloc(&h->dmat, sizeof(T) * m.size()), "hipMalloc DFT matrices");
    hip_check(hipMemcpy(h->dmat, m.data(), sizeof(T) * m.size(), hipMemcpyHostToDevice),
              "hipMemcpy DFT matrices");
    h->dmat_key = key;
    return static_cast<const T*>(h->dmat);
}

// Scratch of tsvt_noalloc (include/tsvd.h): every GPU the library runs on
// holds one copy of this array until the process ends, shared by every
// handle on that GPU.  Host code never takes its name as an address: the
// device address of each GPU's copy is looked up once per device, with that
// device current, when the first handle on it is created (scratch_address).
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<char*> g_scratch_ptr;   // per device; nullptr until looked up

char* scratch_address(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress scratch");
        if (!p) fail(TSVD_E_HIP, "no device address for the scratch array");
        g_scratch_ptr[device] = static_cast<char*>(p);
    }
    return g_scratch_ptr[device];
}

// Kernel families reported by tsvd_profile_read.
enum Kind : int {
    K_DFT_FWD = 0, K_JAC_INIT, K_JAC_SELF, K_JAC_CROSS, K_SVT_W, K_SVT_REBUILD, K_DFT_INV,
    K_CTRL, K_GEMM, K_JAC_PERSIST, K_OTHER, K_COUNT
};
const char* kKindName[K_COUNT] = {"dft_forward", "jacobi_init", "jacobi_self", "jacobi_cross",
                                  "svt_sigma", "svt_rebuild", "dft_inverse", "admm_ctrl",
                                  "warm_gemm", "jacobi_persistent", "other"};
const bool kKindBytes[K_COUNT] = {true, true, false, false, true, false, true, true, false, false, true};

hipEvent_t take_event(tsvd_handle h) {
    if (!h->ev_pool.empty()) {
        hipEvent_t e = h->ev_pool.back();
        h->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "hipEventCreate");
    return e;
}

void prof_harvest(tsvd_handle h) {
    if (h->pending.empty()) return;
    hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    for (auto& p : h->pending) {
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, p.a, p.b), "hipEventElapsedTime");
        auto& g = h->agg[p.kind];
        g.launches += 1;
        g.ms += ms;
        g.work += p.work;
        g.sweeps += p.sweeps;
        g.pairs += p.pairs;
        g.kept += p.kept;
        h->ev_pool.push_back(p.a);
        h->ev_pool.push_back(p.b);
    }
    h->pending.clear();
}

// Run `launch` (which enqueues one kernel on h->stream), timing it when
// profiling is on.  Returns the index of the pending record or -1.
template <typename F>
int prof_launch(tsvd_handle h, int kind, double work, F&& launch) {
    if (!h->prof_on) {
        launch();
        return -1;
    }
    tsvd_handle_s::Pending p{kind, take_event(h), take_event(h), work};
    hip_check(hipEventRecord(p.a, h->stream), "hipEventRecord");
    launch();
    hip_check(hipEventRecord(p.b, h->stream), "hipEventRecord");
    h->pending.push_back(p);
    if (h->pending.size() >= 4096) {
        prof_harvest(h);
        return -1;
    }
    return (int)h->pending.size() - 1;
}

int blk_start_host(int b, int n, int nb) { return (int)(((int64_t)b * n) / nb); }

// column pairs visited by one self launch / one cross round, per slice
int64_t self_pairs(int n, int nb) {
    int64_t p = 0;
    for (int b = 0; b < nb; ++b) {
        const int64_t w = blk_start_host(b + 1, n, nb) - blk_start_host(b, n, nb);
        p += w * (w - 1) / 2;
    }
    return p;
}

int64_t cross_pairs(int n, int nb, int round) {
    int64_t p = 0;
    auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (nb - 1); };
    for (int pr = 0; pr < nb / 2; ++pr) {
        const int bi = player(pr), bj = player(nb - 1 - pr);
        const int64_t wi = blk_start_host(bi + 1, n, nb) - blk_start_host(bi, n, nb);
        const int64_t wj = blk_start_host(bj + 1, n, nb) - blk_start_host(bj, n, nb);
        p += wi * wj;
    }
    return p;
}

struct SweepStats {
    int sweeps = 0;
    bool on_device = false;      // the sweeps were counted into ctrl->sweep_max
    const void* out = nullptr;   // slice buffer holding the prox output
    const void* w = nullptr;     // W = A V (orthogonal columns, sigma_j = ||w_j||)
    const void* v = nullptr;     // V
};

// Jacobi sweeps + shrink + rebuild on the slices in sb.A; output in sb.Z.
//
// Work model of the Jacobi kernels (FP operations): every visited column
// pair costs 28 m + 20 n, one complex dot product over the m slice rows
// (8 m) plus the 2 x 2 complex rotation of both columns' m slice rows and
// n V rows (20 (m + n)), whether or not the rotation is applied; a slice
// sweep visits n (n - 1) / 2 pairs.  Slice sweeps, visited pairs and applied
// rotations are recorded beside it.
template <typename T>
SweepStats run_svt(tsvd_handle h, const Geometry& g, const SvtBuffers<T>& sb, int max_sweeps,
                   WarmState* warm = nullptr, bool want_rank = false, bool rebuild = true) {
    hipStream_t st = h->stream;
    const bool use_warm = warm && warm->enabled && warm->valid;
    const int64_t nn = (int64_t)g.n * g.n, mn = (int64_t)g.m * g.n;
    cplx<T>* work = sb.A;   // Jacobi work array
    cplx<T>* out = sb.Z;    // rebuild output
    int vc = warm ? warm->vcur : 0;
    if (use_warm) {
        if (warm->reorth_every > 0 && warm->iter % warm->reorth_every == 0) {
            // V <- 1.5 V - 0.5 V (V^H V): one Newton-Schulz step towards unitary
            ZGemmArgs<T> gg{};
            gg.A = sb.V[vc]; gg.B = sb.V[vc]; gg.C = sb.G;
            gg.M = gg.N = gg.K = g.n;
            gg.lda = gg.ldb = gg.ldc = gg.ldd = g.n;
            gg.sA = gg.sB = gg.sC = gg.sD = nn;
            gg.alpha = (T)1; gg.beta = (T)0; gg.opA = 1; gg.opB = 0; gg.batch = g.h;
            gg.ctrl = h->ctrl;
            gg.herm = 1;
            prof_launch(h, K_GEMM, 8.0 * g.n * g.n * g.n * g.h, [&] { launch_zgemm(gg, st); });
            launch_check("gemm gram");
            ZGemmArgs<T> gn = gg;
            gn.herm = 0;
            gn.A = sb.V[vc]; gn.B = sb.G; gn.D = sb.V[vc]; gn.C = sb.V[1 - vc];
            gn.alpha = (T)-0.5; gn.beta = (T)1.5; gn.opA = 0;
            prof_launch(h, K_GEMM, 8.0 * g.n * g.n * g.n * g.h, [&] { launch_zgemm(gn, st); });
            launch_check("gemm newton-schulz");
            vc = 1 - vc;
            warm->vcur = vc;
        }
        // pre-rotate: work = A V_prev
        ZGemmArgs<T> ga{};
        ga.A = sb.A; ga.B = sb.V[vc]; ga.C = sb.Z;
        ga.M = g.m; ga.N = g.n; ga.K = g.n;
        ga.lda = g.m; ga.ldb = g.n; ga.ldc = g.m; ga.ldd = g.m;
        ga.sA = mn; ga.sB = nn; ga.sC = mn; ga.sD = mn;
        ga.alpha = (T)1; ga.beta = (T)0; ga.opA = 0; ga.opB = 0; ga.batch = g.h;
        ga.ctrl = h->ctrl;
        prof_launch(h, K_GEMM, 8.0 * g.m * g.n * g.n * g.h, [&] { launch_zgemm(ga, st); });
        launch_check("gemm prerotate");
        work = sb.Z;
        out = sb.A;
    }
    JacArgs<T> ja{};
    ja.A = work;
    ja.V = sb.V[vc];
    ja.m = g.m;
    ja.n = g.n;
    ja.h = g.h;
    ja.reset_v = use_warm ? 0 : 1;
    ja.ctrl = h->ctrl;
    int bw = env_int("TSVD_JACOBI_BW", 0);
    if (bw != 4 && bw != 8 && bw != 16) bw = jacobi_block_width(g.m, g.n, sizeof(T), g.h);
    ja.nb = jacobi_num_blocks(g.n, bw);
    ja.rot = sb.rot;
    ja.sweeps = sb.sweeps;
    ja.tol = (T)jacobi_tol(g.m, sizeof(T));
    ja.rotations = h->rot_counter;
    const int check_every = std::max(1, env_int("TSVD_CHECK_EVERY", 1));
    ensure_host_ints(h, g.h);
    SweepStats stats;
    const double pair_flops = 28.0 * g.m + 20.0 * g.n;
    const double slice_pairs = 0.5 * g.n * (g.n - 1.0);
    const JacPlan plan = jacobi_plan<T>(h, g);
    const bool persist = plan.mode == JacMode::PERSIST;
    bool done_persist = false;
    if (persist) {
        // one launch runs every sweep
        ja.nb = jacobi_persistent_blocks(g.n);
        ja.rotations = h->rot_counter + 1;
        // the init also clears the barrier counters, rotation flags, role
        // ticket and block flags (the error word is cleared once per call)
        ja.clr[0] = sb.pbar;
        ja.nclr[0] = 4 * g.h;
        ja.clr[1] = sb.pbar + 4 * g.h + 1;
        ja.nclr[1] = 1 + g.h * ja.nb;
        prof_launch(h, K_JAC_INIT, (double)g.h * g.n * g.n * sizeof(cplx<T>),
                    [&] { launch_jacobi_init(ja, st); });
        launch_check("jacobi_init");
        ja.clr[0] = ja.clr[1] = nullptr;
        PersistArgs pa{};
        pa.pbar = sb.pbar;
        pa.fro = sb.fro;
        pa.floor_scale = jacobi_floor_scale(g.m, sizeof(T));
        pa.max_sweeps = max_sweeps;
        // about a second of polling; TSVD_PERSIST_SPIN lowers it (tests of the fallback)
        pa.spin_limit = std::max(0, env_int("TSVD_PERSIST_SPIN", 1 << 21));
        pa.spread = env_int("TSVD_SPREAD", 0);
        hipError_t e = hipSuccess;
        const int ip = prof_launch(h, K_JAC_PERSIST, 0.0,
                                   [&] { e = launch_jacobi_persistent(ja, pa, h->cus, st); });
        if (e == hipSuccess) {
            // finishes the SVD only if a wait of the persistent launch gave up
            hip_check(launch_jacobi_slice<T>(plan.bw, plan.rpt, sb.ftab + (work == sb.Z ? 2 : 0) + vc,
                                             sb.fws, 1, g.h, max_sweeps, st),
                      "jacobi fallback");
        }
        if (e == hipSuccess) {
            done_persist = true;
            stats.sweeps = -1;   // known on the device only
            stats.on_device = true;
            if (h->prof_on) {
                // n(n-1)/2 visited pairs per slice per sweep run
                hip_check(hipMemcpyAsync(h->host_ints, sb.sweeps, sizeof(int) * g.h, hipMemcpyDeviceToHost, st),
                          "hipMemcpyAsync sweeps");
                hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
                int64_t sw = 0;
                int smax = 0;
                for (int s = 0; s < g.h; ++s) {
                    sw += h->host_ints[s];
                    smax = std::max(smax, h->host_ints[s]);
                }
                if (ip >= 0) {
                    h->pending[ip].work = pair_flops * slice_pairs * (double)sw;
                    h->pending[ip].sweeps = (double)sw;
                    h->pending[ip].pairs = slice_pairs * (double)sw;
                }
                stats.sweeps = smax;
            }
        } else {
            (void)hipGetLastError();
            if (ip >= 0) {
                // the timing events bracket nothing; drop the record
                h->ev_pool.push_back(h->pending[ip].a);
                h->ev_pool.push_back(h->pending[ip].b);
                h->pending.erase(h->pending.begin() + ip);
            }
        }
    }
    if (plan.mode == JacMode::PAIRS) {
        // one launch runs every sweep, one workgroup per block pair; the init
        // clears the rotation-flag ring, the role ticket, the barrier counters
        // and the block flags (the error word is cleared once per call)
        ja.nb = plan.nb;
        ja.rotations = h->rot_counter + 1;
        ja.clr[0] = sb.pbar;
        ja.nclr[0] = 4 * g.h;
        ja.clr[1] = sb.pbar + 4 * g.h + 1;
        ja.nclr[1] = g.h * (1 + plan.nb);
        prof_launch(h, K_JAC_INIT, (double)g.h * g.n * g.n * sizeof(cplx<T>),
                    [&] { launch_jacobi_init(ja, st); });
        launch_check("jacobi_init");
        ja.clr[0] = ja.clr[1] = nullptr;
        const int entry = (work == sb.Z ? 2 : 0) + vc;
        const int spin = std::max(0, env_int("TSVD_PERSIST_SPIN", 1 << 21));
        const int ip = prof_launch(h, K_JAC_PERSIST, 0.0, [&] {
            hip_check(launch_jacobi_pairs<T>(plan.bw, plan.rpt, sb.ftab + 4 + entry, sb.fws + 2, 1,
                                             g.h * (plan.nb / 2), sb.pbar + 4 * g.h - 1, spin, st),
                      "jacobi block pairs");
        });
        // finishes the SVD only if a wait between the workgroups gave up
        hip_check(launch_jacobi_slice<T>(plan.bw, plan.rpt, sb.ftab + entry, sb.fws, 1, g.h, max_sweeps, st),
                  "jacobi fallback");
        done_persist = true;
        stats.sweeps = -1;   // known on the device only
        stats.on_device = true;
        if (h->prof_on) {
            hip_check(hipMemcpyAsync(h->host_ints, sb.sweeps, sizeof(int) * g.h, hipMemcpyDeviceToHost, st),
                      "hipMemcpyAsync sweeps");
            hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
            int64_t sw = 0;
            int smax = 0;
            for (int s = 0; s < g.h; ++s) {
                sw += h->host_ints[s];
                smax = std::max(smax, h->host_ints[s]);
            }
            if (ip >= 0) {
                h->pending[ip].work = pair_flops * slice_pairs * (double)sw;
                h->pending[ip].sweeps = (double)sw;
                h->pending[ip].pairs = slice_pairs * (double)sw;
            }
            stats.sweeps = smax;
        }
    }
    if (!done_persist && sb.tall) {
        // tall slices: columns in global memory, two launches per round
        const TallPlan tp = jacobi_tall_plan(g.m, g.n, g.h);
        ja.nb = tp.players;
        prof_launch(h, K_JAC_INIT, (double)g.h * g.n * g.n * sizeof(cplx<T>),
                    [&] { launch_jacobi_init(ja, st); });
        launch_check("jacobi_init");
        ja.rotations = h->rot_counter + 1;
        for (int sw = 0; sw < max_sweeps; ++sw) {
            ja.sweep = sw;
            for (int r = 0; r < tp.players - 1; ++r) {
                ja.round = r;
                const int ip = prof_launch(h, K_JAC_CROSS, pair_flops * g.h * (tp.players / 2),
                                           [&] { launch_jacobi_tall_round(ja, tp, sb.tall, st); });
                if (ip >= 0) {
                    h->pending[ip].pairs = (double)g.h * (tp.players / 2);
                    if (r == 0) h->pending[ip].sweeps = g.h;
                }
                launch_check("jacobi_tall");
            }
            stats.sweeps = sw + 1;
            if ((sw + 1) % check_every == 0 || sw + 1 == max_sweeps) {
                hip_check(hipMemcpyAsync(h->host_ints, sb.rot + (sw % 3) * g.h, sizeof(int) * g.h,
                                         hipMemcpyDeviceToHost, st),
                          "hipMemcpyAsync rot");
                hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
                int active = 0;
                for (int s = 0; s < g.h; ++s) active += h->host_ints[s] != 0;
                if (!active) break;
            }
        }
        done_persist = true;
    }
    if (!done_persist) {
    ja.nb = jacobi_num_blocks(g.n, bw);
    prof_launch(h, K_JAC_INIT, (double)g.h * g.n * g.n * sizeof(cplx<T>),
                [&] { launch_jacobi_init(ja, st); });
    launch_check("jacobi_init");
    int active = g.h;   // slices still rotating, as last observed
    for (int sw = 0; sw < max_sweeps; ++sw) {
        ja.sweep = sw;
        ja.rotations = h->rot_counter;
        const double sp = (double)active * self_pairs(g.n, ja.nb);
        const int ip = prof_launch(h, K_JAC_SELF, pair_flops * sp, [&] { launch_jacobi_self(ja, bw, st); });
        if (ip >= 0) {
            h->pending[ip].pairs = sp;
            h->pending[ip].sweeps = active;
        }
        launch_check("jacobi_self");
        ja.rotations = h->rot_counter + 1;
        for (int r = 0; r < ja.nb - 1; ++r) {
            ja.round = r;
            const double cp = (double)active * cross_pairs(g.n, ja.nb, r);
            const int ic = prof_launch(h, K_JAC_CROSS, pair_flops * cp, [&] { launch_jacobi_cross(ja, bw, st); });
            if (ic >= 0) h->pending[ic].pairs = cp;
            launch_check("jacobi_cross");
        }
        stats.sweeps = sw + 1;
        if ((sw + 1) % check_every == 0 || sw + 1 == max_sweeps) {
            hip_check(hipMemcpyAsync(h->host_ints, sb.rot + (sw % 3) * g.h, sizeof(int) * g.h,
                                     hipMemcpyDeviceToHost, st),
                      "hipMemcpyAsync rot");
            hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
            active = 0;
            for (int s = 0; s < g.h; ++s) active += h->host_ints[s] != 0;
            if (!active) break;
        }
    }
    }
    // sigma_j = ||w_j||, then Zhat = W diag((1 - tau/sigma)_+) V^H on the matrix cores
    const int64_t slice_bytes = (int64_t)g.h * g.m * g.n * sizeof(cplx<T>);
    prof_launch(h, K_SVT_W, (double)slice_bytes + (double)g.h * g.n * sizeof(double),
                [&] { launch_svt_sigma(work, g.m, g.n, g.h, sb.sigma, sb.dk, h->ctrl, st); });
    launch_check("svt_sigma");
    ZGemmArgs<T> gr{};
    gr.A = work; gr.B = sb.V[vc]; gr.C = out;
    gr.M = g.m; gr.N = g.n; gr.K = g.n;
    gr.lda = g.m; gr.ldb = g.n; gr.ldc = g.m; gr.ldd = g.m;
    gr.sA = mn; gr.sB = nn; gr.sC = mn; gr.sD = mn;
    gr.alpha = (T)1; gr.beta = (T)0; gr.opA = 0; gr.opB = 1; gr.batch = g.h;
    gr.dk = sb.dk; gr.sdk = g.n; gr.ctrl = h->ctrl;
    gr.bf16x3 = env_int("TSVD_REBUILD_BF16", 0);
    gr.kcompact = env_int("TSVD_REBUILD_KEPT", 1);   // sum over the kept columns only
    if (rebuild) {
        const int ip = prof_launch(h, K_SVT_REBUILD, 8.0 * g.m * g.n * g.n * g.h, [&] { launch_zgemm(gr, st); });
        launch_check("svt_rebuild");
        if (ip >= 0 && !want_rank) {
            // the kept rank of every slice, for the rebuild's useful work
            launch_multirank(sb.sigma, g.n, g.n, g.h, h->ctrl, sb.rank, st);
            hip_check(hipMemcpyAsync(h->host_ints, sb.rank, sizeof(int) * g.h, hipMemcpyDeviceToHost, st),
                      "hipMemcpyAsync rank");
            hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
            double kept = 0.0;
            for (int s = 0; s < g.h; ++s) kept += h->host_ints[s];
            h->pending[ip].kept = kept;
        }
    }
    if (want_rank) {
        launch_multirank(sb.sigma, g.n, g.n, g.h, h->ctrl, sb.rank, st);
        launch_check("multirank");
    }
    if (h->prof_on) {
        // rotation work needs the device counts
        unsigned long long rots[2] = {0, 0};
        hip_check(hipMemcpyAsync(rots, h->rot_counter, sizeof(rots), hipMemcpyDeviceToHost, st),
                  "hipMemcpyAsync rotations");
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        hip_check(hipMemsetAsync(h->rot_counter, 0, 2 * sizeof(unsigned long long), st),
                  "hipMemsetAsync rotations");
        prof_harvest(h);
        h->agg[K_JAC_SELF].rotations += (double)rots[0];
        h->agg[done_persist ? K_JAC_PERSIST : K_JAC_CROSS].rotations += (double)rots[1];
    }
    if (warm) {
        warm->valid = true;
        warm->iter += 1;
    }
    stats.out = out;
    stats.w = work;
    stats.v = sb.V[vc];
    return stats;
}

void put_ctrl(tsvd_handle h, const Ctrl& c) {
    *h->host_ctrl = c;
    hip_check(hipMemcpyAsync(h->ctrl, h->host_ctrl, sizeof(Ctrl), hipMemcpyHostToDevice, h->stream),
              "hipMemcpyAsync ctrl");
    hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
}

Ctrl get_ctrl(tsvd_handle h) {
    hip_check(hipMemcpyAsync(h->host_ctrl, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream),
              "hipMemcpyAsync ctrl");
    hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return *h->host_ctrl;
}

void ensure_mirror(tsvd_handle h) {
    if (h->mirror_host) return;
    hip_check(hipHostMalloc(reinterpret_cast<void**>(&h->mirror_host), 2 * sizeof(Ctrl),
                            hipHostMallocMapped | hipHostMallocCoherent),
              "hipHostMalloc control mirror");
    hip_check(hipHostGetDevicePointer(reinterpret_cast<void**>(&h->mirror_dev), h->mirror_host, 0),
              "hipHostGetDevicePointer");
    for (auto& e : h->mirror_ev) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
}

struct LoopResult {
    Ctrl c;   // the control block after the last iteration
    int sweeps_total = 0, sweeps_last = 0;
};

// The ADMM loop of the single-problem calls.  iteration(k, mirror) queues
// iteration k, its control kernel copying the control block to `mirror`,
// and returns the largest sweep count of its SVDs when the host knows it,
// else -1 (then the device counts them in the control block).  The host
// stays one iteration behind the device: it reads the stop state of
// iteration k - 1 only after queueing iteration k, so the device does not
// wait for the host between iterations; every kernel of an iteration does
// nothing once ctrl->done is set, so the iteration queued after the stop
// changes nothing.
template <typename F>
LoopResult admm_loop(tsvd_handle h, int max_iter, F&& iteration) {
    ensure_mirror(h);
    std::vector<int> host_sweeps;
    host_sweeps.reserve(std::max(max_iter, 0));
    for (int k = 0; k < max_iter; ++k) {
        host_sweeps.push_back(iteration(k, h->mirror_dev + (k & 1)));
        hip_check(hipEventRecord(h->mirror_ev[k & 1], h->stream), "hipEventRecord");
        if (k > 0) {
            hip_check(hipEventSynchronize(h->mirror_ev[(k - 1) & 1]), "hipEventSynchronize");
            if (h->mirror_host[(k - 1) & 1].done) break;
        }
    }
    LoopResult r;
    r.c = get_ctrl(h);
    r.sweeps_total = r.c.sweeps_total;
    r.sweeps_last = r.c.sweeps_last;
    const int iters = std::min<int>(r.c.iter, (int)host_sweeps.size());
    for (int k = 0; k < iters; ++k)
        if (host_sweeps[k] >= 0) r.sweeps_total += host_sweeps[k];
    if (iters > 0 && host_sweeps[iters - 1] >= 0) r.sweeps_last = host_sweeps[iters - 1];
    return r;
}

void clear_flag(tsvd_handle h) { launch_fill<int>(h->flag, 0, 1, h->stream); }

// Error word of the persistent Jacobi launches (pbar[4h]): cleared once per
// call; bit 1 (a wait between workgroups gave up) only makes the fallback
// kernel finish the SVDs, bit 2 (a wait inside a workgroup ran out: a fault)
// fails the call.
template <typename T>
void clear_persist_err(tsvd_handle h, const Geometry& g, const SvtBuffers<T>& sb) {
    launch_fill<int>(sb.pbar + 4 * g.h, 0, 1, h->stream);
}

template <typename T>
void check_persist_err(tsvd_handle h, const Geometry& g, const SvtBuffers<T>& sb) {
    ensure_host_ints(h, 1);
    hip_check(hipMemcpyAsync(h->host_ints, sb.pbar + 4 * g.h, sizeof(int), hipMemcpyDeviceToHost, h->stream),
              "hipMemcpyAsync err");
    hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    if (h->host_ints[0] & 2) fail(TSVD_E_HIP, "a Jacobi step wait inside a workgroup ran out");
}

// largest per-slice sweep count of the last SVD (read after a sync)
bool read_flag(tsvd_handle h) {
    ensure_host_ints(h, 1);
    hip_check(hipMemcpyAsync(h->host_ints, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream),
              "hipMemcpyAsync flag");
    hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return h->host_ints[0] != 0;
}

int elementwise_parts() { return 1024; }

// Checks of a solver state (include/tsvd.h, tsvd_state).
void check_state(const tsvd_state* st, bool rpca) {
    if (!st) return;
    if (!st->z || !st->dual || (rpca && !st->s)) fail(TSVD_E_INVALID, "state: null iterate pointer");
    if (st->iter < 0) fail(TSVD_E_INVALID, "state: iter must be >= 0");
    if (st->load && (!(st->penalty > 0.0) || !std::isfinite(st->penalty) || !(st->dual_scale > 0.0) ||
                     !std::isfinite(st->dual_scale)))
        fail(TSVD_E_INVALID, "state: penalty and dual_scale must be finite and > 0");
}

void copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t st) {
    hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync state");
}

}  // namespace

// t-SVT.  scratch == nullptr: workspace and DFT matrices of the handle
// (allocated or grown as needed); otherwise both are carved from `scratch`
// (the no-allocation entry point), the DFT matrices built on the device.
template <typename T>
void do_tsvt(tsvd_handle h, const void* X, tsvd_shape shape, tsvd_dtype dtype, double tau,
                 tsvd_precision precision, void* Z, int32_t* multirank_host, char* scratch = nullptr) {
        check_handle(h);
        if (!X || !Z) fail(TSVD_E_INVALID, "null tensor pointer");
        if (!(tau >= 0.0) || !std::isfinite(tau)) fail(TSVD_E_INVALID, "tau must be finite and >= 0");
        
        const Geometry g = make_geometry(shape);
        if (!jacobi_supported(g.m, g.n, sizeof(T))) fail(TSVD_E_SHAPE, "slice too large for the Jacobi kernels");
        Device dev(h->device);
        const int nparts = (int)dft_grid(g, dft_inverse_tile(g, EPI_STORE));
        const T* dmat = nullptr;
        SvtBuffers<T> sb;
        if (!scratch) {
            ensure_workspace(h, svt_bytes<T>(g, nparts) + 4096);
            Carver cv{reinterpret_cast<char*>(h->ws)};
            sb = carve_svt<T>(cv, g, nparts);
            dmat = ensure_dft_matrices<T>(h, g);
        } else {
            const int64_t mat_elems = DftDims::of(g.h, g.L).total();
            const size_t need = svt_bytes<T>(g, nparts) + mat_elems * sizeof(T) + 4096;
            if (need > kScratchBytes)
                fail(TSVD_E_NOMEM, "t-SVT of this shape needs " + std::to_string(need) +
                                       " bytes of workspace, over the no-allocation scratch of " +
                                       std::to_string(kScratchBytes) + " bytes");
            Carver cv{scratch};
            sb = carve_svt<T>(cv, g, nparts);
            T* mat = cv.take<T>(mat_elems);
            launch_dft_matrices<T>(mat, g, h->stream);
            launch_check("dft matrices");
            dmat = mat;
        }
        upload_fallback<T>(h, g, sb, 30);
        Ctrl c{};
        c.rho = tau > 0 ? 1.0 / tau : INFINITY;
        c.tau = tau;
        c.dscale = 1.0;
        put_ctrl(h, c);
        clear_flag(h);
        clear_persist_err(h, g, sb);

        FwdArgs<T> fa{};
        fa.x = static_cast<const T*>(X);
        fa.ctrl = h->ctrl;
        fa.mat = dmat;
        fa.out = sb.A;
        fa.nonfinite = h->flag;
        fa.g = g;
        fa.tile = dft_forward_tile(g);
        const double slice_bytes = (double)g.h * g.m * g.n * sizeof(cplx<T>);
        prof_launch(h, K_DFT_FWD, slice_bytes + (double)g.numel * sizeof(T),
                    [&] { launch_dft_forward(PRO_COPY, fa, h->stream); });
        launch_check("dft_forward");
        const SweepStats ss = run_svt<T>(h, g, sb, 30, nullptr, multirank_host != nullptr);
        InvArgs<T> ia{};
        ia.in = static_cast<const cplx<T>*>(ss.out);
        ia.mat = dmat + DftDims::of(g.h, g.L).fwd_size();
        ia.ctrl = h->ctrl;
        ia.g = g;
        ia.tile = dft_inverse_tile(g, EPI_STORE);
        ia.out = static_cast<T*>(Z);
        prof_launch(h, K_DFT_INV, slice_bytes + (double)g.numel * sizeof(T),
                    [&] { launch_dft_inverse(EPI_STORE, ia, h->stream); });
        launch_check("dft_inverse");
        if (multirank_host) {
            ensure_host_ints(h, g.h);
            hip_check(hipMemcpyAsync(h->host_ints, sb.rank, sizeof(int) * g.h, hipMemcpyDeviceToHost,
                                     h->stream),
                      "hipMemcpyAsync rank");
        }
        hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        if (multirank_host) std::memcpy(multirank_host, h->host_ints, sizeof(int) * g.h);
        prof_harvest(h);
        check_persist_err(h, g, sb);
        if (read_flag(h)) fail(TSVD_E_NONFINITE, "non-finite input");
}

// The slice SVDs of M with nothing thresholded (Sec. 2.2, Algorithm 1):
// forward DFT, cold Jacobi (up to 30 sweeps), singular values, and in 4-D
// the conjugate pairs inside the half spectrum mirrored.  `extra` bytes of
// workspace stay free after the SVD buffers for the caller's carver.
template <typename T>
struct SvdStage {
    SvtBuffers<T> sb;
    SweepStats ss;
    Carver cv{nullptr};
    const T* dmat = nullptr;
};

template <typename T>
SvdStage<T> svd_stage(tsvd_handle h, const Geometry& g, const void* X, size_t extra) {
    const int nparts = (int)dft_grid(g, dft_inverse_tile(g, EPI_STORE));
    ensure_workspace(h, svt_bytes<T>(g, nparts) + extra + 4096);
    SvdStage<T> st;
    st.cv = Carver{reinterpret_cast<char*>(h->ws)};
    st.sb = carve_svt<T>(st.cv, g, nparts);
    st.dmat = ensure_dft_matrices<T>(h, g);
    upload_fallback<T>(h, g, st.sb, 30);
    Ctrl c{};
    c.rho = INFINITY;
    c.tau = 0.0;
    c.dscale = 1.0;
    put_ctrl(h, c);
    clear_flag(h);
    clear_persist_err(h, g, st.sb);
    FwdArgs<T> fa{};
    fa.x = static_cast<const T*>(X);
    fa.ctrl = h->ctrl;
    fa.mat = st.dmat;
    fa.out = st.sb.A;
    fa.nonfinite = h->flag;
    fa.g = g;
    fa.tile = dft_forward_tile(g);
    const double slice_bytes = (double)g.h * g.m * g.n * sizeof(cplx<T>);
    prof_launch(h, K_DFT_FWD, slice_bytes + (double)g.numel * sizeof(T),
                [&] { launch_dft_forward(PRO_COPY, fa, h->stream); });
    launch_check("dft_forward");
    st.ss = run_svt<T>(h, g, st.sb, 30, nullptr, false, false);
    launch_tsvd_mirror<T>(static_cast<cplx<T>*>(const_cast<void*>(st.ss.w)),
                          static_cast<cplx<T>*>(const_cast<void*>(st.ss.v)), st.sb.sigma, g, h->stream);
    launch_check("tsvd_mirror");
    return st;
}

// Real inverse transform (EPI_STORE) of h slices of a tensor of geometry gf
// that shares the trailing modes of the DFT matrices in dmat.
template <typename T>
void inverse_store(tsvd_handle h, const Geometry& gf, const T* dmat, const cplx<T>* in, T* out) {
    InvArgs<T> ia{};
    ia.in = in;
    ia.mat = dmat + DftDims::of(gf.h, gf.L).fwd_size();
    ia.ctrl = h->ctrl;
    ia.g = gf;
    ia.tile = dft_inverse_tile(gf, EPI_STORE);
    ia.out = out;
    prof_launch(h, K_DFT_INV, (double)gf.h * gf.m * gf.n * sizeof(cplx<T>) + (double)gf.numel * sizeof(T),
                [&] { launch_dft_inverse(EPI_STORE, ia, h->stream); });
    launch_check("dft_inverse");
}

// The geometry of a tensor with matrix modes a x b and the trailing modes of s.
Geometry factor_geometry(const tsvd_shape& s, int64_t a, int64_t b) {
    tsvd_shape f = s;
    f.n[0] = a;
    f.n[1] = b;
    return make_geometry(f);
}

template <typename T>
void finish_call(tsvd_handle h, const Geometry& g, const SvtBuffers<T>& sb) {
    hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    prof_harvest(h);
    check_persist_err(h, g, sb);
    if (read_flag(h)) fail(TSVD_E_NONFINITE, "non-finite input");
}

template <typename T>
void do_factors(tsvd_handle h, const void* M, tsvd_shape shape, void* U_out, void* S_out, void* V_out) {
    check_handle(h);
    if (!M || !U_out || !S_out || !V_out) fail(TSVD_E_INVALID, "null tensor pointer");
    const Geometry g = make_geometry(shape);
    if (!jacobi_supported(g.m, g.n, sizeof(T))) fail(TSVD_E_SHAPE, "slice too large for the Jacobi kernels");
    Device dev(h->device);
    const int64_t n0 = g.n, n1 = g.n1, n2 = g.n2, hn = (int64_t)g.h * g.n;
    const size_t extra = hn * sizeof(int) + (size_t)g.h * (n1 + n2 + 1) * n0 * sizeof(cplx<T>) + 4 * 256;
    SvdStage<T> st = svd_stage<T>(h, g, M, extra);
    Carver cv = st.cv;
    int* rank = cv.take<int>(hn);
    cplx<T>* Uh = cv.take<cplx<T>>((int64_t)g.h * n1 * n0);
    cplx<T>* Vh = cv.take<cplx<T>>((int64_t)g.h * n2 * n0);
    cplx<T>* Sh = cv.take<cplx<T>>((int64_t)g.h * n0);
    launch_tsvd_rank(st.sb.sigma, g.n, g.h, rank, h->stream);
    launch_tsvd_factors<T>(static_cast<const cplx<T>*>(st.ss.w), static_cast<const cplx<T>*>(st.ss.v), st.sb.sigma,
                           rank, g, Uh, Vh, Sh, h->stream);
    launch_check("tsvd_factors");
    inverse_store<T>(h, factor_geometry(shape, n1, n0), st.dmat, Uh, static_cast<T*>(U_out));
    inverse_store<T>(h, factor_geometry(shape, n2, n0), st.dmat, Vh, static_cast<T*>(V_out));
    inverse_store<T>(h, factor_geometry(shape, n0, 1), st.dmat, Sh, static_cast<T*>(S_out));
    finish_call<T>(h, g, st.sb);
}

template <typename T>
void do_compress(tsvd_handle h, const void* M, tsvd_shape shape, int32_t method, int64_t k, void* M_out,
                 double* ratio_host) {
    check_handle(h);
    if (!M || !M_out) fail(TSVD_E_INVALID, "null tensor pointer");
    if (shape.ndim != 3) fail(TSVD_E_SHAPE, "the compression methods are stated for third-order tensors");
    const Geometry g = make_geometry(shape);
    if (!jacobi_supported(g.m, g.n, sizeof(T))) fail(TSVD_E_SHAPE, "slice too large for the Jacobi kernels");
    const int64_t n0 = g.n, n1 = g.n1, n2 = g.n2, n3 = g.L;
    if (method == TSVD_COMPRESS_TSVD) {
        if (k < 1 || k > n0 * n3) fail(TSVD_E_INVALID, "Method 1 needs 1 <= k <= min(n1, n2) n3");
    } else if (method == TSVD_COMPRESS_TUBAL) {
        if (k < 1 || k > n0) fail(TSVD_E_INVALID, "Method 2 needs 1 <= k <= min(n1, n2)");
    } else {
        fail(TSVD_E_INVALID, "unknown compression method");
    }
    Device dev(h->device);
    const int64_t hn = (int64_t)g.h * g.n;
    SvdStage<T> st = svd_stage<T>(h, g, M, hn * sizeof(int) + 256);
    if (method == TSVD_COMPRESS_TUBAL) {
        Carver cv = st.cv;
        int* rank = cv.take<int>(hn);
        launch_tsvd_rank(st.sb.sigma, g.n, g.h, rank, h->stream);
        launch_tubal_select(rank, hn, (int)k, st.sb.dk, h->stream);
    } else {
        launch_global_select(st.sb.sigma, g, k, st.sb.dk, h->stream);
    }
    launch_check("select");
    // the kept triplets: W diag(d) V^H with d in {0, 1}
    const cplx<T>* W = static_cast<const cplx<T>*>(st.ss.w);
    cplx<T>* out = W == st.sb.A ? st.sb.Z : st.sb.A;
    const int64_t mn = (int64_t)g.m * g.n, nn = (int64_t)g.n * g.n;
    ZGemmArgs<T> gr{};
    gr.A = W; gr.B = static_cast<const cplx<T>*>(st.ss.v); gr.C = out;
    gr.M = g.m; gr.N = g.n; gr.K = g.n;
    gr.lda = g.m; gr.ldb = g.n; gr.ldc = g.m; gr.ldd = g.m;
    gr.sA = mn; gr.sB = nn; gr.sC = mn; gr.sD = mn;
    gr.alpha = (T)1; gr.beta = (T)0; gr.opA = 0; gr.opB = 1; gr.batch = g.h;
    gr.dk = st.sb.dk; gr.sdk = g.n; gr.ctrl = h->ctrl;
    prof_launch(h, K_SVT_REBUILD, 8.0 * g.m * g.n * g.n * g.h, [&] { launch_zgemm(gr, h->stream); });
    launch_check("compress_rebuild");
    inverse_store<T>(h, g, st.dmat, out, static_cast<T*>(M_out));
    finish_call<T>(h, g, st.sb);
    if (ratio_host)
        *ratio_host = method == TSVD_COMPRESS_TSVD ? (double)(n1 * n2 * n3) / ((double)k * (double)(n1 + n2 + 1))
                                                   : (double)(n1 * n2) / ((double)k * (double)(n1 + n2 + 1));
}

template <typename T>
void do_complete(tsvd_handle h, const void* X_obs, const uint8_t* mask, tsvd_shape shape,
                          tsvd_dtype dtype, double rho, double tol, const tsvd_admm_opts* opts,
                          void* X_out, tsvd_info* info_host) {
        const auto t0 = std::chrono::steady_clock::now();
        check_handle(h);
        if (!X_obs || !mask || !X_out) fail(TSVD_E_INVALID, "null tensor pointer");
        if (!(rho > 0.0) || !std::isfinite(rho)) fail(TSVD_E_INVALID, "rho must be > 0");
        if (!(tol >= 0.0) || !std::isfinite(tol)) fail(TSVD_E_INVALID, "tol must be >= 0");
        const AdmmSettings s = settings(opts, 1.1, 1e3, 300);
        if (s.rho_max < rho) fail(TSVD_E_INVALID, "rho_max must be >= rho");
        
        const Geometry g = make_geometry(shape);
        if (!jacobi_supported(g.m, g.n, sizeof(T))) fail(TSVD_E_SHAPE, "slice too large for the Jacobi kernels");
        Device dev(h->device);
        const int tile_i = dft_inverse_tile(g, EPI_COMPLETE);
        const int nparts = (int)std::max<int64_t>(dft_grid(g, tile_i), elementwise_parts());
        const int64_t N = g.numel;
        ensure_workspace(h, svt_bytes<T>(g, nparts) + 4 * (N * sizeof(T) + 256) + 4096);
        Carver cv{reinterpret_cast<char*>(h->ws)};
        SvtBuffers<T> sb = carve_svt<T>(cv, g, nparts);
        T* Zb[2] = {cv.take<T>(N), cv.take<T>(N)};
        T* Qb[2] = {cv.take<T>(N), cv.take<T>(N)};
        const T* dmat = ensure_dft_matrices<T>(h, g);
        hipStream_t st = h->stream;
        const T* Y = static_cast<const T*>(X_obs);
        const tsvd_state* state = s.state;
        check_state(state, false);
        const bool load = state && state->load;
        const int64_t vv_bytes = (int64_t)g.h * g.n * g.n * sizeof(cplx<T>);
        upload_fallback<T>(h, g, sb, s.max_sweeps);
        WarmState warm;
        warm.enabled = env_int("TSVD_WARM", 1) != 0;
        // one Newton-Schulz refresh of V every 2 iterations in the FP32 form, every 4 in FP64
        warm.reorth_every = env_int("TSVD_REORTH_EVERY", sizeof(T) == 4 ? 2 : 4);
        if (load) {
            copy_d2d(Zb[0], state->z, N * sizeof(T), st);
            copy_d2d(Qb[0], state->dual, N * sizeof(T), st);
            warm.iter = state->iter;
            if (state->v) {
                copy_d2d(sb.V[0], state->v, vv_bytes, st);
                warm.valid = true;
            }
        } else {
            launch_fill<T>(Zb[0], 0.0, N, st);
            launch_fill<T>(Qb[0], 0.0, N, st);
        }
        const double rho0 = load ? state->penalty : rho;
        const double ds0 = load ? state->dual_scale : 1.0;
        Ctrl c{};
        c.rho = rho0;
        c.tau = 1.0 / rho0;
        c.dscale = ds0;
        c.dscale_used = ds0;
        c.growth = s.growth;
        c.rho_max = s.rho_max;
        c.rho_used = rho0;
        put_ctrl(h, c);
        launch_sumsq<T>(Y, mask, N, sb.partials, elementwise_parts(), st);
        launch_set_tol(h->ctrl, sb.partials, elementwise_parts(), tol, st);
        launch_check("setup");
        clear_flag(h);
        clear_persist_err(h, g, sb);

        FwdArgs<T> fa{};
        fa.x = Y;
        fa.mask = mask;
        fa.ctrl = h->ctrl;
        fa.mat = dmat;
        fa.out = sb.A;
        fa.nonfinite = h->flag;
        fa.g = g;
        fa.tile = dft_forward_tile(g);
        InvArgs<T> ia{};
        ia.in = sb.Z;
        ia.mat = dmat + DftDims::of(g.h, g.L).fwd_size();
        ia.ctrl = h->ctrl;
        ia.g = g;
        ia.tile = tile_i;
        ia.y = Y;
        ia.mask = mask;
        ia.partials = sb.partials;
        const int inv_parts = (int)dft_grid(g, tile_i);
        const double slice_bytes = (double)g.h * g.m * g.n * sizeof(cplx<T>);
        int sweeps_total = 0, sweeps_last = 0, iters = 0;
        Ctrl hc{};
        std::vector<int> vcur_after;   // V buffer holding each queued iteration's V
        const LoopResult lr = admm_loop(h, s.max_iter, [&](int k, Ctrl* mirror) -> int {
            fa.z = Zb[k % 2];
            fa.dual = Qb[k % 2];
            // Y, mask, Z, Q in; slices out
            prof_launch(h, K_DFT_FWD, slice_bytes + (double)N * (3 * sizeof(T) + 1),
                        [&] { launch_dft_forward(PRO_COMPLETE, fa, st); });
            launch_check("dft_forward");
            const SweepStats ss = run_svt<T>(h, g, sb, s.max_sweeps, &warm);
            ia.in = static_cast<const cplx<T>*>(ss.out);
            ia.out = Zb[(k + 1) % 2];
            ia.z_old = Zb[k % 2];
            ia.dual_old = Qb[k % 2];
            ia.dual_new = Qb[(k + 1) % 2];
            // slices, Y, mask, Z, Q in; Z', Q~ out
            prof_launch(h, K_DFT_INV, slice_bytes + (double)N * (5 * sizeof(T) + 1),
                        [&] { launch_dft_inverse(EPI_COMPLETE, ia, st); });
            launch_check("dft_inverse");
            prof_launch(h, K_CTRL, (double)inv_parts * kNumPartials * sizeof(double),
                        [&] { launch_admm_ctrl(h->ctrl, sb.partials, inv_parts, 0, mirror, st); });
            launch_check("admm_ctrl");
            vcur_after.push_back(warm.vcur);
            return ss.on_device ? -1 : ss.sweeps;
        });
        hc = lr.c;
        iters = hc.iter;
        sweeps_total = lr.sweeps_total;
        sweeps_last = lr.sweeps_last;
        launch_complete_output<T>(Y, mask, Zb[(iters - 1) % 2], Qb[(iters - 1) % 2], h->ctrl,
                                  static_cast<T*>(X_out), N, st);
        launch_check("complete_output");
        if (state && state->save) {
            copy_d2d(state->z, Zb[iters % 2], N * sizeof(T), st);
            copy_d2d(state->dual, Qb[iters % 2], N * sizeof(T), st);
            if (state->v) copy_d2d(state->v, sb.V[vcur_after[iters - 1]], vv_bytes, st);
        }
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        prof_harvest(h);
        check_persist_err(h, g, sb);
        if (hc.nonfinite || read_flag(h)) fail(TSVD_E_NONFINITE, "non-finite input or iterate");
        if (state && state->save) {
            tsvd_state* out = const_cast<tsvd_state*>(state);
            out->penalty = hc.rho;
            out->dual_scale = hc.dscale;
            out->iter = (load ? state->iter : 0) + iters;
        }
        if (info_host) {
            info_host->iters = iters;
            info_host->converged = hc.done ? 1 : 0;
            info_host->sweeps_total = sweeps_total;
            info_host->sweeps_last = sweeps_last;
            info_host->primal = hc.primal;
            info_host->change = hc.change;
            info_host->rho_final = hc.rho_used;
            info_host->seconds =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
}

template <typename T>
void do_trpca(tsvd_handle h, const void* X, tsvd_shape shape, tsvd_dtype dtype, double lambda,
                  double mu, double tol, tsvd_shrink shrink, const tsvd_admm_opts* opts, void* L_out,
                  void* S_out, tsvd_info* info_host) {
        const auto t0 = std::chrono::steady_clock::now();
        check_handle(h);
        if (!X || !L_out || !S_out) fail(TSVD_E_INVALID, "null tensor pointer");
        if (!(lambda > 0.0) || !std::isfinite(lambda)) fail(TSVD_E_INVALID, "lambda must be > 0");
        if (!(mu > 0.0) || !std::isfinite(mu)) fail(TSVD_E_INVALID, "mu must be > 0");
        if (!(tol >= 0.0) || !std::isfinite(tol)) fail(TSVD_E_INVALID, "tol must be >= 0");
        if (shrink != TSVD_SHRINK_L1 && shrink != TSVD_SHRINK_L112) fail(TSVD_E_INVALID, "unknown shrink");
        const AdmmSettings s = settings(opts, 1.2, 1e10, 500);
        if (s.rho_max < mu) fail(TSVD_E_INVALID, "rho_max must be >= mu");
        
        const Geometry g = make_geometry(shape);
        if (!jacobi_supported(g.m, g.n, sizeof(T))) fail(TSVD_E_SHAPE, "slice too large for the Jacobi kernels");
        Device dev(h->device);
        const int epi = shrink == TSVD_SHRINK_L1 ? EPI_RPCA_L1 : EPI_RPCA_L112;
        const int tile_i = dft_inverse_tile(g, epi);
        const int nparts = (int)std::max<int64_t>(dft_grid(g, tile_i), elementwise_parts());
        const int64_t N = g.numel;
        ensure_workspace(h, svt_bytes<T>(g, nparts) + 6 * (N * sizeof(T) + 256) + 4096);
        Carver cv{reinterpret_cast<char*>(h->ws)};
        SvtBuffers<T> sb = carve_svt<T>(cv, g, nparts);
        T* Lb[2] = {cv.take<T>(N), cv.take<T>(N)};
        T* Sb[2] = {cv.take<T>(N), cv.take<T>(N)};
        T* Wb[2] = {cv.take<T>(N), cv.take<T>(N)};
        const T* dmat = ensure_dft_matrices<T>(h, g);
        hipStream_t st = h->stream;
        const T* M = static_cast<const T*>(X);
        const tsvd_state* state = s.state;
        check_state(state, true);
        const bool load = state && state->load;
        const int64_t vv_bytes = (int64_t)g.h * g.n * g.n * sizeof(cplx<T>);
        upload_fallback<T>(h, g, sb, s.max_sweeps);
        WarmState warm;
        warm.enabled = env_int("TSVD_WARM", 1) != 0;
        // one Newton-Schulz refresh of V every 2 iterations in the FP32 form, every 4 in FP64
        warm.reorth_every = env_int("TSVD_REORTH_EVERY", sizeof(T) == 4 ? 2 : 4);
        if (load) {
            copy_d2d(Lb[0], state->z, N * sizeof(T), st);
            copy_d2d(Sb[0], state->s, N * sizeof(T), st);
            copy_d2d(Wb[0], state->dual, N * sizeof(T), st);
            warm.iter = state->iter;
            if (state->v) {
                copy_d2d(sb.V[0], state->v, vv_bytes, st);
                warm.valid = true;
            }
        } else {
            launch_fill<T>(Lb[0], 0.0, N, st);
            launch_fill<T>(Sb[0], 0.0, N, st);
            launch_fill<T>(Wb[0], 0.0, N, st);
        }
        const double mu0 = load ? state->penalty : mu;
        const double ds0 = load ? state->dual_scale : 1.0;
        Ctrl c{};
        c.rho = mu0;
        c.tau = 1.0 / mu0;
        c.dscale = ds0;
        c.dscale_used = ds0;
        c.growth = s.growth;
        c.rho_max = s.rho_max;
        c.lambda = lambda;
        c.shrink = lambda / mu0;
        c.rho_used = mu0;
        put_ctrl(h, c);
        launch_sumsq<T>(M, nullptr, N, sb.partials, elementwise_parts(), st);
        launch_set_tol(h->ctrl, sb.partials, elementwise_parts(), tol, st);
        launch_check("setup");
        clear_flag(h);
        clear_persist_err(h, g, sb);

        FwdArgs<T> fa{};
        fa.x = M;
        fa.ctrl = h->ctrl;
        fa.mat = dmat;
        fa.out = sb.A;
        fa.nonfinite = h->flag;
        fa.g = g;
        fa.tile = dft_forward_tile(g);
        InvArgs<T> ia{};
        ia.in = sb.Z;
        ia.mat = dmat + DftDims::of(g.h, g.L).fwd_size();
        ia.ctrl = h->ctrl;
        ia.g = g;
        ia.tile = tile_i;
        ia.m = M;
        ia.partials = sb.partials;
        const int inv_parts = (int)dft_grid(g, tile_i);
        const double slice_bytes = (double)g.h * g.m * g.n * sizeof(cplx<T>);
        int sweeps_total = 0, sweeps_last = 0, iters = 0;
        Ctrl hc{};
        std::vector<int> vcur_after;   // V buffer holding each queued iteration's V
        const LoopResult lr = admm_loop(h, s.max_iter, [&](int k, Ctrl* mirror) -> int {
            fa.s = Sb[k % 2];
            fa.dual = Wb[k % 2];
            // M, S, W in; slices out
            prof_launch(h, K_DFT_FWD, slice_bytes + (double)N * 3 * sizeof(T),
                        [&] { launch_dft_forward(PRO_RPCA, fa, st); });
            launch_check("dft_forward");
            const SweepStats ss = run_svt<T>(h, g, sb, s.max_sweeps, &warm);
            ia.in = static_cast<const cplx<T>*>(ss.out);
            ia.out = Lb[(k + 1) % 2];
            ia.l_old = Lb[k % 2];
            ia.s_old = Sb[k % 2];
            ia.s_new = Sb[(k + 1) % 2];
            ia.dual_old = Wb[k % 2];
            ia.dual_new = Wb[(k + 1) % 2];
            // slices, M, W, S, L in; L', S', W~ out
            prof_launch(h, K_DFT_INV, slice_bytes + (double)N * 7 * sizeof(T),
                        [&] { launch_dft_inverse(epi, ia, st); });
            launch_check("dft_inverse");
            prof_launch(h, K_CTRL, (double)inv_parts * kNumPartials * sizeof(double),
                        [&] { launch_admm_ctrl(h->ctrl, sb.partials, inv_parts, 1, mirror, st); });
            launch_check("admm_ctrl");
            vcur_after.push_back(warm.vcur);
            return ss.on_device ? -1 : ss.sweeps;
        });
        hc = lr.c;
        iters = hc.iter;
        sweeps_total = lr.sweeps_total;
        sweeps_last = lr.sweeps_last;
        hip_check(hipMemcpyAsync(L_out, Lb[iters % 2], N * sizeof(T), hipMemcpyDeviceToDevice, st),
                  "hipMemcpyAsync L");
        hip_check(hipMemcpyAsync(S_out, Sb[iters % 2], N * sizeof(T), hipMemcpyDeviceToDevice, st),
                  "hipMemcpyAsync S");
        if (state && state->save) {
            copy_d2d(state->z, Lb[iters % 2], N * sizeof(T), st);
            copy_d2d(state->s, Sb[iters % 2], N * sizeof(T), st);
            copy_d2d(state->dual, Wb[iters % 2], N * sizeof(T), st);
            if (state->v) copy_d2d(state->v, sb.V[vcur_after[iters - 1]], vv_bytes, st);
        }
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        prof_harvest(h);
        check_persist_err(h, g, sb);
        if (hc.nonfinite || read_flag(h)) fail(TSVD_E_NONFINITE, "non-finite input or iterate");
        if (state && state->save) {
            tsvd_state* out = const_cast<tsvd_state*>(state);
            out->penalty = hc.rho;
            out->dual_scale = hc.dscale;
            out->iter = (load ? state->iter : 0) + iters;
        }
        if (info_host) {
            info_host->iters = iters;
            info_host->converged = hc.done ? 1 : 0;
            info_host->sweeps_total = sweeps_total;
            info_host->sweeps_last = sweeps_last;
            info_host->primal = hc.primal;
            info_host->change = hc.change;
            info_host->rho_final = hc.rho_used;
            info_host->seconds =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
}

// ---------------------------------------------------------------- C ABI

extern "C" {

tsvd_status tsvd_create(int device, size_t hbm_budget_bytes, tsvd_handle* out) {
    return guarded([&] {
        if (!out) fail(TSVD_E_INVALID, "out is NULL");
        *out = nullptr;
        int count = 0;
        hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
        if (device < 0 || device >= count) fail(TSVD_E_INVALID, "no such device");
        Device dev(device);
        int lds_max = 0;
        if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
                hipSuccess &&
            lds_max > 0)
            jacobi_set_lds_limit((size_t)std::min(lds_max, env_int("TSVD_LDS_LIMIT", lds_max)));
        tsvd_handle h = new tsvd_handle_s();
        h->device = device;
        (void)hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, device);
        h->lds_cap = lds_max > 0 ? (size_t)lds_max : 65536;
        h->budget = hbm_budget_bytes;
        hipError_t e = hipMalloc(reinterpret_cast<void**>(&h->ctrl), sizeof(Ctrl));
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&h->flag), sizeof(int));
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&h->host_ctrl), sizeof(Ctrl), 0);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&h->rot_counter), 2 * sizeof(unsigned long long));
        if (e == hipSuccess) e = hipMemset(h->rot_counter, 0, 2 * sizeof(unsigned long long));
        // host staging sized for every shape, so later calls never allocate it
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&h->host_ints), sizeof(int) * kMaxSlices, 0);
        if (e == hipSuccess) h->host_ints_len = kMaxSlices;
        if (e == hipSuccess) e = hipHostMalloc(&h->host_stage, 4096, 0);
        if (e == hipSuccess) h->host_stage_len = 4096;
        h->agg.assign(K_COUNT, tsvd_handle_s::Agg{});
        if (e != hipSuccess) {
            if (h->ctrl) (void)hipFree(h->ctrl);
            if (h->flag) (void)hipFree(h->flag);
            if (h->rot_counter) (void)hipFree(h->rot_counter);
            if (h->host_ctrl) (void)hipHostFree(h->host_ctrl);
            if (h->host_ints) (void)hipHostFree(h->host_ints);
            if (h->host_stage) (void)hipHostFree(h->host_stage);
            delete h;
            fail(TSVD_E_HIP, std::string("handle allocation: ") + hipGetErrorString(e));
        }
        try {
            h->scratch = scratch_address(device);
        } catch (...) {
            tsvd_destroy(h);
            throw;
        }
        *out = h;
    });
}

tsvd_status tsvd_destroy(tsvd_handle h) {
    if (!h) return TSVD_OK;
    return guarded([&] {
        serve_shutdown(h);
        Device dev(h->device);
        if (h->stream) (void)hipStreamSynchronize(h->stream);
        else (void)hipDeviceSynchronize();
        if (h->ws) (void)hipFree(h->ws);
        if (h->dmat) (void)hipFree(h->dmat);
        if (h->ctrl) (void)hipFree(h->ctrl);
        if (h->flag) (void)hipFree(h->flag);
        if (h->host_ints) (void)hipHostFree(h->host_ints);
        if (h->host_stage) (void)hipHostFree(h->host_stage);
        if (h->host_ctrl) (void)hipHostFree(h->host_ctrl);
        if (h->mirror_host) (void)hipHostFree(h->mirror_host);
        for (auto e : h->mirror_ev)
            if (e) (void)hipEventDestroy(e);
        if (h->rot_counter) (void)hipFree(h->rot_counter);
        for (auto& p : h->pending) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        for (auto e : h->ev_pool) (void)hipEventDestroy(e);
        delete h;
    });
}

tsvd_status tsvd_set_stream(tsvd_handle h, void* hip_stream) {
    return guarded([&] {
        check_handle(h);
        h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    });
}

tsvd_status tsvt(tsvd_handle h, const void* X, tsvd_shape shape, tsvd_dtype dtype, double tau,
                 tsvd_precision precision, void* Z, int32_t* multirank_host) {
    return guarded([&] {
        check_handle(h);
        if (check_precision(dtype, precision))
            do_tsvt<float>(h, X, shape, dtype, tau, precision, Z, multirank_host);
        else
            do_tsvt<double>(h, X, shape, dtype, tau, precision, Z, multirank_host);
    });
}

tsvd_status tsvt_noalloc(tsvd_handle h, const void* X, tsvd_shape shape, tsvd_dtype dtype, double tau,
                         tsvd_precision precision, void* Z, int32_t* multirank_host) {
    return guarded([&] {
        check_handle(h);
        // no events are created for this call: profiling records nothing
        const bool prof = h->prof_on;
        h->prof_on = false;
        struct Restore {
            tsvd_handle h;
            bool prof;
            ~Restore() { h->prof_on = prof; }
        } restore{h, prof};
        if (check_precision(dtype, precision))
            do_tsvt<float>(h, X, shape, dtype, tau, precision, Z, multirank_host, h->scratch);
        else
            do_tsvt<double>(h, X, shape, dtype, tau, precision, Z, multirank_host, h->scratch);
    });
}

tsvd_status tsvd_factors(tsvd_handle h, const void* M, tsvd_shape shape, tsvd_dtype dtype,
                         tsvd_precision precision, void* U_out, void* S_out, void* V_out) {
    return guarded([&] {
        check_handle(h);
        if (check_precision(dtype, precision))
            do_factors<float>(h, M, shape, U_out, S_out, V_out);
        else
            do_factors<double>(h, M, shape, U_out, S_out, V_out);
    });
}

tsvd_status tsvd_compress(tsvd_handle h, const void* M, tsvd_shape shape, tsvd_dtype dtype,
                          tsvd_precision precision, int32_t method, int64_t k, void* M_out,
                          double* ratio_host) {
    return guarded([&] {
        check_handle(h);
        if (check_precision(dtype, precision))
            do_compress<float>(h, M, shape, method, k, M_out, ratio_host);
        else
            do_compress<double>(h, M, shape, method, k, M_out, ratio_host);
    });
}

tsvd_status tsvd_complete(tsvd_handle h, const void* X_obs, const uint8_t* mask, tsvd_shape shape,
                          tsvd_dtype dtype, double rho, double tol, const tsvd_admm_opts* opts,
                          void* X_out, tsvd_info* info_host) {
    return guarded([&] {
        check_handle(h);
        if (check_precision(dtype, opts ? opts->precision : TSVD_PREC_FP64))
            do_complete<float>(h, X_obs, mask, shape, dtype, rho, tol, opts, X_out, info_host);
        else
            do_complete<double>(h, X_obs, mask, shape, dtype, rho, tol, opts, X_out, info_host);
    });
}

tsvd_status trpca(tsvd_handle h, const void* X, tsvd_shape shape, tsvd_dtype dtype, double lambda,
                  double mu, double tol, tsvd_shrink shrink, const tsvd_admm_opts* opts, void* L_out,
                  void* S_out, tsvd_info* info_host) {
    return guarded([&] {
        check_handle(h);
        if (check_precision(dtype, opts ? opts->precision : TSVD_PREC_FP64))
            do_trpca<float>(h, X, shape, dtype, lambda, mu, tol, shrink, opts, L_out, S_out, info_host);
        else
            do_trpca<double>(h, X, shape, dtype, lambda, mu, tol, shrink, opts, L_out, S_out, info_host);
    });
}

tsvd_status tsvd_profile(tsvd_handle h, int enable) {
    return guarded([&] {
        check_handle(h);
        Device dev(h->device);
        prof_harvest(h);
        if (enable) {
            h->agg.assign(K_COUNT, tsvd_handle_s::Agg{});
            hip_check(hipMemsetAsync(h->rot_counter, 0, 2 * sizeof(unsigned long long), h->stream),
                      "hipMemsetAsync rotations");
            hip_check(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        }
        h->prof_on = enable != 0;
    });
}

tsvd_status tsvd_profile_read(tsvd_handle h, tsvd_kernel_stat* out_host, int capacity,
                              int* count_host) {
    return guarded([&] {
        check_handle(h);
        if (!count_host || (capacity > 0 && !out_host)) fail(TSVD_E_INVALID, "null output");
        Device dev(h->device);
        prof_harvest(h);
        int c = 0;
        for (int k = 0; k < K_COUNT; ++k) {
            const auto& g = h->agg[k];
            if (g.launches == 0) continue;
            if (c < capacity) {
                tsvd_kernel_stat& o = out_host[c];
                std::memset(&o, 0, sizeof(o));
                std::snprintf(o.name, sizeof(o.name), "%s", kKindName[k]);
                o.launches = g.launches;
                o.total_ms = g.ms;
                o.work = g.work;
                o.work_is_bytes = kKindBytes[k] ? 1 : 0;
                o.slice_sweeps = g.sweeps;
                o.pairs_visited = g.pairs;
                o.rotations = g.rotations;
                o.kept_rank = g.kept;
            }
            ++c;
        }
        *count_host = c;
    });
}

tsvd_status tsvd_batch_run(tsvd_handle h, const tsvd_problem* probs, int32_t count, tsvd_info* infos_host,
                           int32_t* status_host) {
    return guarded([&] { batch_run(h, probs, count, infos_host, status_host); });
}

tsvd_status tsvd_submit(tsvd_handle h, const tsvd_problem* prob, uint64_t* ticket_host) {
    return guarded([&] { serve_submit(h, prob, ticket_host); });
}

tsvd_status tsvd_poll(tsvd_handle h, uint64_t ticket, tsvd_info* info_host) {
    tsvd_status st = TSVD_OK;
    const tsvd_status g = guarded([&] { st = serve_poll(h, ticket, info_host); });
    return g != TSVD_OK ? g : st;
}

tsvd_status tsvd_cancel(tsvd_handle h, uint64_t ticket) {
    return guarded([&] { serve_cancel(h, ticket); });
}

tsvd_status tsvd_serve_stats_read(tsvd_handle h, tsvd_serve_stats* out_host) {
    return guarded([&] { serve_stats(h, out_host); });
}

const char* tsvd_status_string(tsvd_status s) {
    switch (s) {
        case TSVD_OK: return "ok";
        case TSVD_E_INVALID: return "invalid argument";
        case TSVD_E_SHAPE: return "unsupported or invalid shape";
        case TSVD_E_NOMEM: return "out of memory or over budget";
        case TSVD_E_HIP: return "HIP runtime error";
        case TSVD_E_NONFINITE: return "non-finite value";
        case TSVD_E_UNSUPPORTED: return "unsupported request";
        case TSVD_E_BUSY: return "not finished";
        case TSVD_E_CANCELLED: return "cancelled";
        case TSVD_E_TIMEOUT: return "deadline passed";
    }
    return "unknown status";
}

const char* tsvd_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
