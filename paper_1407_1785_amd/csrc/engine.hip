// Batched and served solves: many completion (Sec. 4) and tensor-RPCA
// (Sec. 5) problems of uneven shapes advance together on one device.
//
// Every phase of an ADMM iteration is one launch over all running problems
// of an element type, driven by per-problem argument tables (kernels.h,
// "problem-table launches"):
//   forward DFT + prologue -> Newton-Schulz V^H V -> Newton-Schulz V update
//   -> pre-rotation A V -> Jacobi SVD (one launch per block-width / row-count
//   / schedule class: one workgroup per slice, or one per block pair of a
//   round with the blocks exchanged inside the launch; the classes run
//   concurrently on side streams, forked from and joined back into the
//   engine's stream) -> singular values -> rebuild
//   -> inverse DFT + epilogue -> control step.
// A problem runs exactly the arithmetic of the single-problem drivers in
// capi.hip: the first iteration's pre-rotation by V = I is an exact copy, so
// it equals their cold start.  Problems whose control step has stopped them
// are skipped by every kernel, so a batch keeps running until the host,
// which reads the control blocks after every two iterations, retires them.
//
// Buffers alternate between two parities (the iterates Z/Q, L/S/W and the
// two V buffers), so two iterations -- one table set per parity -- form one
// period; the period is captured once into a HIP graph and replayed until the
// running set changes (no launch depends on a host decision inside a
// period).  Problems join and leave only between periods.
//
// Device memory: each problem's state is one block of a per-engine arena
// (first-fit allocator, host bookkeeping); admission waits until the block
// fits.  The Jacobi block width of a shape is picked by the tuner below.

#include "arena.h"
#include "host.h"

#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <unordered_set>

namespace tsvd {

namespace {

using Clock = std::chrono::steady_clock;

// Jacobi schedules picked by the tuner (block width and whether the block
// pairs of a round run on one workgroup each), shared by every engine of the
// process and, with TSVD_AUTOTUNE_CACHE set to a file, across processes:
// each decision is one line "arch cus elem_bytes rpt ncls slices bw pairs".
struct TuneChoice {
    int bw = 16;
    bool pairs = false;
};
// (arch, cus, elem bytes, rpt, 32-column class, timed slice count)
using TuneKey = std::tuple<std::string, int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tuned;
std::string g_tune_cache_path;   // the cache file last read

// Reads the cache file (under g_tune_mu) when TSVD_AUTOTUNE_CACHE names a
// file other than the one last read; its entries take precedence over the
// decisions held in memory.  Lines that do not parse end the read.
void read_tune_cache() {
    const char* path = std::getenv("TSVD_AUTOTUNE_CACHE");
    if (!path || !*path || g_tune_cache_path == path) return;
    g_tune_cache_path = path;
    std::FILE* f = std::fopen(path, "r");
    if (!f) return;
    char arch[64];
    int cus, eb, rpt, ncls, ns, bw, pairs;
    while (std::fscanf(f, "%63s %d %d %d %d %d %d %d", arch, &cus, &eb, &rpt, &ncls, &ns, &bw, &pairs) == 8)
        if (bw == 4 || bw == 8 || bw == 16)
            g_tuned[TuneKey{arch, cus, eb, rpt, ncls, ns}] = TuneChoice{bw, pairs != 0};
    std::fclose(f);
}

void append_tune_cache(const TuneKey& k, const TuneChoice& c) {
    const char* path = std::getenv("TSVD_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    std::FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %d %d %d\n", std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k),
                 std::get<3>(k), std::get<4>(k), std::get<5>(k), c.bw, c.pairs ? 1 : 0);
    std::fclose(f);
}

// ------------------------------------------------------------------ problems

struct Spec {
    tsvd_problem p;
    Geometry g;
    AdmmSettings s;
    bool fp32;
};

Spec validate(const tsvd_problem& p) {
    Spec sp{};
    sp.p = p;
    if (p.kind != TSVD_KIND_COMPLETE && p.kind != TSVD_KIND_TRPCA) fail(TSVD_E_INVALID, "unknown problem kind");
    sp.fp32 = check_precision(p.dtype, p.precision);
    if (!p.x || !p.out) fail(TSVD_E_INVALID, "null tensor pointer");
    if (!(p.penalty > 0.0) || !std::isfinite(p.penalty)) fail(TSVD_E_INVALID, "penalty must be > 0");
    if (!(p.tol >= 0.0) || !std::isfinite(p.tol)) fail(TSVD_E_INVALID, "tol must be >= 0");
    if (p.opts.state) fail(TSVD_E_UNSUPPORTED, "the batched and served forms take no solver state");
    if (!(p.deadline_s >= 0.0) || !std::isfinite(p.deadline_s)) fail(TSVD_E_INVALID, "deadline_s must be >= 0");
    tsvd_admm_opts o = p.opts;
    o.precision = p.precision;
    if (p.kind == TSVD_KIND_COMPLETE) {
        if (!p.mask) fail(TSVD_E_INVALID, "null mask");
        sp.s = settings(&o, 1.1, 1e3, 300);
    } else {
        if (!p.out_s) fail(TSVD_E_INVALID, "null S output");
        if (!(p.lambda > 0.0) || !std::isfinite(p.lambda)) fail(TSVD_E_INVALID, "lambda must be > 0");
        if (p.shrink != TSVD_SHRINK_L1 && p.shrink != TSVD_SHRINK_L112) fail(TSVD_E_INVALID, "unknown shrink");
        sp.s = settings(&o, 1.2, 1e10, 500);
    }
    if (sp.s.rho_max < p.penalty) fail(TSVD_E_INVALID, "rho_max must be >= the initial penalty");
    sp.g = make_geometry(p.shape);
    if (jacobi_slice_rpt(sp.g.m, sp.g.n) > jacobi_slice_max_rpt())
        fail(TSVD_E_SHAPE, "slice too large for the batched Jacobi kernel");
    if (sp.g.n < 2) fail(TSVD_E_SHAPE, "batched solves need min(n1, n2) >= 2");
    return sp;
}

struct Result {
    tsvd_status status = TSVD_E_BUSY;
    tsvd_info info{};
};

template <typename T>
struct Slot {
    Spec sp;
    uint64_t ticket = 0;
    Clock::time_point t0;
    size_t off = 0, bytes = 0;
    T* it[3][2] = {};           // completion: Z, Q; RPCA: L, S, W (two parities each)
    cplx<T>* A = nullptr;       // forward DFT output, rebuild output
    cplx<T>* W = nullptr;       // pre-rotation output, Jacobi work array
    cplx<T>* V[2] = {};
    cplx<T>* G = nullptr;
    double* sigma = nullptr;
    double* dk = nullptr;       // shrink factors of the rebuild
    int* sweeps = nullptr;
    int* rot = nullptr;         // pairs-parallel Jacobi: 3 x h rotation flags
    int* bar = nullptr;         // pairs-parallel Jacobi: barrier counters and block flags
    double* fro = nullptr;      // pairs-parallel Jacobi: parts of the slices' Frobenius norms
    double* partials = nullptr;
    Ctrl* ctrl = nullptr;
    int* flag = nullptr;
    T* mat = nullptr;           // forward then inverse DFT matrix of the tube shape
    int tile_f = 0, tile_i = 0, inv_parts = 0, pro = 0, epi = 0;
    int bw = 0, rpt = 0, nb = 0;
    bool pairs = false;         // Jacobi schedule: one workgroup per block pair (else per slice)
};

template <typename T>
size_t slot_layout(Slot<T>& sl, char* base) {
    const Geometry& g = sl.sp.g;
    const bool rpca = sl.sp.p.kind == TSVD_KIND_TRPCA;
    sl.epi = rpca ? (sl.sp.p.shrink == TSVD_SHRINK_L1 ? EPI_RPCA_L1 : EPI_RPCA_L112) : EPI_COMPLETE;
    sl.pro = rpca ? PRO_RPCA : PRO_COMPLETE;
    sl.tile_f = dft_forward_tile(g);
    sl.tile_i = dft_inverse_tile(g, sl.epi);
    sl.inv_parts = (int)dft_grid(g, sl.tile_i);
    const int nparts = std::max(sl.inv_parts, 1024);   // the data-norm pass uses 1024 partials
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = Arena::round(off);
        char* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const int64_t N = g.numel, slice = (int64_t)g.h * g.m * g.n, vv = (int64_t)g.h * g.n * g.n;
    const int nit = rpca ? 3 : 2;
    for (int k = 0; k < nit; ++k)
        for (int q = 0; q < 2; ++q) sl.it[k][q] = reinterpret_cast<T*>(take(N * sizeof(T)));
    sl.A = reinterpret_cast<cplx<T>*>(take(slice * sizeof(cplx<T>)));
    sl.W = reinterpret_cast<cplx<T>*>(take(slice * sizeof(cplx<T>)));
    sl.V[0] = reinterpret_cast<cplx<T>*>(take(vv * sizeof(cplx<T>)));
    sl.V[1] = reinterpret_cast<cplx<T>*>(take(vv * sizeof(cplx<T>)));
    sl.G = reinterpret_cast<cplx<T>*>(take(vv * sizeof(cplx<T>)));
    sl.sigma = reinterpret_cast<double*>(take((int64_t)g.h * g.n * sizeof(double)));
    sl.dk = reinterpret_cast<double*>(take((int64_t)g.h * g.n * sizeof(double)));
    sl.sweeps = reinterpret_cast<int*>(take((int64_t)g.h * sizeof(int)));
    sl.rot = reinterpret_cast<int*>(take((int64_t)3 * g.h * sizeof(int)));
    // sized for the narrowest block width, the most blocks
    sl.bar = reinterpret_cast<int*>(take(jacobi_pairs_words(g.h, jacobi_num_blocks(g.n, 4)) * sizeof(int)));
    sl.fro = reinterpret_cast<double*>(take(jacobi_pairs_fro(g.h, g.n) * sizeof(double)));
    sl.partials = reinterpret_cast<double*>(take((int64_t)nparts * kNumPartials * sizeof(double)));
    sl.ctrl = reinterpret_cast<Ctrl*>(take(sizeof(Ctrl)));
    sl.flag = reinterpret_cast<int*>(take(sizeof(int)));
    sl.mat = reinterpret_cast<T*>(take(DftDims::of(g.h, g.L).total() * sizeof(T)));
    return Arena::round(off);
}

// ------------------------------------------------------------------ tables

// Host images of the argument tables of one parity, packed into one device
// buffer: [args of every phase][wg_start of every phase].
template <typename T>
struct Tables {
    struct Phase {
        size_t args_off = 0, ws_off = 0;
        int nprob = 0, nwg = 0;
        size_t lds = 0;
        int bw = 0, rpt = 0;   // Jacobi classes
        bool pairs = false;    // Jacobi classes: pairs-parallel schedule
        double work = 0.0;     // Jacobi classes: sum over slices of n^2 (m + n)
        int lane = 0;          // Jacobi classes: side stream
    };
    Phase fwd, gram, ns, pre, sig, reb, inv, ctl;
    std::vector<Phase> jac;
    std::vector<char> host;
    char* dev = nullptr;
    size_t dev_cap = 0;
};

template <typename A>
size_t append(std::vector<char>& buf, const std::vector<A>& v) {
    size_t off = (buf.size() + 255) & ~size_t(255);
    buf.resize(off + v.size() * sizeof(A));
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(A));
    return off;
}

// ------------------------------------------------------------------ engine

template <typename T>
class Engine {
public:
    Engine(int device, int cus, size_t lds_cap) : device_(device), cus_(cus), lds_cap_(lds_cap) {}
    ~Engine() { release(); }

    void release() {
        drop_graph();
        for (int q = 0; q < 2; ++q)
            if (tab_[q].dev) (void)hipFree(tab_[q].dev), tab_[q].dev = nullptr;
        if (host_ctrl_) (void)hipHostFree(host_ctrl_), host_ctrl_ = nullptr;
        if (words_) (void)hipFree(words_), words_ = nullptr;
        if (words_host_) (void)hipHostFree(words_host_), words_host_ = nullptr;
        for (int k = 0; k < kLanes; ++k) {
            if (side_[k]) (void)hipStreamDestroy(side_[k]), side_[k] = nullptr;
            if (ev_join_[k]) (void)hipEventDestroy(ev_join_[k]), ev_join_[k] = nullptr;
        }
        if (ev_fork_) (void)hipEventDestroy(ev_fork_), ev_fork_ = nullptr;
        if (stream_) (void)hipStreamDestroy(stream_), stream_ = nullptr;
    }

    void attach(Arena* arena) {
        arena_ = arena;
        if (stream_) return;
        hip_check(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking), "hipStreamCreate");
        for (int k = 0; k < kLanes; ++k) {
            hip_check(hipStreamCreateWithFlags(&side_[k], hipStreamNonBlocking), "hipStreamCreate");
            hip_check(hipEventCreateWithFlags(&ev_join_[k], hipEventDisableTiming), "hipEventCreate");
        }
        hip_check(hipEventCreateWithFlags(&ev_fork_, hipEventDisableTiming), "hipEventCreate");
        // pairs-parallel classes: a role ticket and an error word each,
        // cleared by a fill kernel at the start of every Jacobi phase
        hip_check(hipMalloc(reinterpret_cast<void**>(&words_), sizeof(int) * 2 * kMaxClasses), "hipMalloc words");
        hip_check(hipHostMalloc(reinterpret_cast<void**>(&words_host_), sizeof(int) * 2 * kMaxClasses, 0),
                  "hipHostMalloc words");
    }

    hipStream_t stream() const { return stream_; }
    size_t running() const { return slots_.size(); }
    // Fourier slices of the running problems (their share of the chip)
    int64_t running_slices() const {
        int64_t s = 0;
        for (const Slot<T>& sl : slots_) s += sl.sp.g.h;
        return s;
    }
    int64_t iterations() const { return iterations_; }

    static size_t footprint(const Spec& sp) {
        Slot<T> sl;
        sl.sp = sp;
        return slot_layout(sl, nullptr);
    }

    // Try to admit; false if the arena has no room now.
    bool admit(const Spec& sp, uint64_t ticket, Clock::time_point t0) {
        Slot<T> sl;
        sl.sp = sp;
        sl.ticket = ticket;
        sl.t0 = t0;
        const size_t bytes = slot_layout(sl, nullptr);
        size_t off = 0;
        if (!arena_->take(bytes, &off)) return false;
        sl.off = off;
        sl.bytes = bytes;
        slot_layout(sl, arena_->base() + off);
        try {
            setup(sl);
        } catch (...) {
            arena_->give(off, bytes);
            throw;
        }
        slots_.push_back(sl);
        dirty_ = true;
        return true;
    }

    // Run one period (two iterations) over the running problems.
    void period() {
        if (slots_.empty()) return;
        if (dirty_) rebuild();
        if (graph_exec_) {
            hip_check(hipGraphLaunch(graph_exec_, stream_), "hipGraphLaunch");
        } else {
            iteration(0);
            iteration(1);
        }
        iterations_ += 2;
    }

    // Retire stopped problems: write their outputs and results.
    template <typename F>
    void harvest(F&& done_cb) {
        if (slots_.empty()) return;
        const size_t n = slots_.size();
        ensure_host_ctrl(n);
        for (size_t i = 0; i < n; ++i)
            hip_check(hipMemcpyAsync(host_ctrl_ + i, slots_[i].ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream_),
                      "hipMemcpyAsync ctrl");
        hip_check(hipMemcpyAsync(words_host_, words_, sizeof(int) * 2 * kMaxClasses, hipMemcpyDeviceToHost, stream_),
                  "hipMemcpyAsync words");
        hip_check(hipStreamSynchronize(stream_), "hipStreamSynchronize");
        for (int k = 0; k < kMaxClasses; ++k)
            if (words_host_[2 * k + 1]) fail(TSVD_E_HIP, "a batched Jacobi wait between workgroups gave up");
        std::vector<size_t> stopped;
        for (size_t i = 0; i < n; ++i)
            if (host_ctrl_[i].done) stopped.push_back(i);
        if (stopped.empty()) return;
        std::vector<Ctrl> cs;
        for (size_t i : stopped) cs.push_back(host_ctrl_[i]);
        // outputs, sweep counts and non-finite flags of the stopped problems
        std::vector<int> flags(stopped.size());
        for (size_t k = 0; k < stopped.size(); ++k) {
            Slot<T>& sl = slots_[stopped[k]];
            write_outputs(sl, cs[k]);
            hip_check(hipMemcpyAsync(&flags[k], sl.flag, sizeof(int), hipMemcpyDeviceToHost, stream_),
                      "hipMemcpyAsync flag");
        }
        hip_check(hipStreamSynchronize(stream_), "hipStreamSynchronize");
        const auto now = Clock::now();
        for (size_t k = 0; k < stopped.size(); ++k) {
            Slot<T>& sl = slots_[stopped[k]];
            const Ctrl& c = cs[k];
            Result r;
            r.status = (c.nonfinite || flags[k]) ? TSVD_E_NONFINITE : TSVD_OK;
            r.info.iters = c.iter;
            r.info.converged = c.done == 1 && !c.nonfinite ? 1 : 0;
            r.info.sweeps_total = c.sweeps_total;
            r.info.sweeps_last = c.sweeps_last;
            r.info.primal = c.primal;
            r.info.change = c.change;
            r.info.rho_final = c.rho_used;
            r.info.seconds = std::chrono::duration<double>(now - sl.t0).count();
            done_cb(sl.ticket, r);
        }
        // free in reverse index order so the remaining indices stay valid
        for (auto it = stopped.rbegin(); it != stopped.rend(); ++it) {
            arena_->give(slots_[*it].off, slots_[*it].bytes);
            slots_.erase(slots_.begin() + (long)*it);
        }
        dirty_ = true;
    }

    // Serving: drop the running problems that are cancelled or past their
    // deadline (call between periods, after harvest, when the engine's
    // stream is idle); each is reported with its status.
    template <typename C, typename F>
    void expire(C&& cancelled, Clock::time_point now, F&& done_cb) {
        for (size_t i = slots_.size(); i-- > 0;) {
            const Slot<T>& sl = slots_[i];
            const double dl = sl.sp.p.deadline_s;
            tsvd_status st = TSVD_OK;
            if (cancelled(sl.ticket))
                st = TSVD_E_CANCELLED;
            else if (dl > 0.0 && std::chrono::duration<double>(now - sl.t0).count() > dl)
                st = TSVD_E_TIMEOUT;
            if (st == TSVD_OK) continue;
            Result r;
            r.status = st;
            r.info.seconds = std::chrono::duration<double>(now - sl.t0).count();
            done_cb(sl.ticket, r);
            arena_->give(sl.off, sl.bytes);
            slots_.erase(slots_.begin() + (long)i);
            dirty_ = true;
        }
    }

    // After a device failure: report every running problem with `status`
    // and forget it (no device work is issued).
    template <typename F>
    void abandon(tsvd_status status, F&& done_cb) {
        for (const Slot<T>& sl : slots_) {
            Result r;
            r.status = status;
            done_cb(sl.ticket, r);
            if (arena_) arena_->give(sl.off, sl.bytes);
        }
        slots_.clear();
        dirty_ = true;
    }

private:
    void ensure_host_ctrl(size_t n) {
        if (n <= host_ctrl_len_) return;
        if (host_ctrl_) hip_check(hipHostFree(host_ctrl_), "hipHostFree");
        host_ctrl_ = nullptr;
        hip_check(hipHostMalloc(reinterpret_cast<void**>(&host_ctrl_), sizeof(Ctrl) * n, 0), "hipHostMalloc");
        host_ctrl_len_ = n;
    }

    void setup(Slot<T>& sl) {
        const Geometry& g = sl.sp.g;
        const tsvd_problem& p = sl.sp.p;
        const bool rpca = p.kind == TSVD_KIND_TRPCA;
        const int64_t N = g.numel;
        hipStream_t st = stream_;
        // the DFT matrices and the control block come from host memory: stage
        // them through pinned buffers that outlive the copies (synchronised below)
        const std::vector<T> mat = dft_matrices_host<T>(g);
        Ctrl c{};
        c.rho = p.penalty;
        c.tau = 1.0 / p.penalty;
        c.dscale = 1.0;
        c.dscale_used = 1.0;
        c.growth = sl.sp.s.growth;
        c.rho_max = sl.sp.s.rho_max;
        c.rho_used = p.penalty;
        c.max_iter = sl.sp.s.max_iter;
        if (rpca) {
            c.lambda = p.lambda;
            c.shrink = p.lambda / p.penalty;
        }
        void* staging = nullptr;
        const size_t mat_bytes = Arena::round(mat.size() * sizeof(T));
        hip_check(hipHostMalloc(&staging, mat_bytes + sizeof(Ctrl), 0), "hipHostMalloc");
        std::memcpy(staging, mat.data(), mat.size() * sizeof(T));
        std::memcpy(static_cast<char*>(staging) + mat_bytes, &c, sizeof(Ctrl));
        hip_check(hipMemcpyAsync(sl.mat, staging, mat.size() * sizeof(T), hipMemcpyHostToDevice, st),
                  "hipMemcpyAsync DFT matrices");
        hip_check(hipMemcpyAsync(sl.ctrl, static_cast<char*>(staging) + mat_bytes, sizeof(Ctrl),
                                 hipMemcpyHostToDevice, st),
                  "hipMemcpyAsync ctrl");
        const int nit = rpca ? 3 : 2;
        for (int k = 0; k < nit; ++k) launch_fill<T>(sl.it[k][0], (T)0, N, st);
        launch_set_identity<T>(sl.V[0], g.n, g.h, st);
        launch_fill<int>(sl.flag, 0, 1, st);
        launch_fill<int>(sl.rot, 0, 3 * g.h, st);
        launch_fill<int>(sl.bar, 0, jacobi_pairs_words(g.h, jacobi_num_blocks(g.n, 4)), st);
        launch_sumsq<T>(static_cast<const T*>(p.x), rpca ? nullptr : p.mask, N, sl.partials, 1024, st);
        launch_set_tol(sl.ctrl, sl.partials, 1024, p.tol, st);
        launch_check("problem setup");
        const hipError_t e = hipStreamSynchronize(st);
        (void)hipHostFree(staging);
        hip_check(e, "hipStreamSynchronize");
        // Jacobi launch class
        sl.rpt = jacobi_slice_rpt(g.m, g.n);
        const TuneChoice tc = pick_schedule(g.m, g.n, sl.rpt, g.h);
        sl.bw = tc.bw;
        sl.nb = jacobi_num_blocks(g.n, sl.bw);
        sl.pairs = tc.pairs && sl.nb / 2 >= 2;
        // TSVD_PAIRS_MIN: one workgroup per block pair from that many pairs on
        const int forced = env_int("TSVD_PAIRS_MIN", 0);
        if (forced > 0) sl.pairs = sl.nb / 2 >= forced;
    }

    void write_outputs(Slot<T>& sl, const Ctrl& c) {
        const Geometry& g = sl.sp.g;
        const tsvd_problem& p = sl.sp.p;
        const int64_t N = g.numel;
        const int iters = std::max(c.iter, 1);
        if (p.kind == TSVD_KIND_COMPLETE) {
            // the X-update of the last iteration, from the iterates it started with
            const int q = (iters - 1) % 2;
            launch_complete_output<T>(static_cast<const T*>(p.x), p.mask, sl.it[0][q], sl.it[1][q], sl.ctrl,
                                      static_cast<T*>(p.out), N, stream_);
            launch_check("complete_output");
        } else {
            const int q = iters % 2;
            hip_check(hipMemcpyAsync(p.out, sl.it[0][q], N * sizeof(T), hipMemcpyDeviceToDevice, stream_),
                      "hipMemcpyAsync L");
            hip_check(hipMemcpyAsync(p.out_s, sl.it[1][q], N * sizeof(T), hipMemcpyDeviceToDevice, stream_),
                      "hipMemcpyAsync S");
        }
    }

    // ---- Jacobi schedule tuner
    //
    // Candidates: every block width whose two blocks fit in LDS, each with
    // one workgroup per slice, and, where a slice has two or more block
    // pairs, one workgroup per block pair of a round.  One decision per
    // device, element type, row class, 32-column class and slice count
    // (rounded up to a power of two, at most one per CU): a class runs beside
    // a few others on the side streams, so its latency on its own slices is
    // what the period waits for; timed on one slice per CU instead, the
    // one-workgroup schedule wins classes that the pairs schedule runs twice
    // as fast inside a batch.  The sweep cap is a limit of the method, not a
    // schedule, and is not tuned.
    TuneChoice pick_schedule(int m, int n, int rpt, int h) {
        std::vector<TuneChoice> cand;
        for (int bw : {16, 8, 4}) {
            if (jacobi_slice_lds(bw, rpt, sizeof(T)) + 1024 > lds_cap_) continue;
            cand.push_back(TuneChoice{bw, false});
            if (jacobi_num_blocks(n, bw) / 2 >= 2) cand.push_back(TuneChoice{bw, true});
        }
        if (cand.empty()) fail(TSVD_E_SHAPE, "slice too large for the batched Jacobi kernel");
        const int forced = env_int("TSVD_BATCH_BW", 0);
        if (forced) {
            std::vector<TuneChoice> keep;
            for (const TuneChoice& c : cand)
                if (c.bw == forced) keep.push_back(c);
            if (!keep.empty()) cand = keep;
        }
        if (cand.size() == 1 || env_int("TSVD_TUNE", 1) == 0) {
            // untuned: the widest block, one workgroup per block pair when a
            // slice has two or more
            TuneChoice c = cand[0];
            for (const TuneChoice& d : cand)
                if (d.bw == c.bw && d.pairs) c = d;
            return c;
        }
        hipDeviceProp_t prop{};
        (void)hipGetDeviceProperties(&prop, device_);
        const TuneKey key{std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':')), cus_,
                          (int)sizeof(T), rpt, (n + 31) / 32, tune_slices(h)};
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            read_tune_cache();
            auto hit = g_tuned.find(key);
            if (hit != g_tuned.end()) {
                for (const TuneChoice& c : cand)
                    if (c.bw == hit->second.bw && c.pairs == hit->second.pairs) {
                        tune_log("cached", m, n, rpt, std::get<5>(key), c);
                        return c;
                    }
            }
        }
        const TuneChoice best = tune(m, n, rpt, std::get<5>(key), cand);
        tune_log("chose", m, n, rpt, std::get<5>(key), best);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (g_tuned.find(key) == g_tuned.end()) {
            g_tuned[key] = best;
            append_tune_cache(key, best);
        }
        return best;
    }

    static void tune_log(const char* what, int m, int n, int rpt, int S, const TuneChoice& c) {
        if (env_int("TSVD_TUNE_LOG", 0))
            std::fprintf(stderr, "[tsvd tune] %s m=%d n=%d rpt=%d slices=%d bw=%d pairs=%d\n", what, m, n, rpt, S, c.bw,
                         c.pairs ? 1 : 0);
    }

    int tune_slices(int h) const {
        int s = 1;
        while (s < h && s < cus_) s *= 2;
        return std::min(s, cus_);
    }

    // Time every candidate on S synthetic slices of this shape (pseudo-random
    // entries, V = I, one sweep) and keep the fastest.
    TuneChoice tune(int m, int n, int rpt, int S, const std::vector<TuneChoice>& cand) {
        const int64_t mn = (int64_t)m * n, nn = (int64_t)n * n;
        const int nb_max = jacobi_num_blocks(n, 4);
        const size_t ints = 2 + 3 * (size_t)S + (size_t)jacobi_pairs_words(S, nb_max);
        char* buf = nullptr;
        const size_t cbytes = sizeof(cplx<T>) * (size_t)S * (2 * mn + nn);
        hip_check(hipMalloc(&buf, cbytes + sizeof(int) * ints + 1024), "hipMalloc tuner");
        cplx<T>* A0 = reinterpret_cast<cplx<T>*>(buf);
        cplx<T>* A = A0 + S * mn;
        cplx<T>* V = A + S * mn;
        int* words = reinterpret_cast<int*>(buf + cbytes);
        int* rot = words + 2;
        int* bar = rot + 3 * S;
        JacSliceArgs<T>* dtab = nullptr;
        int* dws = nullptr;
        hip_check(hipMalloc(&dtab, sizeof(JacSliceArgs<T>)), "hipMalloc tuner");
        hip_check(hipMalloc(&dws, 2 * sizeof(int)), "hipMalloc tuner");
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "hipEventCreate");
        hip_check(hipEventCreate(&e1), "hipEventCreate");
        TuneChoice best = cand[0];
        float best_ms = 1e30f;
        try {
            launch_fill_hash<T>(A0, S * mn, 12345u, stream_);
            for (const TuneChoice& c : cand) {
                JacSliceArgs<T> ja{};
                ja.A = A;
                ja.V = V;
                ja.m = m;
                ja.n = n;
                ja.h = S;
                ja.nb = jacobi_num_blocks(n, c.bw);
                ja.tol = (T)jacobi_tol(m, sizeof(T));
                ja.max_sweeps = 1;
                ja.rot = rot;
                ja.bar = bar;
                const int G = c.pairs ? ja.nb / 2 : 1;
                const int ws[2] = {0, S * G};
                hip_check(hipMemcpyAsync(dws, ws, sizeof(ws), hipMemcpyHostToDevice, stream_), "hipMemcpyAsync");
                hip_check(hipMemcpyAsync(dtab, &ja, sizeof(ja), hipMemcpyHostToDevice, stream_), "hipMemcpyAsync");
                hip_check(prepare_jacobi_slice<T>(c.bw, rpt), "jacobi tuner attribute");
                // the best of three runs: the choice should not follow the noise of one
                float ms = 1e30f;
                for (int rep = 0; rep < 3; ++rep) {
                    hip_check(hipMemcpyAsync(A, A0, sizeof(cplx<T>) * S * mn, hipMemcpyDeviceToDevice, stream_),
                              "hipMemcpyAsync");
                    launch_set_identity<T>(V, n, S, stream_);
                    launch_fill<int>(words, 0, (int64_t)ints, stream_);
                    hip_check(hipEventRecord(e0, stream_), "hipEventRecord");
                    if (c.pairs)
                        hip_check(launch_jacobi_pairs<T>(c.bw, rpt, dtab, dws, 1, S * G, words, 1 << 21, stream_),
                                  "jacobi tuner launch");
                    else
                        hip_check(launch_jacobi_slice<T>(c.bw, rpt, dtab, dws, 1, S, 1, stream_),
                                  "jacobi tuner launch");
                    hip_check(hipEventRecord(e1, stream_), "hipEventRecord");
                    hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
                    float one = 0.f;
                    hip_check(hipEventElapsedTime(&one, e0, e1), "hipEventElapsedTime");
                    if (c.pairs) {
                        // a wait between workgroups that gave up (other work on the device):
                        // this timing does not count
                        int gave_up = 0;
                        hip_check(hipMemcpy(&gave_up, words + 1, sizeof(int), hipMemcpyDeviceToHost),
                                  "hipMemcpy tuner");
                        if (gave_up) one = 1e30f;
                    }
                    ms = std::min(ms, one);
                }
                if (env_int("TSVD_TUNE_LOG", 0))
                    std::fprintf(stderr, "[tsvd tune] m=%d n=%d rpt=%d slices=%d bw=%d pairs=%d: %.3f ms\n", m, n, rpt, S, c.bw,
                                 c.pairs ? 1 : 0, ms);
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
        } catch (...) {
            (void)hipStreamSynchronize(stream_);
            (void)hipFree(buf), (void)hipFree(dtab), (void)hipFree(dws);
            (void)hipEventDestroy(e0), (void)hipEventDestroy(e1);
            throw;
        }
        (void)hipFree(buf), (void)hipFree(dtab), (void)hipFree(dws);
        (void)hipEventDestroy(e0), (void)hipEventDestroy(e1);
        return best;
    }

    // ---- tables and graph
    void rebuild() {
        drop_graph();
        for (int q = 0; q < 2; ++q) build_tables(q);
        dirty_ = false;
        if (env_int("TSVD_GRAPH", 1) == 0) return;
        hipGraph_t graph = nullptr;
        hip_check(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        bool ok = true;
        try {
            iteration(0);
            iteration(1);
        } catch (...) {
            ok = false;
        }
        const hipError_t e = hipStreamEndCapture(stream_, &graph);
        if (!ok || e != hipSuccess || !graph) {
            (void)hipGetLastError();
            if (graph) (void)hipGraphDestroy(graph);
            return;   // eager launches from now on for this running set
        }
        if (hipGraphInstantiate(&graph_exec_, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGetLastError();
            graph_exec_ = nullptr;
        }
        (void)hipGraphDestroy(graph);
    }

    void drop_graph() {
        if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
        graph_exec_ = nullptr;
    }

    void build_tables(int par) {
        Tables<T>& tb = tab_[par];
        tb.host.clear();
        tb.jac.clear();
        const int P = par, Q = 1 - par;
        std::vector<FwdArgs<T>> fwd;
        std::vector<InvArgs<T>> inv;
        std::vector<ZGemmArgs<T>> gram, ns, pre, reb;
        std::vector<SigmaArgs<T>> sig;
        std::vector<CtrlArgs> ctl;
        std::vector<int> ws_fwd{0}, ws_inv{0}, ws_gram{0}, ws_ns{0}, ws_pre{0}, ws_reb{0}, ws_sig{0};
        size_t lds_f = 0, lds_i = 0;
        using JKey = std::tuple<int, int, int>;   // (bw, rpt, pairs)
        std::map<JKey, std::pair<std::vector<JacSliceArgs<T>>, std::vector<int>>> jc;
        std::map<JKey, double> jwork;
        for (const Slot<T>& sl : slots_) {
            const Geometry& g = sl.sp.g;
            const tsvd_problem& p = sl.sp.p;
            const bool rpca = p.kind == TSVD_KIND_TRPCA;
            const int64_t mn = (int64_t)g.m * g.n, nn = (int64_t)g.n * g.n;
            FwdArgs<T> fa{};
            fa.x = static_cast<const T*>(p.x);
            fa.mask = rpca ? nullptr : p.mask;
            fa.ctrl = sl.ctrl;
            fa.mat = sl.mat;
            fa.out = sl.A;
            fa.nonfinite = sl.flag;
            fa.g = g;
            fa.tile = sl.tile_f;
            fa.pro = sl.pro;
            if (rpca) {
                fa.s = sl.it[1][P];
                fa.dual = sl.it[2][P];
            } else {
                fa.z = sl.it[0][P];
                fa.dual = sl.it[1][P];
            }
            fwd.push_back(fa);
            ws_fwd.push_back(ws_fwd.back() + (int)dft_grid(g, sl.tile_f));
            lds_f = std::max(lds_f, dft_forward_lds<T>(g, sl.tile_f));
            // Newton-Schulz: G = V^H V, V' = 1.5 V - 0.5 V G
            ZGemmArgs<T> gg{};
            gg.A = sl.V[P];
            gg.B = sl.V[P];
            gg.C = sl.G;
            gg.M = gg.N = gg.K = g.n;
            gg.lda = gg.ldb = gg.ldc = gg.ldd = g.n;
            gg.sA = gg.sB = gg.sC = gg.sD = nn;
            gg.alpha = (T)1;
            gg.beta = (T)0;
            gg.opA = 1;
            gg.opB = 0;
            gg.batch = g.h;
            gg.ctrl = sl.ctrl;
            gram.push_back(gg);
            ws_gram.push_back(ws_gram.back() + zgemm_workgroups(g.n, g.n, g.h));
            ZGemmArgs<T> gn = gg;
            gn.A = sl.V[P];
            gn.B = sl.G;
            gn.D = sl.V[P];
            gn.C = sl.V[Q];
            gn.alpha = (T)-0.5;
            gn.beta = (T)1.5;
            gn.opA = 0;
            ns.push_back(gn);
            ws_ns.push_back(ws_ns.back() + zgemm_workgroups(g.n, g.n, g.h));
            // pre-rotation W = A V'
            ZGemmArgs<T> ga{};
            ga.A = sl.A;
            ga.B = sl.V[Q];
            ga.C = sl.W;
            ga.M = g.m;
            ga.N = g.n;
            ga.K = g.n;
            ga.lda = g.m;
            ga.ldb = g.n;
            ga.ldc = g.m;
            ga.ldd = g.m;
            ga.sA = mn;
            ga.sB = nn;
            ga.sC = mn;
            ga.sD = mn;
            ga.alpha = (T)1;
            ga.beta = (T)0;
            ga.batch = g.h;
            ga.ctrl = sl.ctrl;
            pre.push_back(ga);
            ws_pre.push_back(ws_pre.back() + zgemm_workgroups(g.m, g.n, g.h));
            // Jacobi on (W, V')
            JacSliceArgs<T> ja{};
            ja.A = sl.W;
            ja.V = sl.V[Q];
            ja.m = g.m;
            ja.n = g.n;
            ja.h = g.h;
            ja.nb = sl.nb;
            ja.tol = (T)jacobi_tol(g.m, sizeof(T));
            ja.sweeps = sl.sweeps;
            ja.ctrl = sl.ctrl;
            ja.max_sweeps = sl.sp.s.max_sweeps;
            ja.rot = sl.rot;
            ja.bar = sl.bar;
            ja.floor_scale = jacobi_floor_scale(g.m, sizeof(T));
            ja.fro = sl.fro;
            const JKey key{sl.bw, sl.rpt, sl.pairs ? 1 : 0};
            auto& cls = jc[key];
            if (cls.second.empty()) cls.second.push_back(0);
            cls.first.push_back(ja);
            cls.second.push_back(cls.second.back() + g.h * (sl.pairs ? sl.nb / 2 : 1));
            jwork[key] += (double)g.h * g.n * g.n * (g.m + g.n);
            // singular values and rebuild A = W diag(d) V'^H
            SigmaArgs<T> sa{sl.W, g.m, g.n, g.h, sl.sigma, sl.dk, sl.ctrl};
            sig.push_back(sa);
            ws_sig.push_back(ws_sig.back() + svt_sigma_workgroups(g.n, g.h));
            ZGemmArgs<T> gr = ga;
            gr.A = sl.W;
            gr.B = sl.V[Q];
            gr.C = sl.A;
            gr.opB = 1;
            gr.dk = sl.dk;
            gr.sdk = g.n;
            reb.push_back(gr);
            ws_reb.push_back(ws_reb.back() + zgemm_workgroups(g.m, g.n, g.h));
            // inverse DFT + epilogue
            InvArgs<T> ia{};
            ia.in = sl.A;
            ia.mat = sl.mat + DftDims::of(g.h, g.L).fwd_size();
            ia.ctrl = sl.ctrl;
            ia.g = g;
            ia.tile = sl.tile_i;
            ia.partials = sl.partials;
            ia.epi = sl.epi;
            ia.out = sl.it[0][Q];
            if (rpca) {
                ia.m = static_cast<const T*>(p.x);
                ia.l_old = sl.it[0][P];
                ia.s_old = sl.it[1][P];
                ia.s_new = sl.it[1][Q];
                ia.dual_old = sl.it[2][P];
                ia.dual_new = sl.it[2][Q];
            } else {
                ia.y = static_cast<const T*>(p.x);
                ia.mask = p.mask;
                ia.z_old = sl.it[0][P];
                ia.dual_old = sl.it[1][P];
                ia.dual_new = sl.it[1][Q];
            }
            inv.push_back(ia);
            ws_inv.push_back(ws_inv.back() + sl.inv_parts);
            lds_i = std::max(lds_i, dft_inverse_lds<T>(g, sl.tile_i, sl.epi));
            ctl.push_back(CtrlArgs{sl.ctrl, sl.partials, sl.inv_parts, rpca ? 1 : 0, sl.pairs ? sl.rot : nullptr, g.h,
                                   sl.pairs ? sl.bar : nullptr,
                                   sl.pairs ? (int)jacobi_pairs_words(g.h, sl.nb) : 0});
        }
        auto put = [&](typename Tables<T>::Phase& ph, auto& args, std::vector<int>& ws, size_t lds) {
            ph.args_off = append(tb.host, args);
            ph.ws_off = append(tb.host, ws);
            ph.nprob = (int)args.size();
            ph.nwg = ws.back();
            ph.lds = lds;
        };
        put(tb.fwd, fwd, ws_fwd, lds_f);
        put(tb.gram, gram, ws_gram, 0);
        put(tb.ns, ns, ws_ns, 0);
        put(tb.pre, pre, ws_pre, 0);
        put(tb.sig, sig, ws_sig, 0);
        put(tb.reb, reb, ws_reb, 0);
        put(tb.inv, inv, ws_inv, lds_i);
        std::vector<int> ws_ctl(ctl.size() + 1, 0);
        put(tb.ctl, ctl, ws_ctl, 0);
        tb.ctl.nwg = (int)ctl.size();
        for (auto& kv : jc) {
            typename Tables<T>::Phase ph;
            put(ph, kv.second.first, kv.second.second, 0);
            ph.bw = std::get<0>(kv.first);
            ph.rpt = std::get<1>(kv.first);
            ph.pairs = std::get<2>(kv.first) != 0;
            ph.work = jwork[kv.first];
            hip_check(prepare_jacobi_slice<T>(ph.bw, ph.rpt), "jacobi attribute");
            tb.jac.push_back(ph);
        }
        if ((int)tb.jac.size() > kMaxClasses) fail(TSVD_E_UNSUPPORTED, "too many Jacobi classes");
        // the classes run concurrently on kLanes streams: largest work first,
        // each to the least loaded stream
        std::sort(tb.jac.begin(), tb.jac.end(), [](const auto& a, const auto& b) { return a.work > b.work; });
        double load[kLanes] = {};
        for (auto& ph : tb.jac) {
            int best = 0;
            for (int k = 1; k < kLanes; ++k)
                if (load[k] < load[best]) best = k;
            ph.lane = best;
            load[best] += ph.work;
        }
        if (tb.host.size() > tb.dev_cap) {
            if (tb.dev) hip_check(hipFree(tb.dev), "hipFree tables");
            tb.dev = nullptr;
            tb.dev_cap = std::max(tb.host.size() * 2, (size_t)1 << 16);
            hip_check(hipMalloc(&tb.dev, tb.dev_cap), "hipMalloc tables");
        }
        hip_check(hipMemcpy(tb.dev, tb.host.data(), tb.host.size(), hipMemcpyHostToDevice), "hipMemcpy tables");
        prepare_dft_batched<T>(lds_f, lds_i);
    }

    template <typename A>
    const A* targs(const Tables<T>& tb, const typename Tables<T>::Phase& ph) const {
        return reinterpret_cast<const A*>(tb.dev + ph.args_off);
    }
    const int* tws(const Tables<T>& tb, const typename Tables<T>::Phase& ph) const {
        return reinterpret_cast<const int*>(tb.dev + ph.ws_off);
    }

    void iteration(int par) {
        const Tables<T>& tb = tab_[par];
        hipStream_t st = stream_;
        launch_dft_forward_batched<T>(targs<FwdArgs<T>>(tb, tb.fwd), tws(tb, tb.fwd), tb.fwd.nprob, tb.fwd.nwg,
                                      tb.fwd.lds, st);
        launch_check("batched dft_forward");
        launch_zgemm_batched<T>(targs<ZGemmArgs<T>>(tb, tb.gram), tws(tb, tb.gram), tb.gram.nprob, tb.gram.nwg, st);
        launch_zgemm_batched<T>(targs<ZGemmArgs<T>>(tb, tb.ns), tws(tb, tb.ns), tb.ns.nprob, tb.ns.nwg, st);
        launch_zgemm_batched<T>(targs<ZGemmArgs<T>>(tb, tb.pre), tws(tb, tb.pre), tb.pre.nprob, tb.pre.nwg, st);
        launch_check("batched warm start");
        // role tickets and error words of the pairs-parallel classes
        launch_fill<int>(words_, 0, 2 * kMaxClasses, st);
        // fork: the Jacobi classes on the side streams, then join
        hip_check(hipEventRecord(ev_fork_, st), "hipEventRecord");
        bool used[kLanes] = {};
        for (const auto& ph : tb.jac) used[ph.lane] = true;
        for (int k = 0; k < kLanes; ++k)
            if (used[k]) hip_check(hipStreamWaitEvent(side_[k], ev_fork_, 0), "hipStreamWaitEvent");
        const int spin = std::max(0, env_int("TSVD_PERSIST_SPIN", 1 << 21));
        for (size_t c = 0; c < tb.jac.size(); ++c) {
            const auto& ph = tb.jac[c];
            if (ph.pairs)
                hip_check(launch_jacobi_pairs<T>(ph.bw, ph.rpt, targs<JacSliceArgs<T>>(tb, ph), tws(tb, ph), ph.nprob,
                                                 ph.nwg, words_ + 2 * c, spin, side_[ph.lane]),
                          "batched jacobi pairs");
            else
                hip_check(launch_jacobi_slice<T>(ph.bw, ph.rpt, targs<JacSliceArgs<T>>(tb, ph), tws(tb, ph),
                                                 ph.nprob, ph.nwg, 30, side_[ph.lane]),
                          "batched jacobi");
        }
        for (int k = 0; k < kLanes; ++k)
            if (used[k]) {
                hip_check(hipEventRecord(ev_join_[k], side_[k]), "hipEventRecord");
                hip_check(hipStreamWaitEvent(st, ev_join_[k], 0), "hipStreamWaitEvent");
            }
        launch_svt_sigma_batched<T>(targs<SigmaArgs<T>>(tb, tb.sig), tws(tb, tb.sig), tb.sig.nprob, tb.sig.nwg, st);
        launch_zgemm_batched<T>(targs<ZGemmArgs<T>>(tb, tb.reb), tws(tb, tb.reb), tb.reb.nprob, tb.reb.nwg, st);
        launch_check("batched rebuild");
        launch_dft_inverse_batched<T>(targs<InvArgs<T>>(tb, tb.inv), tws(tb, tb.inv), tb.inv.nprob, tb.inv.nwg,
                                      tb.inv.lds, st);
        launch_admm_ctrl_batched(targs<CtrlArgs>(tb, tb.ctl), tb.ctl.nprob, st);
        launch_check("batched control");
    }

    int device_, cus_;
    size_t lds_cap_;
    static constexpr int kLanes = 3;   // side streams of the Jacobi phase
    Arena* arena_ = nullptr;
    hipStream_t stream_ = nullptr;
    hipStream_t side_[kLanes] = {};
    hipEvent_t ev_fork_ = nullptr, ev_join_[kLanes] = {};
    std::vector<Slot<T>> slots_;
    Tables<T> tab_[2];
    bool dirty_ = true;
    hipGraphExec_t graph_exec_ = nullptr;
    Ctrl* host_ctrl_ = nullptr;
    size_t host_ctrl_len_ = 0;
    static constexpr int kMaxClasses = 64;       // Jacobi classes of a running set
    int* words_ = nullptr;                        // per class: role ticket, error word
    int* words_host_ = nullptr;                   // pinned copy read by harvest
    int64_t iterations_ = 0;
};

size_t default_arena_bytes(size_t budget) {
    if (budget) return budget;
    size_t free_b = 0, total_b = 0;
    hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    return (size_t)(0.9 * (double)free_b);
}

}  // namespace

// ------------------------------------------------------------------ batch

void batch_run(tsvd_handle h, const tsvd_problem* probs, int count, tsvd_info* infos, int32_t* status) {
    check_handle(h);
    if (count < 0 || (count > 0 && !probs)) fail(TSVD_E_INVALID, "bad problem array");
    std::vector<Spec> specs;
    specs.reserve(count);
    for (int i = 0; i < count; ++i) specs.push_back(validate(probs[i]));
    if (count == 0) return;
    const auto t0 = Clock::now();
    Device dev(h->device);
    // arena: everything at once if it fits, else the budget
    size_t need = 0, largest = 0;
    for (const Spec& sp : specs) {
        const size_t b = sp.fp32 ? Engine<float>::footprint(sp) : Engine<double>::footprint(sp);
        need += Arena::round(b);
        largest = std::max(largest, Arena::round(b));
    }
    const size_t cap = std::min(need, default_arena_bytes(h->budget));
    if (largest > cap) fail(TSVD_E_NOMEM, "a problem does not fit the arena");
    char* mem = nullptr;
    hipError_t e = hipMalloc(&mem, cap);
    if (e != hipSuccess) fail(TSVD_E_NOMEM, std::string("hipMalloc arena: ") + hipGetErrorString(e));
    Arena arena;
    arena.reset(mem, cap);
    std::vector<Result> res(count);
    try {
        Engine<float> ef(h->device, h->cus, h->lds_cap);
        Engine<double> ed(h->device, h->cus, h->lds_cap);
        ef.attach(&arena);
        ed.attach(&arena);
        size_t next = 0;
        auto record = [&](uint64_t ticket, const Result& r) { res[ticket] = r; };
        for (;;) {
            // admit in order while the arena has room
            while (next < specs.size()) {
                const Spec& sp = specs[next];
                const bool ok = sp.fp32 ? ef.admit(sp, next, t0) : ed.admit(sp, next, t0);
                if (!ok) break;
                ++next;
            }
            if (ef.running() == 0 && ed.running() == 0) {
                if (next >= specs.size()) break;
                fail(TSVD_E_NOMEM, "arena too small for the next problem");
            }
            ef.period();
            ed.period();
            ef.harvest(record);
            ed.harvest(record);
        }
    } catch (...) {
        (void)hipDeviceSynchronize();
        (void)hipFree(mem);
        throw;
    }
    hip_check(hipFree(mem), "hipFree arena");
    for (int i = 0; i < count; ++i) {
        if (infos) infos[i] = res[i].info;
        if (status) status[i] = res[i].status;
    }
}

// ------------------------------------------------------------------ serving

struct Server {
    explicit Server(tsvd_handle h)
        : handle(h), ef(h->device, h->cus, h->lds_cap), ed(h->device, h->cus, h->lds_cap) {}

    tsvd_handle handle;
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    bool started = false;
    struct Queued {
        uint64_t ticket;
        Spec sp;
        Clock::time_point t0;
    };
    std::deque<Queued> queue;
    std::unordered_map<uint64_t, Result> results;
    std::unordered_set<uint64_t> cancelled;   // running tickets to drop at the next period boundary
    uint64_t next_ticket = 1;
    tsvd_serve_stats stats{};
    std::string worker_error;
    tsvd_status worker_status = TSVD_OK;
    // device side (worker thread only after start)
    Arena arena;
    char* mem = nullptr;
    Engine<float> ef;
    Engine<double> ed;
    // admission stops at this many running Fourier slices (the batched form
    // keeps the chip busy with about a thousand)
    int64_t slice_cap = std::max(1, env_int("TSVD_SERVE_SLICES", 1024));

    void start() {
        if (started) return;
        Device dev(handle->device);
        const size_t cap = default_arena_bytes(handle->budget);
        hipError_t e = hipMalloc(&mem, cap);
        if (e != hipSuccess) fail(TSVD_E_NOMEM, std::string("hipMalloc arena: ") + hipGetErrorString(e));
        arena.reset(mem, cap);
        ef.attach(&arena);
        ed.attach(&arena);
        stats.arena_bytes = (int64_t)cap;
        started = true;
        worker = std::thread([this] { loop(); });
    }

    void shutdown() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv.notify_all();
        if (worker.joinable()) worker.join();
        if (started) {
            Device dev(handle->device);
            ef.release();
            ed.release();
            if (mem) (void)hipFree(mem);
            mem = nullptr;
        }
    }

    void finish(uint64_t ticket, const Result& r) {
        std::lock_guard<std::mutex> lk(mu);
        results[ticket] = r;
        stats.finished += 1;
    }

    void loop() {
        (void)hipSetDevice(handle->device);
        for (;;) {
            std::vector<Queued> take;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || !queue.empty() || ef.running() + ed.running() > 0; });
                if (stop) return;
            }
            try {
                // admit from the head of the queue while the arena has room and
                // the running problems do not yet fill the chip: past about
                // slice_cap Fourier slices the GPU is saturated, and admitting
                // more only makes every running request slower
                {
                    // queued requests past their deadline never start
                    std::lock_guard<std::mutex> lk(mu);
                    const auto now = Clock::now();
                    for (auto it = queue.begin(); it != queue.end();) {
                        const double dl = it->sp.p.deadline_s;
                        if (dl > 0.0 && std::chrono::duration<double>(now - it->t0).count() > dl) {
                            Result& r = results[it->ticket];
                            r.status = TSVD_E_TIMEOUT;
                            r.info.seconds = std::chrono::duration<double>(now - it->t0).count();
                            stats.finished += 1;
                            it = queue.erase(it);
                        } else {
                            ++it;
                        }
                    }
                }
                for (;;) {
                    Queued q;
                    {
                        std::lock_guard<std::mutex> lk(mu);
                        if (queue.empty()) break;
                        q = queue.front();
                    }
                    const int64_t busy = ef.running_slices() + ed.running_slices();
                    if (busy > 0 && busy + q.sp.g.h > slice_cap) break;
                    const bool ok = q.sp.fp32 ? ef.admit(q.sp, q.ticket, q.t0) : ed.admit(q.sp, q.ticket, q.t0);
                    if (!ok) break;
                    std::lock_guard<std::mutex> lk(mu);
                    queue.pop_front();
                }
                ef.period();
                ed.period();
                auto cb = [&](uint64_t t, const Result& r) { finish(t, r); };
                ef.harvest(cb);
                ed.harvest(cb);
                {
                    // cancellations and deadlines of running requests
                    std::unordered_set<uint64_t> drop;
                    {
                        std::lock_guard<std::mutex> lk(mu);
                        drop.swap(cancelled);
                    }
                    auto is_cancelled = [&](uint64_t t) { return drop.count(t) != 0; };
                    const auto now = Clock::now();
                    ef.expire(is_cancelled, now, cb);
                    ed.expire(is_cancelled, now, cb);
                }
                std::lock_guard<std::mutex> lk(mu);
                stats.iterations = ef.iterations() + ed.iterations();
                stats.running = (int64_t)(ef.running() + ed.running());
                stats.peak_running = std::max(stats.peak_running, stats.running);
                stats.queued = (int64_t)queue.size();
                stats.arena_used = (int64_t)arena.used();
            } catch (const Failure& f) {
                // a device failure ends serving: fail every open ticket,
                // queued or running
                std::lock_guard<std::mutex> lk(mu);
                worker_error = f.msg;
                worker_status = f.status;
                for (auto& q : queue) results[q.ticket].status = f.status;
                queue.clear();
                auto fail_cb = [&](uint64_t t, const Result& r) {
                    results[t] = r;
                    stats.finished += 1;
                };
                ef.abandon(f.status, fail_cb);
                ed.abandon(f.status, fail_cb);
                stop = true;
                return;
            }
        }
    }
};

void serve_submit(tsvd_handle h, const tsvd_problem* prob, uint64_t* ticket) {
    check_handle(h);
    if (!prob || !ticket) fail(TSVD_E_INVALID, "null argument");
    const Spec sp = validate(*prob);
    if (!h->server) h->server = new Server(h);
    Server& s = *h->server;
    s.start();
    const size_t bytes = sp.fp32 ? Engine<float>::footprint(sp) : Engine<double>::footprint(sp);
    if (Arena::round(bytes) > s.arena.cap()) fail(TSVD_E_NOMEM, "problem does not fit the serving arena");
    {
        std::lock_guard<std::mutex> lk(s.mu);
        if (s.stop) fail(TSVD_E_HIP, "serving stopped after a device failure: " + s.worker_error);
        *ticket = s.next_ticket++;
        s.results[*ticket] = Result{};
        s.queue.push_back(Server::Queued{*ticket, sp, Clock::now()});
        s.stats.submitted += 1;
    }
    s.cv.notify_all();
}

tsvd_status serve_poll(tsvd_handle h, uint64_t ticket, tsvd_info* info) {
    check_handle(h);
    if (!h->server) fail(TSVD_E_INVALID, "unknown ticket");
    Server& s = *h->server;
    std::lock_guard<std::mutex> lk(s.mu);
    auto it = s.results.find(ticket);
    if (it == s.results.end()) fail(TSVD_E_INVALID, "unknown ticket");
    // a worker stopped by a device failure finishes no open ticket
    if (it->second.status == TSVD_E_BUSY && s.stop && s.worker_status != TSVD_OK)
        it->second.status = s.worker_status;
    if (it->second.status != TSVD_E_BUSY && info) *info = it->second.info;
    return it->second.status;
}

void serve_cancel(tsvd_handle h, uint64_t ticket) {
    check_handle(h);
    if (!h->server) fail(TSVD_E_INVALID, "unknown ticket");
    Server& s = *h->server;
    {
        std::lock_guard<std::mutex> lk(s.mu);
        auto it = s.results.find(ticket);
        if (it == s.results.end()) fail(TSVD_E_INVALID, "unknown ticket");
        if (it->second.status != TSVD_E_BUSY) return;   // already finished
        for (auto q = s.queue.begin(); q != s.queue.end(); ++q) {
            if (q->ticket != ticket) continue;
            it->second.status = TSVD_E_CANCELLED;
            it->second.info.seconds = std::chrono::duration<double>(Clock::now() - q->t0).count();
            s.stats.finished += 1;
            s.queue.erase(q);
            return;
        }
        s.cancelled.insert(ticket);   // running: dropped at the next period boundary
    }
    s.cv.notify_all();
}

void serve_stats(tsvd_handle h, tsvd_serve_stats* out) {
    check_handle(h);
    if (!out) fail(TSVD_E_INVALID, "null argument");
    if (!h->server) {
        *out = tsvd_serve_stats{};
        return;
    }
    std::lock_guard<std::mutex> lk(h->server->mu);
    *out = h->server->stats;
}

void serve_shutdown(tsvd_handle h) {
    if (!h || !h->server) return;
    h->server->shutdown();
    delete h->server;
    h->server = nullptr;
}

}  // namespace tsvd
