// Host-side helpers shared by the C ABI (capi.hip) and the batch / serving
// engine (engine.hip): error plumbing, the handle, geometry and settings.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <new>
#include <string>
#include <vector>

#include "../../include/tsvd.h"
#include "kernels.h"

namespace tsvd {

inline thread_local std::string g_last_error;

struct Failure {
    tsvd_status status;
    std::string msg;
};

[[noreturn]] inline void fail(tsvd_status s, const std::string& msg) { throw Failure{s, msg}; }

inline void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(TSVD_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

inline void launch_check(const char* what) { hip_check(hipGetLastError(), what); }

inline int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}

inline double env_double(const char* name, double dflt) {
    const char* v = std::getenv(name);
    return v && *v ? std::atof(v) : dflt;
}

// Jacobi rotation tolerance of an m-row slice (a pair is rotated when its
// relative off-diagonal exceeds it).  FP64: sqrt(m) eps.  FP32 form:
// 32 sqrt(m) eps32 -- the ADMM recovers the same tensor (relative difference
// to the FP64 path ~8e-6 on the video-shaped workload, bar 1e-4) with fewer
// sweeps than nearer the rounding floor (16 sqrt(m) eps32: 5.7e-6, 3% slower;
// 64: 7.7e-6, 1% faster).  Looser factors cost accuracy where the iterates
// are less benign: at 96 the 256 x 256 x 64 RPCA prefix (15 iterations) is
// 2.1e-4 from the FP64 oracle, over the bar.  TSVD_JACOBI_TOL /
// TSVD_JACOBI_TOL32 override it.
inline double jacobi_tol(int m, int elem_bytes) {
    const double eps = elem_bytes == 4 ? 32.0 * 1.1920928955078125e-07 : 2.220446049250313e-16;
    return env_double(elem_bytes == 4 ? "TSVD_JACOBI_TOL32" : "TSVD_JACOBI_TOL", std::sqrt((double)m) * eps);
}

// Scale of the stopping rule's rounding floor (rot_forces_sweep): m eps^2 of
// the element type, so that the floor is sqrt(m) eps ||A||_F for a slice A.
// TSVD_SWEEP_FLOOR scales it (0 drops the floor: the plain rule).
inline double jacobi_floor_scale(int m, int elem_bytes) {
    const double eps = elem_bytes == 4 ? 1.1920928955078125e-07 : 2.220446049250313e-16;
    return std::max(0.0, env_double("TSVD_SWEEP_FLOOR", 1.0)) * (double)m * eps * eps;
}

// Largest supported sizes (LDS staging of the DFT tiles and Jacobi blocks).
constexpr int kMaxTube = 512;
constexpr int kMaxSlices = 300;
constexpr int64_t kMaxRows = 1 << 18;   // longer matrix mode of a slice (tall slices: global-memory Jacobi)
constexpr size_t kScratchBytes = size_t(64) << 20;   // workspace of tsvt_noalloc, per device

struct Server;   // serving engine of a handle (engine.hip)

// engine.hip
void batch_run(tsvd_handle h, const tsvd_problem* probs, int count, tsvd_info* infos, int32_t* status);
void serve_submit(tsvd_handle h, const tsvd_problem* prob, uint64_t* ticket);
tsvd_status serve_poll(tsvd_handle h, uint64_t ticket, tsvd_info* info);
void serve_cancel(tsvd_handle h, uint64_t ticket);
void serve_stats(tsvd_handle h, tsvd_serve_stats* out);
void serve_shutdown(tsvd_handle h);

}  // namespace tsvd

struct tsvd_handle_s {
    int device = 0;
    size_t budget = 0;
    hipStream_t stream = nullptr;
    // workspace arena: one allocation, carved per call
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // small device objects
    tsvd::Ctrl* ctrl = nullptr;
    int* flag = nullptr;            // non-finite flag
    void* dmat = nullptr;           // DFT matrices of the current tube shape
    int64_t dmat_key = -1;          // (P, Q, element size) they were built for
    // pinned host staging
    int* host_ints = nullptr;
    int host_ints_len = 0;
    void* host_stage = nullptr;     // argument tables uploaded once per call
    size_t host_stage_len = 0;
    tsvd::Ctrl* host_ctrl = nullptr;
    // ADMM loop of the single-problem calls: the control kernel copies the
    // control block into one of two slots of mapped pinned host memory, and
    // an event per slot tells the host when it is complete
    tsvd::Ctrl* mirror_host = nullptr;
    tsvd::Ctrl* mirror_dev = nullptr;   // device address of mirror_host
    hipEvent_t mirror_ev[2] = {nullptr, nullptr};
    // profiling (tsvd_profile)
    struct Pending {
        int kind;
        hipEvent_t a, b;
        double work;
        double sweeps = 0.0, pairs = 0.0;   // Jacobi families: slice sweeps and pairs visited
        double kept = 0.0;                  // rebuild: summed kept rank
    };
    struct Agg {
        int64_t launches = 0;
        double ms = 0.0, work = 0.0;
        double sweeps = 0.0, pairs = 0.0, rotations = 0.0, kept = 0.0;
    };
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<Pending> pending;
    std::vector<Agg> agg;
    unsigned long long* rot_counter = nullptr;   // [0] self, [1] cross
    int cus = 0;
    size_t lds_cap = 0;
    tsvd::Server* server = nullptr;   // batch / serving engine, created on first use
    char* scratch = nullptr;          // device address of this device's no-allocation scratch
};

namespace tsvd {

struct Device {
    explicit Device(int d) {
        hip_check(hipGetDevice(&prev), "hipGetDevice");
        if (prev != d) hip_check(hipSetDevice(d), "hipSetDevice");
        target = d;
    }
    ~Device() {
        if (prev != target) (void)hipSetDevice(prev);
    }
    int prev = 0, target = 0;
};

inline Geometry make_geometry(const tsvd_shape& s) {
    if (s.ndim != 3 && s.ndim != 4) fail(TSVD_E_SHAPE, "ndim must be 3 or 4");
    for (int k = 0; k < s.ndim; ++k)
        if (s.n[k] < 1) fail(TSVD_E_SHAPE, "every dimension must be >= 1");
    Geometry g{};
    g.n1 = s.n[0];
    g.n2 = s.n[1];
    if (s.ndim == 3) {
        g.P = 1;
        g.Q = (int)s.n[2];
        if (s.n[2] > kMaxTube) fail(TSVD_E_SHAPE, "tube length above the supported maximum");
    } else {
        if (s.n[2] * s.n[3] > kMaxTube) fail(TSVD_E_SHAPE, "tube length above the supported maximum");
        g.P = (int)s.n[2];
        g.Q = (int)s.n[3];
    }
    g.L = g.P * g.Q;
    g.Qh = g.Q / 2 + 1;
    g.h = g.P * g.Qh;
    if (g.h > kMaxSlices) fail(TSVD_E_SHAPE, "too many Fourier slices");
    g.trans = g.n1 < g.n2;
    const int64_t m = std::max(g.n1, g.n2), n = std::min(g.n1, g.n2);
    if (m > kMaxRows) fail(TSVD_E_SHAPE, "matrix mode above the supported maximum");
    g.m = (int)m;
    g.n = (int)n;
    g.ntubes = g.n1 * g.n2;
    g.numel = g.ntubes * g.L;
    return g;
}


// FP64 twiddles exp(-2 pi i u / L); the quarter points are exact.
inline std::vector<cplx<double>> twiddles_host(int L);

// The forward and inverse DFT matrices of a tube shape (layout in kernels.h,
// DftDims), forward first, built in FP64 from the twiddles and rounded once
// to the element type.
template <typename T>
inline std::vector<T> dft_matrices_host(const Geometry& g) {
    const DftDims d = DftDims::of(g.h, g.L);
    const std::vector<cplx<double>> tw = twiddles_host(g.L);
    std::vector<T> m((size_t)d.total(), (T)0);
    T* F = m.data();
    T* S = m.data() + d.fwd_size();
    for (int s = 0; s < g.h; ++s) {
        const int k3 = s / g.Qh, k4 = s - k3 * g.Qh;
        const double c = (k4 == 0 || 2 * k4 == g.Q) ? 1.0 : 2.0;
        for (int t = 0; t < g.L; ++t) {
            const int t3 = t / g.Q, t4 = t - t3 * g.Q;
            const int64_t u = ((int64_t)t3 * k3 * g.Q + (int64_t)t4 * k4 * g.P) % g.L;
            F[(int64_t)t * 2 * d.hp + s] = (T)tw[u].re;
            F[(int64_t)t * 2 * d.hp + d.hp + s] = (T)tw[u].im;
            S[(int64_t)(2 * s) * d.Lr + t] = (T)(c / g.L * tw[u].re);
            S[(int64_t)(2 * s + 1) * d.Lr + t] = (T)(c / g.L * tw[u].im);
        }
    }
    return m;
}

inline std::vector<cplx<double>> twiddles_host(int L) {
    std::vector<cplx<double>> tw(L);
    for (int u = 0; u < L; ++u) {
        if ((4 * u) % L == 0) {
            const int q = (4 * u) / L;
            const double c[4] = {1.0, 0.0, -1.0, 0.0}, s[4] = {0.0, -1.0, 0.0, 1.0};
            tw[u] = cplx<double>{c[q], s[q]};
        } else {
            const double a = -2.0 * M_PI * (double)u / (double)L;
            tw[u] = cplx<double>{std::cos(a), std::sin(a)};
        }
    }
    return tw;
}

template <typename F>
inline tsvd_status guarded(F&& f) {
    try {
        f();
        g_last_error.clear();
        return TSVD_OK;
    } catch (const Failure& e) {
        g_last_error = e.msg;
        return e.status;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return TSVD_E_NOMEM;
    } catch (...) {
        g_last_error = "unexpected failure";
        return TSVD_E_HIP;
    }
}

inline void check_handle(tsvd_handle h) {
    if (!h) fail(TSVD_E_INVALID, "null handle");
}

// true for the FP32 form (FP32 data), false for the plain FP64 path
inline bool check_precision(int dtype, int precision) {
    if (dtype != TSVD_F64 && dtype != TSVD_F32) fail(TSVD_E_INVALID, "unknown dtype");
    if (precision != TSVD_PREC_FP64 && precision != TSVD_PREC_FP32)
        fail(TSVD_E_INVALID, "unknown precision");
    if (dtype == TSVD_F64 && precision == TSVD_PREC_FP64) return false;
    if (dtype == TSVD_F32 && precision == TSVD_PREC_FP32) return true;
    fail(TSVD_E_UNSUPPORTED, "FP64 data needs TSVD_PREC_FP64 and FP32 data TSVD_PREC_FP32");
}

struct AdmmSettings {
    double growth, rho_max;
    int max_iter, precision, max_sweeps;
    const tsvd_state* state;
};

inline AdmmSettings settings(const tsvd_admm_opts* o, double growth, double rho_max, int max_iter) {
    AdmmSettings s{growth, rho_max, max_iter, TSVD_PREC_FP64, 30, nullptr};
    if (o) {
        if (o->pad != 0) fail(TSVD_E_INVALID, "opts.pad must be 0");
        s.state = o->state;
        if (o->growth > 0) s.growth = o->growth;
        if (o->rho_max > 0) s.rho_max = o->rho_max;
        if (o->max_iter > 0) s.max_iter = o->max_iter;
        s.precision = o->precision;
        if (o->max_sweeps > 0) s.max_sweeps = o->max_sweeps;
    }
    if (!(s.growth >= 1.0) || !std::isfinite(s.growth)) fail(TSVD_E_INVALID, "growth must be >= 1");
    return s;
}

}  // namespace tsvd
