// Shared definitions of the gfx950 t-SVT library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tsvd {

// Interleaved complex number; the slice workspaces hold arrays of these.
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T re, im;
};

// Shape of one problem as the kernels see it.
//
// The trailing modes of a tube are (P, Q): a 3-D tensor has P = 1, Q = n3;
// a 4-D tensor has P = n3, Q = n4.  The real DFT runs along Q (half
// spectrum Qh = Q/2 + 1 bins) and a full complex DFT along P, so there are
// h = P * Qh Fourier frontal slices; slice s holds bin (k3, k4) =
// (s / Qh, s % Qh).
//
// Every slice is stored column-major with the longer matrix mode as rows:
// m = max(n1, n2) rows, n = min(n1, n2) columns, element (row, col) at
// col * m + row.  trans == false: row = i, col = j (n1 >= n2);
// trans == true: row = j, col = i (n1 < n2), i.e. the slice is transposed,
// which leaves t-SVT unchanged up to the same transpose.
struct Geometry {
    int64_t n1, n2;
    int P, Q, Qh, L, h;
    int m, n;
    bool trans;
    int64_t ntubes, numel;
};

// One launch-wide parameter block of the ADMM drivers, kept in device
// memory so that kernels read the current penalty without a host round trip.
struct Ctrl {
    double rho;        // penalty of the current iteration's prox
    double tau;        // threshold of the current prox = 1 / rho
    double dscale;     // the stored dual is dscale * (value in the buffer)
    double growth;     // penalty growth factor
    double rho_max;    // penalty cap
    double tol_abs;    // tol * ||data||_F
    double shrink;     // S-update threshold lambda / mu (RPCA)
    double lambda;     // RPCA weight
    double primal;     // last primal residual
    double change;     // last change residual
    double rho_used;   // penalty of the last finished iteration
    double dscale_used;  // dual scale of the last finished iteration
    int32_t iter;      // finished iterations
    int32_t done;      // 1 once the stop test passed, 2 at the iteration cap
    int32_t nonfinite; // 1 if a residual was not finite
    int32_t max_iter;  // iteration cap of a problem-table run (0: none)
    int32_t sweep_max;     // problem-table runs: largest sweep count of this iteration's SVDs
    int32_t sweeps_total;  // problem-table runs: sum of sweep_max over finished iterations
    int32_t sweeps_last;   // problem-table runs: sweep_max of the last finished iteration
    int32_t pad;
};

constexpr int kBlock = 256;        // threads per workgroup of the elementwise/DFT kernels
constexpr int kNumPartials = 4;    // residual partial sums per workgroup

}  // namespace tsvd
