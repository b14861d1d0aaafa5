// Launch log: every kernel launch of the multigrid / domain-decomposition path
// goes through EHH_LAUNCH.  While the log is switched on (one preconditioner
// application inside ehh_profile_precondition), each launch is also recorded
// as a closure that launches the same kernel with the same arguments again,
// together with its algorithmic HBM bytes, so that every kernel of a real cycle
// can be replayed and timed on its own.  Switched off, a launch costs one
// relaxed atomic load more.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <functional>

#include "common.hpp"

namespace ehh {

// Algorithmic bytes of one launch: this library's count (every vector entry the
// kernel must read or write once, the operator's compact coefficients once) and
// the per-cell model of the (1,1)-cycle (V unknowns of w bytes per cell per
// source: 3 V w for a half-sweep from e_in, 2 V w from zero, plus C bytes of
// coefficients per cell).
struct LaunchBytes {
    double mine = 0.0;
    double model = 0.0;
};

bool launch_log_on();
// again(stream, start, stop): the launch repeated on stream; with start / stop
// events, they record the dispatch's own begin and end (hipExtLaunchKernel)
using LaunchAgain = std::function<void(hipStream_t, hipEvent_t, hipEvent_t)>;
void launch_log_add(const void* kernel, LaunchBytes bytes, LaunchAgain again);

// Byte counts of the cycle's kernels on a level of geometry g with R sources in
// a precision of es bytes per real.  coef_reals: the level's coefficient reals
// per cell in this library's storage (fine: 4; Galerkin: the symmetric stencil).
inline double level_coef_reals(const Geo& g, bool fine) {
    if (fine) return 4.0 * (double)g.ncell;
    const double nu = (double)(g.N - g.ncell);
    return g.dim == 2 ? nu * (2 * 8 + 6) + (double)g.ncell : nu * (2 * 38 + 18) + (double)g.ncell;
}
// model coefficient bytes per cell: fine 4 reals, Galerkin 29 (2D) / 169 (3D) complex
inline double model_coef_bytes(const Geo& g, bool fine, int es) {
    if (fine) return 4.0 * es;
    return (g.dim == 2 ? 29.0 : 169.0) * 2.0 * es;
}
// red-black half-sweep: b on the colour's rows, e_in (when given) and e_out
inline LaunchBytes bytes_relax(const Geo& g, bool fine, int R, bool with_e, int es, int out_es, double coef_es) {
    const double w = 2.0 * es, nu = (double)(g.N - g.ncell), nc = (double)g.ncell;
    LaunchBytes b;
    b.mine = R * ((nu + nc / 2) * w + (with_e ? g.N * w : 0.0) + g.N * 2.0 * out_es) +
             level_coef_reals(g, fine) * coef_es;
    const double V = g.dim + 1;
    b.model = nc * (R * ((with_e ? 2.0 : 1.0) * V * w + V * 2.0 * out_es) + model_coef_bytes(g, fine, es));
    return b;
}
// y = A x (b == null) or r = b - A x
inline LaunchBytes bytes_apply(const Geo& g, bool fine, int R, bool with_b, int es, double coef_es) {
    const double w = 2.0 * es;
    LaunchBytes b;
    b.mine = R * (with_b ? 3.0 : 2.0) * g.N * w + level_coef_reals(g, fine) * coef_es;
    b.model = (double)g.ncell * (R * (with_b ? 3.0 : 2.0) * (g.dim + 1) * w + model_coef_bytes(g, fine, es));
    return b;
}
// transfers: restriction reads the fine vector and writes the coarse one,
// prolongation reads both and writes the fine one
inline LaunchBytes bytes_transfer(const Geo& gf, const Geo& gc, int R, bool prolong, int es) {
    const double w = 2.0 * es;
    LaunchBytes b;
    b.mine = R * w * ((prolong ? 2.0 : 1.0) * gf.N + gc.N);
    b.model = R * w * (gf.dim + 1) * ((prolong ? 2.0 : 1.0) * gf.ncell + gc.ncell);
    return b;
}
inline LaunchBytes bytes_plain(double v) { return LaunchBytes{v, v}; }

}  // namespace ehh

// Launch kernel K (a parenthesised template-id where it has commas) like
// hipLaunchKernelGGL, with BYTES (a LaunchBytes expression, evaluated only while
// the launch log is on) recorded together with a closure that repeats it.
#define EHH_LAUNCH_B(BYTES, K, GRID, BLOCK, SHMEM, STREAM, ...)                                            \
    do {                                                                                                  \
        hipLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                                   \
        if (::ehh::launch_log_on())                                                                       \
            ::ehh::launch_log_add(reinterpret_cast<const void*>(&K), (BYTES),                              \
                                  [=](hipStream_t ehh_s_, hipEvent_t ehh_e0_, hipEvent_t ehh_e1_) {       \
                                      if (ehh_e0_)                                                        \
                                          hipExtLaunchKernelGGL(K, GRID, BLOCK, SHMEM, ehh_s_, ehh_e0_,   \
                                                                ehh_e1_, 0, __VA_ARGS__);                 \
                                      else                                                                \
                                          hipLaunchKernelGGL(K, GRID, BLOCK, SHMEM, ehh_s_, __VA_ARGS__); \
                                  });                                                                     \
    } while (0)
#define EHH_LAUNCH(K, GRID, BLOCK, SHMEM, STREAM, ...) \
    EHH_LAUNCH_B(::ehh::LaunchBytes{}, K, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__)
