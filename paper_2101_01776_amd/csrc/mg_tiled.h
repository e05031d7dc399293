// Arguments and launchers of the LDS-tiled multigrid kernels (mg_tiled.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "irk_internal.h"

namespace irk {

#define IRK_MAX_CHEB 8
#define IRK_MAX_COARSE_ITERS 64
#define IRK_MAX_SUB_LEVELS 8       // levels of the one-work-group sub-cycle

// One level of a V-cycle: geometry, operator parameters, buffers.
template <class T>
struct MgLevelArgs {
    int nx, ny;
    T h, nu, sigma, dt;
    const T *coef;       // linearization field on this level (nullptr: Poisson)
    const T *b;          // right-hand side (levels > 0)
    T *x;                // iterate on this level (down: written; up: read)
    T *xout;             // up: smoothed iterate (a different buffer than x:
                         // neighbouring tiles read x in their halos)
    T *bc;               // down: restricted residual -> next level's b
    const T *xc;         // up: next level's correction
    T cd[IRK_MAX_CHEB], cr[IRK_MAX_CHEB];   // Chebyshev step coefficients
};

// Finest-level right-hand side taken from float64 Krylov vectors:
// b = a1 v1 + a2 v2 - (a1 mean[0] + a2 mean[1]) (v2, mean optional).
struct MgIn {
    const double *v1 = nullptr;
    double a1 = 1.0;
    const double *v2 = nullptr;
    double a2 = 0.0;
    const double *mean = nullptr;
};

// Finest-level output written as float64: z = x + shift_scale * shift[0];
// carries the right-hand side definition again for the up sweep.
struct MgOut {
    double *z = nullptr;
    const double *shift = nullptr;
    double shift_scale = 0.0;
    const double *v1 = nullptr;
    double a1 = 1.0;
    const double *v2 = nullptr;
    double a2 = 0.0;
    const double *mean_in = nullptr;
};

// Levels l0..L-1 of a V-cycle solved inside one work-group.
template <class T>
struct MgSubArgs {
    int nlev;
    int nx[IRK_MAX_LEVELS], ny[IRK_MAX_LEVELS];
    T h[IRK_MAX_LEVELS];
    T nu, sigma, dt;
    const T *coef[IRK_MAX_LEVELS];
    const T *b0;         // right-hand side of the first level (when MgIn has none)
    T *x0;               // result of the first level (when MgOut has no z)
    int deg, coarse_iters;
    T cd[IRK_MAX_CHEB], cr[IRK_MAX_CHEB];
    T ccd[IRK_MAX_COARSE_ITERS], ccr[IRK_MAX_COARSE_ITERS];
};

template <class T>
void launch_mg_down(hipStream_t st, int opk, const MgLevelArgs<T> &a, const MgIn &in, int deg);
template <class T>
void launch_mg_up(hipStream_t st, int opk, const MgLevelArgs<T> &a, const MgOut &out, int deg);
template <class T>
void launch_mg_subcycle(hipStream_t st, int opk, const MgSubArgs<T> &s, const MgIn &in, const MgOut &out);
// LDS bytes of the one-work-group sub-cycle over levels nx[0..nlev-1]
size_t mg_subcycle_lds_bytes(int opk, int nlev, const int *nx, const int *ny, size_t tsz);

}  // namespace irk
