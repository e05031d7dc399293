// Arguments and launchers of the LDS-tiled multigrid kernels (mg_tiled.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "irk_internal.h"

namespace irk {

#define IRK_MAX_CHEB 8
#define IRK_MAX_COARSE_ITERS 64
#define IRK_MAX_SUB_LEVELS 8       // levels of the one-work-group sub-cycle
#define IRK_SUB_WAVE_PTS 64        // sub-cycle levels this small run on one wave

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
    int nx[IRK_MAX_SUB_LEVELS], ny[IRK_MAX_SUB_LEVELS];
    T h[IRK_MAX_SUB_LEVELS];
    T nu, sigma, dt;
    const T *coef[IRK_MAX_SUB_LEVELS];
    const T *b0;         // right-hand side of the first level (when MgIn has none)
    T *x0;               // result of the first level (when MgOut has no z)
    int deg, coarse_iters;
    int wave_pts;        // levels of at most this many points run on one wave
    T cd[IRK_MAX_CHEB], cr[IRK_MAX_CHEB];
};

// Several jobs of one kernel in one launch (at most IRK_MG_BATCH; the
// argument block stays below the 4 KiB kernel-argument limit).
#define IRK_MG_BATCH 6
template <class T>
struct MgLevelBatch {
    int n;
    int prefix[IRK_MG_BATCH + 1];       // first work-group of each job; prefix[n] = grid
    MgLevelArgs<T> g[IRK_MG_BATCH];
    MgIn in[IRK_MG_BATCH];
    MgOut out[IRK_MG_BATCH];
};
template <class T>
struct MgSubBatch {
    MgSubArgs<T> s[IRK_MG_BATCH];
    MgIn in[IRK_MG_BATCH];
    MgOut out[IRK_MG_BATCH];
};

template <class T>
void launch_mg_down(hipStream_t st, int opk, const MgLevelArgs<T> &a, const MgIn &in, int deg);
template <class T>
void launch_mg_up(hipStream_t st, int opk, const MgLevelArgs<T> &a, const MgOut &out, int deg);
template <class T>
void launch_mg_subcycle(hipStream_t st, int opk, const MgSubArgs<T> &s, const MgIn &in, const MgOut &out);

// Batched launches: n jobs of one kernel (n >= 1; split into launches of at
// most IRK_MG_BATCH jobs of one tile shape each).  Jobs must be independent.
template <class T>
void launch_mg_down_batch(hipStream_t st, int opk, const MgLevelArgs<T> *g, const MgIn *in, int n, int deg);
template <class T>
void launch_mg_up_batch(hipStream_t st, int opk, const MgLevelArgs<T> *g, const MgOut *out, int n, int deg);
template <class T>
void launch_mg_subcycle_batch(hipStream_t st, int opk, const MgSubArgs<T> *s, const MgIn *in, const MgOut *out,
                              int n);
// Exact solve of the periodic Poisson problem -dt Lap_h x = b (mean-free
// part) on an n x n level (n <= IRK_FDM_MAX, a multiple of 4) by fast
// diagonalization: Q is
// the n x n real orthonormal Fourier basis (row = grid index, column = mode),
// lam[k] = 4 sin^2(pi m_k / n) / h^2 its eigenvalues of -D2; one work-group.
#define IRK_FDM_MAX 32
template <class T>
void launch_poisson_fdm(hipStream_t st, int n, T dt, const T *Q, const T *lam, const T *b, T *x);
// LDS bytes of the one-work-group sub-cycle over levels nx[0..nlev-1]
size_t mg_subcycle_lds_bytes(int opk, int nlev, const int *nx, const int *ny, size_t tsz);

}  // namespace irk
