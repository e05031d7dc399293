// The stage residual of equation (stages) / (dae_stage) without a context or
// a caller workspace, for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// allocation).
//
// Its scratch -- the stage values U, the reduction partials and device
// scalars, the forcing tables -- lives in one file-scope device array of
// fixed size, `scratch`.  Host code never passes the array's name to a
// kernel or a copy (on the host that name is only a stand-in for the
// symbol): the device address of each GPU's copy is looked up once per
// device with hipGetSymbolAddress, with that device current, and kept.
// Every call on a GPU shares that GPU's array and keeps the last call's
// contents; nothing in it needs to start at zero (every value is written
// before it is read).  Calls that overlap on one GPU race on it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "irk_internal.h"
#include "kernels.h"

namespace irk {

#define IRK_NOALLOC_MAX_DEVICES 64

static __device__ __align__(256) unsigned char scratch[IRK_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[IRK_NOALLOC_MAX_DEVICES];

// device address of the current device's scratch array (looked up once)
static irk_status scratch_address(void **ptr) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= IRK_NOALLOC_MAX_DEVICES) return IRK_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return IRK_E_DEVICE;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return IRK_OK;
}

// forcing tables sin / cos (2 pi x_i), x_i = i h, and the same in y
__global__ void __launch_bounds__(IRK_WG) k_forcing_tables(double *tab, int nx, int ny, double h) {
    const double two_pi = 2.0 * 3.14159265358979323846;
    const int n = 2 * (nx + ny);
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        double v;
        if (q < nx) v = sin(two_pi * (q * h));
        else if (q < 2 * nx) v = cos(two_pi * ((q - nx) * h));
        else if (q < 2 * nx + ny) v = sin(two_pi * ((q - 2 * nx) * h));
        else v = cos(two_pi * ((q - 2 * nx - ny) * h));
        tab[q] = v;
    }
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace irk

using namespace irk;

extern "C" irk_status irk_eval_residual_noalloc(irk_family family, int s, const irk_operator *op,
                                                const double *u_n, double t_n, double dt, const double *K,
                                                double *F, void *hip_stream) {
    if (!op || !u_n || !K || !F || !(dt > 0) || !std::isfinite(t_n) || s < 1 || s > IRK_MAX_STAGES)
        return IRK_E_ARG;
    if (family == IRK_SDIRK) return IRK_E_UNSUPPORTED;      // its stages are solved one at a time
    if (op->kind < IRK_OP_BURGERS_1D || op->kind > IRK_OP_VSF_2D || op->nx < 3 || !(op->length > 0))
        return IRK_E_ARG;
    const bool one_d = op->kind == IRK_OP_BURGERS_1D;
    if (one_d ? op->ny != 1 : (op->ny != op->nx)) return IRK_E_ARG;
    if (((uintptr_t)u_n | (uintptr_t)K | (uintptr_t)F) & 7) return IRK_E_ARG;
    // scratch: U [s][nf], reduction partials, device scalars, forcing tables;
    // sizes beyond the array are refused before any device call
    const int nvar = op->kind == IRK_OP_VSF_2D ? 2 : 1;
    const size_t npts = (size_t)op->nx * op->ny, nf = nvar * npts;
    const size_t off_U = 0;
    const size_t off_part = align256(off_U + (size_t)s * nf * sizeof(double));
    const size_t off_dv = align256(off_part + (size_t)IRK_RED_BLOCKS * 32 * sizeof(double));
    const size_t off_tab = align256(off_dv + 512 * sizeof(double));
    const size_t total = align256(off_tab + (size_t)2 * (op->nx + op->ny) * sizeof(double));
    if (total > (size_t)IRK_NOALLOC_SCRATCH_BYTES) return IRK_E_NOMEM;

    long double Al[IRK_MAX_STAGES * IRK_MAX_STAGES], bl[IRK_MAX_STAGES], cl[IRK_MAX_STAGES];
    if (!build_tableau_ld(family, s, Al, bl, cl)) return IRK_E_ARG;
    StageCoefs C;
    std::memset(&C, 0, sizeof(C));
    for (int i = 0; i < s * s; ++i) {
        C.A[i] = (double)Al[i];
        C.Tinv[i] = (i / s == i % s) ? 1.0 : 0.0;            // identity transform: F itself
    }
    for (int i = 0; i < s; ++i) {
        C.b[i] = (double)bl[i];
        C.tstage[i] = t_n + (double)cl[i] * dt;
        C.sin_t[i] = std::sin(C.tstage[i]);
        C.cos_t[i] = std::cos(C.tstage[i]);
    }

    void *base = nullptr;
    irk_status e = scratch_address(&base);
    if (e != IRK_OK) return e;
    unsigned char *ws = (unsigned char *)base;
    double *U = (double *)(ws + off_U), *part = (double *)(ws + off_part), *dv = (double *)(ws + off_dv);
    double *tab = (double *)(ws + off_tab);

    DeviceProblem dp;
    std::memset(&dp, 0, sizeof(dp));
    dp.kind = op->kind;
    dp.forcing = op->kind == IRK_OP_NLDIFF_2D ? op->forcing : IRK_FORCING_NONE;
    dp.nvar = nvar;
    dp.g.nx = op->nx;
    dp.g.ny = op->ny;
    dp.g.h = op->length / op->nx;
    dp.g.nu = op->nu;
    dp.sinx = tab;
    dp.cosx = tab + op->nx;
    dp.siny = tab + 2 * op->nx;
    dp.cosy = tab + 2 * op->nx + op->ny;

    hipStream_t st = (hipStream_t)hip_stream;
    (void)hipGetLastError();
    if (dp.forcing != IRK_FORCING_NONE) {
        const int n = 2 * (op->nx + op->ny);
        k_forcing_tables<<<(n + IRK_WG - 1) / IRK_WG, IRK_WG, 0, st>>>(tab, op->nx, op->ny, dp.g.h);
    }
    // U_i = u_n + dt sum_j a_ij k_j (no fold: K is only read)
    launch_stage_prep(st, s, nf, u_n, const_cast<double *>(K), nullptr, U, C, dt, 0);
    if (op->kind == IRK_OP_VSF_2D)
        launch_field_sums(st, U, npts, 2 * s, npts, 1.0 / npts, part, dv + 24, nullptr);
    launch_residual(st, s, dp, U, K, F, C, dv + 24, part, dv, dv + 40);
    return hipGetLastError() == hipSuccess ? IRK_OK : IRK_E_DEVICE;
}
