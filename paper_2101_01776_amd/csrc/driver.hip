// Host driver of the IRK stage solve: workspace layout, the Newton-like loop
// of Algorithm 1 in the real eigenbasis of A0^{-1}, right-preconditioned
// FGMRES per eigen-block with the block lower-triangular preconditioner of
// equation (Lprec), and the geometric-multigrid V-cycle that applies each
// diagonal inverse.  All arithmetic on fields runs in the kernels of
// kernels.hip and mg_tiled.hip; the host does the s x s algebra, the
// Hessenberg least-squares problem and the control flow.
//
// In the eigenbasis the eigen-blocks are independent (no back-substitution),
// so each block's FGMRES solve runs on a "lane" of its own: a HIP stream,
// Krylov bases, multigrid work arrays and reduction scratch.  The host
// interleaves the lanes' FGMRES state machines, so that the kernels of
// different blocks overlap on the device and one lane's host round trip is
// hidden behind the others' device work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "fft_poisson.h"
#include "irk_internal.h"
#include "kernels.h"
#include "mg_tiled.h"

namespace irk {

static inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Multigrid level geometry for a problem (level 0 = the grid).
struct LevelGeom {
    int nlev = 0;
    int nx[IRK_MAX_LEVELS], ny[IRK_MAX_LEVELS];
};

static bool level_geometry(const irk_operator &op, int coarsest, LevelGeom *lg) {
    int nx = op.nx, ny = op.ny;
    const bool one_d = (ny == 1);
    int L = 0;
    while (true) {
        if (L >= IRK_MAX_LEVELS) return false;
        lg->nx[L] = nx;
        lg->ny[L] = ny;
        ++L;
        const bool can = (nx % 2 == 0) && (nx / 2 >= coarsest) &&
                         (one_d || ((ny % 2 == 0) && (ny / 2 >= coarsest)));
        if (!can) break;
        nx /= 2;
        if (!one_d) ny /= 2;
    }
    lg->nlev = L;
    // the coarsest level is solved inside one work-group
    return (size_t)lg->nx[L - 1] * lg->ny[L - 1] <= 1024;
}

// Workspace offsets of one lane (one eigen-block's concurrent solve).
struct LaneLayout {
    size_t V, Z, part, dv;
    size_t tmp;                         // one float64 field (Newton-like (3) pairs), else 0
    size_t lev[IRK_MAX_LEVELS][4];
    size_t ldv;                         // Krylov vector length (block width * field)
    size_t spec;                        // half spectrum of the spectral Poisson solve, else 0
};

// A side stream of a vorticity-streamfunction pair block: the first
// streamfunction row's Poisson V-cycle runs there, concurrently with the
// second row's vorticity V-cycle (which needs only the first vorticity
// component); its own reduction scratch, device scalars and level arrays.
struct AuxLayout {
    bool used = false;
    LaneLayout lay;
};

// Everything irk_create decides before touching the device.
struct Plan {
    irk_operator op;
    irk_options opt;
    EigenBlocks eb;
    int family = 0, s = 0, nvar = 1;
    size_t npts = 0, nf = 0;
    int m = 30;                         // restart length
    LevelGeom lg;
    int l0 = 0;                         // first level of the one-work-group sub-cycle
    int fdm_level = 0;                  // VSF: level of the exact Poisson solve (0: none)
    size_t off_fdm_Q = 0, off_fdm_lam = 0;
    bool fft_psi = false;               // VSF: streamfunction rows solved spectrally on the finest grid
    size_t fft_tsz = 0;                 // bytes per value of that solve's arithmetic
    size_t off_fft_tw = 0, off_fft_lam = 0;
    size_t tsz = 4;                     // bytes per V-cycle scalar
    int nhier = 0;                      // distinct linearization stages
    int hier_stage[IRK_MAX_STAGES];     // hierarchy -> stage index
    int row_hier[IRK_MAX_STAGES];       // transformed row -> hierarchy
    // Newton-like (2), (3): every transformed row r linearizes at the stage
    // weights d_rr (its own hierarchy, built from sum_k d_rr,k U_k) and the
    // block operators carry the weights blk_w
    bool weighted = false;
    double hier_w[IRK_MAX_STAGES][IRK_MAX_STAGES];
    BlockWeights blk_w[IRK_MAX_STAGES];
    // real Schur basis: the blocks of R0 above the diagonal, cpl[i][j] for
    // i < j, applied in the back-substitution
    BlockCouple cpl[IRK_MAX_STAGES][IRK_MAX_STAGES];
    size_t off_K, off_Y, off_Fh, off_U, off_part, off_dv, off_tab, off_K2 = 0;
    size_t off_coef[IRK_MAX_STAGES][IRK_MAX_LEVELS];
    LaneLayout lane[IRK_MAX_STAGES];
    AuxLayout aux[IRK_MAX_STAGES];
    // SDIRK: the method's own tableau; the machinery above runs one stage at
    // a time as a 1-stage method (s = 1, A = [gamma], c = [c_i])
    int sd_s = 0;
    double sd_A[IRK_MAX_STAGES * IRK_MAX_STAGES], sd_b[IRK_MAX_STAGES], sd_c[IRK_MAX_STAGES];
    size_t off_Ksd = 0, off_Uin = 0, off_Uout = 0;
    size_t total = 0;
};

static bool valid_options(const irk_options &o) {
    return o.restart >= 1 && o.restart <= IRK_MAX_RESTART && o.max_krylov >= 1 && o.max_newton >= 1 &&
           (o.newton_like >= 0 && o.newton_like <= 3) && (o.gamma_mode == 0 || o.gamma_mode == 1) &&
           (o.prec_fp32 == 0 || o.prec_fp32 == 1) && o.cheb_degree >= 1 && o.cheb_degree <= 4 &&
           o.mg_coarsest >= 2 && o.coarse_iters >= 1 && o.coarse_iters <= 64 && o.krylov_rtol > 0 &&
           o.krylov_rtol < 1 && o.newton_rtol >= 0 && o.newton_atol >= 0 && (o.batch_mg == 0 || o.batch_mg == 1) &&
           (o.start_extrapolate == 0 || o.start_extrapolate == 1) && (o.krylov_adaptive == 0 || o.krylov_adaptive == 1) &&
           (o.dae_reorder == 0 || o.dae_reorder == 1) && (o.transform == 0 || o.transform == 1) &&
           (o.psi_solve == 0 || o.psi_solve == 1) && (o.lane_threads == 0 || o.lane_threads == 1);
}

static irk_status make_plan(int family, int s, const irk_operator *op, const irk_options *opt, Plan *P) {
    if (!op || s < 1 || s > IRK_MAX_STAGES) return IRK_E_ARG;
    if (family != IRK_GAUSS && family != IRK_RADAU_IIA && family != IRK_LOBATTO_IIIC && family != IRK_SDIRK)
        return IRK_E_ARG;
    P->op = *op;
    if (opt) P->opt = *opt; else irk_default_options(&P->opt);
    if (!valid_options(P->opt)) return IRK_E_ARG;
    const irk_operator &o = P->op;
    if (o.nx < 3 || o.ny < 1 || !(o.length > 0)) return IRK_E_ARG;
    if (o.kind == IRK_OP_BURGERS_1D) {
        if (o.ny != 1 || !(o.nu >= 0)) return IRK_E_ARG;
    } else if (o.kind == IRK_OP_NLDIFF_2D || o.kind == IRK_OP_VSF_2D) {
        if (o.ny != o.nx) return IRK_E_ARG;
        if (o.kind == IRK_OP_VSF_2D && !(o.nu >= 0)) return IRK_E_ARG;
        if (o.kind == IRK_OP_NLDIFF_2D && (o.forcing < 0 || o.forcing > 2)) return IRK_E_ARG;
    } else {
        return IRK_E_ARG;
    }
    const int s_sd = s;
    if (family == IRK_SDIRK) {
        long double A[IRK_MAX_STAGES * IRK_MAX_STAGES], b[IRK_MAX_STAGES], c[IRK_MAX_STAGES];
        if (!build_tableau_ld(family, s, A, b, c)) return IRK_E_ARG;
        P->sd_s = s;
        for (int i = 0; i < s * s; ++i) P->sd_A[i] = (double)A[i];
        for (int i = 0; i < s; ++i) { P->sd_b[i] = (double)b[i]; P->sd_c[i] = (double)c[i]; }
        build_sdirk_stage_block(P->sd_A[0], P->sd_c[0], &P->eb);
        s = 1;
    } else if (P->opt.transform == 1) {
        // the real Schur basis: blocks solved by back-substitution (ODE
        // operators; the DAE's constraint rows are not coupled this way)
        if (o.kind == IRK_OP_VSF_2D) return IRK_E_UNSUPPORTED;
        if (!build_schur_blocks(family, s, &P->eb)) return IRK_E_ARG;
    } else if (!build_eigen_blocks(family, s, &P->eb)) {
        return IRK_E_ARG;
    }
    if (family == IRK_SDIRK && P->opt.transform == 1) return IRK_E_UNSUPPORTED;
    for (int k = 0; k < P->eb.nblocks; ++k)
        if (!(P->eb.eta[k] > 0)) return IRK_E_UNSUPPORTED;     // Assumption 1
    P->family = family;
    P->s = s;
    P->nvar = (o.kind == IRK_OP_VSF_2D) ? 2 : 1;
    P->npts = (size_t)o.nx * o.ny;
    P->nf = P->nvar * P->npts;
    P->m = P->opt.restart;
    if (!level_geometry(o, P->opt.mg_coarsest, &P->lg)) return IRK_E_ARG;
    P->tsz = P->opt.prec_fp32 ? sizeof(float) : sizeof(double);
    // levels from l0 down run inside one work-group with everything in LDS
    // (at most 60 KiB of dynamic LDS -- the kernel's few KiB of static LDS
    // come on top of it --, 4096 points on its finest level and
    // IRK_MAX_SUB_LEVELS levels)
    P->l0 = P->lg.nlev - 1;
    {
        const int opk = o.kind == IRK_OP_NLDIFF_2D ? MG_NLDIFF : (o.kind == IRK_OP_BURGERS_1D ? MG_BURGERS : MG_VSF_OMEGA);
        for (int l = 0; l < P->lg.nlev; ++l) {
            const size_t top = (size_t)P->lg.nx[l] * P->lg.ny[l];
            const int nl = P->lg.nlev - l;
            if (top <= 4096 && nl <= IRK_MAX_SUB_LEVELS &&
                mg_subcycle_lds_bytes(opk, nl, P->lg.nx + l, P->lg.ny + l, P->tsz) <= 60 * 1024) {
                P->l0 = l;
                break;
            }
        }
    }
    // VSF streamfunction rows: the Poisson V-cycles stop at the first level
    // below the finest one of side <= IRK_FDM_MAX and a multiple of 4 (at or
    // above the sub-cycle's) and solve it exactly
    P->fdm_level = 0;
    // ... unless the finest grid is solved spectrally (a power-of-two side
    // the transforms take, option psi_solve = 0), in the V-cycle precision
    P->fft_tsz = (o.kind == IRK_OP_VSF_2D && P->opt.psi_solve == 0 && fft_poisson_supported(o.nx, P->tsz))
                     ? P->tsz : 0;
    P->fft_psi = P->fft_tsz > 0;
    static_assert(2 * 2048 <= IRK_RED_BLOCKS * 32, "the spectral solve's row sums use a lane's partials");
    static_assert(IRK_LANE_PARTIALS >= IRK_RED_BLOCKS * 32, "a lane's partials hold every reduction's");
    if (o.kind == IRK_OP_VSF_2D && !P->fft_psi)
        for (int l = 1; l <= P->l0 && l < P->lg.nlev; ++l)
            if (P->lg.nx[l] <= IRK_FDM_MAX && P->lg.nx[l] % 4 == 0 && P->lg.nx[l] == P->lg.ny[l]) {
                P->fdm_level = l;
                break;
            }

    // linearization of every transformed row (Section 3.2, written in the
    // eigenbasis with d_rq,k = (T^{-1})_rk T_kq): Newton-like (0) the last
    // stage, (1) the stage of the largest |d_rr,k|, each shared by the rows
    // that use it; (2) the weights d_rr of the row itself, (3) also the
    // weights d_rq coupling the two rows of a pair.  A 1-stage problem (and
    // every SDIRK stage) has a single weight 1: all four coincide.
    P->nhier = 0;
    std::memset(P->hier_w, 0, sizeof(P->hier_w));
    std::memset(P->blk_w, 0, sizeof(P->blk_w));
    P->weighted = P->opt.newton_like >= 2 && family != IRK_SDIRK && s > 1;
    if (P->weighted) {
        const double *T = P->eb.T, *Ti = P->eb.Tinv;
        for (int r = 0; r < s; ++r) {
            P->row_hier[r] = r;
            P->hier_stage[r] = P->eb.argmax_stage[r];
            for (int k = 0; k < s; ++k) P->hier_w[r][k] = Ti[r * s + k] * T[k * s + r];
        }
        P->nhier = s;
        for (int b = 0; b < P->eb.nblocks; ++b) {
            const int f = P->eb.first[b], w = P->eb.width[b];
            for (int a = 0; a < w; ++a)
                for (int q = 0; q < w; ++q)
                    if (P->opt.newton_like == 3 || a == q)
                        for (int k = 0; k < s; ++k) P->blk_w[b].w[a][q][k] = Ti[(f + a) * s + k] * T[k * s + f + q];
        }
    } else {
        for (int r = 0; r < s; ++r) {
            const int stage = P->opt.newton_like == 1 ? P->eb.argmax_stage[r] : s - 1;
            int hidx = -1;
            for (int q = 0; q < P->nhier; ++q)
                if (P->hier_stage[q] == stage) hidx = q;
            if (hidx < 0) { hidx = P->nhier++; P->hier_stage[hidx] = stage; }
            P->row_hier[r] = hidx;
        }
        for (int q = 0; q < P->nhier; ++q) P->hier_w[q][P->hier_stage[q]] = 1.0;
    }
    // back-substitution couplings of the real Schur basis: R0_ij M, and under
    // Newton-like (3) also -dt sum_k d_rq,k L(U_k) for rows r of block i and
    // columns q of block j (d_rq,k = (Q0^T)_rk (Q0)_kq; equation (Q0approx))
    std::memset(P->cpl, 0, sizeof(P->cpl));
    if (P->eb.schur) {
        const double *T = P->eb.T, *Ti = P->eb.Tinv;
        for (int i = 0; i < P->eb.nblocks; ++i)
            for (int j = i + 1; j < P->eb.nblocks; ++j) {
                BlockCouple &C = P->cpl[i][j];
                const int fi = P->eb.first[i], fj = P->eb.first[j];
                C.wi = P->eb.width[i];
                C.wj = P->eb.width[j];
                C.jac = P->opt.newton_like == 3 && s > 1;
                for (int a = 0; a < C.wi; ++a)
                    for (int q = 0; q < C.wj; ++q) {
                        C.R[a][q] = P->eb.R[(fi + a) * s + fj + q];
                        if (C.jac)
                            for (int k = 0; k < s; ++k) C.W.w[a][q][k] = Ti[(fi + a) * s + k] * T[k * s + fj + q];
                    }
            }
    }

    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes); return at; };
    const size_t f64 = sizeof(double);
    P->off_K = take(s * P->nf * f64);
    P->off_Y = take(s * P->nf * f64);
    P->off_Fh = take(s * P->nf * f64);
    P->off_U = take(s * P->nf * f64);
    // reduction partials: 512 work-groups x up to 32 values, or the fused
    // stage residual's 2 per tile
    P->off_part = take(std::max((size_t)IRK_RED_BLOCKS * 32, 2 * stage_residual_blocks(o.kind, o.nx, o.ny)) * f64);
    P->off_dv = take(512 * f64);
    // the fused stage residual writes the folded stages to a second buffer
    // (neighbouring tiles still read the first); the two swap roles
    P->off_K2 = (o.kind != IRK_OP_VSF_2D) ? take(s * P->nf * f64) : 0;
    P->off_tab = take((size_t)2 * (o.nx + o.ny) * f64);
    if (P->fdm_level > 0) {
        const size_t n = P->lg.nx[P->fdm_level];
        P->off_fdm_Q = take(n * n * P->tsz);
        P->off_fdm_lam = take(n * P->tsz);
    }
    const size_t spec_bytes = P->fft_psi ? fft_poisson_spectrum_values(o.nx) * P->fft_tsz : 0;
    if (P->fft_psi) {
        P->off_fft_tw = take((size_t)2 * o.nx * P->fft_tsz);  // n complex twiddles
        P->off_fft_lam = take((size_t)o.nx * P->fft_tsz);
    }
    for (int hq = 0; hq < P->nhier; ++hq)
        for (int l = 0; l < P->lg.nlev; ++l)
            P->off_coef[hq][l] = take((size_t)P->lg.nx[l] * P->lg.ny[l] * P->tsz);
    for (int b = 0; b < P->eb.nblocks; ++b) {
        LaneLayout &ln = P->lane[b];
        ln.ldv = (size_t)P->eb.width[b] * P->nf;
        ln.V = take((size_t)(P->m + 1) * ln.ldv * f64);
        ln.Z = take((size_t)P->m * ln.ldv * f64);
        ln.part = take((size_t)IRK_LANE_PARTIALS * f64);
        ln.dv = take(512 * f64);
        ln.tmp = (P->weighted && P->opt.newton_like == 3 && P->eb.width[b] == 2) ? take(P->nf * f64) : 0;
        ln.spec = spec_bytes ? take(spec_bytes) : 0;
        for (int l = 0; l < P->lg.nlev; ++l) {
            const size_t n = (size_t)P->lg.nx[l] * P->lg.ny[l];
            for (int q = 0; q < 4; ++q) ln.lev[l][q] = take(n * P->tsz);
        }
        AuxLayout &ax = P->aux[b];
        ax.used = o.kind == IRK_OP_VSF_2D && P->eb.width[b] == 2 && family != IRK_SDIRK;
        if (ax.used) {
            ax.lay.ldv = ln.ldv;
            ax.lay.part = take((size_t)IRK_RED_BLOCKS * 32 * f64);
            ax.lay.dv = take(512 * f64);
            ax.lay.spec = spec_bytes ? take(spec_bytes) : 0;
            for (int l = 0; l < P->lg.nlev; ++l) {
                const size_t n = (size_t)P->lg.nx[l] * P->lg.ny[l];
                for (int q = 0; q < 4; ++q) ax.lay.lev[l][q] = take(n * P->tsz);
            }
        }
    }
    if (family == IRK_SDIRK) {
        P->off_Ksd = take((size_t)s_sd * P->nf * f64);
        P->off_Uin = take(P->nf * f64);
        P->off_Uout = take(P->nf * f64);
    }
    P->total = off;
    return IRK_OK;
}

}  // namespace irk

using namespace irk;

// slots of the float64 device scalars (per lane, and for the Newton level)
enum {
    DV_RES = 0,        // ||F||^2
    DV_ABS = 1,        // squared norm of |terms of F| (rounding scale)
    DV_CAND = 2,       // Newton level: (||F||^2, |terms|^2) of the starting candidates (6)
    DV_BETA = 4,       // ||r0||^2 of a block solve
    DV_NRM = 5,        // ||w||^2 after orthogonalization (unfused path)
    DV_SUMS = 8,       // field sums (up to 16)
    DV_MEANS = 24,     // VSF stage means (2 s)
    DV_XMEANS = 40,    // VSF matvec input means (4)
    DV_H1 = 64,        // first Gram-Schmidt coefficients (<= 64)
    DV_H2 = 160,       // second pass (<= 64) and the norm
    DV_Y = 256,        // least-squares solution (<= 64)
    DV_GMAX = 480,     // Newton level, VSF: largest one-cell streamfunction difference per stage (s)
};
#define PIN_READ 0          // per-lane pinned staging: readbacks (the reductions write there too)
#define PIN_WRITE 512       // per-lane pinned staging: uploads
#define PIN_LANE 1024       // doubles of pinned staging per lane

struct Lane {
    int blk = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr, done = nullptr;
    hipEvent_t ev_prec = nullptr;       // lane work before a shared V-cycle batch
    double *V = nullptr, *Z = nullptr, *part = nullptr, *dv = nullptr;
    double *tmp = nullptr;              // the (2,1) coupling of Newton-like (3) pairs
    double *pin = nullptr;
    double *pin_dev = nullptr;          // pin as a device address
    size_t ldv = 0;
    const LaneLayout *lay = nullptr;
    // vorticity-streamfunction pairs: the side lane of the first
    // streamfunction row (fork after the first vorticity V-cycle, join before
    // the block operator reads z)
    Lane *aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

struct StepperBase;
struct LaneWorkers;

// Streams, events and pinned host staging a context runs on.  irk_create
// makes a private set; a server makes one per slot when it is created, so
// that admitting a request allocates nothing and waits for nothing.
struct CtxRes {
    int nlanes = 0;                                  // lanes with streams and events
    hipStream_t lane_st[IRK_MAX_STAGES] = {}, aux_st[IRK_MAX_STAGES] = {};
    hipEvent_t ev[IRK_MAX_STAGES] = {}, done[IRK_MAX_STAGES] = {}, prec[IRK_MAX_STAGES] = {};
    hipEvent_t fork[IRK_MAX_STAGES] = {}, join[IRK_MAX_STAGES] = {};
    hipEvent_t ev_main = nullptr, ev_res = nullptr, ev_coef = nullptr;
    double *pinned = nullptr;                        // readback/upload staging, then the upload area
    double *pinned_dev = nullptr;                    // pinned as a device address
    size_t upload = 0;                               // doubles of the upload area
};

struct irk_ctx {
    Plan P;
    hipStream_t stream = nullptr;        // the caller's stream (Newton level)
    unsigned char *ws = nullptr;
    double *K, *Y, *Fh, *U, *part, *dv, *tab;
    double *K2 = nullptr;                // second stage buffer of the fused stage residual
    DeviceProblem dp;
    double *pinned = nullptr;            // host staging: Newton level + lanes (res->pinned)
    double *pinned_dev = nullptr;        // the same as a device address
    CtxRes *res = nullptr;               // streams, events, pinned staging
    bool res_owned = false;              // made by irk_create (else a server slot's)
    hipEvent_t ev_main = nullptr;       // Newton level -> lanes
    hipEvent_t ev_res = nullptr;        // Newton-level readbacks
    hipEvent_t ev_coef = nullptr;       // the Newton iteration's coefficient hierarchies -> V-cycles
    StepperBase *stepper = nullptr;
    LaneWorkers *workers = nullptr;      // host threads of the eigen-block lanes (lane_threads)
    // V-cycle batching: a broker of the context's precision (PrecBroker<T>),
    // private (owned, batches this context's blocks) or a server's (shared)
    void *broker = nullptr;
    bool broker_owned = false;
    Lane lanes[IRK_MAX_STAGES];
    Lane aux_lanes[IRK_MAX_STAGES];
    int nlanes = 0;
    bool have_stages = false;
    bool have_U = false;                 // U holds the stage values of some K
    // the last successful step's output buffer and end time: a step from
    // there continues it, and K (still the previous stages) extrapolates
    const double *next_u = nullptr;
    double next_t = 0, prev_dt = 0;
    bool extrap = false;                  // this step has the third candidate
    double extrap_ratio = 1.0;            // dt / previous dt
    // Chebyshev smoothing coefficients
    double cheb_cd[8], cheb_cr[8];
    double lmax = 2.0, lmin = 0.5;
    irk_stats *st = nullptr;
    double dt = 0;
    // VSF: per hierarchy, a bound on the one-cell differences of the
    // streamfunction it linearizes at (valid for the current Newton
    // iteration's hierarchies); decides where vorticity V-cycles stop
    bool hier_g_valid = false;
    double hier_g[IRK_MAX_STAGES];
    // optional per-kernel timing with HIP events (irk_profile_enable)
    bool prof = false;
    std::vector<std::string> prof_names;
    std::vector<double> prof_ms, prof_bytes;
    std::vector<long> prof_launches;
    struct Rec { int id; double bytes; long n; hipEvent_t e0, e1; };
    std::vector<Rec> prof_pending;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_next = 0;
    // the most recent launches (at most 32, all on one stream) of every
    // kernel group, kept for back-to-back replay timing (irk_profile_replay)
    struct Replay { hipStream_t strm = nullptr; std::vector<std::function<void()>> f; std::vector<double> nbytes; };
    std::map<std::string, Replay> prof_rep;

    template <class T> T *lev(const Lane &ln, int l, int q) { return reinterpret_cast<T *>(ws + ln.lay->lev[l][q]); }
    template <class T> T *coef(int h, int l) { return reinterpret_cast<T *>(ws + P.off_coef[h][l]); }
};

static hipEvent_t prof_event(irk_ctx *c) {
    if (c->ev_next < c->ev_pool.size()) return c->ev_pool[c->ev_next++];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
    c->ev_next = c->ev_pool.size();
    return e;
}

static int prof_id(irk_ctx *c, const std::string &name) {
    for (size_t i = 0; i < c->prof_names.size(); ++i)
        if (c->prof_names[i] == name) return (int)i;
    c->prof_names.push_back(name);
    c->prof_ms.push_back(0.0);
    c->prof_bytes.push_back(0.0);
    c->prof_launches.push_back(0);
    return (int)c->prof_names.size() - 1;
}

// harvest the recorded event pairs (call after every stream has synchronized)
static void prof_harvest(irk_ctx *c) {
    for (auto &r : c->prof_pending) {
        float ms = 0.f;
        if (r.e0 && r.e1 && hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
            c->prof_ms[r.id] += ms;
            c->prof_bytes[r.id] += r.bytes;
            c->prof_launches[r.id] += r.n;
        }
    }
    c->prof_pending.clear();
    c->ev_next = 0;
}

// time one launch site on stream `st`: algorithmic bytes `bytes`, `n` launches
#define PROF(c, st, name, bytes, n, stmt)                                              \
    do {                                                                               \
        if ((c)->prof) {                                                               \
            hipEvent_t e0_ = prof_event(c);                                            \
            if (e0_) (void)hipEventRecord(e0_, (st));                                  \
            stmt;                                                                      \
            hipEvent_t e1_ = prof_event(c);                                            \
            if (e1_) (void)hipEventRecord(e1_, (st));                                  \
            (c)->prof_pending.push_back({prof_id(c, name), (double)(bytes), (long)(n), e0_, e1_}); \
            auto &rp_ = (c)->prof_rep[name];                                           \
            if (rp_.strm != (st)) { rp_.strm = (st); rp_.f.clear(); rp_.nbytes.clear(); }   \
            if (rp_.f.size() >= 32) { rp_.f.erase(rp_.f.begin()); rp_.nbytes.erase(rp_.nbytes.begin()); } \
            rp_.f.push_back([=]() { stmt; });                                          \
            rp_.nbytes.push_back((double)(bytes));                                      \
        } else {                                                                       \
            stmt;                                                                      \
        }                                                                              \
    } while (0)

template <class T> static const char *tname();
template <> const char *tname<float>() { return "float"; }
template <> const char *tname<double>() { return "double"; }
template <class T> static std::string kn(const char *base, int opk = -1) {
    std::string r = std::string(base) + "<" + tname<T>();
    if (opk >= 0) r += "," + std::to_string(opk);
    return r + ">";
}

#define HIP_TRY(x)                                   \
    do {                                             \
        if ((x) != hipSuccess) return IRK_E_DEVICE;  \
    } while (0)

// IRK_DEBUG=1 in the environment traces the Newton iterations on stderr, 2
// also every block solve.
static int debug_level() {
    static const int lvl = [] {
        const char *e = getenv("IRK_DEBUG");
        return e ? atoi(e) : 0;
    }();
    return lvl;
}

// asynchronous readback of a lane's device scalars; completion via ln.ev
static irk_status lane_readback(Lane &ln, int count) {
    HIP_TRY(hipMemcpyAsync(ln.pin + PIN_READ, ln.dv, sizeof(double) * count, hipMemcpyDeviceToHost, ln.stream));
    HIP_TRY(hipEventRecord(ln.ev, ln.stream));
    return IRK_OK;
}

// the same for scalars the reductions already wrote to the lane's pinned
// staging as well (their hout): only the event
static irk_status lane_mark(Lane &ln) {
    HIP_TRY(hipEventRecord(ln.ev, ln.stream));
    return IRK_OK;
}

// upload through the lane's pinned staging; the staging area is only reused
// after a later readback on the same lane has completed
static irk_status lane_write(Lane &ln, double *dev, const double *host, int count) {
    double *stage = ln.pin + PIN_WRITE;
    std::memcpy(stage, host, sizeof(double) * count);
    HIP_TRY(hipMemcpyAsync(dev, stage, sizeof(double) * count, hipMemcpyHostToDevice, ln.stream));
    return IRK_OK;
}

// ---------------------------------------------------------------------------
// One V-cycle on a lane's hierarchy: tiled down sweeps on levels 0..l0-1, the
// rest of the cycle inside one work-group, tiled up sweeps back to level 0.
// The finest level reads its right-hand side from float64 vectors (in) and
// writes the float64 result (out).  A V-cycle is first described as a job
// (all kernel arguments), then either launched on its lane's stream or
// batched with the V-cycles of other lanes (and of other contexts).
// ---------------------------------------------------------------------------
template <class T>
struct VcJob {
    int opk = 0, l0 = 0, deg = 3;
    // how the cycle's coarsest level l0 is solved: the one-work-group
    // sub-cycle (levels l0 and below), D Jacobi sweeps (a diagonally dominant
    // level operator), or exactly (periodic Poisson, fast diagonalization)
    enum Coarse { SUBCYCLE, JACOBI, FDM } coarse = SUBCYCLE;
    const T *fdm_Q = nullptr, *fdm_lam = nullptr, *fdm_b = nullptr;
    T *fdm_x = nullptr;
    double fdm_dt = 0;
    hipStream_t st = nullptr;
    MgLevelArgs<T> lev[IRK_MAX_LEVELS];
    MgSubArgs<T> sub;
    MgIn in;
    MgOut out;
    double by_down[IRK_MAX_LEVELS], by_up[IRK_MAX_LEVELS], by_sub = 0;   // algorithmic bytes
};

// Where a vorticity V-cycle may stop: the first level l >= 1 (above the
// sub-cycle's) whose operator A = sigma - dt (J_A(psi, .) + nu Lap) is
// diagonally dominant with Gershgorin ratio rho_l = sum_q |a_q| / a_c <= 1/4,
// so that D Jacobi sweeps there reduce its error by rho_l^D in the max norm.
// Bound: the advective coefficients of Arakawa's Jacobian are 12 differences
// of psi between points two cells apart (Manhattan) over 12 h^2, and a
// one-cell difference on level l is at most 2^l times the finest level's
// largest one, g (restriction averages with non-negative weights of sum 1):
// sum_q |a_q| <= dt (2 g / (h_0^2 2^l) + 4 nu / h_l^2),
// a_c = sigma + 4 dt nu / h_l^2.  Returns 0 (the full cycle) otherwise.
static int vorticity_coarsest(const irk_ctx *c, int opk, double sigma, double dt, int hier) {
    const Plan &P = c->P;
    if (opk != MG_VSF_OMEGA || hier < 0 || !c->hier_g_valid || c->broker || !(sigma > 0)) return 0;
    const double h0 = P.op.length / P.op.nx, g = c->hier_g[hier];
    for (int l = 1; l < P.l0; ++l) {
        const double hl = h0 * (double)(1 << l);
        const double visc = 4.0 * dt * P.op.nu / (hl * hl);
        const double adv = dt * 2.0 * g / (h0 * h0 * (double)(1 << l));
        if (visc + adv <= 0.25 * (sigma + visc)) return l;
    }
    return 0;
}

template <class T>
static void make_vcjob(irk_ctx *c, Lane &ln, int opk, double sigma, double dtop, int hier, const MgIn &in,
                       const MgOut &out, VcJob<T> *J) {
    const Plan &P = c->P;
    const int L = P.lg.nlev, deg = P.opt.cheb_degree;
    const double nu = P.op.nu;
    const double ts = sizeof(T);
    const int lc = vorticity_coarsest(c, opk, sigma, dtop, hier);
    const bool fdm = opk == MG_POISSON && P.fdm_level > 0;
    const int l0 = lc > 0 ? lc : (fdm ? P.fdm_level : P.l0);
    J->coarse = lc > 0 ? VcJob<T>::JACOBI : (fdm ? VcJob<T>::FDM : VcJob<T>::SUBCYCLE);
    J->opk = opk;
    J->l0 = l0;
    J->deg = deg;
    J->st = ln.stream;
    J->in = in;
    J->out = out;
    auto hl = [&](int l) { return P.op.length / P.op.nx * (double)(1 << l); };
    for (int l = 0; l < l0; ++l) {
        MgLevelArgs<T> &a = J->lev[l];
        a.nx = P.lg.nx[l];
        a.ny = P.lg.ny[l];
        a.h = (T)hl(l);
        a.nu = (T)nu;
        a.sigma = (T)sigma;
        a.dt = (T)dtop;
        a.coef = hier >= 0 ? c->coef<T>(hier, l) : nullptr;
        a.b = c->lev<T>(ln, l, 3);
        a.x = c->lev<T>(ln, l, 0);
        a.xout = c->lev<T>(ln, l, 1);
        a.bc = l + 1 < L ? c->lev<T>(ln, l + 1, 3) : nullptr;
        // the up sweep of level l+1 left its result in buffer 1; the
        // one-work-group sub-cycle leaves it in buffer 0
        a.xc = l + 1 < L ? c->lev<T>(ln, l + 1, l + 1 < l0 ? 1 : 0) : nullptr;
        for (int k = 0; k < IRK_MAX_CHEB; ++k) {
            a.cd[k] = (T)(k < deg ? c->cheb_cd[k] : 0.0);
            a.cr[k] = (T)(k < deg ? c->cheb_cr[k] : 0.0);
        }
        const double np = (double)a.nx * a.ny;
        // algorithmic bytes: the unfused per-level traffic of a 2-D V-cycle
        // (every field read or written once per sweep): a Chebyshev sweep
        // moves 6 fields, residual + full-weighting restriction 3.25,
        // prolongation + correction 2.25, so 12 deg + 5.5 fields per level
        // (41.5 at degree 3); the down launch carries the pre-smoothing and
        // the restriction, the up launch the rest.  The fused kernels move
        // far less (temporal blocking keeps iterates in registers and LDS).
        J->by_down[l] = np * ts * (6.0 * deg + 3.25);
        J->by_up[l] = np * ts * (6.0 * deg + 2.25);
    }
    if (J->coarse == VcJob<T>::FDM) {
        J->fdm_Q = reinterpret_cast<const T *>(c->ws + P.off_fdm_Q);
        J->fdm_lam = reinterpret_cast<const T *>(c->ws + P.off_fdm_lam);
        J->fdm_b = c->lev<T>(ln, l0, 3);
        J->fdm_x = c->lev<T>(ln, l0, 0);
        J->fdm_dt = dtop;
        const double n = P.lg.nx[l0];
        J->by_sub = (3.0 * n * n + n) * ts;            // reads b, Q, lam; writes x
        return;
    }
    if (J->coarse == VcJob<T>::JACOBI) {
        // the coarsest level: D Jacobi sweeps from zero (the down kernel
        // without its residual and restriction), result in buffer 0
        MgLevelArgs<T> &a = J->lev[l0];
        a.nx = P.lg.nx[l0];
        a.ny = P.lg.ny[l0];
        a.h = (T)hl(l0);
        a.nu = (T)nu;
        a.sigma = (T)sigma;
        a.dt = (T)dtop;
        a.coef = c->coef<T>(hier, l0);
        a.b = c->lev<T>(ln, l0, 3);
        a.x = c->lev<T>(ln, l0, 0);
        a.xout = nullptr;
        a.bc = nullptr;
        a.xc = nullptr;
        for (int k = 0; k < IRK_MAX_CHEB; ++k) {
            a.cd[k] = T(0);
            a.cr[k] = (T)(k < deg ? 1.0 : 0.0);
        }
        J->by_down[l0] = (double)a.nx * a.ny * ts * 6.0 * deg;
        J->by_sub = 0;
        return;
    }
    MgSubArgs<T> &sa = J->sub;
    sa.nlev = L - l0;
    double np_all = 0;
    for (int q = 0; q < sa.nlev; ++q) {
        sa.nx[q] = P.lg.nx[l0 + q];
        sa.ny[q] = P.lg.ny[l0 + q];
        sa.h[q] = (T)hl(l0 + q);
        sa.coef[q] = hier >= 0 ? c->coef<T>(hier, l0 + q) : nullptr;
        np_all += (double)sa.nx[q] * sa.ny[q];
    }
    sa.nu = (T)nu;
    sa.sigma = (T)sigma;
    sa.dt = (T)dtop;
    sa.b0 = c->lev<T>(ln, l0, 3);
    sa.x0 = c->lev<T>(ln, l0, 0);
    sa.deg = deg;
    sa.coarse_iters = P.opt.coarse_iters;
    sa.wave_pts = IRK_SUB_WAVE_PTS;
    for (int k = 0; k < IRK_MAX_CHEB; ++k) {
        sa.cd[k] = (T)(k < deg ? c->cheb_cd[k] : 0.0);
        sa.cr[k] = (T)(k < deg ? c->cheb_cr[k] : 0.0);
    }
    J->by_sub = np_all * ts * (12.0 * deg + 5.5);
}

// one job, launched on its lane's stream
template <class T>
static void run_vcjob(irk_ctx *c, const VcJob<T> &J) {
    const int l0 = J.l0, opk = J.opk, deg = J.deg;
    hipStream_t st = J.st;
    for (int l = 0; l < l0; ++l) {
        const MgLevelArgs<T> a = J.lev[l];
        const MgIn in = l == 0 ? J.in : MgIn{};
        PROF(c, st, kn<T>("k_mg_down", opk), J.by_down[l], 1, launch_mg_down<T>(st, opk, a, in, deg));
    }
    if (J.coarse == VcJob<T>::JACOBI) {
        const MgLevelArgs<T> a = J.lev[l0];
        PROF(c, st, kn<T>("k_mg_down", opk), J.by_down[l0], 1, launch_mg_down<T>(st, opk, a, MgIn{}, deg));
    } else if (J.coarse == VcJob<T>::FDM) {
        const int n = c->P.lg.nx[l0];
        PROF(c, st, kn<T>("k_poisson_fdm"), J.by_sub, 1,
             launch_poisson_fdm<T>(st, n, (T)J.fdm_dt, J.fdm_Q, J.fdm_lam, J.fdm_b, J.fdm_x));
    } else {
        const MgSubArgs<T> sa = J.sub;
        const MgIn in = l0 == 0 ? J.in : MgIn{};
        const MgOut out = l0 == 0 ? J.out : MgOut{};
        PROF(c, st, kn<T>("k_mg_subcycle", opk), J.by_sub, 1, launch_mg_subcycle<T>(st, opk, sa, in, out));
    }
    for (int l = l0 - 1; l >= 0; --l) {
        const MgLevelArgs<T> a = J.lev[l];
        const MgOut out = l == 0 ? J.out : MgOut{};
        PROF(c, st, kn<T>("k_mg_up", opk), J.by_up[l], 1, launch_mg_up<T>(st, opk, a, out, deg));
    }
}

// several independent jobs of one operator and degree, one launch per
// V-cycle phase on stream st: down sweeps by depth from the finest level,
// all sub-cycles (one work-group each), up sweeps by depth back to the finest
template <class T>
static void run_vcjobs_batched(irk_ctx *c, hipStream_t st, const std::vector<const VcJob<T> *> &jobs) {
    if (jobs.empty()) return;
    const int opk = jobs[0]->opk, deg = jobs[0]->deg;
    int maxl0 = 0;
    for (auto *J : jobs) maxl0 = std::max(maxl0, J->l0);
    std::vector<MgLevelArgs<T>> g;
    std::vector<MgIn> ins;
    std::vector<MgOut> outs;
    std::vector<MgSubArgs<T>> subs;
    for (int d = 0; d < maxl0; ++d) {
        g.clear();
        ins.clear();
        double by = 0;
        for (auto *J : jobs)
            if (J->l0 > d) {
                g.push_back(J->lev[d]);
                ins.push_back(d == 0 ? J->in : MgIn{});
                by += J->by_down[d];
            }
        const int n = (int)g.size();
        PROF(c, st, kn<T>("k_mg_down", opk), by, 1,
             launch_mg_down_batch<T>(st, opk, g.data(), ins.data(), n, deg));
    }
    {
        subs.clear();
        ins.clear();
        outs.clear();
        double by = 0;
        for (auto *J : jobs) {
            subs.push_back(J->sub);
            ins.push_back(J->l0 == 0 ? J->in : MgIn{});
            outs.push_back(J->l0 == 0 ? J->out : MgOut{});
            by += J->by_sub;
        }
        const int n = (int)subs.size();
        PROF(c, st, kn<T>("k_mg_subcycle", opk), by, 1,
             launch_mg_subcycle_batch<T>(st, opk, subs.data(), ins.data(), outs.data(), n));
    }
    for (int d = maxl0 - 1; d >= 0; --d) {
        g.clear();
        outs.clear();
        double by = 0;
        for (auto *J : jobs)
            if (J->l0 > d) {
                g.push_back(J->lev[d]);
                outs.push_back(d == 0 ? J->out : MgOut{});
                by += J->by_up[d];
            }
        const int n = (int)g.size();
        PROF(c, st, kn<T>("k_mg_up", opk), by, 1, launch_mg_up_batch<T>(st, opk, g.data(), outs.data(), n, deg));
    }
}

template <class T>
static void vcycle(irk_ctx *c, Lane &ln, int opk, double sigma, double dtop, int hier, const MgIn &in,
                   const MgOut &out) {
    VcJob<T> J;
    make_vcjob<T>(c, ln, opk, sigma, dtop, hier, in, out, &J);
    run_vcjob<T>(c, J);
}

static BlockLam block_lam(const EigenBlocks &eb, int blk) {
    BlockLam l;
    l.eta = eb.eta[blk];
    l.c12 = eb.c12[blk];
    l.c21 = eb.c21[blk];
    return l;
}

static int mg_op_of(int kind) {
    return kind == IRK_OP_NLDIFF_2D ? MG_NLDIFF : (kind == IRK_OP_BURGERS_1D ? MG_BURGERS : MG_VSF_OMEGA);
}

// z = (sigma M - dt L_hier)^{-1} (a1 v1 + a2 v2), one V-cycle, for the
// differential variable.
template <class T>
static void prec_component(irk_ctx *c, Lane &ln, double *z, const double *v1, double a1, const double *v2,
                           double a2, double sigma, int hier) {
    MgIn in;
    in.v1 = v1; in.a1 = a1; in.v2 = v2; in.a2 = a2;
    MgOut out;
    out.z = z; out.v1 = v1; out.a1 = a1; out.v2 = v2; out.a2 = a2;
    vcycle<T>(c, ln, mg_op_of(c->P.op.kind), sigma, c->dt, hier, in, out);
}

// VSF streamfunction row of a block: solve B psi = q, B = -dt (Lap - mean),
// q = r_psi + dt (z_omega - mean z_omega).  The mean-free part comes from
// the spectral solve or one Poisson V-cycle on -dt Lap, the mean exactly:
// mean(psi) = mean(r_psi)/dt.  The spectral solve reduces the means itself
// and, with xm, also hands the block matvec the means of its input
// (xm[0] = mean z_omega, xm[1] = mean psi).
template <class T>
static void prec_psi(irk_ctx *c, Lane &ln, double *zpsi, const double *rpsi, const double *zomega,
                     double *xm = nullptr) {
    const size_t npts = c->P.npts;
    double *means = ln.dv + DV_SUMS;            // [0] mean r_psi, [1] mean z_omega
    if (c->P.fft_psi) {
        // exact: the spectral solve on the finest grid.  Bytes: q's two
        // float64 inputs and z (24 per point), the half spectrum written,
        // read, written and read again (4 n (n/2 + 1) complex values)
        const int n = c->P.op.nx;
        const size_t fs = c->P.fft_tsz;
        const double by = 24.0 * npts + 4.0 * fft_poisson_spectrum_values(n) * fs;
        FftPoissonArgs a;
        a.v1 = rpsi; a.a1 = 1.0; a.v2 = zomega; a.a2 = c->dt;
        a.z = zpsi; a.shift_scale = 1.0 / c->dt;
        a.sums = ln.part; a.means = means; a.zmeans = xm;
        unsigned char *ws = c->ws;
        if (fs == sizeof(double)) {
            PROF(c, ln.stream, "k_fft_poisson<double>", by, 1,
                 launch_fft_poisson<double>(ln.stream, n, c->dt, reinterpret_cast<const double *>(ws + c->P.off_fft_tw),
                                            reinterpret_cast<const double *>(ws + c->P.off_fft_lam), a,
                                            reinterpret_cast<double *>(ws + ln.lay->spec)));
        } else {
            PROF(c, ln.stream, "k_fft_poisson<float>", by, 1,
                 launch_fft_poisson<float>(ln.stream, n, (float)c->dt,
                                           reinterpret_cast<const float *>(ws + c->P.off_fft_tw),
                                           reinterpret_cast<const float *>(ws + c->P.off_fft_lam), a,
                                           reinterpret_cast<float *>(ws + ln.lay->spec)));
        }
        return;
    }
    PROF(c, ln.stream, "k_field_sums2", 16.0 * npts, 1,
         launch_field_sums2(ln.stream, rpsi, zomega, npts, 1.0 / npts, ln.part, means));
    MgIn in;
    in.v1 = rpsi; in.a1 = 1.0; in.v2 = zomega; in.a2 = c->dt; in.mean = means;
    MgOut out;
    out.z = zpsi; out.shift = means; out.shift_scale = 1.0 / c->dt;
    out.v1 = rpsi; out.a1 = 1.0; out.v2 = zomega; out.a2 = c->dt; out.mean_in = means;
    vcycle<T>(c, ln, MG_POISSON, 0.0, c->dt, -1, in, out);
}

// z = L_P^{-1} v for the lane's eigen-block: the block lower-triangular
// preconditioner of equation (Lprec) with diagonal inverses (eta M - dt L_a)
// and the Schur complement approximation (gamma M - dt L_b) of equation
// (schur-approx), each applied as one V-cycle; the (2,1) block of D is
// -beta M (phi = beta in the eigenbasis), and with Newton-like (3) also
// -dt sum_k d_21,k L_k.  Returns the number of V-cycles.
template <class T>
static int apply_prec(irk_ctx *c, Lane &ln, const double *v, double *z) {
    const Plan &P = c->P;
    const EigenBlocks &eb = P.eb;
    const int blk = ln.blk;
    const int r = eb.first[blk];
    const size_t nf = P.nf, npts = P.npts;
    const double eta = eb.eta[blk];
    const bool vsf = (P.op.kind == IRK_OP_VSF_2D);
    const int ha = P.row_hier[r];
    int nvc = 0;
    prec_component<T>(c, ln, z, v, 1.0, nullptr, 0.0, eta, ha);
    ++nvc;
    // the first streamfunction row needs z1 only; with a side lane it runs
    // there while the second row's vorticity V-cycle runs here
    const bool fork = vsf && ln.aux && eb.width[blk] == 2;
    if (fork) {
        (void)hipEventRecord(ln.ev_fork, ln.stream);
        (void)hipStreamWaitEvent(ln.aux->stream, ln.ev_fork, 0);
        prec_psi<T>(c, *ln.aux, z + npts, v + npts, z, ln.dv + DV_XMEANS);
        ++nvc;
    } else if (vsf) {
        prec_psi<T>(c, ln, z + npts, v + npts, z, ln.dv + DV_XMEANS);
        ++nvc;
    }
    if (eb.width[blk] == 2) {
        const double gam = P.opt.gamma_mode == 0 ? eb.gamma_star[blk] : eta;
        const int hb = P.row_hier[r + 1];
        if (ln.tmp) {
            // Newton-like (3): the (2,1) block of D is c21 M - dt sum_k
            // d_21,k L_k; its negation applied to z1 joins the right-hand side
            PROF(c, ln.stream, "k_block_matvec_w<" + std::to_string(P.op.kind) + ">",
                 8.0 * P.npts * (2.0 + P.s * P.nvar), 1,
                 launch_block_matvec_w(ln.stream, c->dp, P.s, 1, block_lam(eb, blk), c->dt, c->U, P.blk_w[blk], z,
                                       ln.tmp, nullptr, 1));
            prec_component<T>(c, ln, z + nf, v + nf, 1.0, ln.tmp, 1.0, gam, hb);
        } else {
            // the (2,1) block c21 M (eigenbasis: -beta M) moved to the right
            prec_component<T>(c, ln, z + nf, v + nf, 1.0, z, -eb.c21[blk], gam, hb);
        }
        ++nvc;
        if (vsf) { prec_psi<T>(c, ln, z + nf + npts, v + nf + npts, z + nf, ln.dv + DV_XMEANS + 2); ++nvc; }
    }
    if (fork) {
        (void)hipEventRecord(ln.ev_join, ln.aux->stream);
        (void)hipStreamWaitEvent(ln.stream, ln.ev_join, 0);
    }
    return nvc;
}

static const double *stage_field(irk_ctx *c, int stage) { return c->U + (size_t)stage * c->P.nf; }

// Zero one variable (0: omega, 1: psi) of every component of a VSF block
// vector ([width][omega, psi][npts]).
static void zero_var(irk_ctx *c, Lane &ln, double *x, int var) {
    const Plan &P = c->P;
    for (int comp = 0; comp < P.eb.width[ln.blk]; ++comp)
        PROF(c, ln.stream, "k_fill_f64", 8.0 * P.npts, 1,
             launch_fill(ln.stream, x + comp * P.nf + var * P.npts, 0.0, P.npts));
}

// Preconditioners of the two solves of the reordered DAE block system (eq
// (vsf-system-2), the forward substitution): mode 1, the vorticity system
// alone -- the block-triangular L_P on the omega components, psi parts
// zero; mode 2, the streamfunction rows alone -- one Poisson V-cycle per
// component with the vorticity parts zero.  Returns the V-cycles used.
template <class T>
static int apply_prec_mode(irk_ctx *c, Lane &ln, const double *v, double *z, int mode) {
    if (mode == 0) return apply_prec<T>(c, ln, v, z);
    const Plan &P = c->P;
    const EigenBlocks &eb = P.eb;
    const int blk = ln.blk, r = eb.first[blk], width = eb.width[blk];
    const size_t nf = P.nf, npts = P.npts;
    int nvc = 0;
    if (mode == 1) {
        prec_component<T>(c, ln, z, v, 1.0, nullptr, 0.0, eb.eta[blk], P.row_hier[r]);
        ++nvc;
        if (width == 2) {
            const double gam = P.opt.gamma_mode == 0 ? eb.gamma_star[blk] : eb.eta[blk];
            if (ln.tmp) {
                PROF(c, ln.stream, "k_block_matvec_w<" + std::to_string(P.op.kind) + ">",
                     8.0 * npts * (2.0 + P.s * P.nvar), 1,
                     launch_block_matvec_w(ln.stream, c->dp, P.s, 1, block_lam(eb, blk), c->dt, c->U, P.blk_w[blk],
                                           z, ln.tmp, nullptr, 1));
                prec_component<T>(c, ln, z + nf, v + nf, 1.0, ln.tmp, 1.0, gam, P.row_hier[r + 1]);
            } else {
                prec_component<T>(c, ln, z + nf, v + nf, 1.0, z, -eb.c21[blk], gam, P.row_hier[r + 1]);
            }
            ++nvc;
        }
        zero_var(c, ln, z, 1);
    } else {
        zero_var(c, ln, z, 0);
        for (int comp = 0; comp < width; ++comp) {
            prec_psi<T>(c, ln, z + comp * nf + npts, v + comp * nf + npts, z + comp * nf,
                        ln.dv + DV_XMEANS + 2 * comp);
            ++nvc;
        }
    }
    return nvc;
}

// w = D_b x for the lane's block.  The DAE's constraint rows need the means
// of x: xm_ready says the spectral streamfunction solves that produced x
// (the preconditioner's output, both its variables) already left them.
static void block_matvec(irk_ctx *c, Lane &ln, const double *x, double *w, bool xm_ready = false) {
    const Plan &P = c->P;
    const EigenBlocks &eb = P.eb;
    const int blk = ln.blk;
    const int r = eb.first[blk];
    const int width = eb.width[blk];
    const double *Ua = stage_field(c, P.hier_stage[P.row_hier[r]]);
    const double *Ub = width == 2 ? stage_field(c, P.hier_stage[P.row_hier[r + 1]]) : Ua;
    const double *xm = nullptr;
    if (P.op.kind == IRK_OP_VSF_2D) {
        if (!(xm_ready && P.fft_psi))
            PROF(c, ln.stream, "k_field_sums", 8.0 * 2 * width * P.npts, 1,
                 launch_field_sums(ln.stream, x, P.npts, 2 * width, P.npts, 1.0 / P.npts, ln.part,
                                   ln.dv + DV_XMEANS, nullptr));
        xm = ln.dv + DV_XMEANS;
    }
    if (P.weighted) {
        // reads x, w (width * nvar fields each) and the s stage fields
        const double byw = 8.0 * P.npts * (2.0 * width * P.nvar + P.s * P.nvar);
        PROF(c, ln.stream, "k_block_matvec_w<" + std::to_string(P.op.kind) + ">", byw, 1,
             launch_block_matvec_w(ln.stream, c->dp, P.s, width, block_lam(eb, blk), c->dt, c->U, P.blk_w[blk], x,
                                   w, xm, 0));
        return;
    }
    // reads x and writes w (width * nvar fields each), reads one linearization field per component
    const double by = 8.0 * P.npts * width * (2.0 * P.nvar + 1.0);
    PROF(c, ln.stream, "k_block_matvec<" + std::to_string(P.op.kind) + ">", by, 1,
         launch_block_matvec(ln.stream, c->dp, width, block_lam(eb, blk), c->dt, Ua, Ub, x, w, xm));
}

// The plain block matvec fused with the first Gram-Schmidt pass,
// out[k] = (V_k, w) for the nv basis vectors at V (stride ldv); false
// (nothing issued) where it does not apply: the stage-weighted operators of
// Newton-like (2), (3), more than 16 basis vectors, or the DAE (its 9-point
// matvec ran slower fused: the reduction grid of 512 work-groups leaves too
// few waves to hide the stencil's latency).
static bool block_matvec_dot(irk_ctx *c, Lane &ln, const double *x, double *w, const double *V, size_t ldv, int nv,
                             double *out, double *hout) {
    const Plan &P = c->P;
    if (P.weighted || nv < 1 || nv > 16 || P.op.kind == IRK_OP_VSF_2D) return false;
    const EigenBlocks &eb = P.eb;
    const int blk = ln.blk;
    const int r = eb.first[blk];
    const int width = eb.width[blk];
    const double *Ua = stage_field(c, P.hier_stage[P.row_hier[r]]);
    const double *Ub = width == 2 ? stage_field(c, P.hier_stage[P.row_hier[r + 1]]) : Ua;
    const double *xm = nullptr;
    if (P.op.kind == IRK_OP_VSF_2D) {
        PROF(c, ln.stream, "k_field_sums", 8.0 * 2 * width * P.npts, 1,
             launch_field_sums(ln.stream, x, P.npts, 2 * width, P.npts, 1.0 / P.npts, ln.part, ln.dv + DV_XMEANS,
                               nullptr));
        xm = ln.dv + DV_XMEANS;
    }
    // reads x and writes w (width * nvar fields each), one linearization
    // field per component, and the nv basis vectors
    const double len = (double)width * P.nf;
    const double by = 8.0 * P.npts * width * (2.0 * P.nvar + 1.0) + 8.0 * len * nv;
    PROF(c, ln.stream, "k_block_matvec_dot<" + std::to_string(P.op.kind) + ">", by, 1,
         (void)launch_block_matvec_dot(ln.stream, c->dp, width, block_lam(eb, blk), c->dt, Ua, Ub, x, w, xm, V,
                                       ldv, nv, ln.part, out, hout));
    return true;
}

// ---------------------------------------------------------------------------
// Right-preconditioned FGMRES(m) on D_b y = fhat_b (y in the block's rows of
// Y), classical Gram-Schmidt with reorthogonalization, Givens QR of the
// Hessenberg matrix on the host.  Written as a state machine driven by the
// lane's readbacks so that several lanes can be interleaved.
// ---------------------------------------------------------------------------
template <class T>
struct Fgmres;

// V-cycles of lanes that wait for their preconditioner at the same time
// (the blocks of one step, or the blocks of many requests in a server),
// run as shared launches on the broker's stream; flush() orders them after
// each lane's preceding work, runs the first (and, for 2x2 blocks, second)
// diagonal V-cycles of all of them, and resumes every lane.
template <class T>
struct PrecBroker {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr, done1 = nullptr;     // after both passes; after the first
    std::vector<Fgmres<T> *> pending;
    bool init() {
        return hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
               hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess &&
               hipEventCreateWithFlags(&done1, hipEventDisableTiming) == hipSuccess;
    }
    ~PrecBroker() {
        if (st) (void)hipStreamSynchronize(st);
        if (done) (void)hipEventDestroy(done);
        if (done1) (void)hipEventDestroy(done1);
        if (st) (void)hipStreamDestroy(st);
    }
    void forget(const irk_ctx *c);
    int flush();            // number of lanes resumed
};

template <class T>
struct Fgmres {
    irk_ctx *c = nullptr;
    Lane *ln = nullptr;
    int m = 30, maxit = 200;
    double rtol = 1e-5;
    const double *rhs = nullptr;
    double *sol = nullptr;
    size_t len = 0;
    std::vector<double> H, cs, sn, g, y;
    int j = 0, total = 0, vcycles = 0;
    int omega_total = 0;                // reordered DAE system: iterations of the vorticity solve
    bool first_cycle = true, converged = false, fused = true;
    double beta0 = 0.0;
    enum Phase { WAIT_BETA, WAIT_PREC, WAIT_ITER, DONE } phase = WAIT_BETA;
    // 0: the whole block system; reordered DAE system (eq (vsf-system-2)):
    // 1 the vorticity rows, then 2 the streamfunction rows, the second
    // solve starting from the first's solution (sol keeps accumulating)
    int mode = 0;
    bool beta0_set = false;
    double *pend_v = nullptr, *pend_z = nullptr;    // preconditioner input/output waiting in a broker
    hipEvent_t prec_wait = nullptr;                  // waited on before the first preconditioner application
    irk_status deferred = IRK_OK;                    // error raised while resumed by a broker

    void init(irk_ctx *cc, Lane *l, double rt, int mx) {
        c = cc;
        ln = l;
        const Plan &P = c->P;
        const int r = P.eb.first[ln->blk];
        m = P.m;
        maxit = mx;
        rtol = rt;
        len = (size_t)P.eb.width[ln->blk] * P.nf;
        rhs = c->Fh + (size_t)r * P.nf;
        sol = c->Y + (size_t)r * P.nf;
        H.assign((size_t)(m + 1) * m, 0.0);
        cs.assign(m, 0.0);
        sn.assign(m, 0.0);
        g.assign(m + 1, 0.0);
        y.assign(m, 0.0);
        j = total = vcycles = 0;
        first_cycle = true;
        converged = false;
        beta0 = 0.0;
        beta0_set = false;
        mode = (P.op.kind == IRK_OP_VSF_2D && P.opt.dae_reorder) ? 1 : 0;
        prec_wait = nullptr;
    }

    // after the vorticity solve of the reordered system: the streamfunction
    // rows, from the current sol
    irk_status to_psi() {
        mode = 2;
        omega_total = total;
        first_cycle = false;
        converged = false;
        beta0_set = false;
        j = 0;
        return start();
    }

    // the block operator of the current solve
    void op(const double *x, double *w) {
        block_matvec(c, *ln, x, w, mode != 1);
        if (mode == 1) zero_var(c, *ln, w, 1);
    }

    double *Vv(int k) { return ln->V + (size_t)k * ln->ldv; }
    double *Zv(int k) { return ln->Z + (size_t)k * ln->ldv; }

    // device address of the lane's readback value k (the reductions write
    // there as well as to dv + k)
    double *hb_dev(int k) { return ln->pin_dev + PIN_READ + k; }

    // issue ||r0||^2 (r0 = rhs on the first cycle, rhs - D sol on restarts)
    irk_status start() {
        if (first_cycle && mode == 1) {
            // the vorticity rows of rhs
            if (hipMemcpyAsync(Vv(0), rhs, len * sizeof(double), hipMemcpyDeviceToDevice, ln->stream) != hipSuccess)
                return IRK_E_DEVICE;
            zero_var(c, *ln, Vv(0), 1);
            PROF(c, ln->stream, "k_dot_multi", 8.0 * len, 1,
                 launch_dot_multi(ln->stream, Vv(0), ln->ldv, 0, Vv(0), len, 1, ln->part, ln->dv + DV_BETA,
                                  hb_dev(DV_BETA)));
        } else if (first_cycle) {
            PROF(c, ln->stream, "k_dot_multi", 8.0 * len, 1,
                 launch_dot_multi(ln->stream, Vv(0), ln->ldv, 0, rhs, len, 1, ln->part, ln->dv + DV_BETA, hb_dev(DV_BETA)));
        } else {
            block_matvec(c, *ln, sol, Vv(0));
            PROF(c, ln->stream, "k_axpby", 24.0 * len, 1, launch_axpby(ln->stream, Vv(0), 1.0, rhs, -1.0, Vv(0), len));
            if (mode) zero_var(c, *ln, Vv(0), mode == 1 ? 1 : 0);
            PROF(c, ln->stream, "k_dot_multi", 8.0 * len, 1,
                 launch_dot_multi(ln->stream, Vv(0), ln->ldv, 0, Vv(0), len, 1, ln->part, ln->dv + DV_BETA,
                                  hb_dev(DV_BETA)));
        }
        phase = WAIT_BETA;
        return lane_mark(*ln);
    }

    // one Arnoldi iteration: preconditioner, matvec, CGS2; readback of h.
    // With a broker the preconditioner waits for a shared V-cycle batch.
    irk_status issue_iteration() {
        double *vj = Vv(j), *zj = Zv(j);
        if (prec_wait) {
            // the V-cycles read the coefficient hierarchies, which the Newton
            // level builds while the solve's first sweeps run
            if (hipStreamWaitEvent(ln->stream, prec_wait, 0) != hipSuccess) return IRK_E_DEVICE;
            prec_wait = nullptr;
        }
        if (c->broker && c->P.op.kind != IRK_OP_VSF_2D) {
            pend_v = vj;
            pend_z = zj;
            phase = WAIT_PREC;
            static_cast<PrecBroker<T> *>(c->broker)->pending.push_back(this);
            return IRK_OK;
        }
        vcycles += apply_prec_mode<T>(c, *ln, vj, zj, mode);
        return issue_after_prec();
    }

    // the broker's jobs for this lane: pass 1 the first diagonal V-cycle,
    // pass 2 (2x2 blocks) the second, which reads the first's output
    void prec_jobs(int pass, std::vector<VcJob<T>> &jobs) {
        const Plan &P = c->P;
        const EigenBlocks &eb = P.eb;
        const int blk = ln->blk, r = eb.first[blk];
        const size_t nf = P.nf;
        const int opk = mg_op_of(P.op.kind);
        MgIn in;
        MgOut out;
        if (pass == 1) {
            in.v1 = pend_v; in.a1 = 1.0;
            out.z = pend_z; out.v1 = pend_v; out.a1 = 1.0;
            jobs.emplace_back();
            make_vcjob<T>(c, *ln, opk, eb.eta[blk], c->dt, P.row_hier[r], in, out, &jobs.back());
        } else if (eb.width[blk] == 2) {
            const double gam = P.opt.gamma_mode == 0 ? eb.gamma_star[blk] : eb.eta[blk];
            in.v1 = pend_v + nf; in.a1 = 1.0; in.v2 = pend_z; in.a2 = -eb.c21[blk];
            out.z = pend_z + nf; out.v1 = pend_v + nf; out.a1 = 1.0; out.v2 = pend_z; out.a2 = -eb.c21[blk];
            jobs.emplace_back();
            make_vcjob<T>(c, *ln, opk, gam, c->dt, P.row_hier[r + 1], in, out, &jobs.back());
        }
    }

    // continue after the broker ran this lane's V-cycles
    void resume() {
        vcycles += c->P.eb.width[ln->blk];
        const irk_status e = issue_after_prec();
        if (e != IRK_OK) deferred = e;
    }

    irk_status issue_after_prec() {
        double *zj = Zv(j), *w = Vv(j + 1);
        const int nv = j + 1;
        fused = nv <= 16;
        hipStream_t st = ln->stream;
        double *dv = ln->dv;
        // the matvec, with h1 = V^T w in the same sweep where it applies (the
        // vorticity solve of the reordered system zeroes part of w after the
        // matvec, so there the projection stays a pass of its own)
        const bool with_h1 =
            fused && mode != 1 && block_matvec_dot(c, *ln, zj, w, Vv(0), ln->ldv, nv, dv + DV_H1, hb_dev(DV_H1));
        if (!with_h1) op(zj, w);
        if (fused) {
            // classical Gram-Schmidt twice in three sweeps: h1 = V^T w;
            // w -= V h1 with h2 = V^T w and ||w||^2 in the same sweep;
            // w = (w - V h2) / ||.||.  The coefficients reach the host
            // through the pinned staging as they are reduced, so the event
            // goes in before the last sweep: the host works out the next
            // step while it runs.
            if (!with_h1)
                PROF(c, st, "k_dot_multi", 8.0 * len * (nv + 1), 1,
                     launch_dot_multi(st, Vv(0), ln->ldv, nv, w, len, 0, ln->part, dv + DV_H1, hb_dev(DV_H1)));
            PROF(c, st, "k_axpy_dot", 8.0 * len * (nv + 2), 1,
                 launch_axpy_dot(st, w, Vv(0), ln->ldv, nv, dv + DV_H1, len, ln->part, dv + DV_H2, hb_dev(DV_H2)));
            phase = WAIT_ITER;
            if (lane_mark(*ln) != IRK_OK) return IRK_E_DEVICE;
            PROF(c, st, "k_axpy_scale", 8.0 * len * (nv + 2), 1,
                 launch_axpy_scale(st, w, Vv(0), ln->ldv, nv, dv + DV_H2, dv + DV_H2 + nv, len));
            return IRK_OK;
        } else {
            const int nch = (nv + 15) / 16;   // dot launches (16 basis vectors each)
            PROF(c, st, "k_dot_multi", 8.0 * len * (nv + nch), nch,
                 launch_dot_multi(st, Vv(0), ln->ldv, nv, w, len, 0, ln->part, dv + DV_H1, nullptr));
            PROF(c, st, "k_axpy_multi", 8.0 * len * (nv + 2), 1,
                 launch_axpy_multi(st, w, Vv(0), ln->ldv, nv, dv + DV_H1, len));
            PROF(c, st, "k_dot_multi", 8.0 * len * (nv + nch), nch,
                 launch_dot_multi(st, Vv(0), ln->ldv, nv, w, len, 0, ln->part, dv + DV_H2, nullptr));
            PROF(c, st, "k_axpy_multi", 8.0 * len * (nv + 2), 1,
                 launch_axpy_multi(st, w, Vv(0), ln->ldv, nv, dv + DV_H2, len));
            PROF(c, st, "k_dot_multi", 8.0 * len, 1,
                 launch_dot_multi(st, Vv(0), ln->ldv, 0, w, len, 1, ln->part, dv + DV_NRM, nullptr));
        }
        phase = WAIT_ITER;
        return lane_readback(*ln, DV_Y);
    }

    // least-squares solution of the cycle and the update of sol
    irk_status finish_cycle() {
        for (int i = j - 1; i >= 0; --i) {
            double acc = g[i];
            for (int k = i + 1; k < j; ++k) acc -= H[(size_t)i * m + k] * y[k];
            y[i] = acc / H[(size_t)i * m + i];
        }
        irk_status stt;
        if (first_cycle) {
            // (the vorticity solve's Z vectors have zero psi parts: sol's psi
            // parts start at zero too)
            if ((stt = lane_write(*ln, ln->dv + DV_Y, y.data(), j)) != IRK_OK) return stt;
            PROF(c, ln->stream, "k_lincomb", 8.0 * len * (j + 1), 1,
                 launch_lincomb(ln->stream, sol, Zv(0), ln->ldv, j, ln->dv + DV_Y, len));
        } else {
            for (int i = 0; i < j; ++i) y[i] = -y[i];        // sol += Z y as sol -= Z (-y)
            if ((stt = lane_write(*ln, ln->dv + DV_Y, y.data(), j)) != IRK_OK) return stt;
            PROF(c, ln->stream, "k_axpy_multi", 8.0 * len * (j + 2), 1,
                 launch_axpy_multi(ln->stream, sol, Zv(0), ln->ldv, j, ln->dv + DV_Y, len));
        }
        first_cycle = false;
        if (converged || total >= maxit) {
            phase = DONE;
            return IRK_OK;
        }
        return start();                                        // restart
    }

    // consume the readback that just completed
    irk_status advance() {
        const double *hb = ln->pin + PIN_READ;
        if (phase == WAIT_BETA) {
            const double bnorm = std::sqrt(hb[DV_BETA]);
            if (!std::isfinite(bnorm)) return IRK_E_NONFINITE;
            if (!beta0_set) {
                beta0 = bnorm;
                beta0_set = true;
                if (bnorm == 0.0) {
                    if (first_cycle)
                        PROF(c, ln->stream, "k_fill_f64", 8.0 * len, 1, launch_fill(ln->stream, sol, 0.0, len));
                    phase = DONE;
                    return IRK_OK;
                }
            }
            if (bnorm <= rtol * beta0 || total >= maxit) {
                phase = DONE;
                return IRK_OK;
            }
            PROF(c, ln->stream, "k_scale_copy", 16.0 * len, 1,
                 launch_scale_copy(ln->stream, Vv(0), first_cycle && mode == 0 ? rhs : Vv(0), ln->dv + DV_BETA,
                                   len));
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = bnorm;
            j = 0;
            return issue_iteration();
        }
        // WAIT_ITER: Hessenberg column j
        const int nv = j + 1;
        double hn2 = fused ? hb[DV_H2 + nv] : hb[DV_NRM];
        if (fused)
            for (int i = 0; i < nv; ++i) hn2 -= hb[DV_H2 + i] * hb[DV_H2 + i];
        if (!std::isfinite(hn2)) return IRK_E_NONFINITE;
        const double hn = std::sqrt(std::max(hn2, 0.0));
        for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hb[DV_H1 + i] + hb[DV_H2 + i];
        H[(size_t)(j + 1) * m + j] = hn;
        // apply previous rotations, then a new one that zeroes H[j+1][j]
        for (int i = 0; i < j; ++i) {
            const double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
            H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
            H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
        }
        const double a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
        const double rr = std::hypot(a, b);
        cs[j] = rr > 0 ? a / rr : 1.0;
        sn[j] = rr > 0 ? b / rr : 0.0;
        H[(size_t)j * m + j] = rr;
        H[(size_t)(j + 1) * m + j] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++total;
        if (std::fabs(g[j + 1]) <= rtol * beta0 || hn <= 1e-300) {
            converged = true;
            ++j;
            return finish_cycle();
        }
        if (j + 1 >= m || total >= maxit) {
            ++j;
            return finish_cycle();
        }
        if (!fused)
            PROF(c, ln->stream, "k_scale_copy", 16.0 * len, 1,
                 launch_scale_copy(ln->stream, Vv(j + 1), Vv(j + 1), ln->dv + DV_NRM, len));
        ++j;
        return issue_iteration();
    }
};

template <class T>
void PrecBroker<T>::forget(const irk_ctx *c) {
    pending.erase(std::remove_if(pending.begin(), pending.end(), [c](Fgmres<T> *f) { return f->c == c; }),
                  pending.end());
}

template <class T>
int PrecBroker<T>::flush() {
    if (pending.empty()) return 0;
    std::vector<Fgmres<T> *> batch;
    batch.swap(pending);
    // order after every lane's preceding work
    for (Fgmres<T> *f : batch) {
        if (hipEventRecord(f->ln->ev_prec, f->ln->stream) != hipSuccess ||
            hipStreamWaitEvent(st, f->ln->ev_prec, 0) != hipSuccess)
            f->deferred = IRK_E_DEVICE;
    }
    bool two_passes = false;
    for (int pass = 1; pass <= 2; ++pass) {
        std::vector<VcJob<T>> jobs;
        jobs.reserve(batch.size());
        for (Fgmres<T> *f : batch) f->prec_jobs(pass, jobs);
        if (jobs.empty()) continue;
        if (pass == 2) {
            // lanes of 1x1 blocks are done after the first pass: let them go on
            two_passes = true;
            const bool ok1 = hipEventRecord(done1, st) == hipSuccess;
            for (Fgmres<T> *f : batch) {
                if (f->c->P.eb.width[f->ln->blk] != 1) continue;
                if (!ok1 || hipStreamWaitEvent(f->ln->stream, done1, 0) != hipSuccess) f->deferred = IRK_E_DEVICE;
            }
        }
        // one batched sequence per operator kind and smoothing degree
        std::vector<bool> used(jobs.size(), false);
        for (size_t i = 0; i < jobs.size(); ++i) {
            if (used[i]) continue;
            std::vector<const VcJob<T> *> grp;
            for (size_t k = i; k < jobs.size(); ++k)
                if (!used[k] && jobs[k].opk == jobs[i].opk && jobs[k].deg == jobs[i].deg) {
                    grp.push_back(&jobs[k]);
                    used[k] = true;
                }
            run_vcjobs_batched<T>(batch[0]->c, st, grp);
        }
    }
    const bool ok = hipEventRecord(done, st) == hipSuccess;
    for (Fgmres<T> *f : batch) {
        const bool waited1 = two_passes && f->c->P.eb.width[f->ln->blk] == 1;
        if (!waited1 && (!ok || hipStreamWaitEvent(f->ln->stream, done, 0) != hipSuccess)) f->deferred = IRK_E_DEVICE;
        f->resume();
    }
    return (int)batch.size();
}

// ---------------------------------------------------------------------------
// One step: Algorithm 1 in the eigenbasis.
// ---------------------------------------------------------------------------
static void fill_stage_coefs(const irk_ctx *c, double t_n, double dt, StageCoefs *C) {
    const EigenBlocks &eb = c->P.eb;
    const int s = eb.s;
    std::memset(C, 0, sizeof(*C));
    for (int i = 0; i < s * s; ++i) {
        C->A[i] = eb.A[i];
        C->TLam[i] = -eb.TLam[i];     // the block solves return y = D^{-1} fhat; the correction is -T Lambda y
        C->Tinv[i] = eb.Tinv[i];
    }
    for (int i = 0; i < s; ++i) {
        C->b[i] = eb.b[i];
        C->tstage[i] = t_n + eb.c[i] * dt;
        C->sin_t[i] = std::sin(C->tstage[i]);
        C->cos_t[i] = std::cos(C->tstage[i]);
    }
}

template <class T>
static void setup_hierarchies(irk_ctx *c) {
    const Plan &P = c->P;
    // coefficient field of each hierarchy's linearization: U_m (NLDIFF,
    // Burgers) or Psi_m (VSF) of its stage, or (Newton-like (2), (3)) the
    // row's weighted combination sum_k d_rr,k U_k -- all hierarchies in one
    // launch per level
    const size_t off = P.op.kind == IRK_OP_VSF_2D ? P.npts : 0;
    const int nh = P.nhier;
    T *dst[IRK_MAX_STAGES];
    const T *src[IRK_MAX_STAGES];
    int nread = 0;                       // stage fields read per point (bytes)
    for (int hq = 0; hq < nh; ++hq) {
        dst[hq] = c->coef<T>(hq, 0);
        for (int k = 0; k < P.s; ++k) nread += P.hier_w[hq][k] != 0.0;
    }
    PROF(c, c->stream, kn<T>("k_mix_cast_multi"), (double)P.npts * (8.0 * nread + nh * sizeof(T)), 1,
         launch_mix_cast_multi<T>(c->stream, dst, c->U, P.nf, off, P.s, P.hier_w, nh, P.npts));
    for (int l = 0; l + 1 < P.lg.nlev; ++l) {
        for (int hq = 0; hq < nh; ++hq) {
            src[hq] = c->coef<T>(hq, l);
            dst[hq] = c->coef<T>(hq, l + 1);
        }
        const double np = (double)P.lg.nx[l] * P.lg.ny[l], npc = (double)P.lg.nx[l + 1] * P.lg.ny[l + 1];
        PROF(c, c->stream, kn<T>("k_mg_coef_restrict_multi"), sizeof(T) * (np + npc) * nh, 1,
             launch_mg_coef_restrict_multi<T>(c->stream, P.lg.nx[l], P.lg.ny[l], src, dst, nh));
    }
}

// The Newton-like loop of Algorithm 1 as a resumable state machine: every
// host decision waits on an event instead of blocking, so irk_step can poll
// one machine and the serving loop can poll many.
struct StepperBase {
    virtual ~StepperBase() {}
    virtual void begin(const double *u_n, double t_n, double dt, double rtol, double *u_np1) = 0;
    // advance as far as possible without blocking; true when finished
    virtual bool poll() = 0;
    // on a lane's host thread: block b's solve of this Newton iteration, to
    // its end
    virtual void run_lane(int b) { (void)b; }
    irk_status status = IRK_OK;
    irk_stats stats;
};

// Host threads of a context, one per eigen-block lane (option lane_threads).
// In a Newton iteration each drives its block's FGMRES -- the launches, the
// waits for its readbacks and the host's Hessenberg work -- while the
// calling thread keeps the Newton level: the blocks' launches, the larger
// part of the host's time, are issued in parallel (HIP launches onto
// separate streams from separate threads do not serialize).  A worker waits
// for a request, first spinning (a Newton iteration's blocks follow each
// other closely), then sleeping; runs the lane's solve to its end; and marks
// the request finished.
struct LaneWorkers {
    irk_ctx *c = nullptr;
    int n = 0;
    std::thread th[IRK_MAX_STAGES];
    std::atomic<unsigned> req[IRK_MAX_STAGES];
    std::atomic<unsigned> fin[IRK_MAX_STAGES];
    std::atomic<bool> quit{false};
    std::mutex m;
    std::condition_variable cv;

    LaneWorkers() {
        for (int b = 0; b < IRK_MAX_STAGES; ++b) {
            req[b].store(0);
            fin[b].store(0);
        }
    }
    void request(int b) {
        {
            std::lock_guard<std::mutex> lk(m);
            req[b].store(req[b].load(std::memory_order_relaxed) + 1, std::memory_order_release);
        }
        cv.notify_all();
    }
    bool finished(int b) const {
        return fin[b].load(std::memory_order_acquire) == req[b].load(std::memory_order_relaxed);
    }
    void wait_all() const {
        for (int b = 0; b < n; ++b)
            while (!finished(b)) std::this_thread::yield();
    }
};

template <class T>
struct Stepper : StepperBase {
    irk_ctx *c;
    enum Phase { RES_WAIT, BLOCKS, FINAL_WAIT, DONE } phase = DONE;
    const double *u_n = nullptr;
    double *u_np1 = nullptr;
    double t_n = 0, dt = 0, rtol = 0;
    StageCoefs C;
    int it = 0, fold = 0, flat = 0, active = 0;
    double res0 = -1, thresh = 0, prev = 0;
    // starting stage vectors: the candidates (zero, explicit, extrapolated)
    // are evaluated back to back with one readback of their residuals
    enum Start { START_CANDIDATES, START_CHOSEN } start = START_CHOSEN;
    int ncand = 2;
    Fgmres<T> fg[IRK_MAX_STAGES];
    bool lane_done[IRK_MAX_STAGES];
    bool lane_started[IRK_MAX_STAGES];
    // this Newton iteration's block solves run on the lanes' host threads
    bool threaded = false;
    hipEvent_t coef_wait = nullptr;      // the hierarchies' event the solves' V-cycles wait on
    irk_status lane_err[IRK_MAX_STAGES];
    double block_ktol = 1e-5;

    explicit Stepper(irk_ctx *cc) : c(cc) {}

    bool fail(irk_status e) {
        if (threaded) c->workers->wait_all();      // no lane still issuing work
        threaded = false;
        status = e;
        phase = DONE;
        if (c->broker) static_cast<PrecBroker<T> *>(c->broker)->forget(c);   // lanes left waiting in a batch
        return true;
    }

    // stage values and residual of the current K; its norms go to dv[slot]
    // and the host's pinned[slot] (VSF: the stages' largest one-cell
    // streamfunction differences to dv and pinned[DV_GMAX..]), with
    // (readback) an event behind them
    irk_status issue_residual(int slot = DV_RES, bool readback = true) {
        const Plan &P = c->P;
        const int s = P.s;
        const size_t nf = P.nf;
        if (c->K2 && stage_residual_fused(c->dp)) {
            // one sweep: fold, stage values, residual, transform, norms;
            // the folded stages land in K2, which becomes K
            PROF(c, c->stream, "k_stage_residual<" + std::to_string(s) + "," + std::to_string(P.op.kind) + ">",
                 8.0 * nf * (fold ? 5 * s + 1 : 3 * s + 1), 1,
                 launch_stage_residual(c->stream, s, c->dp, u_n, c->K, c->K2, c->Y, c->U, c->Fh, C, dt, fold,
                                       c->part, c->dv + slot, c->pinned_dev + slot));
            if (fold) std::swap(c->K, c->K2);
        } else {
            issue_residual_unfused(slot);
        }
        if (!readback) return IRK_OK;
        HIP_TRY(hipEventRecord(c->ev_res, c->stream));
        phase = RES_WAIT;
        return IRK_OK;
    }

    // stage preparation and residual as two sweeps (the vorticity-
    // streamfunction DAE: its constraint rows need the stages' means first)
    void issue_residual_unfused(int slot) {
        const Plan &P = c->P;
        const int s = P.s;
        const size_t nf = P.nf;
        if (P.op.kind == IRK_OP_VSF_2D) {
            // the stage values with the stage means the constraint rows need
            PROF(c, c->stream, "k_stage_prep_sums<" + std::to_string(s) + ">",
                 8.0 * nf * (fold ? 4 * s + 1 : 2 * s + 1), 1,
                 launch_stage_prep_sums(c->stream, s, P.npts, u_n, c->K, c->Y, c->U, C, dt, fold, 1.0 / P.npts,
                                        c->part, c->dv + DV_MEANS));
        } else {
            PROF(c, c->stream, "k_stage_prep<" + std::to_string(s) + ">", 8.0 * nf * (fold ? 4 * s + 1 : 2 * s + 1),
                 1, launch_stage_prep(c->stream, s, nf, u_n, c->K, c->Y, c->U, C, dt, fold));
        }
        // reads U and K, writes the transformed residual: 3 s fields
        PROF(c, c->stream, "k_residual<" + std::to_string(s) + "," + std::to_string(P.op.kind) + ">",
             8.0 * nf * 3 * s, 1,
             launch_residual(c->stream, s, c->dp, c->U, c->K, c->Fh, C, c->dv + DV_MEANS, c->part, c->dv + slot,
                             c->dv + DV_GMAX, c->pinned_dev + slot, c->pinned_dev + DV_GMAX));
    }

    void set_zero_start() {
        const Plan &P = c->P;
        PROF(c, c->stream, "k_fill", 8.0 * P.s * P.nf, 1, launch_fill(c->stream, c->K, 0.0, (size_t)P.s * P.nf));
    }
    void set_explicit_start() {
        const Plan &P = c->P;
        PROF(c, c->stream, "k_rhs_init<" + std::to_string(P.s) + "," + std::to_string(P.op.kind) + ">",
             8.0 * P.nf * (1 + P.s), 1,
             launch_rhs_init(c->stream, P.s, c->dp, u_n, c->K, std::sin(t_n), std::cos(t_n)));
    }

    // all candidates evaluated back to back (the last one's stage values and
    // transformed residual stay current), one readback of their norms
    irk_status issue_candidates() {
        const Plan &P = c->P;
        ncand = c->extrap ? 3 : 2;
        set_zero_start();
        irk_status e = issue_residual(DV_CAND, false);
        if (e != IRK_OK) return e;
        set_explicit_start();
        if ((e = issue_residual(DV_CAND + 2, false)) != IRK_OK) return e;
        if (ncand == 3) {
            HIP_TRY(hipMemcpyAsync(c->K, c->Y, (size_t)P.s * P.nf * sizeof(double), hipMemcpyDeviceToDevice,
                                   c->stream));
            if ((e = issue_residual(DV_CAND + 4, false)) != IRK_OK) return e;
        }
        // (each candidate's norms went to pinned[DV_CAND + 2 i]; the last
        // one's streamfunction differences stay in pinned[DV_GMAX..])
        HIP_TRY(hipEventRecord(c->ev_res, c->stream));
        start = START_CANDIDATES;
        phase = RES_WAIT;
        return IRK_OK;
    }

    void begin(const double *un, double tn, double dtt, double rt, double *out) override {
        const Plan &P = c->P;
        const int s = P.s;
        const size_t nf = P.nf;
        u_n = un;
        u_np1 = out;
        t_n = tn;
        dt = dtt;
        rtol = rt;
        std::memset(&stats, 0, sizeof(stats));
        status = IRK_OK;
        fill_stage_coefs(c, t_n, dt, &C);
        c->dt = dt;
        c->st = &stats;
        it = fold = flat = 0;
        res0 = -1;
        thresh = prev = 0;
        // starting stage vectors (Algorithm 1 leaves them open): first K = 0,
        // every stage value at u_n.  On a continued step the previous stage
        // vectors are first carried along their interpolating polynomial
        // into Y (not read before the first Newton correction):
        // k_i = sum_j l_j(1 + c_i dt / dt_prev) k_j^prev
        if (c->extrap) {
            StageCoefs W;
            std::memset(&W, 0, sizeof(W));
            for (int i = 0; i < s; ++i) {
                const double x = 1.0 + P.eb.c[i] * c->extrap_ratio;
                for (int j = 0; j < s; ++j) {
                    double l = 1.0;
                    for (int m = 0; m < s; ++m)
                        if (m != j) l *= (x - P.eb.c[m]) / (P.eb.c[j] - P.eb.c[m]);
                    W.A[i * s + j] = l;
                }
            }
            PROF(c, c->stream, "k_stage_extrap<" + std::to_string(s) + ">", 8.0 * nf * 2 * s, 1,
                 launch_stage_extrap(c->stream, s, nf, c->K, c->Y, W));
        }
        const irk_status e = issue_candidates();
        if (e != IRK_OK) fail(e);
    }

    // the residual norm has arrived: converge, fail, or start the block solves
    bool on_residual() {
        const Plan &P = c->P;
        if (start == START_CANDIDATES) {
            // candidates in order zero, explicit, extrapolated: the smallest
            // residual wins, the earlier one on ties (NaN never wins)
            start = START_CHOSEN;
            double rc[3];
            for (int i = 0; i < ncand; ++i) rc[i] = std::sqrt(c->pinned[DV_CAND + 2 * i]);
            if (!std::isfinite(rc[0])) return fail(IRK_E_NONFINITE);
            int best = 0;
            for (int i = 1; i < ncand; ++i)
                if (rc[i] < rc[best]) best = i;
            stats.start = best;
            if (debug_level())
                fprintf(stderr, "[irk] start candidates: |F(0)| %.6e |F(explicit)| %.6e |F(extrapolated)| %.6e\n",
                        rc[0], rc[1], ncand == 3 ? rc[2] : -1.0);
            if (best == ncand - 1) {
                // the last candidate evaluated: its stage values are current
                c->pinned[DV_RES] = c->pinned[DV_CAND + 2 * best];
                c->pinned[DV_ABS] = c->pinned[DV_CAND + 2 * best + 1];
            } else {
                if (best == 0) set_zero_start();
                else set_explicit_start();
                const irk_status e = issue_residual();
                return e != IRK_OK ? fail(e) : false;
            }
        }
        const double res = std::sqrt(c->pinned[DV_RES]);
        // the residual cannot be resolved below the rounding error of its own
        // evaluation: 64 eps times the norm of the magnitudes of its terms
        const double floor_res = 64.0 * 2.220446049250313e-16 * std::sqrt(c->pinned[DV_ABS]);
        if (!std::isfinite(res)) return fail(IRK_E_NONFINITE);
        if (it == 0) {
            res0 = res;
            const double atol = P.opt.newton_atol > 0 ? P.opt.newton_atol : 1e-14 * res0;
            thresh = rtol * res0 + atol;
            stats.res0 = res0;
        }
        stats.final_res = res;
        if (debug_level())
            fprintf(stderr, "[irk] newton it %d res %.6e thresh %.3e floor %.3e\n", it, res, thresh, floor_res);
        bool converged = res <= std::max(thresh, floor_res);
        stats.acceptance = 0;
        // stagnation within a small factor of the estimated floor: the
        // iteration has reached rounding level
        if (!converged && it > 0 && res <= 16.0 * floor_res && res > 0.25 * prev) {
            converged = true;
            stats.acceptance = 1;
        }
        // safety net: three iterations in a row that reduce the residual by
        // less than 10 % (stagnation, not slow linear convergence, which
        // goes on to the threshold) far below res0 mean the rounding floor
        // was underestimated; reported in stats.acceptance
        flat = (it > 0 && res >= 0.9 * prev) ? flat + 1 : 0;
        if (!converged && flat >= 3 && res <= 1e-8 * res0) {
            converged = true;
            stats.acceptance = 2;
        }
        if (converged) {
            PROF(c, c->stream, "k_final_update<" + std::to_string(P.s) + ">", 8.0 * P.nf * (P.s + 2), 1,
                 launch_final_update(c->stream, P.s, P.nf, u_n, c->K, u_np1, C, dt));
            if (hipEventRecord(c->ev_res, c->stream) != hipSuccess) return fail(IRK_E_DEVICE);
            phase = FINAL_WAIT;
            return false;
        }
        prev = res;
        if (res > 1e8 * std::max(res0, 1e-300) || it >= P.opt.max_newton) return fail(IRK_E_NOCONV);
        // VSF: per hierarchy a bound on its streamfunction's one-cell
        // differences (the stage's, or the weighted sum's), which lets the
        // vorticity V-cycles stop at a diagonally dominant level
        c->hier_g_valid = P.op.kind == IRK_OP_VSF_2D;
        if (c->hier_g_valid)
            for (int h = 0; h < P.nhier; ++h) {
                double g = 0.0;
                for (int k = 0; k < P.s; ++k) g += std::fabs(P.hier_w[h][k]) * c->pinned[DV_GMAX + k];
                c->hier_g[h] = g;
                if (!std::isfinite(g)) c->hier_g_valid = false;
            }
        // the block solves start (||r0||, the first basis vector) as soon as
        // the residual is in; only their V-cycles wait for the coefficient
        // hierarchies built meanwhile (with shared V-cycle batches, which run
        // on other streams, everything waits as before)
        const bool split = !c->broker;
        if (split && hipEventRecord(c->ev_main, c->stream) != hipSuccess) return fail(IRK_E_DEVICE);
        setup_hierarchies<T>(c);
        if (hipEventRecord(split ? c->ev_coef : c->ev_main, c->stream) != hipSuccess) return fail(IRK_E_DEVICE);
        coef_wait = split ? c->ev_coef : nullptr;
        active = c->nlanes;
        // relative Krylov tolerance of the block solves: the fixed one, or
        // (krylov_adaptive) never tighter than a tenth of the reduction the
        // acceptance test still asks of this residual (an inexact Newton
        // forcing term: solving further cannot change the accepted stages)
        double ktol = P.opt.krylov_rtol;
        if (P.opt.krylov_adaptive) ktol = std::min(0.1, std::max(ktol, 0.1 * std::max(thresh, floor_res) / res));
        block_ktol = ktol;
        threaded = c->workers && !c->prof && !c->broker && !P.eb.schur;
        for (int b = 0; b < c->nlanes; ++b) {
            lane_done[b] = false;
            lane_started[b] = false;
            if (hipStreamWaitEvent(c->lanes[b].stream, c->ev_main, 0) != hipSuccess) return fail(IRK_E_DEVICE);
            // real Schur basis: back-substitution, the last block first
            if (P.eb.schur && b != c->nlanes - 1) continue;
            if (threaded) {
                lane_started[b] = true;
                lane_err[b] = IRK_OK;
                fg[b].init(c, &c->lanes[b], block_ktol, c->P.opt.max_krylov);
                fg[b].prec_wait = coef_wait;
                c->workers->request(b);
                continue;
            }
            const irk_status e = start_block(b);
            if (e != IRK_OK) return fail(e);
        }
        phase = BLOCKS;
        return false;
    }

    void run_lane(int b) override {
        irk_status e = fg[b].start();
        while (e == IRK_OK && fg[b].phase != Fgmres<T>::DONE) {
            const hipError_t q = hipEventQuery(c->lanes[b].ev);
            if (q == hipErrorNotReady) {
                std::this_thread::yield();
                continue;
            }
            if (q != hipSuccess) {
                e = IRK_E_DEVICE;
                break;
            }
            e = fg[b].advance();
            // reordered DAE system: the streamfunction rows next
            if (e == IRK_OK && fg[b].phase == Fgmres<T>::DONE && fg[b].mode == 1) e = fg[b].to_psi();
        }
        // launch errors are recorded per host thread
        if (e == IRK_OK && hipGetLastError() != hipSuccess) e = IRK_E_DEVICE;
        lane_err[b] = e;
    }

    irk_status start_block(int b) {
        lane_started[b] = true;
        fg[b].init(c, &c->lanes[b], block_ktol, c->P.opt.max_krylov);
        fg[b].prec_wait = coef_wait;
        return fg[b].start();
    }

    // real Schur basis, block b solved: every earlier block's right-hand side
    // loses its coupling to y_b (on b's stream), then block b - 1 starts
    // after it
    irk_status back_substitute(int b) {
        const Plan &P = c->P;
        const size_t nf = P.nf;
        Lane &ln = c->lanes[b];
        const double *yb = c->Y + (size_t)P.eb.first[b] * nf;
        for (int i = 0; i < b; ++i) {
            const BlockCouple &C = P.cpl[i][b];
            PROF(c, ln.stream, "k_block_couple<" + std::to_string(P.op.kind) + ">",
                 8.0 * nf * (C.wj + 2 * C.wi + (C.jac ? P.s : 0)), 1,
                 launch_block_couple(ln.stream, c->dp, P.s, C, c->dt, c->U, yb, c->Fh + (size_t)P.eb.first[i] * nf));
        }
        HIP_TRY(hipEventRecord(ln.done, ln.stream));
        HIP_TRY(hipStreamWaitEvent(c->lanes[b - 1].stream, ln.done, 0));
        return start_block(b - 1);
    }

    bool poll() override {
        const Plan &P = c->P;
        for (;;) {
            if (phase == DONE) return true;
            if (phase == RES_WAIT || phase == FINAL_WAIT) {
                const hipError_t q = hipEventQuery(c->ev_res);
                if (q == hipErrorNotReady) return false;
                if (q != hipSuccess) return fail(IRK_E_DEVICE);
                if (phase == FINAL_WAIT) {
                    phase = DONE;
                    return true;
                }
                if (on_residual()) return true;
                continue;
            }
            // BLOCKS: advance every lane whose readback has landed
            bool progressed = false;
            for (int b = 0; b < c->nlanes; ++b) {
                if (lane_done[b] || !lane_started[b]) continue;
                irk_status e = IRK_OK;
                if (threaded) {
                    // the lane's host thread ran its solve to the end
                    if (!c->workers->finished(b)) continue;
                    if (lane_err[b] != IRK_OK) return fail(lane_err[b]);
                    progressed = true;
                } else {
                    if (fg[b].deferred != IRK_OK) return fail(fg[b].deferred);
                    if (fg[b].phase == Fgmres<T>::WAIT_PREC) continue;      // in a broker batch
                    const hipError_t q = hipEventQuery(c->lanes[b].ev);
                    if (q == hipErrorNotReady) continue;
                    if (q != hipSuccess) return fail(IRK_E_DEVICE);
                    progressed = true;
                    e = fg[b].advance();
                    if (e != IRK_OK) return fail(e);
                    if (fg[b].phase == Fgmres<T>::DONE && fg[b].mode == 1) {
                        // reordered DAE system: the streamfunction rows next
                        e = fg[b].to_psi();
                        if (e != IRK_OK) return fail(e);
                    }
                }
                if (fg[b].phase == Fgmres<T>::DONE) {
                    lane_done[b] = true;
                    --active;
                    if (P.eb.schur && b > 0) {
                        e = back_substitute(b);
                        if (e != IRK_OK) return fail(e);
                    }
                    if (hipEventRecord(c->lanes[b].done, c->lanes[b].stream) != hipSuccess ||
                        hipStreamWaitEvent(c->stream, c->lanes[b].done, 0) != hipSuccess)
                        return fail(IRK_E_DEVICE);
                    stats.krylov_its += fg[b].total;
                    stats.krylov_its_block[b] += fg[b].total;
                    if (fg[b].mode == 2) stats.krylov_its_psi += fg[b].total - fg[b].omega_total;
                    stats.vcycles += fg[b].vcycles;
                    stats.prec_applications += fg[b].total * P.eb.width[b];
                    if (debug_level() > 1)
                        fprintf(stderr, "[irk]   block %d fgmres its %d beta0 %.3e\n", b, fg[b].total, fg[b].beta0);
                }
            }
            // this context's own broker: run the V-cycles of the blocks that
            // wait now as shared launches (a server flushes its shared one)
            if (c->broker_owned && static_cast<PrecBroker<T> *>(c->broker)->flush() > 0) {
                for (int b = 0; b < c->nlanes; ++b)
                    if (!lane_done[b] && fg[b].deferred != IRK_OK) return fail(fg[b].deferred);
                progressed = true;
            }
            if (active == 0) {
                threaded = false;
                stats.newton_its++;
                fold = 1;
                ++it;
                const irk_status e = issue_residual();
                if (e != IRK_OK) return fail(e);
                continue;
            }
            if (!progressed) return false;
        }
    }
};

// SDIRK (the comparison class): the stages are solved one after another.
// Stage i is the 1-stage problem k_i = N(u' + dt gamma k_i, t_n + c_i dt)
// with u' = u_n + dt sum_{j<i} a_ij k_j, i.e. the machinery above with
// A = [gamma], c = [c_i] on the state u' (one real block, eta = 1/gamma);
// then u_{n+1} = u_n + dt sum_i b_i k_i.
template <class T>
struct SdirkStepper : StepperBase {
    irk_ctx *c;
    Stepper<T> inner;
    enum Phase { STAGE, FINAL_WAIT, DONE } phase = DONE;
    const double *u_n = nullptr;
    double *u_np1 = nullptr;
    double t_n = 0, dt = 0, rtol = 0;
    int stage = 0;

    explicit SdirkStepper(irk_ctx *cc) : c(cc), inner(cc) {}

    double *Ksd() { return reinterpret_cast<double *>(c->ws + c->P.off_Ksd); }

    bool fail(irk_status e) {
        status = e;
        phase = DONE;
        return true;
    }

    void start_stage() {
        Plan &P = c->P;
        P.eb.c[0] = P.sd_c[stage];
        const double *u_in = u_n;
        if (stage > 0) {
            StageCoefs C;
            std::memset(&C, 0, sizeof(C));
            for (int j = 0; j < stage; ++j) C.b[j] = P.sd_A[stage * P.sd_s + j];
            double *uin = reinterpret_cast<double *>(c->ws + P.off_Uin);
            PROF(c, c->stream, "k_final_update<" + std::to_string(stage) + ">", 8.0 * P.nf * (stage + 2), 1,
                 launch_final_update(c->stream, stage, P.nf, u_n, Ksd(), uin, C, dt));
            u_in = uin;
        }
        inner.begin(u_in, t_n, dt, rtol, reinterpret_cast<double *>(c->ws + P.off_Uout));
    }

    void begin(const double *un, double tn, double dtt, double rt, double *out) override {
        u_n = un;
        u_np1 = out;
        t_n = tn;
        dt = dtt;
        rtol = rt;
        stage = 0;
        std::memset(&stats, 0, sizeof(stats));
        status = IRK_OK;
        phase = STAGE;
        start_stage();
    }

    bool poll() override {
        const Plan &P = c->P;
        for (;;) {
            if (phase == DONE) return true;
            if (phase == FINAL_WAIT) {
                const hipError_t q = hipEventQuery(c->ev_res);
                if (q == hipErrorNotReady) return false;
                if (q != hipSuccess) return fail(IRK_E_DEVICE);
                phase = DONE;
                return true;
            }
            if (!inner.poll()) return false;
            const irk_stats &is = inner.stats;
            stats.newton_its += is.newton_its;
            stats.krylov_its += is.krylov_its;
            stats.krylov_its_block[stage] += is.krylov_its;
            stats.krylov_its_psi += is.krylov_its_psi;
            stats.vcycles += is.vcycles;
            stats.prec_applications += is.prec_applications;
            stats.res0 = std::max(stats.res0, is.res0);
            stats.final_res = std::max(stats.final_res, is.final_res);
            stats.acceptance = std::max(stats.acceptance, is.acceptance);
            if (inner.status != IRK_OK) return fail(inner.status);
            if (debug_level())
                fprintf(stderr, "[irk] sdirk stage %d done: newton %d krylov %d res0 %.3e final %.3e\n", stage,
                        is.newton_its, is.krylov_its, is.res0, is.final_res);
            if (hipMemcpyAsync(Ksd() + (size_t)stage * P.nf, c->K, P.nf * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream) != hipSuccess)
                return fail(IRK_E_DEVICE);
            if (++stage < P.sd_s) {
                start_stage();
                continue;
            }
            StageCoefs C;
            std::memset(&C, 0, sizeof(C));
            for (int i = 0; i < P.sd_s; ++i) C.b[i] = P.sd_b[i];
            PROF(c, c->stream, "k_final_update<" + std::to_string(P.sd_s) + ">", 8.0 * P.nf * (P.sd_s + 2), 1,
                 launch_final_update(c->stream, P.sd_s, P.nf, u_n, Ksd(), u_np1, C, dt));
            if (hipEventRecord(c->ev_res, c->stream) != hipSuccess) return fail(IRK_E_DEVICE);
            phase = FINAL_WAIT;
        }
    }
};

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" const char *irk_status_str(irk_status st) {
    switch (st) {
        case IRK_OK: return "ok";
        case IRK_E_ARG: return "invalid argument";
        case IRK_E_NOMEM: return "workspace too small or budget exceeded";
        case IRK_E_NOCONV: return "nonlinear iteration did not converge";
        case IRK_E_NONFINITE: return "non-finite value";
        case IRK_E_DEVICE: return "HIP runtime error";
        case IRK_E_UNSUPPORTED: return "unsupported option combination";
        case IRK_E_BUSY: return "request not finished";
    }
    return "unknown status";
}

extern "C" void irk_default_options(irk_options *o) {
    if (!o) return;
    o->newton_rtol = 1e-12;
    o->newton_atol = 0.0;
    o->krylov_rtol = 1e-5;
    o->restart = 30;
    o->max_krylov = 200;
    o->max_newton = 30;
    o->newton_like = 1;
    o->gamma_mode = 0;
    o->prec_fp32 = 1;
    o->cheb_degree = 3;
    o->mg_coarsest = 16;
    o->coarse_iters = 24;
    o->batch_mg = 0;
    o->start_extrapolate = 1;
    o->krylov_adaptive = 1;
    o->dae_reorder = 0;
    o->transform = 0;
    o->psi_solve = 0;
    o->lane_threads = 1;
}

extern "C" size_t irk_workspace_bytes(irk_family family, int s, const irk_operator *op, const irk_options *opt) {
    Plan P;
    if (make_plan(family, s, op, opt, &P) != IRK_OK) return 0;
    return P.total;
}

// Chebyshev iteration on D^{-1} A with spectrum in [lmin, lmax]: step k
// updates d <- cd[k] d + cr[k] D^{-1} r, x <- x + d (three-term recurrence).
static void chebyshev_coefs(double lmin, double lmax, int n, double *cd, double *cr) {
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sig1 = theta / delta;
    double rho = 1.0 / sig1;
    for (int k = 0; k < n; ++k) {
        if (k == 0) {
            cd[0] = 0.0;
            cr[0] = 1.0 / theta;
        } else {
            const double rn = 1.0 / (2.0 * sig1 - rho);
            cd[k] = rn * rho;
            cr[k] = 2.0 * rn / delta;
            rho = rn;
        }
    }
}

static void set_chebyshev(irk_ctx *c) {
    std::memset(c->cheb_cd, 0, sizeof(c->cheb_cd));
    std::memset(c->cheb_cr, 0, sizeof(c->cheb_cr));
    chebyshev_coefs(c->lmin, c->lmax, c->P.opt.cheb_degree, c->cheb_cd, c->cheb_cr);
}

// doubles of the upload area a problem needs: forcing tables, the Fourier
// basis and eigenvalues of the exactly solved Poisson level
static size_t upload_doubles(const Plan &P) {
    size_t n = (size_t)2 * (P.op.nx + P.op.ny);
    if (P.fdm_level > 0) {
        const size_t m = P.lg.nx[P.fdm_level];
        n += m * m + m;
    }
    if (P.fft_psi) n += (size_t)3 * P.op.nx;
    return n;
}

// Create every stream, event and the pinned staging of a resource set
// (default-priority, non-blocking streams: ordering with the caller's
// stream is explicit, through events).
static irk_status res_create(CtxRes *r, int nlanes, size_t upload) {
    r->nlanes = nlanes;
    r->upload = upload;
    const size_t pin = (size_t)(1 + IRK_MAX_STAGES) * PIN_LANE + upload;
    // fine-grained (coherent) and mapped: the reductions write their results
    // here directly, visible to the host once an event behind them completes
    if (hipHostMalloc((void **)&r->pinned, pin * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess) {
        r->pinned = nullptr;
        return IRK_E_DEVICE;
    }
    if (hipHostGetDevicePointer((void **)&r->pinned_dev, r->pinned, 0) != hipSuccess) return IRK_E_DEVICE;
    auto ev = [](hipEvent_t *e) { return hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess; };
    if (!ev(&r->ev_main) || !ev(&r->ev_res) || !ev(&r->ev_coef)) return IRK_E_DEVICE;
    for (int b = 0; b < nlanes; ++b) {
        if (hipStreamCreateWithFlags(&r->lane_st[b], hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&r->aux_st[b], hipStreamNonBlocking) != hipSuccess || !ev(&r->ev[b]) ||
            !ev(&r->done[b]) || !ev(&r->prec[b]) || !ev(&r->fork[b]) || !ev(&r->join[b]))
            return IRK_E_DEVICE;
    }
    return IRK_OK;
}

// Wait for and release everything res_create made (also a partial set).
static void res_destroy(CtxRes *r) {
    if (!r) return;
    for (int b = 0; b < IRK_MAX_STAGES; ++b) {
        for (hipStream_t st : {r->lane_st[b], r->aux_st[b]})
            if (st) {
                (void)hipStreamSynchronize(st);
                (void)hipStreamDestroy(st);
            }
        for (hipEvent_t e : {r->ev[b], r->done[b], r->prec[b], r->fork[b], r->join[b]})
            if (e) (void)hipEventDestroy(e);
    }
    if (r->ev_main) (void)hipEventDestroy(r->ev_main);
    if (r->ev_coef) (void)hipEventDestroy(r->ev_coef);
    if (r->ev_res) (void)hipEventDestroy(r->ev_res);
    if (r->pinned) (void)hipHostFree(r->pinned);
    *r = CtxRes();
}

static void lane_worker_main(LaneWorkers *W, int b) {
    unsigned seen = 0;
    for (;;) {
        unsigned g = W->req[b].load(std::memory_order_acquire);
        for (int spin = 0; g == seen; ++spin) {
            if (W->quit.load(std::memory_order_acquire)) return;
            if (spin < 20000) {
                std::this_thread::yield();
            } else {
                std::unique_lock<std::mutex> lk(W->m);
                W->cv.wait(lk, [&] {
                    return W->req[b].load(std::memory_order_acquire) != seen || W->quit.load(std::memory_order_acquire);
                });
            }
            g = W->req[b].load(std::memory_order_acquire);
        }
        seen = g;
        W->c->stepper->run_lane(b);
        W->fin[b].store(g, std::memory_order_release);
    }
}

static void stop_workers(irk_ctx *c) {
    LaneWorkers *W = c->workers;
    if (!W) return;
    W->wait_all();
    {
        std::lock_guard<std::mutex> lk(W->m);
        W->quit.store(true, std::memory_order_release);
    }
    W->cv.notify_all();
    for (int b = 0; b < W->n; ++b)
        if (W->th[b].joinable()) W->th[b].join();
    delete W;
    c->workers = nullptr;
}

// a host thread per eigen-block lane, where they can run concurrently (two
// or more blocks of the eigenbasis, no shared V-cycle batches); none if a
// thread cannot be made
static void start_workers(irk_ctx *c) {
    const Plan &P = c->P;
    if (!P.opt.lane_threads || c->nlanes < 2 || P.sd_s > 0 || P.eb.schur || c->broker) return;
    LaneWorkers *W = new (std::nothrow) LaneWorkers();
    if (!W) return;
    W->c = c;
    c->workers = W;
    try {
        for (int b = 0; b < c->nlanes; ++b) {
            W->th[b] = std::thread(lane_worker_main, W, b);
            W->n = b + 1;
        }
    } catch (...) {
        stop_workers(c);
    }
}

static void release(irk_ctx *c) {
    if (!c) return;
    stop_workers(c);
    if (c->broker) {
        if (c->P.opt.prec_fp32) {
            auto *b = static_cast<PrecBroker<float> *>(c->broker);
            if (c->broker_owned) delete b; else b->forget(c);
        } else {
            auto *b = static_cast<PrecBroker<double> *>(c->broker);
            if (c->broker_owned) delete b; else b->forget(c);
        }
        c->broker = nullptr;
    }
    if (c->res_owned) {
        if (c->stream) (void)hipStreamSynchronize(c->stream);
        res_destroy(c->res);
        delete c->res;
    }
    delete c->stepper;
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

// Real orthonormal Fourier basis of the periodic n-point second difference
// on the exact-solve level (columns: the constant, cos and sin pairs of
// modes 1 .. (n-1)/2, and for even n the alternating mode) and its
// eigenvalues 4 sin^2(pi m / n) / h^2, in the V-cycle precision, written to
// `stage` (pinned) and copied to the workspace on the context's stream.
static irk_status upload_fdm_basis(irk_ctx *c, double *stage) {
    const Plan &P = c->P;
    const int n = P.lg.nx[P.fdm_level];
    const double h = P.op.length / P.op.nx * (double)(1 << P.fdm_level);
    const double pi = 3.14159265358979323846;
    const bool f32 = P.tsz == sizeof(float);
    float *qf = reinterpret_cast<float *>(stage);
    double *qd = stage;
    double lam[IRK_FDM_MAX];
    int col = 0;
    auto put = [&](int m, int kind) {          // kind 0: cos (or constant), 1: sin
        const bool single = (m == 0) || (2 * m == n);
        const double sc = single ? std::sqrt(1.0 / n) : std::sqrt(2.0 / n);
        for (int j = 0; j < n; ++j) {
            const double a = 2.0 * pi * m * j / n;
            const double v = sc * (kind == 0 ? std::cos(a) : std::sin(a));
            if (f32) qf[(size_t)j * n + col] = (float)v;
            else qd[(size_t)j * n + col] = v;
        }
        const double sv = std::sin(pi * m / n);
        lam[col] = 4.0 * sv * sv / (h * h);
        ++col;
    };
    put(0, 0);
    for (int m = 1; 2 * m < n; ++m) {
        put(m, 0);
        put(m, 1);
    }
    if (n % 2 == 0) put(n / 2, 0);
    if (col != n) return IRK_E_ARG;
    lam[0] = 0.0;
    const size_t qbytes = (size_t)n * n * P.tsz;
    unsigned char *lstage = reinterpret_cast<unsigned char *>(stage) + qbytes;
    for (int k = 0; k < n; ++k) {
        if (f32) reinterpret_cast<float *>(lstage)[k] = (float)lam[k];
        else reinterpret_cast<double *>(lstage)[k] = lam[k];
    }
    HIP_TRY(hipMemcpyAsync(c->ws + P.off_fdm_Q, stage, qbytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->ws + P.off_fdm_lam, lstage, (size_t)n * P.tsz, hipMemcpyHostToDevice, c->stream));
    return IRK_OK;
}

// Twiddles exp(-2 pi i j / n), j < n, as (re, im) pairs and the
// eigenvalues 4 sin^2(pi m / n) / h^2 of the 1-D periodic second difference
// on the finest grid, in the spectral solve's precision, written to `stage`
// (pinned) and copied to the workspace on the context's stream.
static irk_status upload_fft_tables(irk_ctx *c, double *stage) {
    const Plan &P = c->P;
    const int n = P.op.nx;
    const double h = P.op.length / n;
    const double pi = 3.14159265358979323846;
    const bool f32 = P.fft_tsz == sizeof(float);
    auto put = [&](size_t i, double v) {
        if (f32) reinterpret_cast<float *>(stage)[i] = (float)v;
        else stage[i] = v;
    };
    for (int j = 0; j < n; ++j) {
        const double a = 2.0 * pi * j / n;
        put(2 * (size_t)j, std::cos(a));
        put(2 * (size_t)j + 1, -std::sin(a));
    }
    for (int m = 0; m < n; ++m) {
        const double sv = std::sin(pi * m / n);
        put((size_t)2 * n + m, 4.0 * sv * sv / (h * h));
    }
    const size_t bytes = (size_t)n * P.fft_tsz;
    HIP_TRY(hipMemcpyAsync(c->ws + P.off_fft_tw, stage, 2 * bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->ws + P.off_fft_lam, reinterpret_cast<unsigned char *>(stage) + 2 * bytes, bytes,
                           hipMemcpyHostToDevice, c->stream));
    return IRK_OK;
}

// A new context for a checked plan on a workspace (host only).
static irk_status ctx_new(irk_family family, int s, const irk_operator *op, const irk_options *opt,
                          void *device_workspace, size_t workspace_bytes, irk_ctx **out) {
    *out = nullptr;
    irk_ctx *c = new (std::nothrow) irk_ctx();
    if (!c) return IRK_E_NOMEM;
    irk_status stt = make_plan(family, s, op, opt, &c->P);
    if (stt != IRK_OK) { delete c; return stt; }
    if (!device_workspace || ((uintptr_t)device_workspace & 255) != 0) { delete c; return IRK_E_ARG; }
    if (workspace_bytes < c->P.total) { delete c; return IRK_E_NOMEM; }
    c->ws = (unsigned char *)device_workspace;
    const Plan &P = c->P;
    c->K = (double *)(c->ws + P.off_K);
    c->K2 = P.off_K2 ? (double *)(c->ws + P.off_K2) : nullptr;
    c->Y = (double *)(c->ws + P.off_Y);
    c->Fh = (double *)(c->ws + P.off_Fh);
    c->U = (double *)(c->ws + P.off_U);
    c->part = (double *)(c->ws + P.off_part);
    c->dv = (double *)(c->ws + P.off_dv);
    c->tab = (double *)(c->ws + P.off_tab);
    c->nlanes = P.eb.nblocks;
    *out = c;
    return IRK_OK;
}

// Bind a context to its stream and resource set and enqueue its device
// set-up (forcing tables, Fourier basis, Y = 0) on that stream from the
// pinned upload area; with `wait` the call returns after the set-up has
// completed, else it only enqueues.  private_broker: irk_create's contexts
// batch their own blocks' V-cycles when the option asks for it.
static irk_status ctx_init(irk_ctx *c, hipStream_t stream, CtxRes *r, bool wait, bool private_broker) {
    const Plan &P = c->P;
    if (r->nlanes < c->nlanes || r->upload < upload_doubles(P)) return IRK_E_ARG;
    c->stream = stream;
    c->res = r;
    c->pinned = r->pinned;
    c->pinned_dev = r->pinned_dev;
    c->ev_main = r->ev_main;
    c->ev_coef = r->ev_coef;
    c->ev_res = r->ev_res;
    if (P.sd_s > 0) {
        if (P.opt.prec_fp32) c->stepper = new (std::nothrow) SdirkStepper<float>(c);
        else c->stepper = new (std::nothrow) SdirkStepper<double>(c);
    } else {
        if (P.opt.prec_fp32) c->stepper = new (std::nothrow) Stepper<float>(c);
        else c->stepper = new (std::nothrow) Stepper<double>(c);
    }
    if (!c->stepper) return IRK_E_NOMEM;
    for (int b = 0; b < c->nlanes; ++b) {
        Lane &ln = c->lanes[b];
        const LaneLayout &lay = P.lane[b];
        ln.blk = b;
        ln.lay = &c->P.lane[b];
        ln.ldv = lay.ldv;
        ln.V = (double *)(c->ws + lay.V);
        ln.Z = (double *)(c->ws + lay.Z);
        ln.part = (double *)(c->ws + lay.part);
        ln.dv = (double *)(c->ws + lay.dv);
        ln.tmp = lay.tmp ? (double *)(c->ws + lay.tmp) : nullptr;
        ln.pin = c->pinned + (size_t)(1 + b) * PIN_LANE;
        ln.pin_dev = c->pinned_dev + (size_t)(1 + b) * PIN_LANE;
        ln.stream = r->lane_st[b];
        ln.ev = r->ev[b];
        ln.done = r->done[b];
        ln.ev_prec = r->prec[b];
        if (P.aux[b].used) {
            Lane &ax = c->aux_lanes[b];
            ax.blk = b;
            ax.lay = &c->P.aux[b].lay;
            ax.ldv = ln.ldv;
            ax.part = (double *)(c->ws + ax.lay->part);
            ax.dv = (double *)(c->ws + ax.lay->dv);
            ax.stream = r->aux_st[b];
            ln.ev_fork = r->fork[b];
            ln.ev_join = r->join[b];
            ln.aux = &ax;
        }
    }
    // a private broker batches the V-cycles of this context's blocks
    // (Newton-like (3) pairs apply an operator between their two V-cycles:
    // they are not batched)
    if (private_broker && P.opt.batch_mg && c->nlanes > 1 && P.op.kind != IRK_OP_VSF_2D && P.opt.newton_like != 3 &&
        !P.eb.schur) {
        bool ok;
        if (P.opt.prec_fp32) {
            auto *b = new (std::nothrow) PrecBroker<float>();
            ok = b && b->init();
            c->broker = b;
        } else {
            auto *b = new (std::nothrow) PrecBroker<double>();
            ok = b && b->init();
            c->broker = b;
        }
        c->broker_owned = c->broker != nullptr;
        if (!ok) return IRK_E_DEVICE;
    }
    set_chebyshev(c);
    // device problem descriptor and forcing tables sin/cos(2 pi x_i)
    c->dp.kind = P.op.kind;
    c->dp.forcing = P.op.kind == IRK_OP_NLDIFF_2D ? P.op.forcing : IRK_FORCING_NONE;
    c->dp.nvar = P.nvar;
    c->dp.g.nx = P.op.nx;
    c->dp.g.ny = P.op.ny;
    c->dp.g.h = P.op.length / P.op.nx;
    c->dp.g.nu = P.op.nu;
    const int nx = P.op.nx, ny = P.op.ny;
    double *tab = c->pinned + (size_t)(1 + IRK_MAX_STAGES) * PIN_LANE;   // the upload area
    const double two_pi = 2.0 * 3.14159265358979323846;
    for (int i = 0; i < nx; ++i) {
        tab[i] = std::sin(two_pi * (i * c->dp.g.h));
        tab[nx + i] = std::cos(two_pi * (i * c->dp.g.h));
    }
    for (int j = 0; j < ny; ++j) {
        tab[2 * nx + j] = std::sin(two_pi * (j * c->dp.g.h));
        tab[2 * nx + ny + j] = std::cos(two_pi * (j * c->dp.g.h));
    }
    c->dp.sinx = c->tab;
    c->dp.cosx = c->tab + nx;
    c->dp.siny = c->tab + 2 * nx;
    c->dp.cosy = c->tab + 2 * nx + ny;
    HIP_TRY(hipMemcpyAsync(c->tab, tab, (size_t)2 * (nx + ny) * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (P.fdm_level > 0) {
        const irk_status e = upload_fdm_basis(c, tab + 2 * (nx + ny));
        if (e != IRK_OK) return e;
    }
    if (P.fft_psi) {
        const irk_status e = upload_fft_tables(c, tab + 2 * (nx + ny));
        if (e != IRK_OK) return e;
    }
    launch_fill(c->stream, c->Y, 0.0, (size_t)P.s * P.nf);   // the plan's s (1 for SDIRK)
    HIP_TRY(hipGetLastError());
    if (wait) HIP_TRY(hipStreamSynchronize(c->stream));
    return IRK_OK;
}

extern "C" irk_status irk_create(irk_family family, int s, const irk_operator *op, const irk_options *opt,
                                 void *device_workspace, size_t workspace_bytes, void *hip_stream, irk_ctx **out) {
    if (!out) return IRK_E_ARG;
    irk_ctx *c = nullptr;
    irk_status stt = ctx_new(family, s, op, opt, device_workspace, workspace_bytes, &c);
    if (stt != IRK_OK) return stt;
    (void)hipGetLastError();   // clear an error left by earlier, unrelated HIP calls
    c->res = new (std::nothrow) CtxRes();
    if (!c->res) {
        delete c;
        return IRK_E_NOMEM;
    }
    c->res_owned = true;
    c->stream = (hipStream_t)hip_stream;
    if ((stt = res_create(c->res, c->nlanes, upload_doubles(c->P))) != IRK_OK ||
        (stt = ctx_init(c, (hipStream_t)hip_stream, c->res, true, true)) != IRK_OK) {
        release(c);
        return stt == IRK_E_NOMEM ? IRK_E_NOMEM : IRK_E_DEVICE;
    }
    start_workers(c);
    *out = c;
    return IRK_OK;
}

namespace irk {
// Start one step on a context (non-blocking); poll with step_poll.
irk_status step_begin(irk_ctx *c, const double *u_n, double t_n, double dt, double tol, double *u_np1) {
    if (!c || !u_n || !u_np1 || !(dt > 0) || !std::isfinite(t_n)) return IRK_E_ARG;
    (void)hipGetLastError();
    // a step from the previous step's output buffer at its end time
    // continues it: its stage vectors (still in K) give a third candidate
    c->extrap = c->have_stages && c->P.sd_s == 0 && c->P.opt.start_extrapolate && u_n == c->next_u &&
                t_n == c->next_t;
    c->extrap_ratio = c->extrap ? dt / c->prev_dt : 1.0;
    c->have_stages = false;
    c->have_U = false;
    c->next_u = u_np1;
    c->next_t = t_n + dt;
    c->prev_dt = dt;
    c->stepper->begin(u_n, t_n, dt, tol > 0 ? tol : c->P.opt.newton_rtol, u_np1);
    return IRK_OK;
}

// Advance the step without blocking; returns 1 when finished (status in *st).
int step_poll(irk_ctx *c, irk_status *st, irk_stats *stats) {
    if (!c->stepper->poll()) return 0;
    irk_status s = c->stepper->status;
    if (s == IRK_OK && hipGetLastError() != hipSuccess) s = IRK_E_DEVICE;
    c->have_stages = (s == IRK_OK);
    c->have_U = c->have_stages && c->P.sd_s == 0;
    c->st = nullptr;
    if (st) *st = s;
    if (stats) *stats = c->stepper->stats;
    return 1;
}

// Serving: resource sets made once per slot, contexts bound to them without
// allocating or waiting, and released without waiting (the server releases
// a context only after an event behind all of its work has completed).
void *res_new(int nlanes, size_t upload) {
    CtxRes *r = new (std::nothrow) CtxRes();
    if (!r) return nullptr;
    if (res_create(r, nlanes, upload) != IRK_OK) {
        res_destroy(r);
        delete r;
        return nullptr;
    }
    return r;
}

void res_free(void *r) {
    res_destroy(static_cast<CtxRes *>(r));
    delete static_cast<CtxRes *>(r);
}

// upload doubles a problem needs (0 if the plan is invalid)
size_t res_upload_need(int family, int s, const irk_operator *op, const irk_options *opt) {
    Plan *P = new (std::nothrow) Plan();
    if (!P) return 0;
    const size_t n = make_plan(family, s, op, opt, P) == IRK_OK ? upload_doubles(*P) : 0;
    delete P;
    return n;
}

irk_status create_in_res(int family, int s, const irk_operator *op, const irk_options *opt, void *ws,
                         size_t ws_bytes, hipStream_t stream, void *res, irk_ctx **out) {
    irk_ctx *c = nullptr;
    irk_status stt = ctx_new((irk_family)family, s, op, opt, ws, ws_bytes, &c);
    if (stt != IRK_OK) return stt;
    stt = ctx_init(c, stream, static_cast<CtxRes *>(res), false, false);
    if (stt != IRK_OK) {
        release(c);
        return stt;
    }
    *out = c;
    return IRK_OK;
}

// every stream of a context's resource set, then `ev` recorded on its
// Newton-level stream: behind all of the context's work
irk_status record_all_done(irk_ctx *c, hipEvent_t ev) {
    CtxRes *r = c->res;
    for (int b = 0; b < r->nlanes; ++b) {
        HIP_TRY(hipEventRecord(r->done[b], r->lane_st[b]));
        HIP_TRY(hipStreamWaitEvent(c->stream, r->done[b], 0));
        HIP_TRY(hipEventRecord(r->join[b], r->aux_st[b]));
        HIP_TRY(hipStreamWaitEvent(c->stream, r->join[b], 0));
    }
    HIP_TRY(hipEventRecord(ev, c->stream));
    return IRK_OK;
}

void ctx_free(irk_ctx *c) { release(c); }

// Shared V-cycle brokers for a server: one per precision (fp32 = 1: float).
void *broker_create(int fp32) {
    if (fp32) {
        auto *b = new (std::nothrow) PrecBroker<float>();
        if (b && !b->init()) { delete b; b = nullptr; }
        return b;
    }
    auto *b = new (std::nothrow) PrecBroker<double>();
    if (b && !b->init()) { delete b; b = nullptr; }
    return b;
}

void broker_destroy(void *b, int fp32) {
    if (fp32) delete static_cast<PrecBroker<float> *>(b);
    else delete static_cast<PrecBroker<double> *>(b);
}

int broker_flush(void *b, int fp32) {
    if (!b) return 0;
    return fp32 ? static_cast<PrecBroker<float> *>(b)->flush() : static_cast<PrecBroker<double> *>(b)->flush();
}

// Let a context's blocks join a shared broker (replacing its private one);
// false when the context does not batch (option off, or the DAE operator).
bool attach_broker(irk_ctx *c, void *fp32_broker, void *fp64_broker) {
    if (!c->P.opt.batch_mg || c->P.op.kind == IRK_OP_VSF_2D || c->P.opt.newton_like == 3 || c->P.eb.schur)
        return false;
    if (c->broker_owned) {
        if (c->P.opt.prec_fp32) delete static_cast<PrecBroker<float> *>(c->broker);
        else delete static_cast<PrecBroker<double> *>(c->broker);
    }
    c->broker = c->P.opt.prec_fp32 ? fp32_broker : fp64_broker;
    c->broker_owned = false;
    return c->broker != nullptr;
}
}  // namespace irk

extern "C" irk_status irk_step(irk_ctx *c, const double *u_n, double t_n, double dt, double tol, double *u_np1,
                               irk_stats *stats) {
    irk_status stt = step_begin(c, u_n, t_n, dt, tol, u_np1);
    if (stt != IRK_OK) return stt;
    irk_stats local;
    while (!step_poll(c, &stt, &local)) {
    }
    // the step is complete on the device (also work a failed step left on
    // the block streams)
    for (int b = 0; b < c->nlanes; ++b) {
        (void)hipStreamSynchronize(c->lanes[b].stream);
        if (c->lanes[b].aux) (void)hipStreamSynchronize(c->lanes[b].aux->stream);
    }
    (void)hipStreamSynchronize(c->stream);
    if (c->prof) prof_harvest(c);
    if (stats) *stats = local;
    return stt;
}

extern "C" irk_status irk_profile_enable(irk_ctx *c, int enable) {
    if (!c) return IRK_E_ARG;
    c->prof = enable != 0;
    c->prof_names.clear();
    c->prof_ms.clear();
    c->prof_bytes.clear();
    c->prof_launches.clear();
    c->prof_pending.clear();
    c->prof_rep.clear();
    c->ev_next = 0;
    return IRK_OK;
}

extern "C" irk_status irk_profile_replay(irk_ctx *c, const char *name, int reps, double *avg_ms,
                                         double *avg_bytes) {
    if (!c || !name || reps < 1 || !avg_ms) return IRK_E_ARG;
    auto it = c->prof_rep.find(name);
    if (it == c->prof_rep.end() || it->second.f.empty()) return IRK_E_ARG;
    auto &rp = it->second;
    HIP_TRY(hipDeviceSynchronize());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return IRK_E_DEVICE;
    }
    for (auto &f : rp.f) f();                      // warm
    irk_status st = IRK_OK;
    if (hipEventRecord(e0, rp.strm) != hipSuccess) st = IRK_E_DEVICE;
    for (int r = 0; r < reps && st == IRK_OK; ++r)
        for (auto &f : rp.f) f();
    float ms = 0.f;
    if (st == IRK_OK && (hipEventRecord(e1, rp.strm) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess))
        st = IRK_E_DEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != IRK_OK) return st;
    double by = 0;
    for (double b : rp.nbytes) by += b;
    *avg_ms = ms / ((double)reps * rp.f.size());
    if (avg_bytes) *avg_bytes = by / rp.f.size();
    return IRK_OK;
}

extern "C" int irk_profile_count(irk_ctx *c) { return c ? (int)c->prof_names.size() : 0; }

extern "C" irk_status irk_profile_entry(irk_ctx *c, int idx, char *name, int name_len, long *launches,
                                        double *total_ms, double *total_bytes) {
    if (!c || idx < 0 || idx >= (int)c->prof_names.size() || !name || name_len < 1) return IRK_E_ARG;
    std::snprintf(name, (size_t)name_len, "%s", c->prof_names[idx].c_str());
    if (launches) *launches = c->prof_launches[idx];
    if (total_ms) *total_ms = c->prof_ms[idx];
    if (total_bytes) *total_bytes = c->prof_bytes[idx];
    return IRK_OK;
}

extern "C" irk_status irk_eval_residual(irk_ctx *c, const double *u_n, double t_n, double dt, const double *K,
                                        double *F) {
    if (!c || !u_n || !K || !F || !(dt > 0)) return IRK_E_ARG;
    if (c->P.sd_s > 0) return IRK_E_UNSUPPORTED;        // stages are solved one at a time
    const Plan &P = c->P;
    const int s = P.s;
    const size_t bytes = (size_t)s * P.nf * sizeof(double);
    StageCoefs C;
    fill_stage_coefs(c, t_n, dt, &C);
    c->dt = dt;
    c->have_U = false;
    (void)hipGetLastError();
    HIP_TRY(hipMemcpyAsync(c->K, K, bytes, hipMemcpyDeviceToDevice, c->stream));
    // identity transform: Tinv = I gives F itself
    for (int i = 0; i < s * s; ++i) C.Tinv[i] = (i / s == i % s) ? 1.0 : 0.0;
    if (c->K2 && stage_residual_fused(c->dp)) {
        launch_stage_residual(c->stream, s, c->dp, u_n, c->K, nullptr, c->Y, c->U, F, C, dt, 0, c->part,
                              c->dv + DV_RES);
    } else {
        launch_stage_prep(c->stream, s, P.nf, u_n, c->K, c->Y, c->U, C, dt, 0);
        if (P.op.kind == IRK_OP_VSF_2D)
            launch_field_sums(c->stream, c->U, P.npts, 2 * s, P.npts, 1.0 / P.npts, c->part, c->dv + DV_MEANS,
                              nullptr);
        launch_residual(c->stream, s, c->dp, c->U, c->K, F, C, c->dv + DV_MEANS, c->part, c->dv + DV_RES,
                        c->dv + DV_GMAX);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->have_stages = false;
    c->have_U = true;
    return IRK_OK;
}

extern "C" irk_status irk_apply_block(irk_ctx *c, int block, const double *x, double *y) {
    if (!c || !x || !y) return IRK_E_ARG;
    if (c->P.sd_s > 0) return IRK_E_UNSUPPORTED;
    if (!c->have_U || block < 0 || block >= c->nlanes) return IRK_E_ARG;
    Lane &ln = c->lanes[block];
    (void)hipGetLastError();
    // the stage values were written on the context's stream
    HIP_TRY(hipEventRecord(c->ev_main, c->stream));
    HIP_TRY(hipStreamWaitEvent(ln.stream, c->ev_main, 0));
    block_matvec(c, ln, x, y);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(ln.stream));
    return IRK_OK;
}

extern "C" irk_status irk_get_stages(irk_ctx *c, double *K) {
    if (!c || !K) return IRK_E_ARG;
    if (!c->have_stages) return IRK_E_ARG;
    const double *src = c->P.sd_s > 0 ? reinterpret_cast<const double *>(c->ws + c->P.off_Ksd) : c->K;
    const int ns = c->P.sd_s > 0 ? c->P.sd_s : c->P.s;
    HIP_TRY(hipMemcpyAsync(K, src, (size_t)ns * c->P.nf * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return IRK_OK;
}

extern "C" void irk_destroy(irk_ctx *c) { release(c); }
