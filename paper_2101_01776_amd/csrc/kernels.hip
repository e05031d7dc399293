// HIP kernels of the IRK stage solve for gfx950 (wave64).
//
//   stage_prep      k <- k + (T Lambda (x) I) y ;  U_i = u_n + dt sum_j a_ij k_j
//   residual        F_i = M k_i - N(U_i, t_n + c_i dt) ; fhat = (T^{-1} (x) I) F ;
//                   ||F||^2 (Algorithm 1, equations (stages), (dae_stage))
//   rhs_init        k_i = N(u_n, t_n) (explicit starting candidate)
//   final_update    u_{n+1} = u_n + dt sum_i b_i k_i (equation (update))
//   block_matvec    w = D_b x for a 1x1 or 2x2 eigen-block (equation (diag_blocks))
//   dot / axpy      Arnoldi (classical Gram-Schmidt, two passes)
//   mg_*            geometric-multigrid V-cycle pieces (Chebyshev smoother,
//                   residual + full-weighting restriction, bilinear
//                   prolongation, coarsest-level solve in one work-group)
//
// Reductions are deterministic: per-work-group partial sums in a fixed order,
// then a one-work-group kernel on the same stream sums the partials in a
// fixed order.
#include <hip/hip_runtime.h>

#include <cstring>

#include "irk_internal.h"
#include "kernels.h"
#include "stencils.h"

namespace irk {

static constexpr double kPi = 3.14159265358979323846;

// blockIdx -> tile mapping that keeps consecutive tiles on one XCD (work-
// groups are dealt round-robin over the 8 XCDs, each with its own L2).
__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

// (i, j) of point p of an nx-wide grid, by 32-bit division where p fits
// (64-bit integer division is a long instruction sequence on the GPU)
__device__ __forceinline__ void point_ij(size_t p, int nx, int &i, int &j) {
    if (p <= 0xffffffffu) {
        const unsigned q = (unsigned)p / (unsigned)nx;
        i = (int)((unsigned)p - q * (unsigned)nx);
        j = (int)q;
    } else {
        i = (int)(p % nx);
        j = (int)(p / nx);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// sum over the 256 threads of a work-group; result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double *sh /* >= 4 */) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
    }
    __syncthreads();
    return r;
}

// max over the 256 threads of a work-group; result valid in thread 0
__device__ __forceinline__ double block_max(double v, double *sh /* >= 4 */) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, sh[w]);
    }
    __syncthreads();
    return r;
}

// Each work-group stores its `nv` partial sums; k_reduce_partials (launched
// right after on the same stream) adds them in a fixed order.  The kernel
// boundary makes the partials visible: no device-scope fences, which on a
// multi-XCD device write back L2.
__device__ void finish_partials(const double *myvals, int nv, double *partials, double *out,
                                unsigned *counter) {
    (void)out;
    (void)counter;
    if (threadIdx.x == 0)
        for (int k = 0; k < nv; ++k) partials[(size_t)blockIdx.x * nv + k] = myvals[k];
}

#define DOT_CHUNK 16                  // basis vectors per dot-product launch
#define RED_NV (DOT_CHUNK + 1)        // at most this many values per partial (16 dots and a norm)

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// out[k] = sum over work-groups b of partials[b * nv + k] (nv <= RED_NV) in
// a fixed order: thread t adds b = t, t + 256, ...; each wave reduces by
// shuffles; then waves 0..3 in order.  Every load of a thread is issued
// before its first add (the values sit in another XCD's L2 or in HBM).  The
// last nmax values of a partial are maxima of non-negative values instead:
// they are reduced by max and written to out2[0..nmax).  hout, hout2
// (optional): the same values again in host memory (pinned, fine-grained),
// which the host reads once an event behind this kernel has completed, with
// no copy.
__global__ void __launch_bounds__(256) k_reduce_partials(const double *__restrict__ partials, int nb, int nv,
                                                         int nmax, double *__restrict__ out,
                                                         double *__restrict__ out2, double *hout, double *hout2) {
    __shared__ double sh[4 * RED_NV];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nsum = nv - nmax;
    double a[RED_NV];
#pragma unroll
    for (int k = 0; k < RED_NV; ++k) a[k] = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const double *p = partials + (size_t)b * nv;
#pragma unroll
        for (int k = 0; k < RED_NV; ++k)
            if (k < nv) a[k] = k < nsum ? a[k] + p[k] : fmax(a[k], p[k]);
    }
#pragma unroll
    for (int k = 0; k < RED_NV; ++k)
        if (k < nv) {
            const double v = k < nsum ? wave_sum(a[k]) : wave_max(a[k]);
            if (lane == 0) sh[wid * RED_NV + k] = v;
        }
    __syncthreads();
    const int k = (int)threadIdx.x;
    if (k < nv) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
            t = k < nsum ? t + sh[w * RED_NV + k] : fmax(t, sh[w * RED_NV + k]);
        if (k < nsum) {
            out[k] = t;
            if (hout) hout[k] = t;
        } else {
            out2[k - nsum] = t;
            if (hout2) hout2[k - nsum] = t;
        }
    }
}

// Reduce nv per-thread accumulators over the work-group: every wave reduces
// with shuffles, wave leaders stage their sums in LDS, one barrier, and
// thread k < nv returns value k in `mine` (fixed order: waves 0..3).
// acc[0..nv-1] are values 0..nv-1; when with_norm, acc[NV-1] becomes value nv
// (register arrays are only indexed with compile-time constants).
template <int NV>
__device__ __forceinline__ void block_reduce_multi(const double (&acc)[NV], int nv, bool with_norm,
                                                   double *sh /* [4][NV] */, double &mine) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV - 1; ++k) {
        if (k < nv) {
            const double v = wave_sum(acc[k]);
            if (lane == 0) sh[wid * NV + k] = v;
        }
    }
    if (with_norm) {
        const double v = wave_sum(acc[NV - 1]);
        if (lane == 0) sh[wid * NV + nv] = v;
    }
    __syncthreads();
    const int nout = nv + (with_norm ? 1 : 0);
    mine = 0.0;
    if ((int)threadIdx.x < nout)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mine += sh[w * NV + threadIdx.x];
}

// Work-group partials: thread k < nv stores value k (all in wave 0).
template <int NV>
__device__ __forceinline__ void finish_multi(double mine, int nv, double *partials) {
    if ((int)threadIdx.x < nv) partials[(size_t)blockIdx.x * nv + threadIdx.x] = mine;
}

// ------------------------------------------------------------------------
// Stage preparation (pointwise over the s stage fields).
// ------------------------------------------------------------------------
template <int S>
__global__ void __launch_bounds__(IRK_WG) k_stage_prep(size_t nf, const double *__restrict__ un,
                                                       double *__restrict__ K, const double *__restrict__ Y,
                                                       double *__restrict__ U, StageCoefs C, double dt,
                                                       int fold) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < nf; e += stride) {
        double k[S];
#pragma unroll
        for (int j = 0; j < S; ++j) k[j] = K[j * nf + e];
        if (fold) {
            double y[S];
#pragma unroll
            for (int l = 0; l < S; ++l) y[l] = Y[l * nf + e];
#pragma unroll
            for (int j = 0; j < S; ++j) {
                double acc = k[j];
#pragma unroll
                for (int l = 0; l < S; ++l) acc += C.TLam[j * S + l] * y[l];
                k[j] = acc;
                K[j * nf + e] = acc;
            }
        }
        const double u = un[e];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            double acc = 0;
#pragma unroll
            for (int j = 0; j < S; ++j) acc += C.A[i * S + j] * k[j];
            U[i * nf + e] = u + dt * acc;
        }
    }
}

// ------------------------------------------------------------------------
// N(U) at one point for each operator (float64).
// ------------------------------------------------------------------------
__device__ __forceinline__ double mms_forcing(const DeviceProblem &P, int i, int j, double st, double ct) {
    const double sx = P.sinx[i], cx = P.cosx[i], sy = P.siny[j], cy = P.cosy[j];
    const double S = sx * sy;
    if (P.forcing == IRK_FORCING_MMS) {
        const double G = cx * cx * sy * sy + sx * sx * cy * cy;
        const double u = S * ct;
        const double lap = -8.0 * kPi * kPi * u;
        const double grad2 = 4.0 * kPi * kPi * G * ct * ct;
        return -S * st - ((1.0 + u * u) * lap + 2.0 * u * grad2);
    }
    // discrete manufactured solution: f = du*/dt - N_h(u*)
    const int nx = P.g.nx, ny = P.g.ny;
    const int ip = wrapm(i + 1, nx), im = wrapm(i - 1, nx), jp = wrapm(j + 1, ny), jm = wrapm(j - 1, ny);
    const double inv_h2 = 1.0 / (P.g.h * P.g.h);
    const double fl = nldiff_flux5(S * ct, P.sinx[ip] * sy * ct, P.sinx[im] * sy * ct,
                                   sx * P.siny[jp] * ct, sx * P.siny[jm] * ct, inv_h2);
    return -S * st - fl;
}

// ------------------------------------------------------------------------
// Residual F_i = M k_i - N(U_i), transformed residual and ||F||^2.
// Layout: U, K, Fh are [S][nvar][npts]; means (VSF) = [S][2] (omega, psi).
// ------------------------------------------------------------------------
// VSF: also the largest one-cell difference of every stage's streamfunction,
// max(|Psi(i+1,j) - Psi(i,j)|, |Psi(i,j+1) - Psi(i,j)|) (it bounds the
// advective coefficients of the vorticity operator on every multigrid level),
// as S more per-work-group values reduced by max.
template <int S, int OP>
__global__ void __launch_bounds__(IRK_WG) k_residual(DeviceProblem P, const double *__restrict__ U,
                                                     const double *__restrict__ K, double *__restrict__ Fh,
                                                     StageCoefs C, const double *__restrict__ means,
                                                     double *partials) {
    const int nx = P.g.nx, ny = P.g.ny;
    const size_t npts = (size_t)nx * ny;
    constexpr int NV = (OP == IRK_OP_VSF_2D) ? 2 : 1;
    const size_t nf = NV * npts;
    const double h = P.g.h, inv_h2 = 1.0 / (h * h);
    double sumsq = 0.0, abssq = 0.0;
    double gmax[S];
#pragma unroll
    for (int st = 0; st < S; ++st) gmax[st] = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t p = (size_t)xcd_block() * blockDim.x + threadIdx.x; p < npts; p += stride) {
        int i, j;
        point_ij(p, nx, i, j);
        double F[S][NV];
#pragma unroll
        for (int st = 0; st < S; ++st) {
            const double *Ui = U + st * nf;
            // a: sum of the magnitudes of the terms of F (its rounding scale)
            if constexpr (OP == IRK_OP_NLDIFF_2D) {
                const int ip = wrapm(i + 1, nx), im = wrapm(i - 1, nx), jp = wrapm(j + 1, ny), jm = wrapm(j - 1, ny);
                const double uc = Ui[p], ue = Ui[j * nx + ip], uw = Ui[j * nx + im], un = Ui[jp * nx + i], us = Ui[jm * nx + i];
                double N = nldiff_flux5(uc, ue, uw, un, us, inv_h2);
                double a = nldiff_flux5_abs(uc, ue, uw, un, us, inv_h2);
                if (P.forcing != IRK_FORCING_NONE) {
                    const double f = mms_forcing(P, i, j, C.sin_t[st], C.cos_t[st]);
                    N += f;
                    a += fabs(f);
                }
                const double k = K[st * nf + p];
                F[st][0] = k - N;
                a += fabs(k);
                abssq += a * a;
            } else if constexpr (OP == IRK_OP_BURGERS_1D) {
                const int ip = wrapm(i + 1, nx), im = wrapm(i - 1, nx);
                const double ue = Ui[ip], uw = Ui[im], uc = Ui[p];
                const double N = -(ue * ue - uw * uw) / (4.0 * h) + P.g.nu * (ue - 2.0 * uc + uw) * inv_h2;
                const double k = K[st * nf + p];
                F[st][0] = k - N;
                const double a = fabs(k) + (ue * ue + uw * uw) / (4.0 * h) +
                                 P.g.nu * (fabs(ue) + 2.0 * fabs(uc) + fabs(uw)) * inv_h2;
                abssq += a * a;
            } else {
                double w[3][3], ps[3][3];
                load3x3(Ui, i, j, nx, ny, w);
                load3x3(Ui + npts, i, j, nx, ny, ps);
                const double Nw = arakawa9(ps, w, inv_h2 / 12.0) + P.g.nu * lap5(w, inv_h2);
                const double k = K[st * nf + p];
                F[st][0] = k - Nw;
                // algebraic rows: 0 * l_i - (Lap Psi + Omega - mean Omega - mean Psi)
                F[st][1] = -(lap5(ps, inv_h2) + w[1][1] - means[2 * st] - means[2 * st + 1]);
                const double a0 = fabs(k) + arakawa9_abs(ps, w, inv_h2 / 12.0) +
                                  P.g.nu * (fabs(w[1][2]) + fabs(w[1][0]) + fabs(w[2][1]) + fabs(w[0][1]) + 4.0 * fabs(w[1][1])) * inv_h2;
                const double a1 = (fabs(ps[1][2]) + fabs(ps[1][0]) + fabs(ps[2][1]) + fabs(ps[0][1]) + 4.0 * fabs(ps[1][1])) * inv_h2 +
                                  fabs(w[1][1]) + fabs(means[2 * st]) + fabs(means[2 * st + 1]);
                abssq += a0 * a0 + a1 * a1;
                gmax[st] = fmax(gmax[st], fmax(fabs(ps[1][2] - ps[1][1]), fabs(ps[2][1] - ps[1][1])));
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
#pragma unroll
            for (int st = 0; st < S; ++st) sumsq += F[st][v] * F[st][v];
#pragma unroll
            for (int m = 0; m < S; ++m) {
                double acc = 0;
#pragma unroll
                for (int st = 0; st < S; ++st) acc += C.Tinv[m * S + st] * F[st][v];
                Fh[m * nf + v * npts + p] = acc;
            }
        }
    }
    __shared__ double sh[8];
    double tot[2 + S];
    tot[0] = block_sum(sumsq, sh);
    tot[1] = block_sum(abssq, sh);
    constexpr int NVAL = (OP == IRK_OP_VSF_2D) ? 2 + S : 2;
    if constexpr (OP == IRK_OP_VSF_2D) {
#pragma unroll
        for (int st = 0; st < S; ++st) tot[2 + st] = block_max(gmax[st], sh);
    }
    finish_partials(tot, NVAL, partials, nullptr, nullptr);
}

// ------------------------------------------------------------------------
// Stage values and residual in one sweep (nonlinear diffusion, Burgers):
// for every point of a TX x TY tile and its one-cell halo
//   k_j <- K_j + sum_l (T Lambda)_jl Y_l   (the fold of the previous block
//                                           solves, when fold != 0)
//   U_i  = u_n + dt sum_j a_ij k_j          (in LDS)
// then, on the tile, F_i = k_i - N(U_i, t_n + c_i dt), fhat = (T^{-1} (x) I) F,
// ||F||^2 and the rounding scale of F as per-work-group partials.  U and the
// folded stages go to HBM (Kout: a different buffer than K, which
// neighbouring tiles still read in their halos); fields are read once from
// HBM (the halo from L2): (2s+1) reads and 3s writes per point with the
// fold, (s+1) and 2s without.
// ------------------------------------------------------------------------
template <int S, int OP, int TX, int TY>
__global__ void __launch_bounds__(IRK_WG) k_stage_residual(DeviceProblem P, const double *__restrict__ un,
                                                           const double *__restrict__ K, double *__restrict__ Kout,
                                                           const double *__restrict__ Y, double *__restrict__ U,
                                                           double *__restrict__ Fh, StageCoefs C, double dt,
                                                           int fold, double *partials) {
    constexpr bool TWO_D = (OP == IRK_OP_NLDIFF_2D);
    constexpr int W = TX + 2, HH = TWO_D ? TY + 2 : 1, NW = W * HH;
    static_assert(TX * TY == IRK_WG, "one interior point per thread");
    __shared__ double Us[S][NW];
    __shared__ double Ks[S][TX * TY];
    const int nx = P.g.nx, ny = P.g.ny;
    const size_t nf = (size_t)nx * ny;
    const int tiles_x = (nx + TX - 1) / TX;
    const int tile = xcd_block();
    const int tyi = tile / tiles_x, txi = tile - tyi * tiles_x;
    const int i0 = txi * TX, j0 = TWO_D ? tyi * TY : 0;
    // window: every point of the tile and its halo (periodic wrap)
    for (int q = threadIdx.x; q < NW; q += blockDim.x) {
        const int ia = q % W, ib = q / W;
        const int ri = i0 + ia - 1, rj = TWO_D ? j0 + ib - 1 : 0;
        // periodic wrap without integer division (ri >= -1: one step up,
        // and usually at most one step down)
        int gi = ri < 0 ? ri + nx : ri, gj = TWO_D ? (rj < 0 ? rj + ny : rj) : 0;
        while (gi >= nx) gi -= nx;
        while (gj >= ny) gj -= ny;
        const size_t g = (size_t)gj * nx + gi;
        double k[S];
#pragma unroll
        for (int j = 0; j < S; ++j) k[j] = K[j * nf + g];
        const double u = un[g];
        if (fold) {
            double y[S];
#pragma unroll
            for (int l = 0; l < S; ++l) y[l] = Y[l * nf + g];
#pragma unroll
            for (int j = 0; j < S; ++j) {
                double acc = k[j];
#pragma unroll
                for (int l = 0; l < S; ++l) acc += C.TLam[j * S + l] * y[l];
                k[j] = acc;
            }
        }
#pragma unroll
        for (int i = 0; i < S; ++i) {
            double acc = 0;
#pragma unroll
            for (int j = 0; j < S; ++j) acc += C.A[i * S + j] * k[j];
            Us[i][q] = u + dt * acc;
        }
        const bool inner = ia >= 1 && ia <= TX && (!TWO_D || (ib >= 1 && ib <= TY));
        if (inner) {
            const int pl = (TWO_D ? (ib - 1) * TX : 0) + ia - 1;
#pragma unroll
            for (int j = 0; j < S; ++j) Ks[j][pl] = k[j];
            if (fold && ri < nx && rj < ny) {
#pragma unroll
                for (int j = 0; j < S; ++j) Kout[j * nf + g] = k[j];
            }
        }
    }
    __syncthreads();
    const int pl = threadIdx.x;
    const int li = pl % TX, lj = TWO_D ? pl / TX : 0;
    const int gi = i0 + li, gj = j0 + lj;
    double sumsq = 0.0, abssq = 0.0;
    if (gi < nx && gj < ny) {
        const size_t g = (size_t)gj * nx + gi;
        const int c = (TWO_D ? (lj + 1) * W : 0) + li + 1;
        const double h = P.g.h, inv_h2 = 1.0 / (h * h);
        double F[S];
#pragma unroll
        for (int st = 0; st < S; ++st) {
            const double uc = Us[st][c], ue = Us[st][c + 1], uw = Us[st][c - 1];
            const double k = Ks[st][pl];
            if constexpr (TWO_D) {
                const double unn = Us[st][c + W], us = Us[st][c - W];
                double N = nldiff_flux5(uc, ue, uw, unn, us, inv_h2);
                double a = nldiff_flux5_abs(uc, ue, uw, unn, us, inv_h2);
                if (P.forcing != IRK_FORCING_NONE) {
                    const double f = mms_forcing(P, gi, gj, C.sin_t[st], C.cos_t[st]);
                    N += f;
                    a += fabs(f);
                }
                F[st] = k - N;
                a += fabs(k);
                abssq += a * a;
            } else {
                const double N = -(ue * ue - uw * uw) / (4.0 * h) + P.g.nu * (ue - 2.0 * uc + uw) * inv_h2;
                F[st] = k - N;
                const double a = fabs(k) + (ue * ue + uw * uw) / (4.0 * h) +
                                 P.g.nu * (fabs(ue) + 2.0 * fabs(uc) + fabs(uw)) * inv_h2;
                abssq += a * a;
            }
            U[st * nf + g] = uc;
        }
#pragma unroll
        for (int st = 0; st < S; ++st) sumsq += F[st] * F[st];
#pragma unroll
        for (int m = 0; m < S; ++m) {
            double acc = 0;
#pragma unroll
            for (int st = 0; st < S; ++st) acc += C.Tinv[m * S + st] * F[st];
            Fh[m * nf + g] = acc;
        }
    }
    __shared__ double sh[8];
    double tot[2];
    tot[0] = block_sum(sumsq, sh);
    tot[1] = block_sum(abssq, sh);
    finish_partials(tot, 2, partials, nullptr, nullptr);
}

// k_i <- N(u_n, t_n) on differential rows, 0 on algebraic rows (explicit candidate for the
// starting stage vectors)
template <int S, int OP>
__global__ void __launch_bounds__(IRK_WG) k_rhs_init(DeviceProblem P, const double *__restrict__ un,
                                                     double *__restrict__ K, double st_n, double ct_n) {
    const int nx = P.g.nx, ny = P.g.ny;
    const size_t npts = (size_t)nx * ny;
    constexpr int NV = (OP == IRK_OP_VSF_2D) ? 2 : 1;
    const size_t nf = NV * npts;
    const double h = P.g.h, inv_h2 = 1.0 / (h * h);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t p = (size_t)xcd_block() * blockDim.x + threadIdx.x; p < npts; p += stride) {
        int i, j;
        point_ij(p, nx, i, j);
        double N;
        if constexpr (OP == IRK_OP_NLDIFF_2D) {
            const int ip = wrapm(i + 1, nx), im = wrapm(i - 1, nx), jp = wrapm(j + 1, ny), jm = wrapm(j - 1, ny);
            N = nldiff_flux5(un[p], un[j * nx + ip], un[j * nx + im], un[jp * nx + i], un[jm * nx + i], inv_h2);
            if (P.forcing != IRK_FORCING_NONE) N += mms_forcing(P, i, j, st_n, ct_n);
        } else if constexpr (OP == IRK_OP_BURGERS_1D) {
            const int ip = wrapm(i + 1, nx), im = wrapm(i - 1, nx);
            N = -(un[ip] * un[ip] - un[im] * un[im]) / (4.0 * h) + P.g.nu * (un[ip] - 2.0 * un[p] + un[im]) * inv_h2;
        } else {
            double w[3][3], ps[3][3];
            load3x3(un, i, j, nx, ny, w);
            load3x3(un + npts, i, j, nx, ny, ps);
            N = arakawa9(ps, w, inv_h2 / 12.0) + P.g.nu * lap5(w, inv_h2);
        }
#pragma unroll
        for (int st = 0; st < S; ++st) {
            K[st * nf + p] = N;
            if constexpr (NV == 2) K[st * nf + npts + p] = 0.0;
        }
    }
}

template <int S>
__global__ void __launch_bounds__(IRK_WG) k_final_update(size_t nf, const double *__restrict__ un,
                                                         const double *__restrict__ K, double *__restrict__ out,
                                                         StageCoefs C, double dt) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < nf; e += stride) {
        double acc = 0;
#pragma unroll
        for (int i = 0; i < S; ++i) acc += C.b[i] * K[i * nf + e];
        out[e] = un[e] + dt * acc;
    }
}

// Kx_i = sum_j W_ij K_j over the s stage fields (the extrapolated starting
// stage vectors; W row-major s x s, passed in StageCoefs.A)
template <int S>
__global__ void __launch_bounds__(IRK_WG) k_stage_extrap(size_t nf, const double *__restrict__ K,
                                                         double *__restrict__ Kx, StageCoefs W) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < nf; e += stride) {
        double k[S];
#pragma unroll
        for (int j = 0; j < S; ++j) k[j] = K[j * nf + e];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            double acc = 0;
#pragma unroll
            for (int j = 0; j < S; ++j) acc += W.A[i * S + j] * k[j];
            Kx[i * nf + e] = acc;
        }
    }
}

// sums of `nfields` consecutive fields of length len (VSF means)
__global__ void __launch_bounds__(IRK_WG) k_field_sums(const double *__restrict__ X, size_t ld, int nfields,
                                                       size_t len, double scale, double *partials, double *out,
                                                       unsigned *counter) {
    constexpr int NF = 2 * IRK_MAX_STAGES, UN = 4;
    double acc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    // UN elements per field loaded before the first add (same order as one
    // at a time)
    for (; e + (UN - 1) * stride < len; e += UN * stride) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if (f < nfields) {
                double x[UN];
#pragma unroll
                for (int u = 0; u < UN; ++u) x[u] = X[f * ld + e + u * stride];
#pragma unroll
                for (int u = 0; u < UN; ++u) acc[f] += x[u];
            }
    }
    for (; e < len; e += stride)
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if (f < nfields) acc[f] += X[f * ld + e];
    __shared__ double sh[8];
    double tot[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f)
        if (f < nfields) tot[f] = scale * block_sum(acc[f], sh);
    finish_partials(tot, nfields, partials, out, counter);
}

// sums of two fields of length len at unrelated addresses
__global__ void __launch_bounds__(IRK_WG) k_field_sums2(const double *__restrict__ X0, const double *__restrict__ X1,
                                                        size_t len, double scale, double *partials) {
    double a0 = 0.0, a1 = 0.0;
    constexpr int UN = 4;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; e + (UN - 1) * stride < len; e += UN * stride) {
        double x0[UN], x1[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            x0[u] = X0[e + u * stride];
            x1[u] = X1[e + u * stride];
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            a0 += x0[u];
            a1 += x1[u];
        }
    }
    for (; e < len; e += stride) {
        a0 += X0[e];
        a1 += X1[e];
    }
    __shared__ double sh[8];
    double tot[2];
    tot[0] = scale * block_sum(a0, sh);
    tot[1] = scale * block_sum(a1, sh);
    finish_partials(tot, 2, partials, nullptr, nullptr);
}

// ------------------------------------------------------------------------
// Eigen-block matvec w = D_b x (float64).
//   width 1: w = eta M x - dt L_a x
//   width 2: w_a = eta M x_a + c12 M x_b - dt L_a x_a
//            w_b = c21 M x_a + eta M x_b - dt L_b x_b
// (eigenbasis: c12 = beta, c21 = -beta; real Schur basis: the standardized
// block's phi and -beta^2/phi)
// For VSF each component is (omega, psi); omega rows use the Picard
// linearization K(Psi_m) = J_A(Psi_m, .) + nu Lap, psi rows
// -dt [(x_omega - mean x_omega) + Lap x_psi - mean x_psi] (mass 0).
// ------------------------------------------------------------------------
// One point p of the eigen-block matvec: writes w at p (width * NV fields)
// and returns the written values in wv (component-major: comp * NV + var).
template <int OP>
__device__ __forceinline__ void block_matvec_point(const DeviceProblem &P, int width, const BlockLam &lam, double dt,
                                                   const double *__restrict__ Ua, const double *__restrict__ Ub,
                                                   const double *__restrict__ x, double *__restrict__ w,
                                                   const double *__restrict__ xmeans, size_t p, double (&wv)[4]) {
    const int nx = P.g.nx, ny = P.g.ny;
    const size_t npts = (size_t)nx * ny;
    constexpr int NV = (OP == IRK_OP_VSF_2D) ? 2 : 1;
    const size_t nf = NV * npts;
    const double h = P.g.h, inv_h2 = 1.0 / (h * h);
    int i, j;
    point_ij(p, nx, i, j);
    double Lx[2], xc[2];
    for (int comp = 0; comp < width; ++comp) {
        const double *Uc = comp == 0 ? Ua : Ub;
        const double *xx = x + comp * nf;
        double lx, ld;
        if constexpr (OP == IRK_OP_NLDIFF_2D) nldiff_lin<double, true>(Uc, xx, i, j, nx, ny, inv_h2, lx, ld);
        else if constexpr (OP == IRK_OP_BURGERS_1D) burgers_lin<double, true>(Uc, xx, i, nx, h, P.g.nu, lx, ld);
        else vsf_omega_lin<double, true>(Uc + npts, xx, i, j, nx, ny, h, P.g.nu, lx, ld);
        Lx[comp] = lx;
        xc[comp] = xx[p];
    }
    if (width == 1) {
        wv[0] = lam.eta * xc[0] - dt * Lx[0];
        w[p] = wv[0];
    } else {
        wv[0] = lam.eta * xc[0] + lam.c12 * xc[1] - dt * Lx[0];
        wv[NV] = lam.c21 * xc[0] + lam.eta * xc[1] - dt * Lx[1];
        w[p] = wv[0];
        w[nf + p] = wv[NV];
    }
    if constexpr (NV == 2) {
        for (int comp = 0; comp < width; ++comp) {
            const double *xx = x + comp * nf;
            double lp, ld;
            poisson_lin<double, true>(xx + npts, i, j, nx, ny, h, lp, ld);
            const double mw = xmeans[2 * comp], mp = xmeans[2 * comp + 1];
            const double v = -dt * ((xc[comp] - mw) + lp - mp);
            wv[comp * NV + 1] = v;
            w[comp * nf + npts + p] = v;
        }
    }
}

template <int OP>
__global__ void __launch_bounds__(IRK_WG) k_block_matvec(DeviceProblem P, int width, BlockLam lam,
                                                         double dt, const double *__restrict__ Ua,
                                                         const double *__restrict__ Ub,
                                                         const double *__restrict__ x, double *__restrict__ w,
                                                         const double *__restrict__ xmeans) {
    const size_t npts = (size_t)P.g.nx * P.g.ny;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t p = (size_t)xcd_block() * blockDim.x + threadIdx.x; p < npts; p += stride) {
        double wv[4];
        block_matvec_point<OP>(P, width, lam, dt, Ua, Ub, x, w, xmeans, p, wv);
    }
}

// The DAE's eigen-block matvec over 64 x 4 tiles: a work-group stages, for
// each component, the linearization's streamfunction and both variables of
// x over its tile and a one-cell halo (periodic wrap) in LDS, then every
// thread evaluates its point from there -- its 3x3 neighbourhoods come from
// LDS instead of three times nine loads through the caches.  The arithmetic
// is block_matvec_point's (arakawa9, lap5, the 5-point Laplacian).
constexpr int VM_TX = 64, VM_TY = IRK_WG / VM_TX;
__global__ void __launch_bounds__(IRK_WG) k_block_matvec_vsf(DeviceProblem P, int width, BlockLam lam, double dt,
                                                             const double *__restrict__ Ua,
                                                             const double *__restrict__ Ub,
                                                             const double *__restrict__ x, double *__restrict__ w,
                                                             const double *__restrict__ xmeans) {
    constexpr int HX = VM_TX + 2, HY = VM_TY + 2, HN = HX * HY, PT = (HN + IRK_WG - 1) / IRK_WG;
    __shared__ double sp[2][HN], so[2][HN], sq[2][HN];
    const int nx = P.g.nx, ny = P.g.ny;
    const size_t npts = (size_t)nx * ny, nf = 2 * npts;
    const int tiles_x = (nx + VM_TX - 1) / VM_TX;
    const int t = xcd_block();
    const int ty = t / tiles_x, tx = t - ty * tiles_x;
    const int i0 = tx * VM_TX, j0 = ty * VM_TY;
    for (int comp = 0; comp < width; ++comp) {
        const double *Psi = (comp == 0 ? Ua : Ub) + npts;
        const double *xo = x + comp * nf, *xp = xo + npts;
        double vp[PT], vo[PT], vq[PT];
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int q = u * IRK_WG + (int)threadIdx.x;
            if (q < HN) {
                const int hj = q / HX, hi = q - hj * HX;
                int gi = i0 - 1 + hi, gj = j0 - 1 + hj;
                gi = gi < 0 ? gi + nx : (gi >= nx ? gi % nx : gi);
                gj = gj < 0 ? gj + ny : (gj >= ny ? gj % ny : gj);
                const size_t e = (size_t)gj * nx + gi;
                vp[u] = Psi[e];
                vo[u] = xo[e];
                vq[u] = xp[e];
            }
        }
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int q = u * IRK_WG + (int)threadIdx.x;
            if (q < HN) {
                sp[comp][q] = vp[u];
                so[comp][q] = vo[u];
                sq[comp][q] = vq[u];
            }
        }
    }
    __syncthreads();
    const int li = (int)threadIdx.x % VM_TX, lj = (int)threadIdx.x / VM_TX;
    const int gi = i0 + li, gj = j0 + lj;
    if (gi >= nx || gj >= ny) return;
    const size_t p = (size_t)gj * nx + gi;
    const double h = P.g.h, inv_h2 = 1.0 / (h * h);
    double Lx[2], xc[2];
    for (int comp = 0; comp < width; ++comp) {
        double pp[3][3], ww[3][3];
#pragma unroll
        for (int dj = 0; dj < 3; ++dj)
#pragma unroll
            for (int di = 0; di < 3; ++di) {
                pp[dj][di] = sp[comp][(lj + dj) * HX + li + di];
                ww[dj][di] = so[comp][(lj + dj) * HX + li + di];
            }
        Lx[comp] = arakawa9(pp, ww, inv_h2 / 12.0) + P.g.nu * lap5(ww, inv_h2);
        xc[comp] = ww[1][1];
    }
    if (width == 1) {
        w[p] = lam.eta * xc[0] - dt * Lx[0];
    } else {
        w[p] = lam.eta * xc[0] + lam.c12 * xc[1] - dt * Lx[0];
        w[nf + p] = lam.c21 * xc[0] + lam.eta * xc[1] - dt * Lx[1];
    }
    for (int comp = 0; comp < width; ++comp) {
        const double *q = sq[comp];
        const int c0 = (lj + 1) * HX + li + 1;
        const double lp = (q[c0 + 1] + q[c0 - 1] + q[c0 + HX] + q[c0 - HX] - 4.0 * q[c0]) * inv_h2;
        const double mw = xmeans[2 * comp], mp = xmeans[2 * comp + 1];
        w[comp * nf + npts + p] = -dt * ((xc[comp] - mw) + lp - mp);
    }
}

// The matvec fused with the first Gram-Schmidt pass: w = D_b x and, per
// work-group, the partial sums of (V_k, w) for k < nv (the basis vectors
// V_k at stride ldv, each of width * NV fields), so w is not read back for
// the first projection.  A separate reduction of the partials follows.
template <int OP, int NVMAX>
__global__ void __launch_bounds__(IRK_WG) k_block_matvec_dot(DeviceProblem P, int width, BlockLam lam,
                                                             double dt, const double *__restrict__ Ua,
                                                             const double *__restrict__ Ub,
                                                             const double *__restrict__ x, double *__restrict__ w,
                                                             const double *__restrict__ xmeans,
                                                             const double *__restrict__ V, size_t ldv, int nv,
                                                             double *partials) {
    constexpr int NV = (OP == IRK_OP_VSF_2D) ? 2 : 1;
    const size_t npts = (size_t)P.g.nx * P.g.ny;
    const int nfld = width * NV;
    double acc[NVMAX + 1];
#pragma unroll
    for (int k = 0; k <= NVMAX; ++k) acc[k] = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t p = (size_t)xcd_block() * blockDim.x + threadIdx.x; p < npts; p += stride) {
        double wv[4];
        block_matvec_point<OP>(P, width, lam, dt, Ua, Ub, x, w, xmeans, p, wv);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            if (f < nfld) {
                const size_t e = (size_t)f * npts + p;
#pragma unroll
                for (int k = 0; k < NVMAX; ++k)
                    if (k < nv) acc[k] += V[k * ldv + e] * wv[f];
            }
        }
    }
    __shared__ double sh[4 * (NVMAX + 1)];
    double mine;
    block_reduce_multi<NVMAX + 1>(acc, nv, false, sh, mine);
    finish_multi<NVMAX + 1>(mine, nv, partials);
}

// The nonlinear-diffusion matvec fused with the first Gram-Schmidt pass over
// 64 x 4 tiles: each component's linearization field U and x over the tile
// and its one-cell halo (periodic wrap) staged in LDS, the point's 5-point
// stencils read from there (nldiff_lin's arithmetic), then the partial sums
// of (V_k, w), k < nv <= NVMAX, one per work-group and k.
template <int NVMAX>
__global__ void __launch_bounds__(IRK_WG) k_block_matvec_dot_nl(DeviceProblem P, int width, BlockLam lam,
                                                                double dt, const double *__restrict__ Ua,
                                                                const double *__restrict__ Ub,
                                                                const double *__restrict__ x,
                                                                double *__restrict__ w,
                                                                const double *__restrict__ V, size_t ldv, int nv,
                                                                double *partials) {
    constexpr int HX = VM_TX + 2, HY = VM_TY + 2, HN = HX * HY, PT = (HN + IRK_WG - 1) / IRK_WG;
    __shared__ double su[2][HN], sx[2][HN];
    const int nx = P.g.nx, ny = P.g.ny;
    const size_t npts = (size_t)nx * ny;
    const int tiles_x = (nx + VM_TX - 1) / VM_TX;
    const int t = xcd_block();
    const int ty = t / tiles_x, tx = t - ty * tiles_x;
    const int i0 = tx * VM_TX, j0 = ty * VM_TY;
    for (int comp = 0; comp < width; ++comp) {
        const double *Uc = comp == 0 ? Ua : Ub;
        const double *xc = x + comp * npts;
        double vu[PT], vx[PT];
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int q = u * IRK_WG + (int)threadIdx.x;
            if (q < HN) {
                const int hj = q / HX, hi = q - hj * HX;
                int gi = i0 - 1 + hi, gj = j0 - 1 + hj;
                gi = gi < 0 ? gi + nx : (gi >= nx ? gi % nx : gi);
                gj = gj < 0 ? gj + ny : (gj >= ny ? gj % ny : gj);
                const size_t e = (size_t)gj * nx + gi;
                vu[u] = Uc[e];
                vx[u] = xc[e];
            }
        }
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int q = u * IRK_WG + (int)threadIdx.x;
            if (q < HN) {
                su[comp][q] = vu[u];
                sx[comp][q] = vx[u];
            }
        }
    }
    __syncthreads();
    const int li = (int)threadIdx.x % VM_TX, lj = (int)threadIdx.x / VM_TX;
    const int gi = i0 + li, gj = j0 + lj;
    double acc[NVMAX + 1];
#pragma unroll
    for (int k = 0; k <= NVMAX; ++k) acc[k] = 0.0;
    if (gi < nx && gj < ny) {
        const size_t p = (size_t)gj * nx + gi;
        const double h = P.g.h, inv_h2 = 1.0 / (h * h);
        const int c0 = (lj + 1) * HX + li + 1;
        const int nb[4] = {c0 + 1, c0 - 1, c0 + HX, c0 - HX};     // e, w, n, s as nldiff_lin
        double Lx[2], xcv[2], wv[2];
        for (int comp = 0; comp < width; ++comp) {
            const double uc = su[comp][c0], xcc = sx[comp][c0];
            double lx = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double un = su[comp][nb[q]];
                const double kf = 1.0 + 0.5 * (uc * uc + un * un);
                const double du = un - uc;
                const double xn = sx[comp][nb[q]];
                lx += kf * (xn - xcc) + du * (uc * xcc + un * xn);
            }
            Lx[comp] = lx * inv_h2;
            xcv[comp] = xcc;
        }
        if (width == 1) {
            wv[0] = lam.eta * xcv[0] - dt * Lx[0];
            w[p] = wv[0];
        } else {
            wv[0] = lam.eta * xcv[0] + lam.c12 * xcv[1] - dt * Lx[0];
            wv[1] = lam.c21 * xcv[0] + lam.eta * xcv[1] - dt * Lx[1];
            w[p] = wv[0];
            w[npts + p] = wv[1];
        }
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            if (f < width) {
                const size_t e = (size_t)f * npts + p;
#pragma unroll
                for (int k = 0; k < NVMAX; ++k)
                    if (k < nv) acc[k] += V[k * ldv + e] * wv[f];
            }
        }
    }
    __shared__ double shr[4 * (NVMAX + 1)];
    double mine;
    block_reduce_multi<NVMAX + 1>(acc, nv, false, shr, mine);
    finish_multi<NVMAX + 1>(mine, nv, partials);
}

// Eigen-block operator with stage-weighted linearizations (Newton-like (2),
// (3)): L_kb = L(U_k) x_b at the point for every stage k and component b,
//   coupling = 0:  w_a = eta M x_a (+ c12 M x_1 | + c21 M x_0)
//                        - dt sum_b sum_k W[a][b][k] L_kb
//                  (the algebraic rows of the DAE as in k_block_matvec);
//   coupling = 1:  w = -c21 M x_0 + dt sum_k W[1][0][k] L_k0 on the
//                  differential variable only (the negated (2,1) block of the
//                  pair applied to x_0: the second row's right-hand side of
//                  the block-triangular preconditioner).
template <int OP, int S>
__global__ void __launch_bounds__(IRK_WG) k_block_matvec_w(DeviceProblem P, int width, BlockLam lam,
                                                           double dt, const double *__restrict__ U,
                                                           BlockWeights W, const double *__restrict__ x,
                                                           double *__restrict__ w,
                                                           const double *__restrict__ xmeans, int coupling) {
    const int nx = P.g.nx, ny = P.g.ny;
    const size_t npts = (size_t)nx * ny;
    constexpr int NV = (OP == IRK_OP_VSF_2D) ? 2 : 1;
    const size_t nf = NV * npts;
    const double h = P.g.h, inv_h2 = 1.0 / (h * h);
    const int nin = coupling ? 1 : width;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t p = (size_t)xcd_block() * blockDim.x + threadIdx.x; p < npts; p += stride) {
        int i, j;
        point_ij(p, nx, i, j);
        double acc[2] = {0.0, 0.0}, xc[2] = {0.0, 0.0};
        for (int b = 0; b < nin; ++b) {
            const double *xx = x + b * nf;
            xc[b] = xx[p];
#pragma unroll
            for (int k = 0; k < S; ++k) {
                const double *Uk = U + (size_t)k * nf;
                double lx, ld;
                if constexpr (OP == IRK_OP_NLDIFF_2D) nldiff_lin<double, true>(Uk, xx, i, j, nx, ny, inv_h2, lx, ld);
                else if constexpr (OP == IRK_OP_BURGERS_1D) burgers_lin<double, true>(Uk, xx, i, nx, h, P.g.nu, lx, ld);
                else vsf_omega_lin<double, true>(Uk + npts, xx, i, j, nx, ny, h, P.g.nu, lx, ld);
                if (coupling) {
                    acc[0] += W.w[1][0][k] * lx;
                } else {
                    acc[0] += W.w[0][b][k] * lx;
                    if (width == 2) acc[1] += W.w[1][b][k] * lx;
                }
            }
        }
        if (coupling) {
            w[p] = -lam.c21 * xc[0] + dt * acc[0];
            continue;
        }
        if (width == 1) {
            w[p] = lam.eta * xc[0] - dt * acc[0];
        } else {
            w[p] = lam.eta * xc[0] + lam.c12 * xc[1] - dt * acc[0];
            w[nf + p] = lam.c21 * xc[0] + lam.eta * xc[1] - dt * acc[1];
        }
        if constexpr (NV == 2) {
            for (int comp = 0; comp < width; ++comp) {
                const double *xx = x + comp * nf;
                double lp, ld;
                poisson_lin<double, true>(xx + npts, i, j, nx, ny, h, lp, ld);
                const double mw = xmeans[2 * comp], mp = xmeans[2 * comp + 1];
                w[comp * nf + npts + p] = -dt * ((xc[comp] - mw) + lp - mp);
            }
        }
    }
}

// ------------------------------------------------------------------------
// Block back-substitution in the real Schur basis (ODE operators): the
// right-hand side of block i loses the coupling to the solved block j,
//   f_a <- f_a - sum_b (R_ab y_b - dt sum_k W[a][b][k] L(U_k) y_b),
// a < wi, b < wj (the Jacobian terms only when C.jac).
// ------------------------------------------------------------------------
template <int OP, int S>
__global__ void __launch_bounds__(IRK_WG) k_block_couple(DeviceProblem P, BlockCouple C, double dt,
                                                         const double *__restrict__ U, const double *__restrict__ y,
                                                         double *__restrict__ f) {
    const int nx = P.g.nx, ny = P.g.ny;
    const size_t nf = (size_t)nx * ny;
    const double h = P.g.h, inv_h2 = 1.0 / (h * h);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t p = (size_t)xcd_block() * blockDim.x + threadIdx.x; p < nf; p += stride) {
        int i, j;
        point_ij(p, nx, i, j);
        double acc[2] = {0.0, 0.0};
        for (int b = 0; b < C.wj; ++b) {
            const double *yb = y + b * nf;
            const double yc = yb[p];
            for (int a = 0; a < C.wi; ++a) acc[a] += C.R[a][b] * yc;
            if (C.jac) {
#pragma unroll
                for (int k = 0; k < S; ++k) {
                    const double *Uk = U + (size_t)k * nf;
                    double lx, ld;
                    if constexpr (OP == IRK_OP_NLDIFF_2D) nldiff_lin<double, true>(Uk, yb, i, j, nx, ny, inv_h2, lx, ld);
                    else burgers_lin<double, true>(Uk, yb, i, nx, h, P.g.nu, lx, ld);
                    for (int a = 0; a < C.wi; ++a) acc[a] -= dt * C.W.w[a][b][k] * lx;
                }
            }
        }
        for (int a = 0; a < C.wi; ++a) f[a * nf + p] -= acc[a];
    }
}

// ------------------------------------------------------------------------
// Arnoldi kernels
// ------------------------------------------------------------------------
// out[k] = <V_k, w> for k < nv (nv <= 16); out[nv] = <w, w> when with_norm
// (The reduction kernels run on at most 512 work-groups, so each thread
// covers many elements: UN of them are loaded before the first is used, in
// the same order e, e + stride, e + 2 stride, ... as one at a time, so the
// sums are the same; NVMAX x UN values in flight per thread.)
template <int NVMAX, int UN>
__global__ void __launch_bounds__(IRK_WG) k_dot_multi(const double *__restrict__ V, size_t ldv, int nv,
                                                      const double *__restrict__ w, size_t len, int with_norm,
                                                      double *partials) {
    double acc[NVMAX + 1];
#pragma unroll
    for (int k = 0; k <= NVMAX; ++k) acc[k] = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x;
    for (; e + (UN - 1) * stride < len; e += UN * stride) {
        double we[UN], v[UN][NVMAX];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            we[u] = w[e + u * stride];
#pragma unroll
            for (int k = 0; k < NVMAX; ++k)
                if (k < nv) v[u][k] = V[k * ldv + e + u * stride];
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
#pragma unroll
            for (int k = 0; k < NVMAX; ++k)
                if (k < nv) acc[k] += v[u][k] * we[u];
            if (with_norm) acc[NVMAX] += we[u] * we[u];
        }
    }
    for (; e < len; e += stride) {
        const double we = w[e];
#pragma unroll
        for (int k = 0; k < NVMAX; ++k)
            if (k < nv) acc[k] += V[k * ldv + e] * we;
        if (with_norm) acc[NVMAX] += we * we;
    }
    __shared__ double sh[4 * (NVMAX + 1)];
    const int nout = nv + (with_norm ? 1 : 0);
    double mine;
    block_reduce_multi<NVMAX + 1>(acc, nv, with_norm != 0, sh, mine);
    finish_multi<NVMAX + 1>(mine, nout, partials);
}

// Second Gram-Schmidt pass fused with the first update (one sweep over V):
//   w <- w - sum_k h1[k] V_k ;  h2[k] = <V_k, w> ;  out[nv] = <w, w>
// (out = h2 followed by the norm).
template <int NVMAX, int UN>
__global__ void __launch_bounds__(IRK_WG) k_axpy_dot(double *__restrict__ w, const double *__restrict__ V,
                                                     size_t ldv, int nv, const double *__restrict__ h1,
                                                     size_t len, double *partials) {
    double acc[NVMAX + 1];
    double hk[NVMAX];
#pragma unroll
    for (int k = 0; k <= NVMAX; ++k) acc[k] = 0.0;
#pragma unroll
    for (int k = 0; k < NVMAX; ++k) hk[k] = k < nv ? h1[k] : 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x;
    for (; e + (UN - 1) * stride < len; e += UN * stride) {
        double we[UN], v[UN][NVMAX];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            we[u] = w[e + u * stride];
#pragma unroll
            for (int k = 0; k < NVMAX; ++k)
                if (k < nv) v[u][k] = V[k * ldv + e + u * stride];
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
#pragma unroll
            for (int k = 0; k < NVMAX; ++k)
                if (k < nv) we[u] -= hk[k] * v[u][k];
            w[e + u * stride] = we[u];
#pragma unroll
            for (int k = 0; k < NVMAX; ++k)
                if (k < nv) acc[k] += v[u][k] * we[u];
            acc[NVMAX] += we[u] * we[u];
        }
    }
    for (; e < len; e += stride) {
        double v[NVMAX];
        double we = w[e];
#pragma unroll
        for (int k = 0; k < NVMAX; ++k)
            if (k < nv) {
                v[k] = V[k * ldv + e];
                we -= hk[k] * v[k];
            }
        w[e] = we;
#pragma unroll
        for (int k = 0; k < NVMAX; ++k)
            if (k < nv) acc[k] += v[k] * we;
        acc[NVMAX] += we * we;
    }
    __shared__ double sh[4 * (NVMAX + 1)];
    double mine;
    block_reduce_multi<NVMAX + 1>(acc, nv, true, sh, mine);
    finish_multi<NVMAX + 1>(mine, nv + 1, partials);
}

// Final update and normalization of the new Arnoldi vector:
//   w <- (w - sum_k h2[k] V_k) / sqrt(nrm2 - sum_k h2[k]^2)
// (the norm of the twice-orthogonalized vector by Pythagoras: V orthonormal).
__global__ void __launch_bounds__(IRK_WG) k_axpy_scale(double *__restrict__ w, const double *__restrict__ V,
                                                       size_t ldv, int nv, const double *__restrict__ h2,
                                                       const double *__restrict__ nrm2, size_t len) {
    double hs = 0.0;
    for (int k = 0; k < nv; ++k) hs += h2[k] * h2[k];
    const double nn = *nrm2 - hs;
    const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < len; e += stride) {
        double acc = w[e];
        for (int k = 0; k < nv; ++k) acc -= h2[k] * V[k * ldv + e];
        w[e] = acc * inv;
    }
}

// w <- w - sum_k h[k] V_k
__global__ void __launch_bounds__(IRK_WG) k_axpy_multi(double *__restrict__ w, const double *__restrict__ V,
                                                       size_t ldv, int nv, const double *__restrict__ hcoef,
                                                       size_t len) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < len; e += stride) {
        double acc = w[e];
        for (int k = 0; k < nv; ++k) acc -= hcoef[k] * V[k * ldv + e];
        w[e] = acc;
    }
}

// dst <- sum_k c[k] V_k
__global__ void __launch_bounds__(IRK_WG) k_lincomb(double *__restrict__ dst, const double *__restrict__ V,
                                                    size_t ldv, int nv, const double *__restrict__ c, size_t len) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < len; e += stride) {
        double acc = 0;
        for (int k = 0; k < nv; ++k) acc += c[k] * V[k * ldv + e];
        dst[e] = acc;
    }
}

// dst <- src / sqrt(*nrm2)
__global__ void __launch_bounds__(IRK_WG) k_scale_copy(double *__restrict__ dst, const double *__restrict__ src,
                                                       const double *__restrict__ nrm2, size_t len) {
    const double inv = 1.0 / sqrt(*nrm2);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < len; e += stride) dst[e] = src[e] * inv;
}

// dst <- a x + b y  (dst may alias x or y)
__global__ void __launch_bounds__(IRK_WG) k_axpby(double *dst, double a, const double *x, double b,
                                                  const double *y, size_t len) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < len; e += stride) dst[e] = a * x[e] + b * y[e];
}

__global__ void k_zero_u32(unsigned *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// ------------------------------------------------------------------------
// Multigrid (precision T).  Level operator A = sigma M - dt L(coef) with the
// operator's linearization rediscretized at the level spacing; a coarse
// coefficient is the full-weighting restriction of the fine one.
// ------------------------------------------------------------------------
// The coefficient hierarchies of one Newton iteration together: blockIdx.y
// selects the hierarchy (its fields are read from the argument block with a
// uniform index).
template <class T>
struct CoefSet {
    const T *src[IRK_MAX_STAGES];
    T *dst[IRK_MAX_STAGES];
};

template <class T>
__global__ void __launch_bounds__(IRK_WG) k_mg_coef_restrict_multi(int nxf, int nyf, CoefSet<T> p) {
    const T *__restrict__ cf = p.src[blockIdx.y];
    T *__restrict__ cc = p.dst[blockIdx.y];
    const int nxc = nxf / 2, nyc = (nyf > 1) ? nyf / 2 : 1;
    const size_t npc = (size_t)nxc * nyc;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const T wgt[3] = {T(0.25), T(0.5), T(0.25)};
    for (size_t q = (size_t)xcd_block() * blockDim.x + threadIdx.x; q < npc; q += stride) {
        int I, J;
        point_ij(q, nxc, I, J);
        T acc = 0;
        if (nyf == 1) {
            for (int a = -1; a <= 1; ++a) acc += wgt[a + 1] * cf[wrapm(2 * I + a, nxf)];
        } else {
            for (int bb = -1; bb <= 1; ++bb)
                for (int a = -1; a <= 1; ++a)
                    acc += wgt[a + 1] * wgt[bb + 1] * cf[(size_t)wrapm(2 * J + bb, nyf) * nxf + wrapm(2 * I + a, nxf)];
        }
        cc[q] = acc;
    }
}

// dst_h = (T) sum_k w[h][k] U_k[off + e] for every hierarchy h = blockIdx.y
// (zero weights skipped: a one-hot row reads one stage field)
template <class T>
struct MixSet {
    T *dst[IRK_MAX_STAGES];
    double w[IRK_MAX_STAGES][IRK_MAX_STAGES];
};

template <class T>
__global__ void __launch_bounds__(IRK_WG) k_mix_cast_multi(const double *__restrict__ U, size_t nf, size_t off,
                                                           int s, MixSet<T> m, size_t len) {
    const int h = blockIdx.y;
    T *__restrict__ dst = m.dst[h];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < len; e += stride) {
        double acc = 0.0;
        for (int k = 0; k < s; ++k) {
            const double wk = m.w[h][k];
            if (wk != 0.0) acc += wk * U[(size_t)k * nf + off + e];
        }
        dst[e] = (T)acc;
    }
}

// b0 = T(a1 v1 + a2 v2 - (a1 m[0] + a2 m[1]))   (v2 and m may be null; m holds
// the means of v1, v2 when the result must be mean-free)
template <class T>
__global__ void __launch_bounds__(IRK_WG) k_mg_cast_in(T *__restrict__ b0, const double *__restrict__ v1,
                                                       double a1, const double *__restrict__ v2, double a2,
                                                       const double *__restrict__ m, size_t len) {
    double shift = 0.0;
    if (m) shift = a1 * m[0] + (v2 ? a2 * m[1] : 0.0);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < len; e += stride) {
        double v = a1 * v1[e];
        if (v2) v += a2 * v2[e];
        b0[e] = (T)(v - shift);
    }
}

// z = a * double(x) + c * shift[0]   (shift may be null)
template <class T>
__global__ void __launch_bounds__(IRK_WG) k_mg_cast_out(double *__restrict__ z, const T *__restrict__ x, double a,
                                                        const double *__restrict__ shift, double c, size_t len) {
    const double off = shift ? c * shift[0] : 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < len; e += stride)
        z[e] = a * (double)x[e] + off;
}

__global__ void __launch_bounds__(IRK_WG) k_fill_f64(double *__restrict__ p, double v, size_t len) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += stride) p[e] = v;
}

// ------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------
static inline unsigned grid_for(size_t n, unsigned cap = 8192) {
    size_t g = (n + IRK_WG - 1) / IRK_WG;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

void launch_stage_prep(hipStream_t st, int s, size_t nf, const double *un, double *K, const double *Y, double *U,
                       const StageCoefs &C, double dt, int fold) {
    const unsigned g = grid_for(nf);
    switch (s) {
        case 1: k_stage_prep<1><<<g, IRK_WG, 0, st>>>(nf, un, K, Y, U, C, dt, fold); break;
        case 2: k_stage_prep<2><<<g, IRK_WG, 0, st>>>(nf, un, K, Y, U, C, dt, fold); break;
        case 3: k_stage_prep<3><<<g, IRK_WG, 0, st>>>(nf, un, K, Y, U, C, dt, fold); break;
        case 4: k_stage_prep<4><<<g, IRK_WG, 0, st>>>(nf, un, K, Y, U, C, dt, fold); break;
        case 5: k_stage_prep<5><<<g, IRK_WG, 0, st>>>(nf, un, K, Y, U, C, dt, fold); break;
    }
}

static void reduce_partials(hipStream_t st, const double *partials, unsigned nb, int nv, double *out,
                            int nmax = 0, double *out2 = nullptr, double *hout = nullptr, double *hout2 = nullptr) {
    k_reduce_partials<<<1, 256, 0, st>>>(partials, (int)nb, nv, nmax, out, out2, hout, hout2);
}

// The stage preparation of a two-variable field (the DAE: omega, psi) with
// the per-work-group partial sums of every stage's omega and psi, times
// scale (the stage means the residual needs), in the same sweep.  The same
// stage arithmetic as k_stage_prep; point p carries elements p and npts + p.
template <int S>
__global__ void __launch_bounds__(IRK_WG) k_stage_prep_sums(size_t npts, const double *__restrict__ un,
                                                            double *__restrict__ K, const double *__restrict__ Y,
                                                            double *__restrict__ U, StageCoefs C, double dt,
                                                            int fold, double scale, double *partials) {
    const size_t nf = 2 * npts;
    double acc[2 * S + 1];
#pragma unroll
    for (int k = 0; k <= 2 * S; ++k) acc[k] = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t p = (size_t)xcd_block() * blockDim.x + threadIdx.x; p < npts; p += stride) {
#pragma unroll
        for (int var = 0; var < 2; ++var) {
            const size_t e = var * npts + p;
            double k[S];
#pragma unroll
            for (int j = 0; j < S; ++j) k[j] = K[j * nf + e];
            if (fold) {
                double y[S];
#pragma unroll
                for (int l = 0; l < S; ++l) y[l] = Y[l * nf + e];
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    double a = k[j];
#pragma unroll
                    for (int l = 0; l < S; ++l) a += C.TLam[j * S + l] * y[l];
                    k[j] = a;
                    K[j * nf + e] = a;
                }
            }
            const double u = un[e];
#pragma unroll
            for (int i = 0; i < S; ++i) {
                double a = 0;
#pragma unroll
                for (int j = 0; j < S; ++j) a += C.A[i * S + j] * k[j];
                const double v = u + dt * a;
                U[i * nf + e] = v;
                acc[2 * i + var] += v;
            }
        }
    }
    __shared__ double sh[4 * (2 * S + 1)];
    double mine;
    block_reduce_multi<2 * S + 1>(acc, 2 * S, false, sh, mine);
    finish_multi<2 * S + 1>(mine * scale, 2 * S, partials);
}

void launch_stage_prep_sums(hipStream_t st, int s, size_t npts, const double *un, double *K, const double *Y,
                            double *U, const StageCoefs &C, double dt, int fold, double scale, double *partials,
                            double *out) {
    const unsigned g = grid_for(npts, IRK_RED_BLOCKS);
    switch (s) {
        case 1: k_stage_prep_sums<1><<<g, IRK_WG, 0, st>>>(npts, un, K, Y, U, C, dt, fold, scale, partials); break;
        case 2: k_stage_prep_sums<2><<<g, IRK_WG, 0, st>>>(npts, un, K, Y, U, C, dt, fold, scale, partials); break;
        case 3: k_stage_prep_sums<3><<<g, IRK_WG, 0, st>>>(npts, un, K, Y, U, C, dt, fold, scale, partials); break;
        case 4: k_stage_prep_sums<4><<<g, IRK_WG, 0, st>>>(npts, un, K, Y, U, C, dt, fold, scale, partials); break;
        case 5: k_stage_prep_sums<5><<<g, IRK_WG, 0, st>>>(npts, un, K, Y, U, C, dt, fold, scale, partials); break;
    }
    reduce_partials(st, partials, g, 2 * s, out);
}

template <int S>
static void residual_s(hipStream_t st, const DeviceProblem &P, const double *U, const double *K, double *Fh,
                       const StageCoefs &C, const double *means, double *partials, double *out, double *gmax,
                       double *hout, double *hgmax) {
    const size_t npts = (size_t)P.g.nx * P.g.ny;
    const unsigned g = grid_for(npts, IRK_RED_BLOCKS);
    if (P.kind == IRK_OP_NLDIFF_2D) {
        k_residual<S, IRK_OP_NLDIFF_2D><<<g, IRK_WG, 0, st>>>(P, U, K, Fh, C, means, partials);
        reduce_partials(st, partials, g, 2, out, 0, nullptr, hout);
    } else if (P.kind == IRK_OP_BURGERS_1D) {
        k_residual<S, IRK_OP_BURGERS_1D><<<g, IRK_WG, 0, st>>>(P, U, K, Fh, C, means, partials);
        reduce_partials(st, partials, g, 2, out, 0, nullptr, hout);
    } else {
        k_residual<S, IRK_OP_VSF_2D><<<g, IRK_WG, 0, st>>>(P, U, K, Fh, C, means, partials);
        reduce_partials(st, partials, g, 2 + S, out, S, gmax, hout, hgmax);
    }
}

void launch_residual(hipStream_t st, int s, const DeviceProblem &P, const double *U, const double *K, double *Fh,
                     const StageCoefs &C, const double *means, double *partials, double *out, double *gmax,
                     double *hout, double *hgmax) {
    switch (s) {
        case 1: residual_s<1>(st, P, U, K, Fh, C, means, partials, out, gmax, hout, hgmax); break;
        case 2: residual_s<2>(st, P, U, K, Fh, C, means, partials, out, gmax, hout, hgmax); break;
        case 3: residual_s<3>(st, P, U, K, Fh, C, means, partials, out, gmax, hout, hgmax); break;
        case 4: residual_s<4>(st, P, U, K, Fh, C, means, partials, out, gmax, hout, hgmax); break;
        case 5: residual_s<5>(st, P, U, K, Fh, C, means, partials, out, gmax, hout, hgmax); break;
    }
}

template <int S>
static void stage_residual_s(hipStream_t st, const DeviceProblem &P, const double *un, const double *K,
                             double *Kout, const double *Y, double *U, double *Fh, const StageCoefs &C, double dt,
                             int fold, double *partials, double *out, double *hout) {
    unsigned g;
    if (P.kind == IRK_OP_NLDIFF_2D) {
        if (P.g.nx >= 64) {
            g = (unsigned)(((P.g.nx + 63) / 64) * ((P.g.ny + 3) / 4));
            k_stage_residual<S, IRK_OP_NLDIFF_2D, 64, 4><<<g, IRK_WG, 0, st>>>(P, un, K, Kout, Y, U, Fh, C, dt, fold,
                                                                            partials);
        } else {
            g = (unsigned)(((P.g.nx + 15) / 16) * ((P.g.ny + 15) / 16));
            k_stage_residual<S, IRK_OP_NLDIFF_2D, 16, 16><<<g, IRK_WG, 0, st>>>(P, un, K, Kout, Y, U, Fh, C, dt,
                                                                             fold, partials);
        }
    } else {
        g = (unsigned)((P.g.nx + 255) / 256);
        k_stage_residual<S, IRK_OP_BURGERS_1D, 256, 1><<<g, IRK_WG, 0, st>>>(P, un, K, Kout, Y, U, Fh, C, dt, fold,
                                                                          partials);
    }
    reduce_partials(st, partials, g, 2, out, 0, nullptr, hout);
}

bool stage_residual_fused(const DeviceProblem &P) {
    return P.kind == IRK_OP_NLDIFF_2D || P.kind == IRK_OP_BURGERS_1D;
}

size_t stage_residual_blocks(int kind, int nx, int ny) {
    if (kind == IRK_OP_NLDIFF_2D)
        return nx >= 64 ? (size_t)((nx + 63) / 64) * ((ny + 3) / 4) : (size_t)((nx + 15) / 16) * ((ny + 15) / 16);
    return (size_t)(nx + 255) / 256;
}

void launch_stage_residual(hipStream_t st, int s, const DeviceProblem &P, const double *un, const double *K,
                           double *Kout, const double *Y, double *U, double *Fh, const StageCoefs &C, double dt,
                           int fold, double *partials, double *out, double *hout) {
    switch (s) {
        case 1: stage_residual_s<1>(st, P, un, K, Kout, Y, U, Fh, C, dt, fold, partials, out, hout); break;
        case 2: stage_residual_s<2>(st, P, un, K, Kout, Y, U, Fh, C, dt, fold, partials, out, hout); break;
        case 3: stage_residual_s<3>(st, P, un, K, Kout, Y, U, Fh, C, dt, fold, partials, out, hout); break;
        case 4: stage_residual_s<4>(st, P, un, K, Kout, Y, U, Fh, C, dt, fold, partials, out, hout); break;
        case 5: stage_residual_s<5>(st, P, un, K, Kout, Y, U, Fh, C, dt, fold, partials, out, hout); break;
    }
}

template <int S>
static void rhs_init_s(hipStream_t st, const DeviceProblem &P, const double *un, double *K, double s_n, double c_n) {
    const size_t npts = (size_t)P.g.nx * P.g.ny;
    const unsigned g = grid_for(npts);
    if (P.kind == IRK_OP_NLDIFF_2D) k_rhs_init<S, IRK_OP_NLDIFF_2D><<<g, IRK_WG, 0, st>>>(P, un, K, s_n, c_n);
    else if (P.kind == IRK_OP_BURGERS_1D) k_rhs_init<S, IRK_OP_BURGERS_1D><<<g, IRK_WG, 0, st>>>(P, un, K, s_n, c_n);
    else k_rhs_init<S, IRK_OP_VSF_2D><<<g, IRK_WG, 0, st>>>(P, un, K, s_n, c_n);
}

void launch_rhs_init(hipStream_t st, int s, const DeviceProblem &P, const double *un, double *K, double sin_tn,
                     double cos_tn) {
    switch (s) {
        case 1: rhs_init_s<1>(st, P, un, K, sin_tn, cos_tn); break;
        case 2: rhs_init_s<2>(st, P, un, K, sin_tn, cos_tn); break;
        case 3: rhs_init_s<3>(st, P, un, K, sin_tn, cos_tn); break;
        case 4: rhs_init_s<4>(st, P, un, K, sin_tn, cos_tn); break;
        case 5: rhs_init_s<5>(st, P, un, K, sin_tn, cos_tn); break;
    }
}

void launch_final_update(hipStream_t st, int s, size_t nf, const double *un, const double *K, double *out,
                         const StageCoefs &C, double dt) {
    const unsigned g = grid_for(nf);
    switch (s) {
        case 1: k_final_update<1><<<g, IRK_WG, 0, st>>>(nf, un, K, out, C, dt); break;
        case 2: k_final_update<2><<<g, IRK_WG, 0, st>>>(nf, un, K, out, C, dt); break;
        case 3: k_final_update<3><<<g, IRK_WG, 0, st>>>(nf, un, K, out, C, dt); break;
        case 4: k_final_update<4><<<g, IRK_WG, 0, st>>>(nf, un, K, out, C, dt); break;
        case 5: k_final_update<5><<<g, IRK_WG, 0, st>>>(nf, un, K, out, C, dt); break;
    }
}

void launch_stage_extrap(hipStream_t st, int s, size_t nf, const double *K, double *Kx, const StageCoefs &W) {
    const unsigned g = grid_for(nf);
    switch (s) {
        case 1: k_stage_extrap<1><<<g, IRK_WG, 0, st>>>(nf, K, Kx, W); break;
        case 2: k_stage_extrap<2><<<g, IRK_WG, 0, st>>>(nf, K, Kx, W); break;
        case 3: k_stage_extrap<3><<<g, IRK_WG, 0, st>>>(nf, K, Kx, W); break;
        case 4: k_stage_extrap<4><<<g, IRK_WG, 0, st>>>(nf, K, Kx, W); break;
        case 5: k_stage_extrap<5><<<g, IRK_WG, 0, st>>>(nf, K, Kx, W); break;
    }
}

void launch_field_sums(hipStream_t st, const double *X, size_t ld, int nfields, size_t len, double scale,
                       double *partials, double *out, unsigned *ctr) {
    const unsigned g = grid_for(len, IRK_RED_BLOCKS);
    k_field_sums<<<g, IRK_WG, 0, st>>>(X, ld, nfields, len, scale, partials, out, ctr);
    reduce_partials(st, partials, g, nfields, out);
}

void launch_field_sums2(hipStream_t st, const double *X0, const double *X1, size_t len, double scale,
                        double *partials, double *out) {
    const unsigned g = grid_for(len, IRK_RED_BLOCKS);
    k_field_sums2<<<g, IRK_WG, 0, st>>>(X0, X1, len, scale, partials);
    reduce_partials(st, partials, g, 2, out);
}

template <int OP, int NVMAX>
static void block_matvec_dot_op(hipStream_t st, unsigned g, const DeviceProblem &P, int width, const BlockLam &lam,
                                double dt, const double *Ua, const double *Ub, const double *x, double *w,
                                const double *xmeans, const double *V, size_t ldv, int nv, double *partials) {
    k_block_matvec_dot<OP, NVMAX><<<g, IRK_WG, 0, st>>>(P, width, lam, dt, Ua, Ub, x, w, xmeans, V, ldv, nv, partials);
}

template <int OP>
static void block_matvec_dot_nv(hipStream_t st, unsigned g, const DeviceProblem &P, int width, const BlockLam &lam,
                                double dt, const double *Ua, const double *Ub, const double *x, double *w,
                                const double *xmeans, const double *V, size_t ldv, int nv, double *partials) {
    if (nv <= 4) block_matvec_dot_op<OP, 4>(st, g, P, width, lam, dt, Ua, Ub, x, w, xmeans, V, ldv, nv, partials);
    else if (nv <= 8) block_matvec_dot_op<OP, 8>(st, g, P, width, lam, dt, Ua, Ub, x, w, xmeans, V, ldv, nv, partials);
    else block_matvec_dot_op<OP, DOT_CHUNK>(st, g, P, width, lam, dt, Ua, Ub, x, w, xmeans, V, ldv, nv, partials);
}

bool launch_block_matvec_dot(hipStream_t st, const DeviceProblem &P, int width, const BlockLam &lam, double dt,
                             const double *Ua, const double *Ub, const double *x, double *w, const double *xmeans,
                             const double *V, size_t ldv, int nv, double *partials, double *out, double *hout) {
    if (nv < 1 || nv > DOT_CHUNK) return false;
    const size_t npts = (size_t)P.g.nx * P.g.ny;
    if (P.kind == IRK_OP_NLDIFF_2D) {
        // over LDS tiles while their partials (one per tile and basis vector) fit
        const unsigned tiles = (unsigned)(((P.g.nx + VM_TX - 1) / VM_TX) * ((P.g.ny + VM_TY - 1) / VM_TY));
        if ((size_t)tiles * nv <= IRK_LANE_PARTIALS) {
            if (nv <= 4)
                k_block_matvec_dot_nl<4><<<tiles, IRK_WG, 0, st>>>(P, width, lam, dt, Ua, Ub, x, w, V, ldv, nv,
                                                                   partials);
            else if (nv <= 8)
                k_block_matvec_dot_nl<8><<<tiles, IRK_WG, 0, st>>>(P, width, lam, dt, Ua, Ub, x, w, V, ldv, nv,
                                                                   partials);
            else
                k_block_matvec_dot_nl<DOT_CHUNK><<<tiles, IRK_WG, 0, st>>>(P, width, lam, dt, Ua, Ub, x, w, V, ldv,
                                                                           nv, partials);
            reduce_partials(st, partials, tiles, nv, out, 0, nullptr, hout);
            return true;
        }
    }
    const unsigned g = grid_for(npts, IRK_MATVEC_DOT_BLOCKS);    // partials: g * nv <= IRK_LANE_PARTIALS
    if (P.kind == IRK_OP_NLDIFF_2D)
        block_matvec_dot_nv<IRK_OP_NLDIFF_2D>(st, g, P, width, lam, dt, Ua, Ub, x, w, xmeans, V, ldv, nv, partials);
    else if (P.kind == IRK_OP_BURGERS_1D)
        block_matvec_dot_nv<IRK_OP_BURGERS_1D>(st, g, P, width, lam, dt, Ua, Ub, x, w, xmeans, V, ldv, nv, partials);
    else
        block_matvec_dot_nv<IRK_OP_VSF_2D>(st, g, P, width, lam, dt, Ua, Ub, x, w, xmeans, V, ldv, nv, partials);
    reduce_partials(st, partials, g, nv, out, 0, nullptr, hout);
    return true;
}

void launch_block_matvec(hipStream_t st, const DeviceProblem &P, int width, const BlockLam &lam, double dt,
                         const double *Ua, const double *Ub, const double *x, double *w, const double *xmeans) {
    const size_t npts = (size_t)P.g.nx * P.g.ny;
    const unsigned g = grid_for(npts);
    if (P.kind == IRK_OP_NLDIFF_2D)
        k_block_matvec<IRK_OP_NLDIFF_2D><<<g, IRK_WG, 0, st>>>(P, width, lam, dt, Ua, Ub, x, w, xmeans);
    else if (P.kind == IRK_OP_BURGERS_1D)
        k_block_matvec<IRK_OP_BURGERS_1D><<<g, IRK_WG, 0, st>>>(P, width, lam, dt, Ua, Ub, x, w, xmeans);
    else {
        const unsigned tiles = (unsigned)(((P.g.nx + VM_TX - 1) / VM_TX) * ((P.g.ny + VM_TY - 1) / VM_TY));
        k_block_matvec_vsf<<<tiles, IRK_WG, 0, st>>>(P, width, lam, dt, Ua, Ub, x, w, xmeans);
    }
}

template <int OP>
static void block_matvec_w_op(hipStream_t st, const DeviceProblem &P, int s, int width, const BlockLam &lam,
                              double dt, const double *U, const BlockWeights &W, const double *x, double *w,
                              const double *xmeans, int coupling) {
    const unsigned g = grid_for((size_t)P.g.nx * P.g.ny);
    switch (s) {
        case 1: k_block_matvec_w<OP, 1><<<g, IRK_WG, 0, st>>>(P, width, lam, dt, U, W, x, w, xmeans, coupling); break;
        case 2: k_block_matvec_w<OP, 2><<<g, IRK_WG, 0, st>>>(P, width, lam, dt, U, W, x, w, xmeans, coupling); break;
        case 3: k_block_matvec_w<OP, 3><<<g, IRK_WG, 0, st>>>(P, width, lam, dt, U, W, x, w, xmeans, coupling); break;
        case 4: k_block_matvec_w<OP, 4><<<g, IRK_WG, 0, st>>>(P, width, lam, dt, U, W, x, w, xmeans, coupling); break;
        case 5: k_block_matvec_w<OP, 5><<<g, IRK_WG, 0, st>>>(P, width, lam, dt, U, W, x, w, xmeans, coupling); break;
    }
}

void launch_block_matvec_w(hipStream_t st, const DeviceProblem &P, int s, int width, const BlockLam &lam,
                           double dt, const double *U, const BlockWeights &W, const double *x, double *w,
                           const double *xmeans, int coupling) {
    if (P.kind == IRK_OP_NLDIFF_2D)
        block_matvec_w_op<IRK_OP_NLDIFF_2D>(st, P, s, width, lam, dt, U, W, x, w, xmeans, coupling);
    else if (P.kind == IRK_OP_BURGERS_1D)
        block_matvec_w_op<IRK_OP_BURGERS_1D>(st, P, s, width, lam, dt, U, W, x, w, xmeans, coupling);
    else
        block_matvec_w_op<IRK_OP_VSF_2D>(st, P, s, width, lam, dt, U, W, x, w, xmeans, coupling);
}

template <int OP>
static void block_couple_op(hipStream_t st, const DeviceProblem &P, int s, const BlockCouple &C, double dt,
                            const double *U, const double *y, double *f) {
    const unsigned g = grid_for((size_t)P.g.nx * P.g.ny);
    switch (s) {
        case 1: k_block_couple<OP, 1><<<g, IRK_WG, 0, st>>>(P, C, dt, U, y, f); break;
        case 2: k_block_couple<OP, 2><<<g, IRK_WG, 0, st>>>(P, C, dt, U, y, f); break;
        case 3: k_block_couple<OP, 3><<<g, IRK_WG, 0, st>>>(P, C, dt, U, y, f); break;
        case 4: k_block_couple<OP, 4><<<g, IRK_WG, 0, st>>>(P, C, dt, U, y, f); break;
        case 5: k_block_couple<OP, 5><<<g, IRK_WG, 0, st>>>(P, C, dt, U, y, f); break;
    }
}

void launch_block_couple(hipStream_t st, const DeviceProblem &P, int s, const BlockCouple &C, double dt,
                         const double *U, const double *y, double *f) {
    if (P.kind == IRK_OP_NLDIFF_2D) block_couple_op<IRK_OP_NLDIFF_2D>(st, P, s, C, dt, U, y, f);
    else if (P.kind == IRK_OP_BURGERS_1D) block_couple_op<IRK_OP_BURGERS_1D>(st, P, s, C, dt, U, y, f);
}

void launch_dot_multi(hipStream_t st, const double *V, size_t ldv, int nv, const double *w, size_t len,
                      int with_norm, double *partials, double *out, double *hout) {
    // chunks of DOT_CHUNK vectors; the norm (if any) rides on the last chunk
    int done = 0;
    do {
        const int c = (nv - done) > DOT_CHUNK ? DOT_CHUNK : (nv - done);
        const int last = (done + c == nv);
        const unsigned g = grid_for(len, IRK_RED_BLOCKS);
        const int wn = last ? with_norm : 0;
        if (c <= 4) k_dot_multi<4, 4><<<g, IRK_WG, 0, st>>>(V + done * ldv, ldv, c, w, len, wn, partials);
        else if (c <= 8) k_dot_multi<8, 2><<<g, IRK_WG, 0, st>>>(V + done * ldv, ldv, c, w, len, wn, partials);
        else k_dot_multi<DOT_CHUNK, 1><<<g, IRK_WG, 0, st>>>(V + done * ldv, ldv, c, w, len, wn, partials);
        reduce_partials(st, partials, g, c + wn, out + done, 0, nullptr, hout ? hout + done : nullptr);
        done += c;
    } while (done < nv);
}

void launch_axpy_dot(hipStream_t st, double *w, const double *V, size_t ldv, int nv, const double *h1, size_t len,
                     double *partials, double *out, double *hout) {
    const unsigned g = grid_for(len, IRK_RED_BLOCKS);
    if (nv <= 4) k_axpy_dot<4, 4><<<g, IRK_WG, 0, st>>>(w, V, ldv, nv, h1, len, partials);
    else if (nv <= 8) k_axpy_dot<8, 2><<<g, IRK_WG, 0, st>>>(w, V, ldv, nv, h1, len, partials);
    else k_axpy_dot<DOT_CHUNK, 1><<<g, IRK_WG, 0, st>>>(w, V, ldv, nv, h1, len, partials);
    reduce_partials(st, partials, g, nv + 1, out, 0, nullptr, hout);
}

void launch_axpy_scale(hipStream_t st, double *w, const double *V, size_t ldv, int nv, const double *h2,
                       const double *nrm2, size_t len) {
    k_axpy_scale<<<grid_for(len), IRK_WG, 0, st>>>(w, V, ldv, nv, h2, nrm2, len);
}

void launch_axpy_multi(hipStream_t st, double *w, const double *V, size_t ldv, int nv, const double *h, size_t len) {
    k_axpy_multi<<<grid_for(len), IRK_WG, 0, st>>>(w, V, ldv, nv, h, len);
}

void launch_lincomb(hipStream_t st, double *dst, const double *V, size_t ldv, int nv, const double *c, size_t len) {
    k_lincomb<<<grid_for(len), IRK_WG, 0, st>>>(dst, V, ldv, nv, c, len);
}

void launch_scale_copy(hipStream_t st, double *dst, const double *src, const double *nrm2, size_t len) {
    k_scale_copy<<<grid_for(len), IRK_WG, 0, st>>>(dst, src, nrm2, len);
}

void launch_axpby(hipStream_t st, double *dst, double a, const double *x, double b, const double *y, size_t len) {
    k_axpby<<<grid_for(len), IRK_WG, 0, st>>>(dst, a, x, b, y, len);
}

void launch_zero_u32(hipStream_t st, unsigned *p, int n) { k_zero_u32<<<1, 256, 0, st>>>(p, n); }

void launch_fill(hipStream_t st, double *p, double v, size_t len) {
    k_fill_f64<<<grid_for(len), IRK_WG, 0, st>>>(p, v, len);
}

template <class T>
void launch_mg_coef_restrict_multi(hipStream_t st, int nxf, int nyf, const T *const *src, T *const *dst, int n) {
    CoefSet<T> p;
    std::memset(&p, 0, sizeof(p));
    for (int h = 0; h < n; ++h) { p.src[h] = src[h]; p.dst[h] = dst[h]; }
    const size_t npc = (size_t)(nxf / 2) * (nyf > 1 ? nyf / 2 : 1);
    k_mg_coef_restrict_multi<T><<<dim3(grid_for(npc), n), IRK_WG, 0, st>>>(nxf, nyf, p);
}

template <class T>
void launch_mix_cast_multi(hipStream_t st, T *const *dst, const double *U, size_t nf, size_t off, int s,
                           const double (*w)[IRK_MAX_STAGES], int n, size_t len) {
    MixSet<T> m;
    std::memset(&m, 0, sizeof(m));
    for (int h = 0; h < n; ++h) {
        m.dst[h] = dst[h];
        for (int k = 0; k < s; ++k) m.w[h][k] = w[h][k];
    }
    k_mix_cast_multi<T><<<dim3(grid_for(len), n), IRK_WG, 0, st>>>(U, nf, off, s, m, len);
}

template <class T>
void launch_mg_cast_in(hipStream_t st, T *b0, const double *v1, double a1, const double *v2, double a2,
                       const double *means, size_t len) {
    k_mg_cast_in<T><<<grid_for(len), IRK_WG, 0, st>>>(b0, v1, a1, v2, a2, means, len);
}

template <class T>
void launch_mg_cast_out(hipStream_t st, double *z, const T *x, double a, const double *shift, double c,
                        size_t len) {
    k_mg_cast_out<T><<<grid_for(len), IRK_WG, 0, st>>>(z, x, a, shift, c, len);
}

#define INST(T)                                                                                                    \
    template void launch_mg_cast_in<T>(hipStream_t, T *, const double *, double, const double *, double,           \
                                       const double *, size_t);                                                    \
    template void launch_mg_cast_out<T>(hipStream_t, double *, const T *, double, const double *, double, size_t); \
    template void launch_mg_coef_restrict_multi<T>(hipStream_t, int, int, const T *const *, T *const *, int);     \
    template void launch_mix_cast_multi<T>(hipStream_t, T *const *, const double *, size_t, size_t, int,           \
                                           const double (*)[IRK_MAX_STAGES], int, size_t);
INST(float)
INST(double)
#undef INST

}  // namespace irk
