// Host-callable launchers of the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "irk_internal.h"

namespace irk {

// operator of a multigrid hierarchy (the diagonal block being inverted)
enum MgOp { MG_NLDIFF = 0, MG_BURGERS = 1, MG_VSF_OMEGA = 2, MG_POISSON = 3 };

void launch_stage_prep(hipStream_t st, int s, size_t nf, const double *un, double *K, const double *Y, double *U,
                       const StageCoefs &C, double dt, int fold);
// The same for a two-variable field of npts points per variable (the DAE),
// with out[2 i + var] = scale * sum of stage i's variable var (omega 0, psi 1)
// through per-work-group partials and their reduction, in the same sweep
void launch_stage_prep_sums(hipStream_t st, int s, size_t npts, const double *un, double *K, const double *Y,
                            double *U, const StageCoefs &C, double dt, int fold, double scale, double *partials,
                            double *out);
// out[0] = ||F||^2, out[1] = squared norm of the magnitudes of F's terms;
// VSF also gmax[0..s): each stage's largest one-cell streamfunction
// difference.  hout, hgmax (optional): the same values in pinned
// fine-grained host memory as well (the reductions write both), which the
// host reads once an event behind the launch has completed.  Every launcher
// below with an hout argument does the same for its out.
void launch_residual(hipStream_t st, int s, const DeviceProblem &P, const double *U, const double *K, double *Fh,
                     const StageCoefs &C, const double *means, double *partials, double *out, double *gmax,
                     double *hout = nullptr, double *hgmax = nullptr);
// Stage values and residual in one sweep (nonlinear diffusion and Burgers
// only: stage_residual_fused): with fold, k = K + (T Lambda (x) I) Y is
// written to Kout (not K); U, the transformed residual Fh and out[0..1] as
// launch_residual.  The partials hold stage_residual_blocks(kind, nx, ny) x 2
// values.
bool stage_residual_fused(const DeviceProblem &P);
size_t stage_residual_blocks(int kind, int nx, int ny);
void launch_stage_residual(hipStream_t st, int s, const DeviceProblem &P, const double *un, const double *K,
                           double *Kout, const double *Y, double *U, double *Fh, const StageCoefs &C, double dt,
                           int fold, double *partials, double *out, double *hout = nullptr);
void launch_rhs_init(hipStream_t st, int s, const DeviceProblem &P, const double *un, double *K, double sin_tn,
                     double cos_tn);
// Kx_i = sum_j W.A[i][j] K_j (s stage fields of length nf; Kx must not alias K)
void launch_stage_extrap(hipStream_t st, int s, size_t nf, const double *K, double *Kx, const StageCoefs &W);
void launch_final_update(hipStream_t st, int s, size_t nf, const double *un, const double *K, double *out,
                         const StageCoefs &C, double dt);
void launch_field_sums(hipStream_t st, const double *X, size_t ld, int nfields, size_t len, double scale,
                       double *partials, double *out, unsigned *ctr);
// out[0] = scale * sum X0, out[1] = scale * sum X1 (len each)
void launch_field_sums2(hipStream_t st, const double *X0, const double *X1, size_t len, double scale,
                        double *partials, double *out);
void launch_block_matvec(hipStream_t st, const DeviceProblem &P, int width, const BlockLam &lam, double dt,
                         const double *Ua, const double *Ub, const double *x, double *w, const double *xmeans);
// The same matvec fused with the first Gram-Schmidt pass: out[k] = (V_k, w)
// for k < nv (basis vectors at stride ldv), through per-work-group partials
// (up to IRK_MATVEC_DOT_BLOCKS work-groups: partials holds IRK_LANE_PARTIALS
// values) and their reduction; false (nothing launched) when nv > 16
bool launch_block_matvec_dot(hipStream_t st, const DeviceProblem &P, int width, const BlockLam &lam, double dt,
                             const double *Ua, const double *Ub, const double *x, double *w, const double *xmeans,
                             const double *V, size_t ldv, int nv, double *partials, double *out,
                             double *hout = nullptr);
// Eigen-block operator with stage-weighted linearizations (U: the s stage
// fields); coupling = 1 gives -c21 M x_0 + dt sum_k W[1][0][k] L(U_k) x_0 on
// the differential variable instead
void launch_block_matvec_w(hipStream_t st, const DeviceProblem &P, int s, int width, const BlockLam &lam,
                           double dt, const double *U, const BlockWeights &W, const double *x, double *w,
                           const double *xmeans, int coupling);
// f (block i's wi components) -= (R_ij M - dt sum_k W L(U_k)) y (block j's wj
// components): the back-substitution of the real Schur basis (ODE operators)
void launch_block_couple(hipStream_t st, const DeviceProblem &P, int s, const BlockCouple &C, double dt,
                         const double *U, const double *y, double *f);
void launch_dot_multi(hipStream_t st, const double *V, size_t ldv, int nv, const double *w, size_t len,
                      int with_norm, double *partials, double *out, double *hout = nullptr);
void launch_axpy_multi(hipStream_t st, double *w, const double *V, size_t ldv, int nv, const double *h, size_t len);
// w <- w - V h1, then h2 = V^T w and ||w||^2 into out[0..nv] (nv <= 16)
void launch_axpy_dot(hipStream_t st, double *w, const double *V, size_t ldv, int nv, const double *h1, size_t len,
                     double *partials, double *out, double *hout = nullptr);
// w <- (w - V h2) / sqrt(nrm2 - |h2|^2)
void launch_axpy_scale(hipStream_t st, double *w, const double *V, size_t ldv, int nv, const double *h2,
                       const double *nrm2, size_t len);
void launch_lincomb(hipStream_t st, double *dst, const double *V, size_t ldv, int nv, const double *c, size_t len);
void launch_scale_copy(hipStream_t st, double *dst, const double *src, const double *nrm2, size_t len);
void launch_axpby(hipStream_t st, double *dst, double a, const double *x, double b, const double *y, size_t len);
void launch_zero_u32(hipStream_t st, unsigned *p, int n);
void launch_fill(hipStream_t st, double *p, double v, size_t len);

// every hierarchy's restriction of one level in one launch (n <= IRK_MAX_STAGES)
template <class T>
void launch_mg_coef_restrict_multi(hipStream_t st, int nxf, int nyf, const T *const *src, T *const *dst, int n);
// dst[h] = (T) sum_k w[h][k] U[k * nf + off + e] for h < n, in one launch
template <class T>
void launch_mix_cast_multi(hipStream_t st, T *const *dst, const double *U, size_t nf, size_t off, int s,
                           const double (*w)[IRK_MAX_STAGES], int n, size_t len);
template <class T>
void launch_mg_cast_in(hipStream_t st, T *b0, const double *v1, double a1, const double *v2, double a2,
                       const double *means, size_t len);
template <class T>
void launch_mg_cast_out(hipStream_t st, double *z, const T *x, double a, const double *shift, double c,
                        size_t len);

}  // namespace irk
