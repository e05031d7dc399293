// Device-side stencils of the three semi-discrete operators and of their
// linearizations.  Periodic grids, fields row-major [ny][nx], x fastest.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace irk {

__device__ __forceinline__ int wrapm(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// ---------------------------------------------------------------------------
// Nonlinear diffusion: N(u)_c = h^{-2} sum_faces kappa_f (u_nb - u_c),
// kappa(u) = 1 + u^2, kappa_f = (kappa(u_c) + kappa(u_nb)) / 2.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T nldiff_flux5(T uc, T ue, T uw, T un, T us, T inv_h2) {
    const T kc = T(1) + uc * uc;
    T sacc = T(0.5) * (kc + T(1) + ue * ue) * (ue - uc);
    sacc += T(0.5) * (kc + T(1) + uw * uw) * (uw - uc);
    sacc += T(0.5) * (kc + T(1) + un * un) * (un - uc);
    sacc += T(0.5) * (kc + T(1) + us * us) * (us - uc);
    return sacc * inv_h2;
}

// sum of the magnitudes of the four face terms (rounding scale of the flux)
template <class T>
__device__ __forceinline__ T nldiff_flux5_abs(T uc, T ue, T uw, T un, T us, T inv_h2) {
    const T kc = T(1) + uc * uc;
    T sacc = T(0.5) * (kc + T(1) + ue * ue) * fabs(ue - uc);
    sacc += T(0.5) * (kc + T(1) + uw * uw) * fabs(uw - uc);
    sacc += T(0.5) * (kc + T(1) + un * un) * fabs(un - uc);
    sacc += T(0.5) * (kc + T(1) + us * us) * fabs(us - uc);
    return sacc * inv_h2;
}

// Linearization L(U) x = h^{-2} sum_f [kappa_f (x_nb - x_c)
//                                      + (U_nb - U_c)(U_c x_c + U_nb x_nb)]
// (kappa'(u) = 2u), and its diagonal coefficient.
template <class T, bool HAS_X>
__device__ __forceinline__ void nldiff_lin(const T *U, const T *x, int i, int j, int nx, int ny,
                                           T inv_h2, T &Lx, T &Ld) {
    const int ip = wrapm(i + 1, nx), im = wrapm(i - 1, nx);
    const int jp = wrapm(j + 1, ny), jm = wrapm(j - 1, ny);
    const int c = j * nx + i;
    const int nb[4] = {j * nx + ip, j * nx + im, jp * nx + i, jm * nx + i};
    const T uc = U[c];
    const T xc = HAS_X ? x[c] : T(0);
    T lx = 0, ld = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const T un = U[nb[q]];
        const T kf = T(1) + T(0.5) * (uc * uc + un * un);
        const T du = un - uc;
        if (HAS_X) {
            const T xn = x[nb[q]];
            lx += kf * (xn - xc) + du * (uc * xc + un * xn);
        }
        ld += -kf + du * uc;
    }
    Lx = lx * inv_h2;
    Ld = ld * inv_h2;
}

// ---------------------------------------------------------------------------
// Burgers: N(u)_i = -(u_{i+1}^2 - u_{i-1}^2)/(4h) + nu (u_{i+1} - 2u_i + u_{i-1})/h^2
// Linearization L(U) x = -(U_{i+1} x_{i+1} - U_{i-1} x_{i-1})/(2h) + nu D2 x.
// ---------------------------------------------------------------------------
template <class T, bool HAS_X>
__device__ __forceinline__ void burgers_lin(const T *U, const T *x, int i, int nx, T h, T nu,
                                            T &Lx, T &Ld) {
    const int ip = wrapm(i + 1, nx), im = wrapm(i - 1, nx);
    const T inv_h2 = T(1) / (h * h);
    if (HAS_X) {
        Lx = -(U[ip] * x[ip] - U[im] * x[im]) / (T(2) * h) + nu * (x[ip] - T(2) * x[i] + x[im]) * inv_h2;
    } else {
        Lx = T(0);
    }
    Ld = T(-2) * nu * inv_h2;
}

// ---------------------------------------------------------------------------
// Arakawa's Jacobian J_A(p, w) ~ p_x w_y - p_y w_x: mean of the three
// second-order forms J++, J+x, Jx+ (energy- and enstrophy-conserving).
// Arguments are the 3x3 neighbourhoods a[dj+1][di+1] = a(i+di, j+dj).
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T arakawa9(const T p[3][3], const T w[3][3], T inv_12h2) {
    // shorthand: P(dj,di)
#define PP(dj, di) p[(dj) + 1][(di) + 1]
#define WW(dj, di) w[(dj) + 1][(di) + 1]
    const T jpp = (PP(0, 1) - PP(0, -1)) * (WW(1, 0) - WW(-1, 0)) - (PP(1, 0) - PP(-1, 0)) * (WW(0, 1) - WW(0, -1));
    const T jpx = PP(0, 1) * (WW(1, 1) - WW(-1, 1)) - PP(0, -1) * (WW(1, -1) - WW(-1, -1))
                - PP(1, 0) * (WW(1, 1) - WW(1, -1)) + PP(-1, 0) * (WW(-1, 1) - WW(-1, -1));
    const T jxp = WW(1, 0) * (PP(1, 1) - PP(1, -1)) - WW(-1, 0) * (PP(-1, 1) - PP(-1, -1))
                - WW(0, 1) * (PP(1, 1) - PP(-1, 1)) + WW(0, -1) * (PP(1, -1) - PP(-1, -1));
#undef PP
#undef WW
    return (jpp + jpx + jxp) * inv_12h2;
}

// sum of the magnitudes of the products that make up arakawa9 (the scale of
// its rounding error)
template <class T>
__device__ __forceinline__ T arakawa9_abs(const T p[3][3], const T w[3][3], T inv_12h2) {
#define PP(dj, di) p[(dj) + 1][(di) + 1]
#define WW(dj, di) w[(dj) + 1][(di) + 1]
    const T jpp = fabs((PP(0, 1) - PP(0, -1)) * (WW(1, 0) - WW(-1, 0))) + fabs((PP(1, 0) - PP(-1, 0)) * (WW(0, 1) - WW(0, -1)));
    const T jpx = fabs(PP(0, 1) * (WW(1, 1) - WW(-1, 1))) + fabs(PP(0, -1) * (WW(1, -1) - WW(-1, -1)))
                + fabs(PP(1, 0) * (WW(1, 1) - WW(1, -1))) + fabs(PP(-1, 0) * (WW(-1, 1) - WW(-1, -1)));
    const T jxp = fabs(WW(1, 0) * (PP(1, 1) - PP(1, -1))) + fabs(WW(-1, 0) * (PP(-1, 1) - PP(-1, -1)))
                + fabs(WW(0, 1) * (PP(1, 1) - PP(-1, 1))) + fabs(WW(0, -1) * (PP(1, -1) - PP(-1, -1)));
#undef PP
#undef WW
    return (jpp + jpx + jxp) * inv_12h2;
}

template <class T>
__device__ __forceinline__ void load3x3(const T *a, int i, int j, int nx, int ny, T out[3][3]) {
    const int is[3] = {wrapm(i - 1, nx), i, wrapm(i + 1, nx)};
    const int js[3] = {wrapm(j - 1, ny), j, wrapm(j + 1, ny)};
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
        for (int di = 0; di < 3; ++di) out[dj][di] = a[js[dj] * nx + is[di]];
}

template <class T>
__device__ __forceinline__ T lap5(const T a[3][3], T inv_h2) {
    return (a[1][2] + a[1][0] + a[2][1] + a[0][1] - T(4) * a[1][1]) * inv_h2;
}

// Vorticity block of the Picard linearization: K(Psi) x = J_A(Psi, x) + nu Lap x
template <class T, bool HAS_X>
__device__ __forceinline__ void vsf_omega_lin(const T *Psi, const T *x, int i, int j, int nx, int ny,
                                              T h, T nu, T &Lx, T &Ld) {
    const T inv_h2 = T(1) / (h * h);
    if (HAS_X) {
        T p[3][3], w[3][3];
        load3x3(Psi, i, j, nx, ny, p);
        load3x3(x, i, j, nx, ny, w);
        Lx = arakawa9(p, w, inv_h2 / T(12)) + nu * lap5(w, inv_h2);
    } else {
        Lx = T(0);
    }
    Ld = T(-4) * nu * inv_h2;      // J_A(Psi, .) has no centre coefficient
}

// Streamfunction block: Lap x (5-point)
template <class T, bool HAS_X>
__device__ __forceinline__ void poisson_lin(const T *x, int i, int j, int nx, int ny, T h, T &Lx, T &Ld) {
    const T inv_h2 = T(1) / (h * h);
    if (HAS_X) {
        const int ip = wrapm(i + 1, nx), im = wrapm(i - 1, nx);
        const int jp = wrapm(j + 1, ny), jm = wrapm(j - 1, ny);
        Lx = (x[j * nx + ip] + x[j * nx + im] + x[jp * nx + i] + x[jm * nx + i] - T(4) * x[j * nx + i]) * inv_h2;
    } else {
        Lx = T(0);
    }
    Ld = T(-4) * inv_h2;
}

}  // namespace irk
