// Geometric-multigrid V-cycle kernels with LDS tiles (gfx950, wave64).
//
// A V-cycle on levels 0..L-1 (2:1 coarsening, full-weighting restriction,
// (bi)linear prolongation, rediscretized level operators A = sigma M - dt L)
// is issued as
//   k_mg_down<l>  for every "tiled" level l < l0: Chebyshev pre-smoothing of
//                 degree D from x = 0, the residual b - A x, and its
//                 full-weighting restriction to the next level's b -- one
//                 launch; the tile plus a halo of D+2 cells lives in LDS and
//                 the D smoothing steps run on shrinking regions (temporal
//                 blocking), so x, d and the residual never touch HBM;
//   k_mg_subcycle for levels l0..L-1 (all small): the whole remaining
//                 V-cycle inside one work-group with every level in LDS,
//                 including the coarsest-level Chebyshev solve;
//   k_mg_up<l>    for l = l0-1..0: prolongation of the coarse correction and
//                 post-smoothing of degree D, one launch.
// The finest level reads its right-hand side directly from the float64
// Krylov vector(s) and writes the float64 preconditioned vector, so the
// precision casts cost no launches.
#include <hip/hip_runtime.h>

#include "irk_internal.h"
#include "kernels.h"
#include "mg_tiled.h"
#include "stencils.h"

namespace irk {

__device__ __forceinline__ int wrap_any(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

__device__ __forceinline__ int xcd_tile() {
    const int nb = gridDim.x, b = blockIdx.x;
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

// Level operator on an LDS window: neighbours at +-1 (x) and +-W (y); the
// window is already periodically unwrapped, so no index wrapping.
template <class T, int OPK, bool HAS_X>
__device__ __forceinline__ void lds_op(const T *cf, const T *x, int c, int W, T inv_h2, T h, T nu, T &Lx,
                                       T &Ld) {
    if constexpr (OPK == MG_NLDIFF) {
        const int nb[4] = {c + 1, c - 1, c + W, c - W};
        const T uc = cf[c];
        const T xc = HAS_X ? x[c] : T(0);
        T lx = 0, ld = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T un = cf[nb[q]];
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
    } else if constexpr (OPK == MG_BURGERS) {
        Lx = HAS_X ? (-(cf[c + 1] * x[c + 1] - cf[c - 1] * x[c - 1]) / (T(2) * h) +
                      nu * (x[c + 1] - T(2) * x[c] + x[c - 1]) * inv_h2)
                   : T(0);
        Ld = T(-2) * nu * inv_h2;
    } else if constexpr (OPK == MG_VSF_OMEGA) {
        if (HAS_X) {
            T p[3][3], w[3][3];
#pragma unroll
            for (int dj = 0; dj < 3; ++dj)
#pragma unroll
                for (int di = 0; di < 3; ++di) {
                    p[dj][di] = cf[c + (dj - 1) * W + (di - 1)];
                    w[dj][di] = x[c + (dj - 1) * W + (di - 1)];
                }
            Lx = arakawa9(p, w, inv_h2 / T(12)) + nu * lap5(w, inv_h2);
        } else {
            Lx = T(0);
        }
        Ld = T(-4) * nu * inv_h2;
    } else {
        Lx = HAS_X ? (x[c + 1] + x[c - 1] + x[c + W] + x[c - W] - T(4) * x[c]) * inv_h2 : T(0);
        Ld = T(-4) * inv_h2;
    }
}

// Iterate over the sub-box of a window: columns [a0, a1), rows [b0, b1).
// (column and row are advanced incrementally: no division per point)
#define FOR_BOX(a0, a1, b0, b1, W, ...)                                    \
    do {                                                                   \
        const int bw_ = (a1) - (a0), bn_ = bw_ * ((b1) - (b0));            \
        const int sx_ = (int)blockDim.x % bw_, sy_ = (int)blockDim.x / bw_; \
        int ca_ = (int)threadIdx.x % bw_, cb_ = (int)threadIdx.x / bw_;    \
        for (int q_ = threadIdx.x; q_ < bn_; q_ += blockDim.x) {           \
            const int ia = (a0) + ca_, ib = (b0) + cb_;                    \
            const int c = ib * (W) + ia;                                   \
            __VA_ARGS__;                                                   \
            ca_ += sx_;                                                    \
            cb_ += sy_;                                                    \
            if (ca_ >= bw_) { ca_ -= bw_; ++cb_; }                         \
        }                                                                  \
    } while (0)

// Points p = j * nx + i of an nx-wide level, strided over the work-group,
// with (i, j) advanced incrementally.
#define FOR_PTS(np_, nx_, ...)                                             \
    do {                                                                   \
        const int w_ = (nx_);                                              \
        const int sx_ = (int)blockDim.x % w_, sy_ = (int)blockDim.x / w_;  \
        int i = (int)threadIdx.x % w_, j = (int)threadIdx.x / w_;          \
        for (int p = threadIdx.x; p < (np_); p += blockDim.x) {            \
            __VA_ARGS__;                                                   \
            i += sx_;                                                      \
            j += sy_;                                                      \
            if (i >= w_) { i -= w_; ++j; }                                 \
        }                                                                  \
    } while (0)

// ---------------------------------------------------------------------------
// Down: pre-smoothing from x = 0, residual, restriction.
// ---------------------------------------------------------------------------
template <class T, int OPK, int TX, int TY, int D>
__global__ void __launch_bounds__(256) k_mg_down(MgLevelArgs<T> g, MgIn in) {
    constexpr int H = D + 2;                                   // halo of the window
    const bool two_d = g.ny > 1;
    const int hy = two_d ? H : 0;
    constexpr int W = TX + 2 * H;
    const int Hh = (two_d ? TY : 1) + 2 * hy;
    extern __shared__ unsigned char smem_raw[];
    T *cf = reinterpret_cast<T *>(smem_raw);
    T *bb = cf + W * Hh;
    T *xa = bb + W * Hh;
    T *xb = xa + W * Hh;
    T *dd = xb + W * Hh;

    const int tiles_x = (g.nx + TX - 1) / TX;
    const int tile = xcd_tile();
    const int ty = tile / tiles_x, tx = tile % tiles_x;
    const int i0 = tx * TX, j0 = ty * (two_d ? TY : 1);
    const int nx = g.nx, ny = g.ny;
    const T inv_h2 = T(1) / (g.h * g.h);

    // load coefficient (full window) and right-hand side (window minus 1)
    FOR_BOX(0, W, 0, Hh, W, {
        const int gi = wrap_any(i0 - H + ia, nx), gj = two_d ? wrap_any(j0 - hy + ib, ny) : 0;
        const size_t gidx = (size_t)gj * nx + gi;
        cf[c] = g.coef ? g.coef[gidx] : T(0);
        T rhs;
        if (in.v1) {
            double v = in.a1 * in.v1[gidx];
            if (in.v2) v += in.a2 * in.v2[gidx];
            if (in.mean) v -= in.a1 * in.mean[0] + (in.v2 ? in.a2 * in.mean[1] : 0.0);
            rhs = (T)v;
        } else {
            rhs = g.b[gidx];
        }
        bb[c] = rhs;
    });
    __syncthreads();

    // D Chebyshev steps on shrinking regions R(D+1) ... R(2)
    T *xcur = xa, *xnext = xb;
    for (int k = 0; k < D; ++k) {
        const int r = D + 1 - k;                 // region half-width added to the tile
        const int ax0 = H - r, ax1 = H + TX + r;
        const int by0 = two_d ? hy - r : 0, by1 = two_d ? hy + TY + r : 1;
        const T cd = g.cd[k], cr = g.cr[k];
        if (k == 0) {
            FOR_BOX(ax0, ax1, by0, by1, W, {
                T Lx, Ld;
                lds_op<T, OPK, false>(cf, nullptr, c, W, inv_h2, g.h, g.nu, Lx, Ld);
                const T diag = g.sigma - g.dt * Ld;
                const T dn = cr * bb[c] / diag;
                dd[c] = dn;
                xnext[c] = dn;
            });
        } else {
            FOR_BOX(ax0, ax1, by0, by1, W, {
                T Lx, Ld;
                lds_op<T, OPK, true>(cf, xcur, c, W, inv_h2, g.h, g.nu, Lx, Ld);
                const T xc = xcur[c];
                const T rr = bb[c] - (g.sigma * xc - g.dt * Lx);
                const T diag = g.sigma - g.dt * Ld;
                const T dn = cd * dd[c] + cr * rr / diag;
                dd[c] = dn;
                xnext[c] = xc + dn;
            });
        }
        __syncthreads();
        T *t = xcur;
        xcur = xnext;
        xnext = t;
    }
    // write the smoothed iterate on the tile
    FOR_BOX(H, H + TX, hy, hy + (two_d ? TY : 1), W, {
        const int gi = i0 + (ia - H), gj = j0 + (ib - hy);
        if (gi < nx && gj < ny) g.x[(size_t)gj * nx + gi] = xcur[c];
    });
    // residual on R(1) into dd
    FOR_BOX(H - 1, H + TX + 1, two_d ? hy - 1 : 0, two_d ? hy + TY + 1 : 1, W, {
        T Lx, Ld;
        lds_op<T, OPK, true>(cf, xcur, c, W, inv_h2, g.h, g.nu, Lx, Ld);
        dd[c] = bb[c] - (g.sigma * xcur[c] - g.dt * Lx);
    });
    __syncthreads();
    // full-weighting restriction to coarse points whose fine node lies in the tile
    const int nxc = nx / 2, nyc = two_d ? ny / 2 : 1;
    constexpr int CX = TX / 2;
    const int CY = two_d ? TY / 2 : 1;
    for (int q = threadIdx.x; q < CX * CY; q += blockDim.x) {
        const int I = i0 / 2 + q % CX, J = (two_d ? j0 / 2 : 0) + q / CX;
        if (I >= nxc || J >= nyc) continue;
        const int ca = H + 2 * (q % CX), cb = two_d ? hy + 2 * (q / CX) : 0;
        const int c = cb * W + ca;
        T acc;
        if (two_d) {
            acc = T(0.25) * dd[c] +
                  T(0.125) * (dd[c - 1] + dd[c + 1] + dd[c - W] + dd[c + W]) +
                  T(0.0625) * (dd[c - W - 1] + dd[c - W + 1] + dd[c + W - 1] + dd[c + W + 1]);
        } else {
            acc = T(0.5) * dd[c] + T(0.25) * (dd[c - 1] + dd[c + 1]);
        }
        g.bc[(size_t)J * nxc + I] = acc;
    }
}

// ---------------------------------------------------------------------------
// Up: prolongation of the coarse correction, then post-smoothing.
// ---------------------------------------------------------------------------
template <class T, int OPK, int TX, int TY, int D>
__global__ void __launch_bounds__(256) k_mg_up(MgLevelArgs<T> g, MgOut out) {
    constexpr int H = D;                                       // halo of the window
    const bool two_d = g.ny > 1;
    const int hy = two_d ? H : 0;
    constexpr int W = TX + 2 * H;
    const int Hh = (two_d ? TY : 1) + 2 * hy;
    extern __shared__ unsigned char smem_raw[];
    T *cf = reinterpret_cast<T *>(smem_raw);
    T *bb = cf + W * Hh;
    T *xa = bb + W * Hh;
    T *xb = xa + W * Hh;
    T *dd = xb + W * Hh;

    const int tiles_x = (g.nx + TX - 1) / TX;
    const int tile = xcd_tile();
    const int ty = tile / tiles_x, tx = tile % tiles_x;
    const int i0 = tx * TX, j0 = ty * (two_d ? TY : 1);
    const int nx = g.nx, ny = g.ny;
    const int nxc = nx / 2, nyc = two_d ? ny / 2 : 1;
    const T inv_h2 = T(1) / (g.h * g.h);

    FOR_BOX(0, W, 0, Hh, W, {
        const int gi = wrap_any(i0 - H + ia, nx), gj = two_d ? wrap_any(j0 - hy + ib, ny) : 0;
        const size_t gidx = (size_t)gj * nx + gi;
        cf[c] = g.coef ? g.coef[gidx] : T(0);
        T rhs;
        if (out.v1) {
            double v = out.a1 * out.v1[gidx];
            if (out.v2) v += out.a2 * out.v2[gidx];
            if (out.mean_in) v -= out.a1 * out.mean_in[0] + (out.v2 ? out.a2 * out.mean_in[1] : 0.0);
            rhs = (T)v;
        } else {
            rhs = g.b[gidx];
        }
        bb[c] = rhs;
        // prolongation: coarse node I sits at fine 2I
        const int I0 = gi >> 1, I1 = (gi & 1) ? (I0 + 1 == nxc ? 0 : I0 + 1) : I0;
        T e;
        if (two_d) {
            const int J0 = gj >> 1, J1 = (gj & 1) ? (J0 + 1 == nyc ? 0 : J0 + 1) : J0;
            e = T(0.25) * (g.xc[(size_t)J0 * nxc + I0] + g.xc[(size_t)J0 * nxc + I1] +
                           g.xc[(size_t)J1 * nxc + I0] + g.xc[(size_t)J1 * nxc + I1]);
        } else {
            e = T(0.5) * (g.xc[I0] + g.xc[I1]);
        }
        xa[c] = g.x[gidx] + e;
    });
    __syncthreads();
    T *xcur = xa, *xnext = xb;
    for (int k = 0; k < D; ++k) {
        const int r = D - 1 - k;
        const int ax0 = H - r, ax1 = H + TX + r;
        const int by0 = two_d ? hy - r : 0, by1 = two_d ? hy + TY + r : 1;
        const T cd = g.cd[k], cr = g.cr[k];
        FOR_BOX(ax0, ax1, by0, by1, W, {
            T Lx, Ld;
            lds_op<T, OPK, true>(cf, xcur, c, W, inv_h2, g.h, g.nu, Lx, Ld);
            const T xc = xcur[c];
            const T rr = bb[c] - (g.sigma * xc - g.dt * Lx);
            const T diag = g.sigma - g.dt * Ld;
            const T dn = (k == 0 ? T(0) : cd * dd[c]) + cr * rr / diag;
            dd[c] = dn;
            xnext[c] = xc + dn;
        });
        __syncthreads();
        T *t = xcur;
        xcur = xnext;
        xnext = t;
    }
    FOR_BOX(H, H + TX, hy, hy + (two_d ? TY : 1), W, {
        const int gi = i0 + (ia - H), gj = j0 + (ib - hy);
        if (gi < nx && gj < ny) {
            const size_t gidx = (size_t)gj * nx + gi;
            if (out.z) out.z[gidx] = (double)xcur[c] + (out.shift ? out.shift_scale * out.shift[0] : 0.0);
            else g.xout[gidx] = xcur[c];
        }
    });
}

// ---------------------------------------------------------------------------
// The V-cycle on levels l0..L-1 in one work-group, every level in LDS.
// ---------------------------------------------------------------------------
// Gershgorin ratio sum_{j != i} |a_ij| / |a_ii| of row i of A = sigma M - dt L
// on a level (periodic), from the operator's stencil coefficients.
template <class T, int OPK>
__device__ T row_ratio(const T *cf, int i, int j, int nx, int ny, T h, T nu, T sigma, T dt) {
    const T inv_h2 = T(1) / (h * h);
    if constexpr (OPK == MG_NLDIFF) {
        const int ip = wrapm(i + 1, nx), im = wrapm(i - 1, nx), jp = wrapm(j + 1, ny), jm = wrapm(j - 1, ny);
        const int nb[4] = {j * nx + ip, j * nx + im, jp * nx + i, jm * nx + i};
        const T uc = cf[j * nx + i];
        T off = 0, ld = 0;
        for (int q = 0; q < 4; ++q) {
            const T un = cf[nb[q]];
            const T kf = T(1) + T(0.5) * (uc * uc + un * un);
            const T du = un - uc;
            off += fabs(dt * inv_h2 * (kf + du * un));
            ld += -kf + du * uc;
        }
        return off / fabs(sigma - dt * ld * inv_h2);
    } else if constexpr (OPK == MG_BURGERS) {
        const int ip = wrapm(i + 1, nx), im = wrapm(i - 1, nx);
        const T off = fabs(dt * (-cf[ip] / (T(2) * h) + nu * inv_h2)) + fabs(dt * (cf[im] / (T(2) * h) + nu * inv_h2));
        return off / fabs(sigma + T(2) * dt * nu * inv_h2);
    } else if constexpr (OPK == MG_VSF_OMEGA) {
        T p[3][3], e[3][3];
        for (int dj = 0; dj < 3; ++dj)
            for (int di = 0; di < 3; ++di) {
                p[dj][di] = cf[wrapm(j + dj - 1, ny) * nx + wrapm(i + di - 1, nx)];
                e[dj][di] = T(0);
            }
        T off = 0;
        for (int dj = 0; dj < 3; ++dj)
            for (int di = 0; di < 3; ++di) {
                if (dj == 1 && di == 1) continue;
                e[dj][di] = T(1);
                T cnb = arakawa9(p, e, inv_h2 / T(12));
                if (dj == 1 || di == 1) cnb += nu * inv_h2;
                e[dj][di] = T(0);
                off += fabs(dt * cnb);
            }
        return off / fabs(sigma + T(4) * dt * nu * inv_h2);
    } else {
        return sigma == T(0) ? T(1) : T(4) * dt * inv_h2 / fabs(sigma + T(4) * dt * inv_h2);
    }
}

template <class T, int OPK>
__device__ void wg_cheb(const T *cf, T *x, const T *b, T *r, T *d, int nx, int ny, T h, T nu, T sigma, T dt,
                        const T *cd, const T *cr, int nsteps, bool from_zero) {
    const int np = nx * ny;
    const T inv_h2 = T(1) / (h * h);
    for (int k = 0; k < nsteps; ++k) {
        // r <- D^{-1} (b - A x)
        FOR_PTS(np, nx, {
            T Lx, Ld;
            T xc = from_zero && k == 0 ? T(0) : x[p];
            if (OPK == MG_VSF_OMEGA) {
                T pp[3][3], ww[3][3];
                for (int dj = 0; dj < 3; ++dj)
                    for (int di = 0; di < 3; ++di) {
                        const int q = wrap_any(j + dj - 1, ny) * nx + wrap_any(i + di - 1, nx);
                        pp[dj][di] = cf[q];
                        ww[dj][di] = (from_zero && k == 0) ? T(0) : x[q];
                    }
                Lx = arakawa9(pp, ww, inv_h2 / T(12)) + nu * lap5(ww, inv_h2);
                Ld = T(-4) * nu * inv_h2;
            } else if (from_zero && k == 0) {
                level_op<T, OPK, false>(cf, x, i, j, nx, ny, h, nu, Lx, Ld);
            } else {
                level_op<T, OPK, true>(cf, x, i, j, nx, ny, h, nu, Lx, Ld);
            }
            r[p] = (b[p] - (sigma * xc - dt * Lx)) / (sigma - dt * Ld);
        });
        __syncthreads();
        for (int p = threadIdx.x; p < np; p += blockDim.x) {
            const T dn = (k == 0 ? T(0) : cd[k] * d[p]) + cr[k] * r[p];
            d[p] = dn;
            x[p] = (from_zero && k == 0 ? T(0) : x[p]) + dn;
        }
        __syncthreads();
    }
}

template <class T, int OPK>
__global__ void __launch_bounds__(1024) k_mg_subcycle(MgSubArgs<T> s, MgIn in, MgOut out) {
    extern __shared__ unsigned char smem_raw[];
    T *base = reinterpret_cast<T *>(smem_raw);
    // per level: x, b, coef (consecutive blocks); then shared scratch r, d
    // sized for the finest level.  Level pointers are recomputed from the
    // sizes (uniform scalar arithmetic) instead of being kept in an array.
    auto lev_base = [&](int l) {
        size_t off = 0;
        for (int q = 0; q < l; ++q) off += 3 * (size_t)s.nx[q] * s.ny[q];
        return base + off;
    };
#define X(l) (lev_base(l))
#define B(l) (lev_base(l) + (size_t)s.nx[l] * s.ny[l])
#define C(l) (lev_base(l) + 2 * (size_t)s.nx[l] * s.ny[l])
    T *R = lev_base(s.nlev);
    T *Dv = R + s.nx[0] * s.ny[0];
    const int np0 = s.nx[0] * s.ny[0];
    for (int p = threadIdx.x; p < np0; p += blockDim.x) {
        T rhs;
        if (in.v1) {
            double v = in.a1 * in.v1[p];
            if (in.v2) v += in.a2 * in.v2[p];
            if (in.mean) v -= in.a1 * in.mean[0] + (in.v2 ? in.a2 * in.mean[1] : 0.0);
            rhs = (T)v;
        } else {
            rhs = s.b0[p];
        }
        B(0)[p] = rhs;
    }
    for (int l = 0; l < s.nlev; ++l) {
        const int np = s.nx[l] * s.ny[l];
        for (int p = threadIdx.x; p < np; p += blockDim.x) C(l)[p] = s.coef[l] ? s.coef[l][p] : T(0);
    }
    __syncthreads();
    const int L = s.nlev;
    for (int l = 0; l < L - 1; ++l) {
        const int nx = s.nx[l], ny = s.ny[l], np = nx * ny;
        wg_cheb<T, OPK>(C(l), X(l), B(l), R, Dv, nx, ny, s.h[l], s.nu, s.sigma, s.dt, s.cd, s.cr, s.deg, true);
        // residual into R, then full weighting into B(l+1)
        FOR_PTS(np, nx, {
            T Lx, Ld;
            level_op<T, OPK, true>(C(l), X(l), i, j, nx, ny, s.h[l], s.nu, Lx, Ld);
            R[p] = B(l)[p] - (s.sigma * X(l)[p] - s.dt * Lx);
        });
        __syncthreads();
        const int nxc = s.nx[l + 1], nyc = s.ny[l + 1];
        FOR_PTS(nxc * nyc, nxc, {
            const int I = i, J = j, q = p;
            T acc;
            if (ny > 1) {
                acc = 0;
                for (int bj = -1; bj <= 1; ++bj)
                    for (int ai = -1; ai <= 1; ++ai) {
                        const T w = (ai == 0 ? T(0.5) : T(0.25)) * (bj == 0 ? T(0.5) : T(0.25));
                        acc += w * R[wrap_any(2 * J + bj, ny) * nx + wrap_any(2 * I + ai, nx)];
                    }
            } else {
                acc = T(0.5) * R[2 * I] + T(0.25) * (R[wrap_any(2 * I - 1, nx)] + R[wrap_any(2 * I + 1, nx)]);
            }
            B(l + 1)[q] = acc;
        });
        __syncthreads();
    }
    {
        // coarsest level: Chebyshev iteration on a Gershgorin interval
        // [1 - rho, 1 + rho] of D^{-1} A computed here; the singular periodic
        // Poisson operator (rho = 1) is solved on mean-free data with the
        // interval's lower end at its smallest nonzero eigenvalue
        const int l = L - 1, nx = s.nx[l], ny = s.ny[l], np = nx * ny;
        __shared__ double red[16];
        const bool singular = (OPK == MG_POISSON && s.sigma == T(0));
        if (singular) {
            double acc = 0;
            for (int p = threadIdx.x; p < np; p += blockDim.x) acc += (double)B(l)[p];
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
            __syncthreads();
            double tot = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += red[w];
            const T m = (T)(tot / np);
            __syncthreads();
            for (int p = threadIdx.x; p < np; p += blockDim.x) B(l)[p] -= m;
            __syncthreads();
        }
        double rho = 0.0;
        FOR_PTS(np, nx, rho = fmax(rho, (double)row_ratio<T, OPK>(C(l), i, j, nx, ny, s.h[l], s.nu, s.sigma, s.dt)));
        for (int off = 32; off > 0; off >>= 1) rho = fmax(rho, __shfl_xor(rho, off, 64));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rho;
        __syncthreads();
        rho = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) rho = fmax(rho, red[w]);
        __syncthreads();
        double lmin = 1.0 - rho, lmax = 1.0 + rho;
        if (singular || lmin < 0.05) {
            const double sx = sin(3.14159265358979323846 / nx), sy = ny > 1 ? sin(3.14159265358979323846 / ny) : 1.0;
            lmin = fmax(0.5 * fmin(sx * sx, sy * sy), 0.02);
        }
        // steps for a 1e-3 reduction of the Chebyshev bound 2 r^k
        const double kap = lmax / lmin, sq = sqrt(kap);
        const double rr = (sq - 1.0) / (sq + 1.0);
        int iters = rr > 0.0 ? (int)ceil(log(2000.0) / -log(rr)) : 1;
        iters = iters < 2 ? 2 : (iters > s.coarse_iters ? s.coarse_iters : iters);
        __shared__ T ccd[IRK_MAX_COARSE_ITERS], ccr[IRK_MAX_COARSE_ITERS];
        if (threadIdx.x == 0) {
            const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
            const double sig1 = theta / delta;
            double rho_k = 1.0 / sig1;
            for (int k = 0; k < iters; ++k) {
                if (k == 0) { ccd[0] = T(0); ccr[0] = (T)(1.0 / theta); }
                else {
                    const double rn = 1.0 / (2.0 * sig1 - rho_k);
                    ccd[k] = (T)(rn * rho_k);
                    ccr[k] = (T)(2.0 * rn / delta);
                    rho_k = rn;
                }
            }
        }
        __syncthreads();
        wg_cheb<T, OPK>(C(l), X(l), B(l), R, Dv, nx, ny, s.h[l], s.nu, s.sigma, s.dt, ccd, ccr, iters, true);
    }
    for (int l = L - 2; l >= 0; --l) {
        const int nx = s.nx[l], ny = s.ny[l], np = nx * ny;
        const int nxc = s.nx[l + 1], nyc = s.ny[l + 1];
        FOR_PTS(np, nx, {
            const int I0 = i >> 1, I1 = (i & 1) ? (I0 + 1 == nxc ? 0 : I0 + 1) : I0;
            T e;
            if (ny > 1) {
                const int J0 = j >> 1, J1 = (j & 1) ? (J0 + 1 == nyc ? 0 : J0 + 1) : J0;
                e = T(0.25) * (X(l + 1)[J0 * nxc + I0] + X(l + 1)[J0 * nxc + I1] + X(l + 1)[J1 * nxc + I0] +
                               X(l + 1)[J1 * nxc + I1]);
            } else {
                e = T(0.5) * (X(l + 1)[I0] + X(l + 1)[I1]);
            }
            X(l)[p] += e;
        });
        __syncthreads();
        wg_cheb<T, OPK>(C(l), X(l), B(l), R, Dv, nx, ny, s.h[l], s.nu, s.sigma, s.dt, s.cd, s.cr, s.deg, false);
    }
    for (int p = threadIdx.x; p < np0; p += blockDim.x) {
        if (out.z) out.z[p] = (double)X(0)[p] + (out.shift ? out.shift_scale * out.shift[0] : 0.0);
        else s.x0[p] = X(0)[p];
    }
}
#undef X
#undef B
#undef C

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <class T, int OPK, int TX, int TY>
static void down_t(hipStream_t st, const MgLevelArgs<T> &a, const MgIn &in, int deg) {
    const int tiles = ((a.nx + TX - 1) / TX) * (a.ny > 1 ? (a.ny + TY - 1) / TY : 1);
    const int H = deg + 2;
    const size_t shm = (size_t)5 * (TX + 2 * H) * ((a.ny > 1 ? TY : 1) + (a.ny > 1 ? 2 * H : 0)) * sizeof(T);
    switch (deg) {
        case 1: k_mg_down<T, OPK, TX, TY, 1><<<tiles, 256, shm, st>>>(a, in); break;
        case 2: k_mg_down<T, OPK, TX, TY, 2><<<tiles, 256, shm, st>>>(a, in); break;
        case 3: k_mg_down<T, OPK, TX, TY, 3><<<tiles, 256, shm, st>>>(a, in); break;
        default: k_mg_down<T, OPK, TX, TY, 4><<<tiles, 256, shm, st>>>(a, in); break;
    }
}

template <class T, int OPK, int TX, int TY>
static void up_t(hipStream_t st, const MgLevelArgs<T> &a, const MgOut &out, int deg) {
    const int tiles = ((a.nx + TX - 1) / TX) * (a.ny > 1 ? (a.ny + TY - 1) / TY : 1);
    const int H = deg;
    const size_t shm = (size_t)5 * (TX + 2 * H) * ((a.ny > 1 ? TY : 1) + (a.ny > 1 ? 2 * H : 0)) * sizeof(T);
    switch (deg) {
        case 1: k_mg_up<T, OPK, TX, TY, 1><<<tiles, 256, shm, st>>>(a, out); break;
        case 2: k_mg_up<T, OPK, TX, TY, 2><<<tiles, 256, shm, st>>>(a, out); break;
        case 3: k_mg_up<T, OPK, TX, TY, 3><<<tiles, 256, shm, st>>>(a, out); break;
        default: k_mg_up<T, OPK, TX, TY, 4><<<tiles, 256, shm, st>>>(a, out); break;
    }
}

// tile shape per level size: wide tiles on big levels, small tiles (more
// work-groups) on small ones; 1-D levels use 256-point strips
template <class T, int OPK>
static void down_dispatch(hipStream_t st, const MgLevelArgs<T> &a, const MgIn &in, int deg) {
    if (a.ny == 1) down_t<T, OPK, 256, 1>(st, a, in, deg);
    else if (a.nx >= 128) down_t<T, OPK, 32, 8>(st, a, in, deg);
    else down_t<T, OPK, 16, 8>(st, a, in, deg);
}

template <class T, int OPK>
static void up_dispatch(hipStream_t st, const MgLevelArgs<T> &a, const MgOut &out, int deg) {
    if (a.ny == 1) up_t<T, OPK, 256, 1>(st, a, out, deg);
    else if (a.nx >= 128) up_t<T, OPK, 32, 8>(st, a, out, deg);
    else up_t<T, OPK, 16, 8>(st, a, out, deg);
}

template <class T>
void launch_mg_down(hipStream_t st, int opk, const MgLevelArgs<T> &a, const MgIn &in, int deg) {
    switch (opk) {
        case MG_NLDIFF: down_dispatch<T, MG_NLDIFF>(st, a, in, deg); break;
        case MG_BURGERS: down_dispatch<T, MG_BURGERS>(st, a, in, deg); break;
        case MG_VSF_OMEGA: down_dispatch<T, MG_VSF_OMEGA>(st, a, in, deg); break;
        default: down_dispatch<T, MG_POISSON>(st, a, in, deg); break;
    }
}

template <class T>
void launch_mg_up(hipStream_t st, int opk, const MgLevelArgs<T> &a, const MgOut &out, int deg) {
    switch (opk) {
        case MG_NLDIFF: up_dispatch<T, MG_NLDIFF>(st, a, out, deg); break;
        case MG_BURGERS: up_dispatch<T, MG_BURGERS>(st, a, out, deg); break;
        case MG_VSF_OMEGA: up_dispatch<T, MG_VSF_OMEGA>(st, a, out, deg); break;
        default: up_dispatch<T, MG_POISSON>(st, a, out, deg); break;
    }
}

template <class T>
size_t mg_subcycle_lds_bytes(const MgSubArgs<T> &s) {
    size_t n = 0;
    for (int l = 0; l < s.nlev; ++l) n += 3 * (size_t)s.nx[l] * s.ny[l];
    n += 2 * (size_t)s.nx[0] * s.ny[0];
    return n * sizeof(T);
}

template <class T>
void launch_mg_subcycle(hipStream_t st, int opk, const MgSubArgs<T> &s, const MgIn &in, const MgOut &out) {
    const size_t shm = mg_subcycle_lds_bytes(s);
    const int np0 = s.nx[0] * s.ny[0];
    const unsigned nt = np0 >= 1024 ? 1024 : ((np0 + 63) / 64) * 64;
    switch (opk) {
        case MG_NLDIFF: k_mg_subcycle<T, MG_NLDIFF><<<1, nt, shm, st>>>(s, in, out); break;
        case MG_BURGERS: k_mg_subcycle<T, MG_BURGERS><<<1, nt, shm, st>>>(s, in, out); break;
        case MG_VSF_OMEGA: k_mg_subcycle<T, MG_VSF_OMEGA><<<1, nt, shm, st>>>(s, in, out); break;
        default: k_mg_subcycle<T, MG_POISSON><<<1, nt, shm, st>>>(s, in, out); break;
    }
}

template void launch_mg_down<float>(hipStream_t, int, const MgLevelArgs<float> &, const MgIn &, int);
template void launch_mg_down<double>(hipStream_t, int, const MgLevelArgs<double> &, const MgIn &, int);
template void launch_mg_up<float>(hipStream_t, int, const MgLevelArgs<float> &, const MgOut &, int);
template void launch_mg_up<double>(hipStream_t, int, const MgLevelArgs<double> &, const MgOut &, int);
template void launch_mg_subcycle<float>(hipStream_t, int, const MgSubArgs<float> &, const MgIn &, const MgOut &);
template void launch_mg_subcycle<double>(hipStream_t, int, const MgSubArgs<double> &, const MgIn &, const MgOut &);
template size_t mg_subcycle_lds_bytes<float>(const MgSubArgs<float> &);
template size_t mg_subcycle_lds_bytes<double>(const MgSubArgs<double> &);

}  // namespace irk
