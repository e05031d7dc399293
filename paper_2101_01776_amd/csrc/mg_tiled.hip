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
//
// Each kernel first turns the level's linearization field into the explicit
// stencil of A on its LDS window, scaled by the Jacobi diagonal:
// a~_q = A_q / A_c for the NS off-diagonal neighbours q, A_c, and
// b~ = b / A_c.  A Chebyshev step is then d <- cd d + cr (b~ - x - sum_q
// a~_q x_q), x <- x + d: a few fused multiply-adds per point instead of
// re-deriving the nonlinear face coefficients and dividing by the diagonal in
// every sweep (the sweeps are bound by vector-ALU issue, not by memory).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "irk_internal.h"
#include "kernels.h"
#include "mg_tiled.h"
#include "stencils.h"

namespace irk {

// index wrap for i in [-n, 2n)
__device__ __forceinline__ int wrap2(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// 1 / x for the Jacobi scaling of a level stencil: float32 uses the
// hardware reciprocal (within 1 ulp; the diagonal is at least sigma > 0, far
// from denormals) instead of the correctly rounded division sequence,
// float64 divides
template <class T>
__device__ __forceinline__ T stencil_rcp(T x) {
    if constexpr (sizeof(T) == sizeof(float)) return __builtin_amdgcn_rcpf(x);
    else return T(1) / x;
}

__device__ __forceinline__ int xcd_tile() {
    const int nb = gridDim.x, b = blockIdx.x;
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

// Off-diagonal neighbours of the level stencils: 5-point operators use
// E, W, N, S; 1-D Burgers E, W; the vorticity operator (Arakawa Jacobian +
// viscous Laplacian) all eight.
template <int OPK>
struct StencilShape {
    static constexpr int NS = (OPK == MG_VSF_OMEGA) ? 8 : (OPK == MG_BURGERS ? 2 : 4);
};

// neighbour q at (di, dj): E(+1,0) W(-1,0) N(0,+1) S(0,-1) NE NW SE SW
__device__ __forceinline__ int nb_off(int q, int W) {
    switch (q) {
        case 0: return 1;
        case 1: return -1;
        case 2: return W;
        case 3: return -W;
        case 4: return W + 1;
        case 5: return W - 1;
        case 6: return -W + 1;
        default: return -W - 1;
    }
}

// Stencil of A = sigma M - dt L at point c of an array with row stride W
// (neighbours at c + nb_off(q, W) must exist): off-diagonals a[q], diagonal ac.
template <class T, int OPK>
__device__ __forceinline__ void build_stencil(const T *cf, int c, int W, T inv_h2, T h, T nu, T sigma, T dt,
                                              T (&a)[StencilShape<OPK>::NS], T &ac) {
    if constexpr (OPK == MG_NLDIFF) {
        // L x = h^-2 sum_f [kf (x_nb - x_c) + (u_nb - u_c)(u_c x_c + u_nb x_nb)],
        // kf = 1 + (u_c^2 + u_nb^2)/2: coefficient of x_nb is kf + du u_nb, of
        // x_c the sum of -kf + du u_c
        const T uc = cf[c];
        T ld = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T un = cf[c + nb_off(q, W)];
            const T kf = T(1) + T(0.5) * (uc * uc + un * un);
            const T du = un - uc;
            a[q] = -dt * inv_h2 * (kf + du * un);
            ld += -kf + du * uc;
        }
        ac = sigma - dt * inv_h2 * ld;
    } else if constexpr (OPK == MG_BURGERS) {
        const T i2h = T(0.5) / h;
        a[0] = -dt * (-cf[c + 1] * i2h + nu * inv_h2);
        a[1] = -dt * (cf[c - 1] * i2h + nu * inv_h2);
        ac = sigma + T(2) * dt * nu * inv_h2;
    } else if constexpr (OPK == MG_VSF_OMEGA) {
        // coefficients of x in J_A(psi, x) (the three second-order forms of
        // Arakawa's Jacobian, divided by 12 h^2) plus nu times the 5-point
        // Laplacian; psi(di, dj) = cf[c + dj W + di]
#define PS(dj, di) cf[c + (dj) * W + (di)]
        const T k = inv_h2 / T(12), v = nu * inv_h2;
        T L[8];
        L[0] = (-(PS(1, 0) - PS(-1, 0)) - (PS(1, 1) - PS(-1, 1))) * k + v;      // E
        L[1] = ((PS(1, 0) - PS(-1, 0)) + (PS(1, -1) - PS(-1, -1))) * k + v;     // W
        L[2] = ((PS(0, 1) - PS(0, -1)) + (PS(1, 1) - PS(1, -1))) * k + v;       // N
        L[3] = (-(PS(0, 1) - PS(0, -1)) - (PS(-1, 1) - PS(-1, -1))) * k + v;    // S
        L[4] = (PS(0, 1) - PS(1, 0)) * k;                                       // NE
        L[5] = (PS(1, 0) - PS(0, -1)) * k;                                      // NW
        L[6] = (PS(-1, 0) - PS(0, 1)) * k;                                      // SE
        L[7] = (PS(0, -1) - PS(-1, 0)) * k;                                     // SW
#undef PS
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] = -dt * L[q];
        ac = sigma + T(4) * dt * v;
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = -dt * inv_h2;
        ac = sigma + T(4) * dt * inv_h2;
    }
}


// (t / w, t % w) for 0 <= t < 2^20, 1 <= w <= 2^16 with a float reciprocal
// (the quotient estimate is off by at most one; one correction each way)
// instead of the integer division sequence
__device__ __forceinline__ void divmod_small(int t, int w, int &q, int &r) {
    q = (int)((float)t * __builtin_amdgcn_rcpf((float)w));
    r = t - q * w;
    if (r < 0) { r += w; --q; }
    if (r >= w) { r -= w; ++q; }
}

// Points p = j * nx + i of an nx-wide level, strided over the work-group,
// with (i, j) advanced incrementally.
#define FOR_PTS(np_, nx_, ...)                                             \
    do {                                                                   \
        const int w_ = (nx_);                                              \
        const int sx_ = (int)blockDim.x % w_, sy_ = (int)blockDim.x / w_;  \
        int i, j;                                                          \
        divmod_small((int)threadIdx.x, w_, j, i);                          \
        for (int p = threadIdx.x; p < (np_); p += blockDim.x) {            \
            __VA_ARGS__;                                                   \
            i += sx_;                                                      \
            j += sy_;                                                      \
            if (i >= w_) { i -= w_; ++j; }                                 \
        }                                                                  \
    } while (0)

// The window points a thread loads: q = threadIdx.x + 256 k, k < NPT, with
// their periodic global coordinates (clamped to a valid point when q lies
// past the window, so every address is in bounds).
template <int NPT>
struct WindowIndex {
    int gi[NPT], gj[NPT];
    size_t gidx[NPT];
    int npl_;
    template <int W, int H>
    __device__ __forceinline__ void init(int npl, int i0, int j0, int nx, int ny, bool two_d) {
        npl_ = npl;
        const int hy = two_d ? H : 0;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int qq = q(k) < npl ? q(k) : 0;
            const int ia = qq % W, ib = qq / W;
            gi[k] = wrap2(i0 - H + ia, nx);
            gj[k] = two_d ? wrap2(j0 - hy + ib, ny) : 0;
            gidx[k] = (size_t)gj[k] * nx + gi[k];
        }
    }
    __device__ __forceinline__ int q(int k) const { return (int)threadIdx.x + 256 * k; }
    __device__ __forceinline__ bool ok(int k) const { return q(k) < npl_; }
};

template <int NPT, class T>
__device__ __forceinline__ void load_field(const T *f, const WindowIndex<NPT> &wi, T (&v)[NPT]) {
    if (f) {
#pragma unroll
        for (int k = 0; k < NPT; ++k) v[k] = f[wi.gidx[k]];
    } else {
#pragma unroll
        for (int k = 0; k < NPT; ++k) v[k] = T(0);
    }
}

// right-hand side a1 v1 + a2 v2 - (a1 mean[0] + a2 mean[1]) from float64
// vectors (v2 and mean optional), or the level's own b when v1 is null
template <class T, int NPT>
__device__ __forceinline__ void load_rhs(const double *v1, double a1, const double *v2, double a2,
                                         const double *mean, const T *b, const WindowIndex<NPT> &wi,
                                         T (&rv)[NPT]) {
    if (v1) {
        double v[NPT], w[NPT];
#pragma unroll
        for (int k = 0; k < NPT; ++k) v[k] = v1[wi.gidx[k]];
        if (v2) {
#pragma unroll
            for (int k = 0; k < NPT; ++k) w[k] = v2[wi.gidx[k]];
        }
        const double m = mean ? a1 * mean[0] + (v2 ? a2 * mean[1] : 0.0) : 0.0;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            double t = a1 * v[k];
            if (v2) t += a2 * w[k];
            rv[k] = (T)(t - m);
        }
    } else {
#pragma unroll
        for (int k = 0; k < NPT; ++k) rv[k] = b[wi.gidx[k]];
    }
}

// LDS of a tiled kernel's window (npl = window points): the linearization
// field (later the residual) and two iterates.  Everything else a point
// needs -- its scaled stencil, b~ and the Chebyshev direction -- stays in
// the registers of the thread that owns the point (window point q belongs
// to thread q mod 256, the same thread that loaded it).
__host__ __device__ constexpr int tile_arrays() { return 3; }

// Scaled stencil rows of a thread's window points (all but the outer ring
// of the window): a~_q = A_q / A_c in a, A_c in ac, b~ = b / A_c in bv.
template <class T, int OPK, int NPT, int W>
__device__ __forceinline__ void own_stencils(const T *cf, const WindowIndex<NPT> &wi, int Hh, bool two_d,
                                             const MgLevelArgs<T> &g, T inv_h2,
                                             T (&a)[NPT][StencilShape<OPK>::NS], T (&ac)[NPT], T (&bv)[NPT]) {
    constexpr int NS = StencilShape<OPK>::NS;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int q = wi.q(k), ia = q % W, ib = q / W;
        const bool inner = wi.ok(k) && ia >= 1 && ia < W - 1 && (!two_d || (ib >= 1 && ib < Hh - 1));
        if (inner) {
            build_stencil<T, OPK>(cf, q, W, inv_h2, g.h, g.nu, g.sigma, g.dt, a[k], ac[k]);
            const T inv = stencil_rcp(ac[k]);
#pragma unroll
            for (int m = 0; m < NS; ++m) a[k][m] *= inv;
            bv[k] *= inv;
        } else {
#pragma unroll
            for (int m = 0; m < NS; ++m) a[k][m] = T(0);
            ac[k] = T(1);
        }
    }
}

// b~ - x - sum_q a~_q x_q at window point c (D^{-1}(b - A x))
template <class T, int OPK, int W>
__device__ __forceinline__ T own_jres(const T (&a)[StencilShape<OPK>::NS], T bv, const T *x, int c, T xv) {
    constexpr int NS = StencilShape<OPK>::NS;
    T r = bv - xv;
#pragma unroll
    for (int m = 0; m < NS; ++m) r -= a[m] * x[c + nb_off(m, W)];
    return r;
}

// ---------------------------------------------------------------------------
// Down: pre-smoothing from x = 0, residual, restriction.
// ---------------------------------------------------------------------------
template <class T, int OPK, int TX, int TY, int D>
__device__ __forceinline__ void mg_down_body(const MgLevelArgs<T> &g, const MgIn &in, const int tile) {
    constexpr int NS = StencilShape<OPK>::NS;
    constexpr int H = D + 2;                                   // halo of the window
    constexpr bool two_d = OPK != MG_BURGERS;                 // (1-D Burgers: ny == 1)
    const int hy = two_d ? H : 0;
    constexpr int W = TX + 2 * H;
    const int Hh = (two_d ? TY : 1) + 2 * hy;
    const int npl = W * Hh;
    extern __shared__ unsigned char smem_raw[];
    T *cf = reinterpret_cast<T *>(smem_raw);
    T *xa = cf + npl;
    T *xb = xa + npl;

    const int tiles_x = (g.nx + TX - 1) / TX;
    const int ty = tile / tiles_x, tx = tile % tiles_x;
    const int i0 = tx * TX, j0 = ty * (two_d ? TY : 1);
    const int nx = g.nx, ny = g.ny;
    const T inv_h2 = T(1) / (g.h * g.h);

    // load the linearization field and the right-hand side on the window:
    // every load of the thread is issued before the first one is used
    constexpr int NPT = (W * (TY + 2 * H) + 255) / 256;
    WindowIndex<NPT> wi;
    wi.template init<W, H>(npl, i0, j0, nx, ny, two_d);
    T bv[NPT];
    {
        T cfv[NPT];
        load_field<NPT>(g.coef, wi, cfv);
        load_rhs<T, NPT>(in.v1, in.a1, in.v2, in.a2, in.mean, g.b, wi, bv);
#pragma unroll
        for (int k = 0; k < NPT; ++k)
            if (wi.ok(k)) cf[wi.q(k)] = cfv[k];
    }
    __syncthreads();
    T a[NPT][NS], ac[NPT];
    own_stencils<T, OPK, NPT, W>(cf, wi, Hh, two_d, g, inv_h2, a, ac, bv);

    // D Chebyshev steps on shrinking regions R(D+1) ... R(2) (the thread's
    // own points inside the region)
    T dv[NPT];
    T *xcur = xa, *xnext = xb;
    for (int st = 0; st < D; ++st) {
        const int r = D + 1 - st;                // region half-width added to the tile
        const int ax0 = H - r, ax1 = H + TX + r;
        const int by0 = two_d ? hy - r : 0, by1 = two_d ? hy + TY + r : 1;
        const T cd = g.cd[st], cr = g.cr[st];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int c = wi.q(k), ia = c % W, ib = c / W;
            if (wi.ok(k) && ia >= ax0 && ia < ax1 && ib >= by0 && ib < by1) {
                if (st == 0) {
                    const T dn = cr * bv[k];
                    dv[k] = dn;
                    xnext[c] = dn;
                } else {
                    const T xv = xcur[c];
                    const T dn = cd * dv[k] + cr * own_jres<T, OPK, W>(a[k], bv[k], xcur, c, xv);
                    dv[k] = dn;
                    xnext[c] = xv + dn;
                }
            }
        }
        __syncthreads();
        T *t = xcur;
        xcur = xnext;
        xnext = t;
    }
    // write the smoothed iterate on the tile; residual b - A x on R(1)
    // (not on the coarsest level of a cycle that stops here: bc == nullptr,
    // the same for the whole work-group)
    const bool restrict_down = g.bc != nullptr;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int c = wi.q(k), ia = c % W, ib = c / W;
        if (!wi.ok(k)) continue;
        const T xv = xcur[c];
        if (ia >= H && ia < H + TX && ib >= hy && ib < hy + (two_d ? TY : 1)) {
            const int gi = i0 + (ia - H), gj = j0 + (ib - hy);
            if (gi < nx && gj < ny) g.x[(size_t)gj * nx + gi] = xv;
        }
        if (restrict_down && ia >= H - 1 && ia < H + TX + 1 && (!two_d || (ib >= hy - 1 && ib < hy + TY + 1)))
            xnext[c] = ac[k] * own_jres<T, OPK, W>(a[k], bv[k], xcur, c, xv);
    }
    if (!restrict_down) return;
    __syncthreads();
    const T *rr = xnext;
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
            acc = T(0.25) * rr[c] +
                  T(0.125) * (rr[c - 1] + rr[c + 1] + rr[c - W] + rr[c + W]) +
                  T(0.0625) * (rr[c - W - 1] + rr[c - W + 1] + rr[c + W - 1] + rr[c + W + 1]);
        } else {
            acc = T(0.5) * rr[c] + T(0.25) * (rr[c - 1] + rr[c + 1]);
        }
        g.bc[(size_t)J * nxc + I] = acc;
    }
}

// ---------------------------------------------------------------------------
// Up: prolongation of the coarse correction, then post-smoothing.
// ---------------------------------------------------------------------------
template <class T, int OPK, int TX, int TY, int D>
__device__ __forceinline__ void mg_up_body(const MgLevelArgs<T> &g, const MgOut &out, const int tile) {
    constexpr int NS = StencilShape<OPK>::NS;
    constexpr int H = D;                                       // halo of the window
    constexpr bool two_d = OPK != MG_BURGERS;                 // (1-D Burgers: ny == 1)
    const int hy = two_d ? H : 0;
    constexpr int W = TX + 2 * H;
    const int Hh = (two_d ? TY : 1) + 2 * hy;
    const int npl = W * Hh;
    extern __shared__ unsigned char smem_raw[];
    T *cf = reinterpret_cast<T *>(smem_raw);
    T *xa = cf + npl;
    T *xb = xa + npl;

    const int tiles_x = (g.nx + TX - 1) / TX;
    const int ty = tile / tiles_x, tx = tile % tiles_x;
    const int i0 = tx * TX, j0 = ty * (two_d ? TY : 1);
    const int nx = g.nx, ny = g.ny;
    const int nxc = nx / 2, nyc = two_d ? ny / 2 : 1;
    const T inv_h2 = T(1) / (g.h * g.h);

    constexpr int NPT = (W * (TY + 2 * H) + 255) / 256;
    WindowIndex<NPT> wi;
    wi.template init<W, H>(npl, i0, j0, nx, ny, two_d);
    T bv[NPT];
    {
        T cfv[NPT], xv[NPT], ev[NPT];
        load_field<NPT>(g.coef, wi, cfv);
        load_field<NPT>(g.x, wi, xv);
        // prolongation of the coarse correction: coarse node I sits at fine 2I
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int gi = wi.gi[k], gj = wi.gj[k];
            const int I0 = gi >> 1, I1 = (gi & 1) ? (I0 + 1 == nxc ? 0 : I0 + 1) : I0;
            if (two_d) {
                const int J0 = gj >> 1, J1 = (gj & 1) ? (J0 + 1 == nyc ? 0 : J0 + 1) : J0;
                ev[k] = T(0.25) * (g.xc[(size_t)J0 * nxc + I0] + g.xc[(size_t)J0 * nxc + I1] +
                                   g.xc[(size_t)J1 * nxc + I0] + g.xc[(size_t)J1 * nxc + I1]);
            } else {
                ev[k] = T(0.5) * (g.xc[I0] + g.xc[I1]);
            }
        }
        load_rhs<T, NPT>(out.v1, out.a1, out.v2, out.a2, out.mean_in, g.b, wi, bv);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (wi.ok(k)) {
                cf[wi.q(k)] = cfv[k];
                xa[wi.q(k)] = xv[k] + ev[k];
            }
        }
    }
    __syncthreads();
    T a[NPT][NS], ac[NPT];
    own_stencils<T, OPK, NPT, W>(cf, wi, Hh, two_d, g, inv_h2, a, ac, bv);
    T dv[NPT];
    T *xcur = xa, *xnext = xb;
    for (int st = 0; st < D; ++st) {
        const int r = D - 1 - st;
        const int ax0 = H - r, ax1 = H + TX + r;
        const int by0 = two_d ? hy - r : 0, by1 = two_d ? hy + TY + r : 1;
        const T cd = g.cd[st], cr = g.cr[st];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int c = wi.q(k), ia = c % W, ib = c / W;
            if (wi.ok(k) && ia >= ax0 && ia < ax1 && ib >= by0 && ib < by1) {
                const T xv = xcur[c];
                const T dn = (st == 0 ? T(0) : cd * dv[k]) + cr * own_jres<T, OPK, W>(a[k], bv[k], xcur, c, xv);
                dv[k] = dn;
                xnext[c] = xv + dn;
            }
        }
        __syncthreads();
        T *t = xcur;
        xcur = xnext;
        xnext = t;
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int c = wi.q(k), ia = c % W, ib = c / W;
        if (!wi.ok(k) || ia < H || ia >= H + TX || ib < hy || ib >= hy + (two_d ? TY : 1)) continue;
        const int gi = i0 + (ia - H), gj = j0 + (ib - hy);
        if (gi < nx && gj < ny) {
            const size_t gidx = (size_t)gj * nx + gi;
            if (out.z) out.z[gidx] = (double)xcur[c] + (out.shift ? out.shift_scale * out.shift[0] : 0.0);
            else g.xout[gidx] = xcur[c];
        }
    }
}

// ---------------------------------------------------------------------------
// The V-cycle on levels l0..L-1 in one work-group, every level in LDS.
// ---------------------------------------------------------------------------
// Periodic neighbour indices of point (i, j) on an nx x ny level, in the
// order of nb_off.
template <int OPK>
__device__ __forceinline__ void nb_index(int i, int j, int nx, int ny, int (&idx)[StencilShape<OPK>::NS]) {
    const int ip = wrap2(i + 1, nx), im = wrap2(i - 1, nx);
    if constexpr (OPK == MG_BURGERS) {
        idx[0] = ip;
        idx[1] = im;
    } else {
        const int jp = wrap2(j + 1, ny), jm = wrap2(j - 1, ny);
        idx[0] = j * nx + ip;
        idx[1] = j * nx + im;
        idx[2] = jp * nx + i;
        idx[3] = jm * nx + i;
        if constexpr (StencilShape<OPK>::NS == 8) {
            idx[4] = jp * nx + ip;
            idx[5] = jp * nx + im;
            idx[6] = jm * nx + ip;
            idx[7] = jm * nx + im;
        }
    }
}

// Scaled stencil row p of a periodic level from its padded field (point c
// of the padded array); b~ scaled too when bl is given.
template <class T, int OPK>
__device__ __forceinline__ void store_level_stencil(const T *pad, int c, int pw, T inv_h2, T h, T nu, T sigma, T dt,
                                                    T *at, int np, int p, T *acl, T *bl) {
    constexpr int NS = StencilShape<OPK>::NS;
    T a[NS], ac;
    build_stencil<T, OPK>(pad, c, pw, inv_h2, h, nu, sigma, dt, a, ac);
    const T inv = stencil_rcp(ac);
#pragma unroll
    for (int q = 0; q < NS; ++q) at[q * np + p] = a[q] * inv;
    acl[p] = ac;
    if (bl) bl[p] *= inv;
}

// D^{-1}(b - A x) at point p of a periodic level
template <class T, int OPK>
__device__ __forceinline__ T level_jres(const T *At, int np, const T *bt, const T *x, int p, int i, int j, int nx,
                                        int ny) {
    constexpr int NS = StencilShape<OPK>::NS;
    int idx[NS];
    nb_index<OPK>(i, j, nx, ny, idx);
    T r = bt[p] - x[p];
#pragma unroll
    for (int q = 0; q < NS; ++q) r -= At[q * np + p] * x[idx[q]];
    return r;
}

// A crew runs one level's sweeps: the whole work-group (separated by
// barriers), or its first wave alone, whose lanes run in lockstep so that
// wave-scope fences order its LDS accesses (no barrier, no idle waves to
// wait for on levels of at most a few hundred points).
struct CrewGroup {
    static constexpr bool size_is_wave = false;
    static __device__ __forceinline__ int tid() { return (int)threadIdx.x; }
    static __device__ __forceinline__ int size() { return (int)blockDim.x; }
    static __device__ __forceinline__ void sync() { __syncthreads(); }
};
struct CrewWave {
    static constexpr bool size_is_wave = true;
    static __device__ __forceinline__ int tid() { return (int)(threadIdx.x & 63); }
    static __device__ __forceinline__ int size() { return 64; }
    static __device__ __forceinline__ void sync() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
};

// FOR_PTS over the members of a crew
#define FOR_PTS_C(C_, np_, nx_, ...)                                       \
    do {                                                                   \
        const int w_ = (nx_), n_ = C_::size(), t_ = C_::tid();             \
        const int sx_ = n_ % w_, sy_ = n_ / w_;                            \
        int i, j;                                                          \
        divmod_small(t_, w_, j, i);                                        \
        for (int p = t_; p < (np_); p += n_) {                             \
            __VA_ARGS__;                                                   \
            i += sx_;                                                      \
            j += sy_;                                                      \
            if (i >= w_) { i -= w_; ++j; }                                 \
        }                                                                  \
    } while (0)

// sum / max over a crew, result in every member (red: >= 16 doubles of LDS)
template <class C>
__device__ __forceinline__ double crew_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if constexpr (C::size_is_wave) {
        return v;
    } else {
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        double t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        __syncthreads();
        return t;
    }
}
template <class C>
__device__ __forceinline__ double crew_max(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if constexpr (C::size_is_wave) {
        return v;
    } else {
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        double t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = fmax(t, red[w]);
        __syncthreads();
        return t;
    }
}

// The work-group form of the Chebyshev steps below with each thread's points
// (p = tid + u blockDim, at most MAXP of them) fixed across the steps: their
// scaled stencil rows, b~, Chebyshev directions and neighbour indices stay in
// registers, so a step reads only the iterate from LDS (the point and its
// neighbours) and does no index arithmetic.  The same operations in the same
// order as the generic form.  With R non-null, the scaled residual
// R = Ac (b~ - x - sum_q a~_q x_q) of the result is written after the last
// step (R may be the ping-pong buffer xn).
template <class T, int OPK, int MAXP>
__device__ void wg_cheb_reg(const T *At, const T *bt, T *x, T *xn, int nx, int ny, const T *cd, const T *cr,
                            int nsteps, bool from_zero, T *R, const T *Ac) {
    constexpr int NS = StencilShape<OPK>::NS;
    const int np = nx * ny, nt = (int)blockDim.x, tid = (int)threadIdx.x;
    T a[MAXP][NS], b[MAXP], d[MAXP];
    int nb[MAXP][NS];
#pragma unroll
    for (int u = 0; u < MAXP; ++u) {
        const int p = tid + u * nt;
        const int pp = p < np ? p : 0;
        const int j = pp / nx, i = pp - j * nx;       // once per level
        nb_index<OPK>(i, j, nx, ny, nb[u]);
#pragma unroll
        for (int q = 0; q < NS; ++q) a[u][q] = At[q * np + pp];
        b[u] = bt[pp];
        d[u] = T(0);
    }
    T *xc = x, *xo = xn;
    for (int k = 0; k < nsteps; ++k) {
        const T cdk = cd[k], crk = cr[k];
#pragma unroll
        for (int u = 0; u < MAXP; ++u) {
            const int p = tid + u * nt;
            if (p < np) {
                T xv, dn;
                if (from_zero && k == 0) {
                    xv = T(0);
                    dn = crk * b[u];
                } else {
                    xv = xc[p];
                    T r = b[u] - xv;
#pragma unroll
                    for (int q = 0; q < NS; ++q) r -= a[u][q] * xc[nb[u][q]];
                    dn = (k == 0 ? T(0) : cdk * d[u]) + crk * r;
                }
                d[u] = dn;
                xo[p] = xv + dn;
            }
        }
        __syncthreads();
        T *t = xc;
        xc = xo;
        xo = t;
    }
    if (xc != x) {
#pragma unroll
        for (int u = 0; u < MAXP; ++u) {
            const int p = tid + u * nt;
            if (p < np) x[p] = xc[p];
        }
        __syncthreads();
    }
    if (R) {
#pragma unroll
        for (int u = 0; u < MAXP; ++u) {
            const int p = tid + u * nt;
            if (p < np) {
                T r = b[u] - x[p];
#pragma unroll
                for (int q = 0; q < NS; ++q) r -= a[u][q] * x[nb[u][q]];
                R[p] = Ac[p] * r;
            }
        }
    }
}

// points per thread of a work-group crew on an np-point level (the
// register form takes up to 2 points of a 5- or 3-point stencil: more, or
// the 9-point vorticity stencil, would spill; those keep the generic form)
__device__ __forceinline__ int group_points(int np) { return (np + (int)blockDim.x - 1) / (int)blockDim.x; }

// nsteps Chebyshev steps on a level; x and xn alternate (one crew sync per
// step), the result is left in x.
template <class T, int OPK, class C>
__device__ void wg_cheb(const T *At, const T *bt, T *x, T *xn, T *d, int nx, int ny, const T *cd, const T *cr,
                        int nsteps, bool from_zero) {
    const int np = nx * ny;
    if constexpr (!C::size_is_wave && StencilShape<OPK>::NS <= 4) {
        const int per = group_points(np);
        if (per <= 1) return wg_cheb_reg<T, OPK, 1>(At, bt, x, xn, nx, ny, cd, cr, nsteps, from_zero, nullptr, nullptr);
        if (per == 2) return wg_cheb_reg<T, OPK, 2>(At, bt, x, xn, nx, ny, cd, cr, nsteps, from_zero, nullptr, nullptr);
    }
    T *xc = x, *xo = xn;
    for (int k = 0; k < nsteps; ++k) {
        if (from_zero && k == 0) {
            for (int p = C::tid(); p < np; p += C::size()) {
                const T dn = cr[0] * bt[p];
                d[p] = dn;
                xo[p] = dn;
            }
        } else {
            FOR_PTS_C(C, np, nx, {
                const T xv = xc[p];
                const T dn = (k == 0 ? T(0) : cd[k] * d[p]) + cr[k] * level_jres<T, OPK>(At, np, bt, xc, p, i, j, nx, ny);
                d[p] = dn;
                xo[p] = xv + dn;
            });
        }
        C::sync();
        T *t = xc;
        xc = xo;
        xo = t;
    }
    if (xc != x) {
        for (int p = C::tid(); p < np; p += C::size()) x[p] = xc[p];
        C::sync();
    }
}

// one sub-cycle level on the way down: pre-smoothing from zero, residual,
// full weighting into the next level's scaled right-hand side
template <class T, int OPK, class C>
__device__ void sub_down(const MgSubArgs<T> &s, int l, const T *At, const T *Ac, const T *bt, T *x, T *R, T *Dv,
                         const T *acc_c, T *bc) {
    const int nx = s.nx[l], ny = s.ny[l], np = nx * ny;
    bool done = false;
    if constexpr (!C::size_is_wave && StencilShape<OPK>::NS <= 4) {
        // smoothing and the residual with the points' stencils in registers
        const int per = group_points(np);
        done = per <= 2;
        if (per <= 1) wg_cheb_reg<T, OPK, 1>(At, bt, x, R, nx, ny, s.cd, s.cr, s.deg, true, R, Ac);
        else if (per == 2) wg_cheb_reg<T, OPK, 2>(At, bt, x, R, nx, ny, s.cd, s.cr, s.deg, true, R, Ac);
    }
    if (!done) {
        wg_cheb<T, OPK, C>(At, bt, x, R, Dv, nx, ny, s.cd, s.cr, s.deg, true);
        FOR_PTS_C(C, np, nx, R[p] = Ac[p] * level_jres<T, OPK>(At, np, bt, x, p, i, j, nx, ny));
    }
    C::sync();
    const int nxc = s.nx[l + 1], nyc = s.ny[l + 1];
    FOR_PTS_C(C, nxc * nyc, nxc, {
        T acc;
        if (ny > 1) {
            const int im = wrap2(2 * i - 1, nx), ip = 2 * i + 1, jm = wrap2(2 * j - 1, ny), jp = 2 * j + 1;
            acc = T(0.25) * R[2 * j * nx + 2 * i] +
                  T(0.125) * (R[2 * j * nx + im] + R[2 * j * nx + ip] + R[jm * nx + 2 * i] + R[jp * nx + 2 * i]) +
                  T(0.0625) * (R[jm * nx + im] + R[jm * nx + ip] + R[jp * nx + im] + R[jp * nx + ip]);
        } else {
            acc = T(0.5) * R[2 * i] + T(0.25) * (R[wrap2(2 * i - 1, nx)] + R[2 * i + 1]);
        }
        bc[p] = acc / acc_c[p];
    });
    C::sync();
}

// one sub-cycle level on the way up: add the (bi)linear interpolation of the
// coarse correction, post-smooth
template <class T, int OPK, class C>
__device__ void sub_up(const MgSubArgs<T> &s, int l, const T *At, const T *bt, T *xl, const T *xcl, T *R, T *Dv) {
    const int nx = s.nx[l], ny = s.ny[l], np = nx * ny;
    const int nxc = s.nx[l + 1], nyc = s.ny[l + 1];
    FOR_PTS_C(C, np, nx, {
        const int I0 = i >> 1, I1 = (i & 1) ? (I0 + 1 == nxc ? 0 : I0 + 1) : I0;
        T e;
        if (ny > 1) {
            const int J0 = j >> 1, J1 = (j & 1) ? (J0 + 1 == nyc ? 0 : J0 + 1) : J0;
            e = T(0.25) * (xcl[J0 * nxc + I0] + xcl[J0 * nxc + I1] + xcl[J1 * nxc + I0] + xcl[J1 * nxc + I1]);
        } else {
            e = T(0.5) * (xcl[I0] + xcl[I1]);
        }
        xl[p] += e;
    });
    C::sync();
    wg_cheb<T, OPK, C>(At, bt, xl, R, Dv, nx, ny, s.cd, s.cr, s.deg, false);
}

// coarsest level: Chebyshev iteration on the Gershgorin interval
// [1 - rho, 1 + rho] of D^{-1} A (rho = max row sum of |a~_q|); the
// singular periodic Poisson operator (rho = 1) is solved on mean-free data
// with the interval's lower end at its smallest nonzero eigenvalue
template <class T, int OPK, class C>
__device__ void sub_coarse(const MgSubArgs<T> &s, int l, const T *At, T *bt, T *x, T *R, T *Dv) {
    constexpr int NS = StencilShape<OPK>::NS;
    const int nx = s.nx[l], ny = s.ny[l], np = nx * ny;
    __shared__ double red[16];
    const bool singular = (OPK == MG_POISSON && s.sigma == T(0));
    if (singular) {
        double acc = 0;
        for (int p = C::tid(); p < np; p += C::size()) acc += (double)bt[p];
        const T m = (T)(crew_sum<C>(acc, red) / np);
        for (int p = C::tid(); p < np; p += C::size()) bt[p] -= m;
        C::sync();
    }
    double rho = 0.0;
    for (int p = C::tid(); p < np; p += C::size()) {
        double rs = 0.0;
#pragma unroll
        for (int q = 0; q < NS; ++q) rs += fabs((double)At[q * np + p]);
        rho = fmax(rho, rs);
    }
    rho = crew_max<C>(rho, red);
    double lmin = 1.0 - rho, lmax = 1.0 + rho;
    if (singular || lmin < 0.05) {
        // sin(pi / n) from its Taylor series (a heuristic lower end only)
        auto sin_pi_over = [](int n) {
            const double x = 3.14159265358979323846 / n, x2 = x * x;
            return x * (1.0 - x2 / 6.0 * (1.0 - x2 / 20.0 * (1.0 - x2 / 42.0)));
        };
        const double sx = sin_pi_over(nx), sy = ny > 1 ? sin_pi_over(ny) : 1.0;
        lmin = fmax(0.5 * fmin(sx * sx, sy * sy), 0.02);
    }
    // steps for a 1e-3 reduction of the Chebyshev bound 2 r^k
    const double kap = lmax / lmin, sq = sqrt(kap);
    const double rr = (sq - 1.0) / (sq + 1.0);
    int iters = rr > 0.0 ? (int)ceil(log(2000.0) / -log(rr)) : 1;
    iters = iters < 2 ? 2 : (iters > s.coarse_iters ? s.coarse_iters : iters);
    // Chebyshev step coefficients, one per member from the closed form of
    // the recurrence rho_k = 1 / (2 sigma1 - rho_{k-1}), rho_0 = 1/sigma1:
    // rho_k = T_k(sigma1) / T_{k+1}(sigma1)
    //       = e^{-a} (1 + e^{-2ka}) / (1 + e^{-2(k+1)a}),  a = acosh(sigma1);
    // step k: d <- rho_k rho_{k-1} d + (2 rho_k / delta) r  (k = 0: r / theta)
    __shared__ T ccd[IRK_MAX_COARSE_ITERS], ccr[IRK_MAX_COARSE_ITERS];
    if (C::tid() < iters) {
        const int k = C::tid();
        const double theta = 0.5 * (lmax + lmin), delta = fmax(0.5 * (lmax - lmin), 1e-12 * theta);
        const double sig1 = theta / delta;
        const double a = log(sig1 + sqrt(sig1 * sig1 - 1.0));
        auto rho_k = [&](int m) {
            return exp(-a) * (1.0 + exp(-2.0 * m * a)) / (1.0 + exp(-2.0 * (m + 1) * a));
        };
        if (k == 0) {
            ccd[0] = T(0);
            ccr[0] = (T)(1.0 / theta);
        } else {
            const double rk = rho_k(k);
            ccd[k] = (T)(rk * rho_k(k - 1));
            ccr[k] = (T)(2.0 * rk / delta);
        }
    }
    C::sync();
    wg_cheb<T, OPK, C>(At, bt, x, R, Dv, nx, ny, ccd, ccr, iters, true);
}

template <class T, int OPK>
__device__ __forceinline__ void mg_subcycle_body(const MgSubArgs<T> &s, const MgIn &in, const MgOut &out) {
    constexpr int NS = StencilShape<OPK>::NS;
    extern __shared__ unsigned char smem_raw[];
    T *base = reinterpret_cast<T *>(smem_raw);
    // per level: x, b~, A_c, then NS scaled off-diagonals; after the levels:
    // scratch R and Dv sized for the first level, and a padded copy of a
    // level's linearization field for building its stencil.  Level pointers
    // are recomputed from the sizes (uniform scalar arithmetic).
    auto lev_base = [&](int l) {
        size_t off = 0;
        for (int q = 0; q < l; ++q) off += (3 + NS) * (size_t)s.nx[q] * s.ny[q];
        return base + off;
    };
    auto npts = [&](int l) { return s.nx[l] * s.ny[l]; };
#define X(l) (lev_base(l))
#define B(l) (lev_base(l) + npts(l))
#define AC(l) (lev_base(l) + 2 * npts(l))
#define AT(l) (lev_base(l) + 3 * npts(l))
    const int np0 = npts(0);
    T *R = lev_base(s.nlev);
    T *Dv = R + np0;
    T *Pad = Dv + np0;            // per-level padded fields, consecutive
    const int L = s.nlev;
    const bool two_d = s.ny[0] > 1;
    // padded level l: (nx + 2) x (ny + 2) (2-D) or nx + 2 points, periodic
    // ring; offsets recomputed from the sizes (no private arrays)
    auto pad_size = [&](int l) { return (s.nx[l] + 2) * (two_d ? s.ny[l] + 2 : 1); };
    auto pad_off = [&](int l) {
        int off = 0;
        for (int q = 0; q < l; ++q) off += pad_size(q);
        return off;
    };
    const int ptot = pad_off(L);
    // every global load is issued before its value is used: the first
    // level's right-hand side, then the linearization fields of all levels
    // in batches of SB points per thread
    constexpr int SB = 4;
    T bv[SB];
    {
#pragma unroll
        for (int k = 0; k < SB; ++k) {
            const int p0 = (int)threadIdx.x + k * (int)blockDim.x;
            const int p = p0 < np0 ? p0 : 0;
            if (in.v1) {
                double v = in.a1 * in.v1[p];
                if (in.v2) v += in.a2 * in.v2[p];
                if (in.mean) v -= in.a1 * in.mean[0] + (in.v2 ? in.a2 * in.mean[1] : 0.0);
                bv[k] = (T)v;
            } else {
                bv[k] = s.b0[p];
            }
        }
    }
    for (int base = 0; base < ptot; base += SB * (int)blockDim.x) {
        T v[SB];
        int dst[SB];
#pragma unroll
        for (int k = 0; k < SB; ++k) {
            const int q = base + (int)threadIdx.x + k * (int)blockDim.x;
            dst[k] = q < ptot ? q : -1;
            // level of q (compile-time indexed search: no private arrays)
            int nx = s.nx[0], ny = s.ny[0], off = 0, offm = 0;
            const T *cl = s.coef[0];
#pragma unroll
            for (int m = 0; m < IRK_MAX_SUB_LEVELS; ++m) {
                if (m < L && q >= offm) {
                    nx = s.nx[m];
                    ny = s.ny[m];
                    off = offm;
                    cl = s.coef[m];
                }
                if (m < L) offm += pad_size(m);
            }
            const int pw = nx + 2;
            const int loc = q < ptot ? q - off : 0;
            const int gi = wrap2(loc % pw - 1, nx), gj = two_d ? wrap2(loc / pw - 1, ny) : 0;
            v[k] = cl ? cl[gj * nx + gi] : T(0);
        }
#pragma unroll
        for (int k = 0; k < SB; ++k)
            if (dst[k] >= 0) Pad[dst[k]] = v[k];
    }
#pragma unroll
    for (int k = 0; k < SB; ++k) {
        const int p = (int)threadIdx.x + k * (int)blockDim.x;
        if (p < np0) B(0)[p] = bv[k];
    }
    __syncthreads();
    // scaled stencils of every level (levels are independent: one barrier)
    for (int l = 0; l < L; ++l) {
        const int nx = s.nx[l], ny = s.ny[l];
        const int pw = nx + 2;
        const T inv_h2 = T(1) / (s.h[l] * s.h[l]);
        T *at = AT(l), *acl = AC(l), *bl = B(l);
        const T *pad = Pad + pad_off(l);
        const int np = nx * ny;
        FOR_PTS(np, nx, store_level_stencil<T, OPK>(pad, (two_d ? (j + 1) * pw : 0) + i + 1, pw, inv_h2, s.h[l],
                                                      s.nu, s.sigma, s.dt, at, np, p, acl, l == 0 ? bl : nullptr));
    }
    __syncthreads();
    // levels of at most s.wave_pts points (and everything coarser) run on
    // the first wave alone; the larger ones on the whole work-group
    int lw = L - 1;
    while (lw > 0 && npts(lw - 1) <= s.wave_pts) --lw;
    if (npts(lw) > s.wave_pts) lw = L;
    const int lg = lw < L - 1 ? lw : L - 1;        // levels 0..lg-1 go down as a group
    for (int l = 0; l < lg; ++l)
        sub_down<T, OPK, CrewGroup>(s, l, AT(l), AC(l), B(l), X(l), R, Dv, AC(l + 1), B(l + 1));
    if (lw < L) {
        if (threadIdx.x < 64) {
            for (int l = lw; l < L - 1; ++l)
                sub_down<T, OPK, CrewWave>(s, l, AT(l), AC(l), B(l), X(l), R, Dv, AC(l + 1), B(l + 1));
            sub_coarse<T, OPK, CrewWave>(s, L - 1, AT(L - 1), B(L - 1), X(L - 1), R, Dv);
            for (int l = L - 2; l >= lw; --l) sub_up<T, OPK, CrewWave>(s, l, AT(l), B(l), X(l), X(l + 1), R, Dv);
        }
        __syncthreads();
    } else {
        sub_coarse<T, OPK, CrewGroup>(s, L - 1, AT(L - 1), B(L - 1), X(L - 1), R, Dv);
    }
    for (int l = lg - 1; l >= 0; --l) sub_up<T, OPK, CrewGroup>(s, l, AT(l), B(l), X(l), X(l + 1), R, Dv);
    for (int p = threadIdx.x; p < np0; p += blockDim.x) {
        if (out.z) out.z[p] = (double)X(0)[p] + (out.shift ? out.shift_scale * out.shift[0] : 0.0);
        else s.x0[p] = X(0)[p];
    }
}
#undef X
#undef B
#undef AC
#undef AT

// ---------------------------------------------------------------------------
// kernels: one job per launch, or a batch of jobs (same operator, precision
// and tile shape; different grids, shifts, linearizations and vectors) in
// one launch -- work-group b runs tile b - prefix[e] of job e.  Job fields
// are selected with compile-time indices (no dynamically indexed copies).
// ---------------------------------------------------------------------------
template <class T, int OPK, int TX, int TY, int D>
__global__ void __launch_bounds__(256) k_mg_down(MgLevelArgs<T> g, MgIn in) {
    mg_down_body<T, OPK, TX, TY, D>(g, in, xcd_tile());
}

template <class T, int OPK, int TX, int TY, int D>
__global__ void __launch_bounds__(256) k_mg_up(MgLevelArgs<T> g, MgOut out) {
    mg_up_body<T, OPK, TX, TY, D>(g, out, xcd_tile());
}

template <class T, int OPK>
__global__ void __launch_bounds__(1024) k_mg_subcycle(MgSubArgs<T> s, MgIn in, MgOut out) {
    mg_subcycle_body<T, OPK>(s, in, out);
}

// job of global tile t: largest e with prefix[e] <= t (uniform)
__device__ __forceinline__ int batch_job(const int (&prefix)[IRK_MG_BATCH + 1], int n, int t) {
    int e = 0;
#pragma unroll
    for (int q = 1; q < IRK_MG_BATCH; ++q)
        if (q < n && t >= prefix[q]) e = q;
    return e;
}

template <class T, int OPK, int TX, int TY, int D>
__global__ void __launch_bounds__(256) k_mg_down_batch(MgLevelBatch<T> b) {
    const int t = xcd_tile();
    const int e = batch_job(b.prefix, b.n, t);
    MgLevelArgs<T> g = b.g[0];
    MgIn in = b.in[0];
    int p0 = b.prefix[0];
#pragma unroll
    for (int q = 1; q < IRK_MG_BATCH; ++q)
        if (q == e) { g = b.g[q]; in = b.in[q]; p0 = b.prefix[q]; }
    mg_down_body<T, OPK, TX, TY, D>(g, in, t - p0);
}

template <class T, int OPK, int TX, int TY, int D>
__global__ void __launch_bounds__(256) k_mg_up_batch(MgLevelBatch<T> b) {
    const int t = xcd_tile();
    const int e = batch_job(b.prefix, b.n, t);
    MgLevelArgs<T> g = b.g[0];
    MgOut out = b.out[0];
    int p0 = b.prefix[0];
#pragma unroll
    for (int q = 1; q < IRK_MG_BATCH; ++q)
        if (q == e) { g = b.g[q]; out = b.out[q]; p0 = b.prefix[q]; }
    mg_up_body<T, OPK, TX, TY, D>(g, out, t - p0);
}

template <class T, int OPK>
__global__ void __launch_bounds__(1024) k_mg_subcycle_batch(MgSubBatch<T> b) {
    // job = work-group; its arguments are read in place (uniform index into
    // the kernel arguments)
    const int e = blockIdx.x;
    mg_subcycle_body<T, OPK>(b.s[e], b.in[e], b.out[e]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static unsigned subcycle_threads(int np0);
template <class T, int OPK, int TX, int TY>
static void down_t(hipStream_t st, const MgLevelArgs<T> &a, const MgIn &in, int deg) {
    const int tiles = ((a.nx + TX - 1) / TX) * (a.ny > 1 ? (a.ny + TY - 1) / TY : 1);
    const int H = deg + 2;
    const size_t shm = (size_t)tile_arrays() * (TX + 2 * H) *
                       ((a.ny > 1 ? TY : 1) + (a.ny > 1 ? 2 * H : 0)) * sizeof(T);
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
    const size_t shm = (size_t)tile_arrays() * (TX + 2 * H) *
                       ((a.ny > 1 ? TY : 1) + (a.ny > 1 ? 2 * H : 0)) * sizeof(T);
    switch (deg) {
        case 1: k_mg_up<T, OPK, TX, TY, 1><<<tiles, 256, shm, st>>>(a, out); break;
        case 2: k_mg_up<T, OPK, TX, TY, 2><<<tiles, 256, shm, st>>>(a, out); break;
        case 3: k_mg_up<T, OPK, TX, TY, 3><<<tiles, 256, shm, st>>>(a, out); break;
        default: k_mg_up<T, OPK, TX, TY, 4><<<tiles, 256, shm, st>>>(a, out); break;
    }
}

// tile shape per level size: 32x16 tiles on levels of side >= 1024 (less
// halo per point where there are work-groups enough to fill the chip),
// 32x8 down to side 128, 16x8 (more work-groups) below; 1-D levels use
// 256-point strips
// The window loads wrap indices once (wrap2), valid when the window of
// every tile stays within [-n, 2n): tiles * T + halo <= 2 n and halo <= n.
static bool window_fits(int n, int t, int halo) {
    const int tiles = (n + t - 1) / t;
    return halo <= n && tiles * t + halo <= 2 * n;
}

template <class T, int OPK>
static void down_dispatch(hipStream_t st, const MgLevelArgs<T> &a, const MgIn &in, int deg) {
    const int H = (deg > 4 ? 4 : deg) + 2;
    if (a.ny == 1) {
        if (window_fits(a.nx, 256, H)) down_t<T, OPK, 256, 1>(st, a, in, deg);
        else down_t<T, OPK, 64, 1>(st, a, in, deg);
    } else if (a.nx >= 1024 && window_fits(a.nx, 32, H) && window_fits(a.ny, 16, H)) {
        down_t<T, OPK, 32, 16>(st, a, in, deg);
    } else if (a.nx >= 128 && window_fits(a.nx, 32, H) && window_fits(a.ny, 8, H)) {
        down_t<T, OPK, 32, 8>(st, a, in, deg);
    } else {
        down_t<T, OPK, 16, 8>(st, a, in, deg);
    }
}

template <class T, int OPK>
static void up_dispatch(hipStream_t st, const MgLevelArgs<T> &a, const MgOut &out, int deg) {
    const int H = deg > 4 ? 4 : deg;
    if (a.ny == 1) {
        if (window_fits(a.nx, 256, H)) up_t<T, OPK, 256, 1>(st, a, out, deg);
        else up_t<T, OPK, 64, 1>(st, a, out, deg);
    } else if (a.nx >= 1024 && window_fits(a.nx, 32, H) && window_fits(a.ny, 16, H)) {
        up_t<T, OPK, 32, 16>(st, a, out, deg);
    } else if (a.nx >= 128 && window_fits(a.nx, 32, H) && window_fits(a.ny, 8, H)) {
        up_t<T, OPK, 32, 8>(st, a, out, deg);
    } else {
        up_t<T, OPK, 16, 8>(st, a, out, deg);
    }
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

static int stencil_ns(int opk) {
    return opk == MG_VSF_OMEGA ? 8 : (opk == MG_BURGERS ? 2 : 4);
}

size_t mg_subcycle_lds_bytes(int opk, int nlev, const int *nx, const int *ny, size_t tsz) {
    size_t n = 0;
    for (int l = 0; l < nlev; ++l) n += (size_t)(3 + stencil_ns(opk)) * nx[l] * ny[l];
    n += 2 * (size_t)nx[0] * ny[0];
    for (int l = 0; l < nlev; ++l) n += (size_t)(nx[l] + 2) * (ny[0] > 1 ? ny[l] + 2 : 1);
    return n * tsz;
}

template <class T>
void launch_mg_subcycle(hipStream_t st, int opk, const MgSubArgs<T> &s, const MgIn &in, const MgOut &out) {
    const size_t shm = mg_subcycle_lds_bytes(opk, s.nlev, s.nx, s.ny, sizeof(T));
    const unsigned nt = subcycle_threads(s.nx[0] * s.ny[0]);
    switch (opk) {
        case MG_NLDIFF: k_mg_subcycle<T, MG_NLDIFF><<<1, nt, shm, st>>>(s, in, out); break;
        case MG_BURGERS: k_mg_subcycle<T, MG_BURGERS><<<1, nt, shm, st>>>(s, in, out); break;
        case MG_VSF_OMEGA: k_mg_subcycle<T, MG_VSF_OMEGA><<<1, nt, shm, st>>>(s, in, out); break;
        default: k_mg_subcycle<T, MG_POISSON><<<1, nt, shm, st>>>(s, in, out); break;
    }
}

// ---------------------------------------------------------------------------
// batched launchers
// ---------------------------------------------------------------------------
// tile shape class of a level (the one launch_mg_down/up would use):
// 0 = 32x8 (2-D) or 256-point strips (1-D), 1 = 16x8 or 64-point strips
template <class T>
static int shape_class(const MgLevelArgs<T> &a, int halo) {
    if (a.ny == 1) return window_fits(a.nx, 256, halo) ? 0 : 1;
    if (a.nx >= 1024 && window_fits(a.nx, 32, halo) && window_fits(a.ny, 16, halo)) return 2;
    return (a.nx >= 128 && window_fits(a.nx, 32, halo) && window_fits(a.ny, 8, halo)) ? 0 : 1;
}

template <class T, int OPK, int TX, int TY, bool DOWN>
static void level_batch_t(hipStream_t st, MgLevelBatch<T> &b, int deg) {
    const bool two_d = b.g[0].ny > 1;
    int acc = 0;
    for (int e = 0; e < b.n; ++e) {
        b.prefix[e] = acc;
        acc += ((b.g[e].nx + TX - 1) / TX) * (two_d ? (b.g[e].ny + TY - 1) / TY : 1);
    }
    for (int e = b.n; e <= IRK_MG_BATCH; ++e) b.prefix[e] = acc;
    const int H = DOWN ? deg + 2 : deg;
    const int arrays = tile_arrays();
    const size_t shm = (size_t)arrays * (TX + 2 * H) * ((two_d ? TY : 1) + (two_d ? 2 * H : 0)) * sizeof(T);
    if (DOWN) {
        switch (deg) {
            case 1: k_mg_down_batch<T, OPK, TX, TY, 1><<<acc, 256, shm, st>>>(b); break;
            case 2: k_mg_down_batch<T, OPK, TX, TY, 2><<<acc, 256, shm, st>>>(b); break;
            case 3: k_mg_down_batch<T, OPK, TX, TY, 3><<<acc, 256, shm, st>>>(b); break;
            default: k_mg_down_batch<T, OPK, TX, TY, 4><<<acc, 256, shm, st>>>(b); break;
        }
    } else {
        switch (deg) {
            case 1: k_mg_up_batch<T, OPK, TX, TY, 1><<<acc, 256, shm, st>>>(b); break;
            case 2: k_mg_up_batch<T, OPK, TX, TY, 2><<<acc, 256, shm, st>>>(b); break;
            case 3: k_mg_up_batch<T, OPK, TX, TY, 3><<<acc, 256, shm, st>>>(b); break;
            default: k_mg_up_batch<T, OPK, TX, TY, 4><<<acc, 256, shm, st>>>(b); break;
        }
    }
}

template <class T, int OPK, bool DOWN>
static void level_batch_dispatch(hipStream_t st, const MgLevelArgs<T> *g, const MgIn *in, const MgOut *out, int n,
                                 int deg) {
    const int halo = DOWN ? (deg > 4 ? 4 : deg) + 2 : (deg > 4 ? 4 : deg);
    for (int cls = 0; cls < 3; ++cls) {
        MgLevelBatch<T> b;
        std::memset(&b, 0, sizeof(b));
        b.n = 0;
        auto flush = [&]() {
            if (b.n == 0) return;
            const bool one_d = b.g[0].ny == 1;
            if (cls == 2) {
                level_batch_t<T, OPK, 32, 16, DOWN>(st, b, deg);
            } else if (cls == 0) {
                if (one_d) level_batch_t<T, OPK, 256, 1, DOWN>(st, b, deg);
                else level_batch_t<T, OPK, 32, 8, DOWN>(st, b, deg);
            } else {
                if (one_d) level_batch_t<T, OPK, 64, 1, DOWN>(st, b, deg);
                else level_batch_t<T, OPK, 16, 8, DOWN>(st, b, deg);
            }
            std::memset(&b, 0, sizeof(b));
            b.n = 0;
        };
        for (int i = 0; i < n; ++i) {
            if (shape_class(g[i], halo) != cls) continue;
            b.g[b.n] = g[i];
            if (in) b.in[b.n] = in[i];
            if (out) b.out[b.n] = out[i];
            if (++b.n == IRK_MG_BATCH) flush();
        }
        flush();
    }
}

template <class T>
void launch_mg_down_batch(hipStream_t st, int opk, const MgLevelArgs<T> *g, const MgIn *in, int n, int deg) {
    switch (opk) {
        case MG_NLDIFF: level_batch_dispatch<T, MG_NLDIFF, true>(st, g, in, nullptr, n, deg); break;
        case MG_BURGERS: level_batch_dispatch<T, MG_BURGERS, true>(st, g, in, nullptr, n, deg); break;
        case MG_VSF_OMEGA: level_batch_dispatch<T, MG_VSF_OMEGA, true>(st, g, in, nullptr, n, deg); break;
        default: level_batch_dispatch<T, MG_POISSON, true>(st, g, in, nullptr, n, deg); break;
    }
}

template <class T>
void launch_mg_up_batch(hipStream_t st, int opk, const MgLevelArgs<T> *g, const MgOut *out, int n, int deg) {
    switch (opk) {
        case MG_NLDIFF: level_batch_dispatch<T, MG_NLDIFF, false>(st, g, nullptr, out, n, deg); break;
        case MG_BURGERS: level_batch_dispatch<T, MG_BURGERS, false>(st, g, nullptr, out, n, deg); break;
        case MG_VSF_OMEGA: level_batch_dispatch<T, MG_VSF_OMEGA, false>(st, g, nullptr, out, n, deg); break;
        default: level_batch_dispatch<T, MG_POISSON, false>(st, g, nullptr, out, n, deg); break;
    }
}

// threads of a sub-cycle work-group: about half a point per thread on a
// 32^2 first level, one per point below (measured fastest); at least np0 / 4
// (the first level's right-hand side is loaded four points per thread)
static unsigned subcycle_threads(int np0) {
    return np0 >= 2048 ? 1024 : (np0 >= 1024 ? 512 : (unsigned)(((np0 + 63) / 64) * 64));
}

template <class T>
void launch_mg_subcycle_batch(hipStream_t st, int opk, const MgSubArgs<T> *s, const MgIn *in, const MgOut *out,
                              int n) {
    for (int i0 = 0; i0 < n; i0 += IRK_MG_BATCH) {
        const int cnt = std::min(IRK_MG_BATCH, n - i0);
        MgSubBatch<T> b;
        std::memset(&b, 0, sizeof(b));
        size_t shm = 0;
        unsigned nt = 64;
        for (int e = 0; e < cnt; ++e) {
            b.s[e] = s[i0 + e];
            b.in[e] = in[i0 + e];
            b.out[e] = out[i0 + e];
            shm = std::max(shm, mg_subcycle_lds_bytes(opk, s[i0 + e].nlev, s[i0 + e].nx, s[i0 + e].ny, sizeof(T)));
            nt = std::max(nt, subcycle_threads(s[i0 + e].nx[0] * s[i0 + e].ny[0]));
        }
        switch (opk) {
            case MG_NLDIFF: k_mg_subcycle_batch<T, MG_NLDIFF><<<cnt, nt, shm, st>>>(b); break;
            case MG_BURGERS: k_mg_subcycle_batch<T, MG_BURGERS><<<cnt, nt, shm, st>>>(b); break;
            case MG_VSF_OMEGA: k_mg_subcycle_batch<T, MG_VSF_OMEGA><<<cnt, nt, shm, st>>>(b); break;
            default: k_mg_subcycle_batch<T, MG_POISSON><<<cnt, nt, shm, st>>>(b); break;
        }
    }
}

// ---------------------------------------------------------------------------
// Exact coarsest-level solve of the periodic 5-point Poisson problem
// -dt Lap_h x = b (its constant mode dropped: b's mean is ignored and x is
// mean-free) on an n x n level, n <= IRK_FDM_MAX, by fast diagonalization:
// -Lap_h = S (x) I + I (x) S with S = Q diag(lam) Q^T the 1-D periodic second
// difference (Q a real orthonormal Fourier basis), so
//   x = Q [ (Q^T B Q)_ab / (dt (lam_a + lam_b)) ] Q^T,   (a, b) != (0, 0).
// One work-group; Q (row stride n + 1 in LDS: both its rows and columns are
// read conflict-free), the field and one temporary live in LDS; four dense
// n x n x n products, each output a dot product of length n.  The side is a
// template parameter, so every loop below is unrolled and no load waits on a
// branch.
// ---------------------------------------------------------------------------
// One dense n x n x n product phase of the fast diagonalization: thread t
// computes row r = t / (N / 4) and the four columns c0 .. c0 + 3 of
// out[r][c] = sum_k a(r, k) b(k, c), where a(r, k) is read as A[r * LD + k]
// (ATR: A[k * LD + r]) and b(k, c) as B[k * LD + c] (BTR: B[c * LD + k]).
template <class T, int N, bool ATR, bool BTR>
__device__ __forceinline__ void fdm_product(const T *A, const T *B, int r, int c0, T (&acc)[4]) {
    constexpr int LD = N + 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = T(0);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const T a = ATR ? A[k * LD + r] : A[r * LD + k];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += a * (BTR ? B[(c0 + q) * LD + k] : B[k * LD + c0 + q]);
    }
}

template <class T, int N>
__global__ void __launch_bounds__(256) k_poisson_fdm(T dt, const T *__restrict__ Q, const T *__restrict__ lam,
                                                     const T *__restrict__ b, T *__restrict__ x) {
    static_assert(N % 4 == 0 && N <= IRK_FDM_MAX, "side a multiple of 4, at most IRK_FDM_MAX");
    constexpr int LD = N + 1, NN = N * N, PER = (NN + 255) / 256, GROUPS = N / 4;
    __shared__ T Qs[N * LD], Fa[N * LD], Fb[N * LD], ls[N];
    const int t = threadIdx.x;
    // every global load of the kernel is issued before the first is used
    T qv[PER], bv[PER], lv = T(0);
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int q = t + 256 * p;
        qv[p] = q < NN ? Q[q] : T(0);
        bv[p] = q < NN ? b[q] : T(0);
    }
    if (t < N) lv = lam[t];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int q = t + 256 * p;
        if (q < NN) {
            const int r = q / N, c = q % N;
            Qs[r * LD + c] = qv[p];
            Fa[r * LD + c] = bv[p];
        }
    }
    if (t < N) ls[t] = lv;
    __syncthreads();
    // N / 4 column groups per row: the threads cover N * N / 4 <= 256 groups
    const bool on = t < N * GROUPS;
    const int r = on ? t / GROUPS : 0, c0 = on ? 4 * (t % GROUPS) : 0;
    T acc[4];
    // Fb = B Q
    if (on) {
        fdm_product<T, N, false, false>(Fa, Qs, r, c0, acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) Fb[r * LD + c0 + q] = acc[q];
    }
    __syncthreads();
    // Fa = (Q^T Fb) ./ (dt (lam_a + lam_b)), the constant mode dropped
    if (on) {
        fdm_product<T, N, true, false>(Qs, Fb, r, c0, acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = c0 + q;
            Fa[r * LD + c] = (r == 0 && c == 0) ? T(0) : acc[q] / (dt * (ls[r] + ls[c]));
        }
    }
    __syncthreads();
    // Fb = Fa Q^T
    if (on) {
        fdm_product<T, N, false, true>(Fa, Qs, r, c0, acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) Fb[r * LD + c0 + q] = acc[q];
    }
    __syncthreads();
    // x = Q Fb
    if (on) {
        fdm_product<T, N, false, false>(Qs, Fb, r, c0, acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) x[r * N + c0 + q] = acc[q];
    }
}

template <class T>
void launch_poisson_fdm(hipStream_t st, int n, T dt, const T *Q, const T *lam, const T *b, T *x) {
    switch (n) {
#define IRK_FDM_CASE(N) \
    case N: k_poisson_fdm<T, N><<<1, 256, 0, st>>>(dt, Q, lam, b, x); break;
        IRK_FDM_CASE(4) IRK_FDM_CASE(8) IRK_FDM_CASE(12) IRK_FDM_CASE(16)
        IRK_FDM_CASE(20) IRK_FDM_CASE(24) IRK_FDM_CASE(28) IRK_FDM_CASE(32)
#undef IRK_FDM_CASE
    default: break;                     // the level choice admits no other side
    }
}

template void launch_poisson_fdm<float>(hipStream_t, int, float, const float *, const float *, const float *,
                                        float *);
template void launch_poisson_fdm<double>(hipStream_t, int, double, const double *, const double *,
                                         const double *, double *);

template void launch_mg_down_batch<float>(hipStream_t, int, const MgLevelArgs<float> *, const MgIn *, int, int);
template void launch_mg_down_batch<double>(hipStream_t, int, const MgLevelArgs<double> *, const MgIn *, int, int);
template void launch_mg_up_batch<float>(hipStream_t, int, const MgLevelArgs<float> *, const MgOut *, int, int);
template void launch_mg_up_batch<double>(hipStream_t, int, const MgLevelArgs<double> *, const MgOut *, int, int);
template void launch_mg_subcycle_batch<float>(hipStream_t, int, const MgSubArgs<float> *, const MgIn *,
                                              const MgOut *, int);
template void launch_mg_subcycle_batch<double>(hipStream_t, int, const MgSubArgs<double> *, const MgIn *,
                                               const MgOut *, int);
template void launch_mg_down<float>(hipStream_t, int, const MgLevelArgs<float> &, const MgIn &, int);
template void launch_mg_down<double>(hipStream_t, int, const MgLevelArgs<double> &, const MgIn &, int);
template void launch_mg_up<float>(hipStream_t, int, const MgLevelArgs<float> &, const MgOut &, int);
template void launch_mg_up<double>(hipStream_t, int, const MgLevelArgs<double> &, const MgOut &, int);
template void launch_mg_subcycle<float>(hipStream_t, int, const MgSubArgs<float> &, const MgIn &, const MgOut &);
template void launch_mg_subcycle<double>(hipStream_t, int, const MgSubArgs<double> &, const MgIn &, const MgOut &);

}  // namespace irk
