// Spectral solve of the periodic Poisson problem -dt Lap_h x = q on the
// finest grid, for the streamfunction rows of the vorticity-streamfunction
// DAE (their block operator is the constant-coefficient 5-point Laplacian).
//
// The discrete Fourier modes e^{2 pi i (a x + b y)} diagonalize the periodic
// 5-point Laplacian: -Lap_h has eigenvalue lam_a + lam_b with
// lam_m = 4 sin^2(pi m / n) / h^2, so x^_ab = q^_ab / (dt (lam_a + lam_b)),
// the constant mode (a, b) = (0, 0) dropped.  Three launches:
//   k_fft_rows_fwd  rows 2r and 2r+1 of q, each less its own mean, packed
//                   as one complex row (q_2r + i q_2r+1), transformed in LDS,
//                   then separated by Hermitian symmetry into the half
//                   spectra (modes 0..n/2) of both rows; the row sums of
//                   the inputs go to a small buffer;
//   k_fft_cols      one column (mode k) of the half spectrum: transform,
//                   divide by dt (lam_a + lam_k) n^2, inverse transform;
//                   column 0 is rebuilt from the row sums (the row sums of q
//                   less n times its mean), which it also reduces to the
//                   means;
//   k_fft_rows_inv  rows 2r and 2r+1 again: their full spectra rebuilt from
//                   the halves (X_{n-k} = conj X_k), packed as X + i Y, one
//                   inverse transform whose real and imaginary parts are the
//                   two real rows of x.
// The transforms are mixed radix-4/2 Stockham passes in LDS (vectors, their
// ping-pong copies and the twiddles), compiled per side; the half spectrum
// (n (n/2 + 1) complex values, column-major) is the only intermediate in
// memory.
#include <hip/hip_runtime.h>

#include "fft_poisson.h"

namespace irk {

namespace {

constexpr int FFT_NT = 256;
constexpr size_t FFT_LDS_MAX = 64 * 1024;

// The vectors in LDS carry one padding slot per 2^FFT_PAD values: index i
// lives at pidx(i).  The radix-4 passes write with strides 4, 16, ... and
// without it several lanes of a wave hit one LDS bank (up to 16-way).
constexpr int FFT_PAD = 4;
__host__ __device__ constexpr int padded(int n) { return n + (n >> FFT_PAD); }
__device__ __forceinline__ int pidx(int i) { return i + (i >> FFT_PAD); }

template <class T>
struct cx {
    T re, im;
};

template <class T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) {
    return {a.re + b.re, a.im + b.im};
}
template <class T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) {
    return {a.re - b.re, a.im - b.im};
}

int log2_exact(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return (1 << l) == n ? l : -1;
}

// LDS bytes of a row work-group (one row pair: a complex vector and its
// ping-pong copy, padded) with the n - 1 stage twiddles, and of a column
// work-group (one column, its copy, the twiddles, the n eigenvalues)
size_t row_lds(int n, size_t tsz) { return (2 * (size_t)padded(n) + n) * 2 * tsz; }
size_t col_lds(int n, size_t tsz) { return row_lds(n, tsz) + n * tsz; }

// XCD-aware work-group order: consecutive logical indices on one XCD (work
// groups are dealt to the 8 XCDs round-robin; neighbours share cache lines
// of the half spectrum); the identity unless the grid is a multiple of 8
__device__ __forceinline__ int xcd_order() {
    const int nb = gridDim.x, b = blockIdx.x;
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

// Sums of NV values over the work-group in a fixed order (each wave by
// shuffles, then the waves in order), returned to every thread.  sh: NV
// values per wave.
template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV], double *sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
        if (lane == 0) sh[wid * NV + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < FFT_NT / 64; ++w) t += sh[w * NV + k];
        v[k] = t;
    }
}

}  // namespace

bool fft_poisson_supported(int n, size_t tsz) {
    if (n < IRK_FFT_MIN || n > 2048 || log2_exact(n) < 0) return false;
    return row_lds(n, tsz) <= FFT_LDS_MAX && col_lds(n, tsz) <= FFT_LDS_MAX;
}

size_t fft_poisson_spectrum_values(int n) { return (size_t)2 * n * (n / 2 + 1); }

// Mixed radix-4/2 Stockham transform (self-sorting: natural order in and
// out) of one vector of length N = 2^LG in X (padded: value i at pidx(i));
// Y is the ping-pong buffer, tw the stage twiddle table (load_twiddles).  A
// stage of radix r (4 while N / Ns >= 4, a last radix-2 stage for odd LG)
// and span Ns takes x[j + q N/r], q < r, times w^(q k N / (r Ns)) with
// k = j mod Ns and w = exp(-2 pi i / N), through an r-point DFT into
// y[(j - k) r + k + q Ns].  INV: conjugate twiddles and DFTs (unnormalized
// inverse).  The size is a template parameter: every stage and thread loop
// is unrolled.  Returns the buffer holding the result.
template <class T, bool INV, int LG>
__device__ __forceinline__ cx<T> *fft_lds(cx<T> *X, cx<T> *Y, const cx<T> *tw) {
    constexpr int N = 1 << LG;
#pragma unroll
    for (int lgNs = 0; lgNs < LG;) {
        const bool r4 = LG - lgNs >= 2;
        const int lgr = r4 ? 2 : 1;
        const int lgm = LG - lgr, m = 1 << lgm;          // butterflies
        const int Ns = 1 << lgNs;
#pragma unroll
        for (int t0 = 0; t0 < m; t0 += FFT_NT) {
            const int j = t0 + (int)threadIdx.x;
            if (m % FFT_NT == 0 || j < m) {
                const int k = j & (Ns - 1);
                const int base = ((j - k) << lgr) + k;
                auto twq = [&](int q) {
                    cx<T> w = tw[(Ns - 1) + (q - 1) * Ns + k];
                    if (INV) w.im = -w.im;
                    return w;
                };
                if (r4) {
                    cx<T> a0 = X[pidx(j)], a1 = X[pidx(j + m)], a2 = X[pidx(j + 2 * m)], a3 = X[pidx(j + 3 * m)];
                    a1 = cmul(a1, twq(1));
                    a2 = cmul(a2, twq(2));
                    a3 = cmul(a3, twq(3));
                    const cx<T> s0 = cadd(a0, a2), s1 = csub(a0, a2), s2 = cadd(a1, a3), s3 = csub(a1, a3);
                    // forward: y1 = s1 - i s3, y3 = s1 + i s3 (inverse: swapped)
                    const cx<T> mi = {s3.im, -s3.re};
                    Y[pidx(base)] = cadd(s0, s2);
                    Y[pidx(base + Ns)] = INV ? csub(s1, mi) : cadd(s1, mi);
                    Y[pidx(base + 2 * Ns)] = csub(s0, s2);
                    Y[pidx(base + 3 * Ns)] = INV ? cadd(s1, mi) : csub(s1, mi);
                } else {
                    cx<T> a0 = X[pidx(j)], a1 = cmul(X[pidx(j + m)], twq(1));
                    Y[pidx(base)] = cadd(a0, a1);
                    Y[pidx(base + Ns)] = csub(a0, a1);
                }
            }
        }
        __syncthreads();
        cx<T> *t = X;
        X = Y;
        Y = t;
        lgNs += lgr;
    }
    return X;
}

// The stage twiddle table in LDS: stage span Ns (the radix-4 stages' spans
// are powers of 4, and so is the last radix-2 stage's for odd LG) keeps
// w^((q k) N / (r Ns)) for q = 1 .. r - 1, k < Ns at (Ns - 1) + (q - 1) Ns + k
// -- consecutive in k, so a stage's lanes read consecutive entries -- n - 1
// values in all, gathered from the n natural twiddles twg (w^j as (re, im)).
template <class T, int N>
__device__ __forceinline__ void load_twiddles(const T *__restrict__ twg, cx<T> *tw) {
    constexpr int LG = __builtin_ctz(N);
#pragma unroll
    for (int e0 = 0; e0 < N - 1; e0 += FFT_NT) {
        const int e = e0 + (int)threadIdx.x;
        if (e < N - 1) {
            const int v = e + 1;
            const int lgNs = (31 - __builtin_clz(v)) & ~1;
            const int lgr = ((LG & 1) && lgNs == LG - 1) ? 1 : 2;
            const int q = v >> lgNs, k = v - (q << lgNs);
            const int idx = (q * k) << (LG - lgr - lgNs);
            tw[e] = {twg[2 * idx], twg[2 * idx + 1]};
        }
    }
}

// Half spectrum layout: column-major, spec[k n + r] for mode k <= n/2 of
// row r (the column pass reads and writes whole contiguous columns).
template <class T, int LG>
__global__ void __launch_bounds__(FFT_NT) k_fft_rows_fwd(const T *__restrict__ twg, FftPoissonArgs in,
                                                         cx<T> *__restrict__ spec) {
    constexpr int N = 1 << LG, HALF = N / 2, PT = (N + FFT_NT - 1) / FFT_NT;
    extern __shared__ unsigned char smem_raw[];
    __shared__ double red[4 * (FFT_NT / 64)];
    cx<T> *X = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *Y = X + padded(N);
    cx<T> *tw = Y + padded(N);
    const size_t r0 = 2 * (size_t)xcd_order();
    // rows r0, r0 + 1 of v1 and v2 (every global load in flight before the
    // first is used), their sums in float64, and q = a1 v1 + a2 v2 less the
    // row's mean, packed q_r0 + i q_r0+1
    const double *p1 = in.v1 + r0 * N;
    double qa[PT], qb[PT], va[PT], vb[PT];
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int j = (u * FFT_NT + (int)threadIdx.x) & (N - 1);
        qa[u] = p1[j];
        qb[u] = p1[N + j];
    }
    if (in.v2) {
        const double *p2 = in.v2 + r0 * N;
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int j = (u * FFT_NT + (int)threadIdx.x) & (N - 1);
            va[u] = p2[j];
            vb[u] = p2[N + j];
        }
    } else {
#pragma unroll
        for (int u = 0; u < PT; ++u) va[u] = vb[u] = 0.0;
    }
    load_twiddles<T, N>(twg, tw);
    double sm[4] = {0.0, 0.0, 0.0, 0.0};       // sums of v1 row a, row b, v2 row a, row b
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        if (N % FFT_NT == 0 || u * FFT_NT + (int)threadIdx.x < N) {
            sm[0] += qa[u];
            sm[1] += qb[u];
            sm[2] += va[u];
            sm[3] += vb[u];
        }
    }
    block_sums<4>(sm, red);
    if (threadIdx.x == 0) {
        in.sums[2 * r0] = sm[0];
        in.sums[2 * r0 + 1] = sm[2];
        in.sums[2 * r0 + 2] = sm[1];
        in.sums[2 * r0 + 3] = sm[3];
    }
    const double ma = (in.a1 * sm[0] + in.a2 * sm[2]) / N, mb = (in.a1 * sm[1] + in.a2 * sm[3]) / N;
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int j = u * FFT_NT + (int)threadIdx.x;
        if (N % FFT_NT == 0 || j < N)
            X[pidx(j)] = {(T)(in.a1 * qa[u] + in.a2 * va[u] - ma), (T)(in.a1 * qb[u] + in.a2 * vb[u] - mb)};
    }
    __syncthreads();
    const cx<T> *R = fft_lds<T, false, LG>(X, Y, tw);
    // Z = FFT(q_a + i q_b): Q_a,k = (Z_k + conj Z_{n-k}) / 2,
    // Q_b,k = -i (Z_k - conj Z_{n-k}) / 2, stored side by side
    for (int k = threadIdx.x; k <= HALF; k += FFT_NT) {
        const cx<T> z = R[pidx(k)], zr = R[pidx((N - k) & (N - 1))];
        cx<T> *dst = spec + (size_t)k * N + r0;
        dst[0] = {T(0.5) * (z.re + zr.re), T(0.5) * (z.im - zr.im)};
        dst[1] = {T(0.5) * (z.im + zr.im), T(0.5) * (zr.re - z.re)};
    }
}

template <class T, int LG>
__global__ void __launch_bounds__(FFT_NT) k_fft_cols(const T *__restrict__ twg, const T *__restrict__ lamg, T dt,
                                                     FftPoissonArgs in, cx<T> *__restrict__ spec) {
    constexpr int N = 1 << LG, PT = (N + FFT_NT - 1) / FFT_NT;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *X = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *Y = X + padded(N);
    cx<T> *tw = Y + padded(N);
    T *lam = reinterpret_cast<T *>(tw + N);
    const int k = blockIdx.x;                     // mode of the column, 0..n/2
    cx<T> *col = spec + (size_t)k * N;
    cx<T> v[PT];
    T lv[PT];
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int r = (u * FFT_NT + (int)threadIdx.x) & (N - 1);
        v[u] = col[r];
        lv[u] = lamg[r];
    }
    if (k == 0) {
        // column 0 holds the row sums of q less n times its mean (the rows'
        // own means were subtracted before their transforms): rebuilt here
        // in float64 from the row sums, which also give the means
        __shared__ double red[2 * (FFT_NT / 64)];
        double sr[PT][2];
        double sm[2] = {0.0, 0.0};
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int r = (u * FFT_NT + (int)threadIdx.x) & (N - 1);
            sr[u][0] = in.sums[2 * r];
            sr[u][1] = in.sums[2 * r + 1];
        }
#pragma unroll
        for (int u = 0; u < PT; ++u)
            if (N % FFT_NT == 0 || u * FFT_NT + (int)threadIdx.x < N) {
                sm[0] += sr[u][0];
                sm[1] += sr[u][1];
            }
        block_sums<2>(sm, red);
        const double nm = (in.a1 * sm[0] + in.a2 * sm[1]) / N;
#pragma unroll
        for (int u = 0; u < PT; ++u) v[u] = {(T)(in.a1 * sr[u][0] + in.a2 * sr[u][1] - nm), T(0)};
        if (threadIdx.x == 0) {
            const double inv = 1.0 / ((double)N * N);
            in.means[0] = sm[0] * inv;
            in.means[1] = sm[1] * inv;
            if (in.zmeans) {
                in.zmeans[0] = sm[1] * inv;
                in.zmeans[1] = in.shift_scale * sm[0] * inv;
            }
        }
    }
    load_twiddles<T, N>(twg, tw);
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int r = u * FFT_NT + (int)threadIdx.x;
        if (N % FFT_NT == 0 || r < N) {
            X[pidx(r)] = v[u];
            lam[r] = lv[u];
        }
    }
    __syncthreads();
    cx<T> *R = fft_lds<T, false, LG>(X, Y, tw);
    cx<T> *O = R == X ? Y : X;
    // mode (a, k): times 1 / (dt (lam_a + lam_k) n^2) (the n^2 of the two
    // unnormalized inverse transforms), the constant mode dropped
    const T inv_n2 = T(1) / ((T)N * (T)N);
    const T lk = lam[k];
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int a = u * FFT_NT + (int)threadIdx.x;
        if (N % FFT_NT == 0 || a < N) {
            const T s = (a == 0 && k == 0) ? T(0) : inv_n2 / (dt * (lam[a] + lk));
            R[pidx(a)] = {R[pidx(a)].re * s, R[pidx(a)].im * s};
        }
    }
    __syncthreads();
    R = fft_lds<T, true, LG>(R, O, tw);
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int r = u * FFT_NT + (int)threadIdx.x;
        if (N % FFT_NT == 0 || r < N) col[r] = R[pidx(r)];
    }
}

template <class T, int LG>
__global__ void __launch_bounds__(FFT_NT) k_fft_rows_inv(const T *__restrict__ twg, const cx<T> *__restrict__ spec,
                                                         FftPoissonArgs out) {
    constexpr int N = 1 << LG, HALF = N / 2, PT = (N + FFT_NT - 1) / FFT_NT;
    constexpr int PH = (HALF + 1 + FFT_NT - 1) / FFT_NT;
    extern __shared__ unsigned char smem_raw[];
    cx<T> *X = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *Y = X + padded(N);
    cx<T> *tw = Y + padded(N);
    const size_t r0 = 2 * (size_t)xcd_order();
    // the full spectra of rows r0, r0 + 1 (X_{n-k} = conj X_k), packed
    // X + i Y: a loaded mode k fills entries k and n - k
    cx<T> ha[PH], hb[PH];
#pragma unroll
    for (int u = 0; u < PH; ++u) {
        int k = u * FFT_NT + (int)threadIdx.x;
        k = k <= HALF ? k : HALF;
        ha[u] = spec[(size_t)k * N + r0];
        hb[u] = spec[(size_t)k * N + r0 + 1];
    }
    load_twiddles<T, N>(twg, tw);
#pragma unroll
    for (int u = 0; u < PH; ++u) {
        const int k = u * FFT_NT + (int)threadIdx.x;
        if (k <= HALF) {
            const cx<T> a = ha[u], b = hb[u];
            X[pidx(k)] = {a.re - b.im, a.im + b.re};
            if (k > 0 && k < HALF) X[pidx(N - k)] = {a.re + b.im, b.re - a.im};
        }
    }
    __syncthreads();
    const cx<T> *R = fft_lds<T, true, LG>(X, Y, tw);
    const double shift = out.shift_scale * out.means[0];
    double *z = out.z + r0 * N;
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int j = u * FFT_NT + (int)threadIdx.x;
        if (N % FFT_NT == 0 || j < N) {
            z[j] = (double)R[pidx(j)].re + shift;
            z[N + j] = (double)R[pidx(j)].im + shift;
        }
    }
}

template <class T, int LG>
static void launch_fft_sized(hipStream_t st, T dt, const T *tw, const T *lam, const FftPoissonArgs &a, cx<T> *sp) {
    constexpr int N = 1 << LG;
    k_fft_rows_fwd<T, LG><<<N / 2, FFT_NT, row_lds(N, sizeof(T)), st>>>(tw, a, sp);
    k_fft_cols<T, LG><<<N / 2 + 1, FFT_NT, col_lds(N, sizeof(T)), st>>>(tw, lam, dt, a, sp);
    k_fft_rows_inv<T, LG><<<N / 2, FFT_NT, row_lds(N, sizeof(T)), st>>>(tw, sp, a);
}

template <class T>
void launch_fft_poisson(hipStream_t st, int n, T dt, const T *tw, const T *lam, const FftPoissonArgs &a, T *spec) {
    cx<T> *sp = reinterpret_cast<cx<T> *>(spec);
    switch (log2_exact(n)) {
        case 4: launch_fft_sized<T, 4>(st, dt, tw, lam, a, sp); break;
        case 5: launch_fft_sized<T, 5>(st, dt, tw, lam, a, sp); break;
        case 6: launch_fft_sized<T, 6>(st, dt, tw, lam, a, sp); break;
        case 7: launch_fft_sized<T, 7>(st, dt, tw, lam, a, sp); break;
        case 8: launch_fft_sized<T, 8>(st, dt, tw, lam, a, sp); break;
        case 9: launch_fft_sized<T, 9>(st, dt, tw, lam, a, sp); break;
        case 10: launch_fft_sized<T, 10>(st, dt, tw, lam, a, sp); break;
        case 11:
            if (sizeof(T) == sizeof(float)) launch_fft_sized<T, 11>(st, dt, tw, lam, a, sp);
            break;
        default: break;                       // fft_poisson_supported admits no other side
    }
}

template void launch_fft_poisson<float>(hipStream_t, int, float, const float *, const float *, const FftPoissonArgs &,
                                        float *);
template void launch_fft_poisson<double>(hipStream_t, int, double, const double *, const double *,
                                         const FftPoissonArgs &, double *);

}  // namespace irk
