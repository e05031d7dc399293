// Spectral solve of the periodic Poisson problem -dt Lap_h x = q on the
// finest grid, for the streamfunction rows of the vorticity-streamfunction
// DAE (their block operator is the constant-coefficient 5-point Laplacian).
//
// The discrete Fourier modes e^{2 pi i (a x + b y)} diagonalize the periodic
// 5-point Laplacian: -Lap_h has eigenvalue lam_a + lam_b with
// lam_m = 4 sin^2(pi m / n) / h^2, so x^_ab = q^_ab / (dt (lam_a + lam_b)),
// the constant mode (a, b) = (0, 0) dropped.  Three launches:
//   k_fft_rows_fwd  rows 2r and 2r+1 of q packed as one complex row
//                   (q_2r + i q_2r+1), transformed in LDS, then separated by
//                   Hermitian symmetry into the half spectra (modes 0..n/2)
//                   of both rows; two row pairs per work-group;
//   k_fft_cols      one column (mode k) of the half spectrum: transform,
//                   divide by dt (lam_a + lam_k) n^2, inverse transform;
//   k_fft_rows_inv  rows 2r and 2r+1 again: their full spectra rebuilt from
//                   the halves (X_{n-k} = conj X_k), packed as X + i Y, one
//                   inverse transform whose real and imaginary parts are the
//                   two real rows of x.
// The transforms are mixed radix-4/2 Stockham passes in LDS (vectors, their
// ping-pong copies and the twiddles); the half spectrum (n (n/2 + 1) complex
// values, column-major) is the only intermediate in memory.
#include <hip/hip_runtime.h>

#include "fft_poisson.h"

namespace irk {

namespace {

constexpr int FFT_NT = 256;
constexpr size_t FFT_LDS_MAX = 64 * 1024;

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

// LDS bytes of a row work-group holding p row pairs (each a complex vector
// and its ping-pong copy) and the n twiddles
size_t row_lds(int n, int p, size_t tsz) { return (2 * (size_t)p * n + n) * 2 * tsz; }
// ... of a column work-group: one column, its copy, the twiddles, the n
// eigenvalues
size_t col_lds(int n, size_t tsz) { return (3 * (size_t)n) * 2 * tsz + n * tsz; }

// row pairs per work-group of the row passes: two (four rows: the half
// spectrum's column-major stores and loads move 4 consecutive values) when
// they fit the LDS budget
int rows_pairs_per_group(int n, size_t tsz) { return row_lds(n, 2, tsz) <= FFT_LDS_MAX ? 2 : 1; }

// XCD-aware work-group order: consecutive logical indices on one XCD (work
// groups are dealt to the 8 XCDs round-robin; neighbours share cache lines
// of the half spectrum); the identity unless the grid is a multiple of 8
__device__ __forceinline__ int xcd_order() {
    const int nb = gridDim.x, b = blockIdx.x;
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

}  // namespace

bool fft_poisson_supported(int n, size_t tsz) {
    if (n < IRK_FFT_MIN || log2_exact(n) < 0) return false;
    return row_lds(n, 1, tsz) <= FFT_LDS_MAX && col_lds(n, tsz) <= FFT_LDS_MAX;
}

size_t fft_poisson_spectrum_values(int n) { return (size_t)2 * n * (n / 2 + 1); }

// Mixed radix-4/2 Stockham transform (self-sorting: natural order in and
// out) of nvec vectors of length n = 2^k stored one after another in X; Y is
// the ping-pong buffer, tw the n twiddles w^j = exp(-2 pi i j / n).  A stage
// of radix r (4 while n / Ns >= 4, a last radix-2 stage for odd k) and span
// Ns takes x[j + q n/r], q < r, times w^(q k n / (r Ns)) with k = j mod Ns,
// through an r-point DFT into y[(j - k) r + k + q Ns].  INV: conjugate
// twiddles and DFTs (unnormalized inverse).  Returns the buffer holding the
// result.
template <class T, bool INV>
__device__ cx<T> *fft_lds(cx<T> *X, cx<T> *Y, int n, int lg2n, int nvec, const cx<T> *tw) {
    int Ns = 1, lgNs = 0;
    while (Ns < n) {
        const bool r4 = lg2n - lgNs >= 2;
        const int lgr = r4 ? 2 : 1;
        const int lgm = lg2n - lgr, m = 1 << lgm;        // butterflies per vector
        const int lgstep = lg2n - lgr - lgNs;            // twiddle step n / (r Ns)
        const int total = nvec << lgm;
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            const int v = t >> lgm, j = t & (m - 1);
            const cx<T> *x = X + (v << lg2n);
            cx<T> *y = Y + (v << lg2n);
            const int k = j & (Ns - 1);
            const int base = ((j - k) << lgr) + k;
            auto twq = [&](int q) {
                cx<T> w = tw[(q * k) << lgstep];
                if (INV) w.im = -w.im;
                return w;
            };
            if (r4) {
                cx<T> a0 = x[j], a1 = x[j + m], a2 = x[j + 2 * m], a3 = x[j + 3 * m];
                if (k) {
                    a1 = cmul(a1, twq(1));
                    a2 = cmul(a2, twq(2));
                    a3 = cmul(a3, twq(3));
                }
                const cx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
                // forward: y1 = t1 - i t3, y3 = t1 + i t3 (inverse: swapped)
                const cx<T> mi = {t3.im, -t3.re};
                y[base] = cadd(t0, t2);
                y[base + Ns] = INV ? csub(t1, mi) : cadd(t1, mi);
                y[base + 2 * Ns] = csub(t0, t2);
                y[base + 3 * Ns] = INV ? cadd(t1, mi) : csub(t1, mi);
            } else {
                cx<T> a0 = x[j], a1 = x[j + m];
                if (k) a1 = cmul(a1, twq(1));
                y[base] = cadd(a0, a1);
                y[base + Ns] = csub(a0, a1);
            }
        }
        __syncthreads();
        cx<T> *t = X;
        X = Y;
        Y = t;
        Ns <<= lgr;
        lgNs += lgr;
    }
    return X;
}

template <class T>
__device__ __forceinline__ void load_twiddles(const T *__restrict__ twg, cx<T> *tw, int n) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) tw[j] = {twg[2 * j], twg[2 * j + 1]};
}

// rows 2r, 2r+1 of q = a1 v1 + a2 v2 for the P row pairs of a work-group,
// packed q_2r + i q_2r+1, into LDS vectors X + p n; every global load of a
// batch is in flight before the first LDS store
template <class T, int P>
__device__ __forceinline__ void load_row_pairs(int n, size_t r0, const MgIn &in, cx<T> *X) {
    constexpr int B = 8;
    const int items = P * n;                      // complex points
    for (int i0 = 0; i0 < items; i0 += B * FFT_NT) {
        double qa[B], qb[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int it = i0 + u * FFT_NT + (int)threadIdx.x;
            const int ii = it < items ? it : 0;
            const int p = ii / n, j = ii - p * n;
            const size_t o = (r0 + 2 * p) * n + j;
            qa[u] = in.a1 * in.v1[o];
            qb[u] = in.a1 * in.v1[o + n];
            if (in.v2) {
                qa[u] += in.a2 * in.v2[o];
                qb[u] += in.a2 * in.v2[o + n];
            }
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int it = i0 + u * FFT_NT + (int)threadIdx.x;
            if (it < items) X[it] = {(T)qa[u], (T)qb[u]};
        }
    }
}

// Half spectrum layout: column-major, spec[k n + r] for mode k <= n/2 of
// row r (the column pass reads and writes whole contiguous columns).
template <class T, int P>
__global__ void __launch_bounds__(FFT_NT) k_fft_rows_fwd(int n, int lg2n, const T *__restrict__ twg, MgIn in,
                                                         cx<T> *__restrict__ spec) {
    extern __shared__ unsigned char smem_raw[];
    cx<T> *X = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *Y = X + P * n;
    cx<T> *tw = Y + P * n;
    const int half = n >> 1;
    const size_t r0 = (size_t)(2 * P) * xcd_order();
    load_row_pairs<T, P>(n, r0, in, X);
    load_twiddles(twg, tw, n);
    __syncthreads();
    const cx<T> *R = fft_lds<T, false>(X, Y, n, lg2n, P, tw);
    // Z = FFT(q_a + i q_b): Q_a,k = (Z_k + conj Z_{n-k}) / 2,
    // Q_b,k = -i (Z_k - conj Z_{n-k}) / 2; the 2P rows of mode k are stored
    // together
    for (int k = threadIdx.x; k <= half; k += blockDim.x) {
        cx<T> o[2 * P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const cx<T> z = R[p * n + k], zr = R[p * n + ((n - k) & (n - 1))];
            o[2 * p] = {T(0.5) * (z.re + zr.re), T(0.5) * (z.im - zr.im)};
            o[2 * p + 1] = {T(0.5) * (z.im + zr.im), T(0.5) * (zr.re - z.re)};
        }
        cx<T> *dst = spec + (size_t)k * n + r0;
#pragma unroll
        for (int q = 0; q < 2 * P; ++q) dst[q] = o[q];
    }
}

template <class T>
__global__ void __launch_bounds__(FFT_NT) k_fft_cols(int n, int lg2n, const T *__restrict__ twg,
                                                     const T *__restrict__ lamg, T dt, cx<T> *__restrict__ spec) {
    extern __shared__ unsigned char smem_raw[];
    cx<T> *X = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *Y = X + n;
    cx<T> *tw = Y + n;
    T *lam = reinterpret_cast<T *>(tw + n);
    const int k = blockIdx.x;                     // mode of the column, 0..n/2
    cx<T> *col = spec + (size_t)k * n;
    {
        constexpr int B = 8;
        for (int i0 = 0; i0 < n; i0 += B * FFT_NT) {
            cx<T> v[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int r = i0 + u * FFT_NT + (int)threadIdx.x;
                v[u] = col[r < n ? r : 0];
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int r = i0 + u * FFT_NT + (int)threadIdx.x;
                if (r < n) X[r] = v[u];
            }
        }
    }
    load_twiddles(twg, tw, n);
    for (int j = threadIdx.x; j < n; j += blockDim.x) lam[j] = lamg[j];
    __syncthreads();
    cx<T> *R = fft_lds<T, false>(X, Y, n, lg2n, 1, tw);
    cx<T> *O = R == X ? Y : X;
    // mode (a, k): times 1 / (dt (lam_a + lam_k) n^2) (the n^2 of the two
    // unnormalized inverse transforms), the constant mode dropped
    const T inv_n2 = T(1) / ((T)n * (T)n);
    const T lk = lam[k];
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const T s = (a == 0 && k == 0) ? T(0) : inv_n2 / (dt * (lam[a] + lk));
        R[a] = {R[a].re * s, R[a].im * s};
    }
    __syncthreads();
    R = fft_lds<T, true>(R, O, n, lg2n, 1, tw);
    for (int r = threadIdx.x; r < n; r += blockDim.x) col[r] = R[r];
}

template <class T, int P>
__global__ void __launch_bounds__(FFT_NT) k_fft_rows_inv(int n, int lg2n, const T *__restrict__ twg,
                                                         const cx<T> *__restrict__ spec, MgOut out) {
    extern __shared__ unsigned char smem_raw[];
    cx<T> *X = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *Y = X + P * n;
    cx<T> *tw = Y + P * n;
    const int half = n >> 1;
    const size_t r0 = (size_t)(2 * P) * xcd_order();
    // the full spectra of the 2P real rows (X_{n-k} = conj X_k), each pair
    // packed X + i Y: a loaded mode k fills entries k and n - k
    for (int k = threadIdx.x; k <= half; k += blockDim.x) {
        cx<T> h[2 * P];
        const cx<T> *src = spec + (size_t)k * n + r0;
#pragma unroll
        for (int q = 0; q < 2 * P; ++q) h[q] = src[q];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const cx<T> a = h[2 * p], b = h[2 * p + 1];
            X[p * n + k] = {a.re - b.im, a.im + b.re};
            if (k > 0 && k < half) X[p * n + n - k] = {a.re + b.im, b.re - a.im};
        }
    }
    load_twiddles(twg, tw, n);
    __syncthreads();
    const cx<T> *R = fft_lds<T, true>(X, Y, n, lg2n, P, tw);
    const double shift = out.shift ? out.shift_scale * out.shift[0] : 0.0;
    for (int it = threadIdx.x; it < P * n; it += blockDim.x) {
        const int p = it / n, j = it - p * n;
        double *z = out.z + (r0 + 2 * p) * n + j;
        z[0] = (double)R[it].re + shift;
        z[n] = (double)R[it].im + shift;
    }
}

template <class T, int P>
static void launch_rows(hipStream_t st, int n, int lg2n, const T *tw, const MgIn &in, const MgOut &out,
                        cx<T> *sp, bool inverse) {
    const size_t shm = row_lds(n, P, sizeof(T));
    const int grid = n / (2 * P);
    if (!inverse) k_fft_rows_fwd<T, P><<<grid, FFT_NT, shm, st>>>(n, lg2n, tw, in, sp);
    else k_fft_rows_inv<T, P><<<grid, FFT_NT, shm, st>>>(n, lg2n, tw, sp, out);
}

template <class T>
void launch_fft_poisson(hipStream_t st, int n, T dt, const T *tw, const T *lam, const MgIn &in, const MgOut &out,
                        T *spec) {
    const int lg2n = log2_exact(n);
    cx<T> *sp = reinterpret_cast<cx<T> *>(spec);
    const int P = rows_pairs_per_group(n, sizeof(T));
    if (P == 2) launch_rows<T, 2>(st, n, lg2n, tw, in, out, sp, false);
    else launch_rows<T, 1>(st, n, lg2n, tw, in, out, sp, false);
    k_fft_cols<T><<<n / 2 + 1, FFT_NT, col_lds(n, sizeof(T)), st>>>(n, lg2n, tw, lam, dt, sp);
    if (P == 2) launch_rows<T, 2>(st, n, lg2n, tw, in, out, sp, true);
    else launch_rows<T, 1>(st, n, lg2n, tw, in, out, sp, true);
}

template void launch_fft_poisson<float>(hipStream_t, int, float, const float *, const float *, const MgIn &,
                                        const MgOut &, float *);
template void launch_fft_poisson<double>(hipStream_t, int, double, const double *, const double *, const MgIn &,
                                         const MgOut &, double *);

}  // namespace irk
