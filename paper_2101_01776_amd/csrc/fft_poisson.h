// Spectral solve of the periodic Poisson problem of the streamfunction rows
// on the finest grid (fft_poisson.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace irk {

// Sides the spectral solve takes: powers of two from IRK_FFT_MIN up to
// 2048 in float32, 1024 in float64 (a work-group's vectors, their ping-pong
// copies, the twiddles and the eigenvalues in at most 64 KiB of LDS).
#define IRK_FFT_MIN 16
bool fft_poisson_supported(int n, size_t tsz);

// T values of the half-spectrum buffer of an n x n grid: n rows of n/2 + 1
// complex entries.
size_t fft_poisson_spectrum_values(int n);

// Arguments of the spectral solve: q = a1 v1 + a2 v2 (v2 optional), the
// float64 result z = x + shift_scale mean(v1), with x the mean-free solution.
// The means come from the solve itself: the work-group of a row pair adds
// its rows in float64 and subtracts each row's mean of q before the
// transforms (a large mean rounded to the transform precision would swamp
// the other modes), and the column pass of mode 0 rebuilds that column from
// the row sums, also in float64.
struct FftPoissonArgs {
    const double *v1 = nullptr;
    double a1 = 1.0;
    const double *v2 = nullptr;
    double a2 = 0.0;
    double *z = nullptr;
    double shift_scale = 0.0;
    double *sums = nullptr;     // scratch, 2 n values: per row, the sums of v1 and v2
    double *means = nullptr;    // written: mean v1, mean v2
    double *zmeans = nullptr;   // optional, written: mean v2, mean z (= shift_scale mean v1)
};

// Solves -dt Lap_h x = q on the periodic n x n grid (5-point Laplacian,
// spacing h; the constant mode of q is dropped and x is mean-free) and writes
// a.z as above (the transforms run in T).
// tw: the n twiddles exp(-2 pi i j / n) as (re, im) pairs; lam: the n
// eigenvalues 4 sin^2(pi m / n) / h^2 of the 1-D second difference; spec:
// fft_poisson_spectrum_values(n) values of scratch.  Three launches on st:
// row transforms of row pairs packed as one complex row (with the row
// sums), column transforms with the division by dt (lam_a + lam_b) and the
// inverse column transforms (mode 0 also reduces the row sums to the means),
// and the inverse row transforms.
template <class T>
void launch_fft_poisson(hipStream_t st, int n, T dt, const T *tw, const T *lam, const FftPoissonArgs &a, T *spec);

}  // namespace irk
