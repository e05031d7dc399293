// Spectral solve of the periodic Poisson problem of the streamfunction rows
// on the finest grid (fft_poisson.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "mg_tiled.h"

namespace irk {

// Sides the spectral solve takes: powers of two from IRK_FFT_MIN up to
// 2048 in float32, 1024 in float64 (a work-group's vectors, their ping-pong
// copies, the twiddles and the eigenvalues in at most 64 KiB of LDS).
#define IRK_FFT_MIN 16
bool fft_poisson_supported(int n, size_t tsz);

// T values of the half-spectrum buffer of an n x n grid: n rows of n/2 + 1
// complex entries.
size_t fft_poisson_spectrum_values(int n);

// Solves -dt Lap_h x = q on the periodic n x n grid (5-point Laplacian,
// spacing h; the constant mode of q is dropped and x is mean-free), with
// q = in.a1 in.v1 + in.a2 in.v2 - (in.a1 in.mean[0] + in.a2 in.mean[1])
// (in.v2 and in.mean optional; the mean is subtracted in float64 before the
// transforms, which run in T), and writes
// out.z = x + out.shift_scale * out.shift[0] (out.shift optional) in float64.
// tw: the n twiddles exp(-2 pi i j / n) as (re, im) pairs; lam: the n
// eigenvalues 4 sin^2(pi m / n) / h^2 of the 1-D second difference; spec:
// fft_poisson_spectrum_values(n) values of scratch.  Three launches on st:
// row transforms of row pairs packed as one complex row, column transforms
// with the division by dt (lam_a + lam_b) and the inverse column
// transforms, and the inverse row transforms.
template <class T>
void launch_fft_poisson(hipStream_t st, int n, T dt, const T *tw, const T *lam, const MgIn &in, const MgOut &out,
                        T *spec);

}  // namespace irk
