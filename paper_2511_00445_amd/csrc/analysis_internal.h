// Internal interface of the observables' kernels (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace tana {

// za = phi + i omega_c, zb = u_c, zc = Qxx + i Qxy from an exported state [7][n][n].
hipError_t launch_pack(const float* state, int n, float2* za, float2* zb, float2* zc, hipStream_t st);
// 2D FFT (unnormalised; inverse = conjugate twiddles) of the n x n complex array
// `in` (overwritten), n = 2^logn, written TRANSPOSED to `out` (out[x][y] = F[y][x]):
// row transforms, one transpose, row transforms.  Power spectra and shell sums
// are symmetric in the two axes, and the transposed-layout inverse of a
// transposed array is the natural-layout inverse, so the second transpose of
// each transform is never needed.
hipError_t launch_fft2t(float2* in, float2* out, int n, int logn, bool inverse, const float2* tw, hipStream_t st);
// Table of the n / 2 forward twiddles exp(-2 pi i k / n) used by launch_fft2t.
hipError_t launch_twiddles(float2* tw, int n, hipStream_t st);
// Power spectra and the inverse-transform inputs of the correlations (see k_power).
hipError_t launch_power(const float2* za, const float2* zb, const float2* zc, int n, float* pE, float* pS,
                        float2* w0, float2* w1, hipStream_t st);
// Shell sums of up to three inputs (element e at in_c[stride * e]) into out[4][ns]
// (three sums and the counts); mean: divide by the value at the origin and by the
// count (correlation maps).  partial: 3 ns nb doubles, pcount: ns nb ints, nb = ceil(n / 256) row blocks.
hipError_t launch_shells(const float* in0, const float* in1, const float* in2, int stride, int n, int ns, bool mean,
                         double* partial, int* pcount, double* out, hipStream_t st);
// W = k^2 E into out[2 ns ..) and L into out[4 ns].
hipError_t launch_finish_spectra(double* out, int n, int ns, hipStream_t st);
int reduce_blocks(int n);
hipError_t launch_overlaps(const float* s0, const float* s1, int n, double* partial, double* out, hipStream_t st);
// Defect counts (exact integers carried in doubles): out[0] = +1/2, out[1] = -1/2.
hipError_t launch_defects(const float* state, int n, double* partial, double* out, hipStream_t st);

}  // namespace tana
