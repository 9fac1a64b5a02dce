/* On-device observables of the two-fluid active-nematic solver (Results section):
 * C ABI.
 *
 * Every function takes solver states as exported by tfan_export_state: device
 * float32 arrays [7][n][n] (phi, Qxx, Qxy, u_a,x, u_a,y, u_p,x, u_p,y), x fastest,
 * on a square periodic grid with n a power of two in [8, 4096].
 *
 * Definitions: mixed velocity u_c = c1 u_a + c2 u_p (c1 = (1 + phi)/2,
 * c2 = 1 - c1); mixed vorticity omega_c = d_x u_c,y - d_y u_c,x (central
 * differences); hat f = FFT(f) / n^2 with wavevector index m in (-n/2, n/2]^2;
 * shell s of m (or of a displacement r, minimum image) = the integer nearest to
 * |m|, s = 0 .. tfan_analysis_shells(n) - 1.
 *   E(s) = 1/2 sum_{shell s} |hat u_c|^2   kinetic-energy spectrum
 *   W(s) = k_s^2 E(s), k_s = 2 pi s / n     enstrophy spectrum
 *   S(s) = sum_{shell s} |hat phi|^2        phase-field spectrum
 *   L    = 2 pi sum_{s>0} S(s) / sum_{s>0} k_s S(s)   domain length
 *   C_f(s) = shell mean over displacements r of <f(x) . f(x + r)> / <f . f> for
 *            f = delta u_c, delta omega_c (fluctuations about the mean) and Q
 *            (Q : Q' = 2 (Qxx Qxx' + Qxy Qxy'))   spatial correlations
 *   +-1/2 defects: director angle atan2(Qxy, Qxx) / 2; around each elementary
 *            plaquette the angle differences wrapped into [-pi/2, pi/2) sum to
 *            +pi (+1/2 defect), -pi (-1/2) or 0.
 * Spectra and correlations use a float32 FFT; sums over shells and sites are
 * float64 in a fixed order (results are deterministic).
 *
 * Ownership: the caller owns the device workspace (256-byte aligned, at least
 * tfan_analysis_workspace_bytes(n)), the state arrays and all host outputs.  All
 * work runs on the handle's stream; every function that returns host values
 * synchronises it.  Return codes are those of tfan.h.
 */
#ifndef TFAN_ANALYSIS_H
#define TFAN_ANALYSIS_H

#include <stddef.h>
#include <stdint.h>

#include "tfan.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tfan_analysis tfan_analysis;

/* Number of shells for an n x n grid (largest shell index + 1); 0 if n is invalid. */
int32_t tfan_analysis_shells(int32_t n);

/* Workspace for an n x n grid; 0 if n is not a power of two in [8, 4096]. */
size_t tfan_analysis_workspace_bytes(int32_t n);

/* TFAN_EINVAL (bad n, unaligned workspace) / TFAN_ENOMEM (workspace too small). */
int tfan_analysis_create(int32_t n, void* dev_workspace, size_t bytes, void* hip_stream, tfan_analysis** out);

/* E, W, S and the number of wavevectors per shell (host arrays of
 * tfan_analysis_shells(n) doubles; any may be NULL) and L (may be NULL). */
int tfan_analysis_spectra(tfan_analysis* a, const float* state, double* E, double* W, double* S, double* count,
                          double* L);

/* Shell-averaged spatial correlations C_uu, C_ww, C_QQ and the number of
 * displacements per shell (host arrays of tfan_analysis_shells(n) doubles; any
 * may be NULL). */
int tfan_analysis_correlations(tfan_analysis* a, const float* state, double* Cuu, double* Cww, double* CQQ,
                               double* count);

/* Site means for the temporal correlations between states s0 and s1:
 * out[0] = <u_c . u_c'>, out[1] = <|u_c|^2>, out[2] = <omega_c omega_c'>,
 * out[3] = <omega_c^2>, out[4] = <Q : Q'>, out[5] = <Q : Q> (unprimed = s0). */
int tfan_analysis_overlaps(tfan_analysis* a, const float* s0, const float* s1, double* out);

/* Numbers of +1/2 and -1/2 defects. */
int tfan_analysis_defects(tfan_analysis* a, const float* state, int64_t* plus, int64_t* minus);

/* Everything above for one state in one call, the three forward transforms
 * computed once: the same values as tfan_analysis_spectra, _correlations and
 * _defects on that state (bitwise: the same kernels).  The shell counts of the
 * spectra and of the correlations are the same numbers (wavevectors and
 * minimum-image displacements fall in the same shells) and are returned once.
 * Array arguments as above, any may be NULL; plus and minus may be NULL. */
int tfan_analysis_all(tfan_analysis* a, const float* state, double* E, double* W, double* S, double* L,
                      double* Cuu, double* Cww, double* CQQ, double* count, int64_t* plus, int64_t* minus);

/* Allocation-free variant of tfan_analysis_overlaps, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc): no handle and no workspace.  Same inputs and the same
 * six site means in out[6] (host array), computed by the same kernels on
 * hip_stream (hipStream_t, NULL = default stream) of the current device; the
 * call synchronises that stream.  The block partials live in a fixed array of
 * 49,200 bytes inside the library, one copy per GPU, held until the process
 * ends; the call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine).  Sizes: n a power of two in [8, 4096] (the reduction uses at most
 * 1024 blocks), else TFAN_EINVAL.  Calls that overlap on one GPU (other threads
 * or streams) share that array and race: serialise them.  The message of the
 * last failure: tfan_analysis_noalloc_last_error(). */
int tfan_analysis_overlaps_noalloc(int32_t n, const float* s0, const float* s1, double* out, void* hip_stream);
const char* tfan_analysis_noalloc_last_error(void);

int tfan_analysis_sync(tfan_analysis* a);
void tfan_analysis_destroy(tfan_analysis* a);
const char* tfan_analysis_last_error(const tfan_analysis* a);

#ifdef __cplusplus
}
#endif
#endif
