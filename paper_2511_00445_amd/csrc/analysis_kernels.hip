// gfx950 kernels of the on-device observables (Results section): packing of the
// exported state into complex fields, a radix-2 2D FFT (one row per block in LDS,
// tiled transposes), power spectra, shell sums, spatial-correlation maps,
// temporal-correlation overlaps and the winding-number defect count.
#include "analysis_internal.h"

namespace tana {
namespace {

__device__ __forceinline__ int wrapn(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Nearest integer to sqrt(m2) for an integer m2 >= 0, exactly: (s + 1/2)^2 =
// s^2 + s + 1/4, so the nearest integer is s + 1 once m2 >= s^2 + s + 1.
__device__ __forceinline__ int shell_of(int m2) {
  int s = (int)sqrtf((float)m2);
  while (s * s > m2) --s;
  while ((s + 1) * (s + 1) <= m2) ++s;
  return (m2 >= s * s + s + 1) ? s + 1 : s;
}
// Signed frequency (or minimum-image displacement) of index i; only |.| is used.
__device__ __forceinline__ int freq(int i, int n) { return i <= n / 2 ? i : i - n; }

// Mixed velocity u_c = c1 u_a + c2 u_p at site (y, x) of an exported state.
__device__ __forceinline__ float2 mixed(const float* __restrict__ s, size_t n2, int idx) {
  const float c1 = 0.5f * (1.f + s[idx]);
  const float c2 = 1.f - c1;
  return make_float2(c1 * s[3 * n2 + idx] + c2 * s[5 * n2 + idx], c1 * s[4 * n2 + idx] + c2 * s[6 * n2 + idx]);
}
// Mixed vorticity d_x u_c,y - d_y u_c,x (central differences) at (y, x).
__device__ __forceinline__ float vort(const float* __restrict__ s, int n, int y, int x) {
  const size_t n2 = (size_t)n * n;
  const float2 e = mixed(s, n2, y * n + wrapn(x + 1, n)), w = mixed(s, n2, y * n + wrapn(x - 1, n));
  const float2 no = mixed(s, n2, wrapn(y + 1, n) * n + x), so = mixed(s, n2, wrapn(y - 1, n) * n + x);
  return 0.5f * (e.y - w.y) - 0.5f * (no.x - so.x);
}

// za = phi + i omega_c, zb = u_c,x + i u_c,y, zc = Qxx + i Qxy.
__global__ void k_pack(const float* __restrict__ s, int n, float2* __restrict__ za, float2* __restrict__ zb,
                       float2* __restrict__ zc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * n) return;
  const int y = i / n, x = i - y * n;
  const size_t n2 = (size_t)n * n;
  const float2 u = mixed(s, n2, i);
  za[i] = make_float2(s[i], vort(s, n, y, x));
  zb[i] = u;
  zc[i] = make_float2(s[n2 + i], s[2 * n2 + i]);
}

// FFT of every row (one block per row), unnormalised; INV uses the conjugate
// twiddles w_k = exp(+2 pi i k / n), both from the table of k_twiddles (the
// values sincospif gives, computed once per handle instead of once per row).
// Bit-reversed load into LDS, then the radix-2 decimation-in-time stages in
// pairs: a thread takes four points, applies the
// butterflies of two consecutive stages in registers and writes them back, so a
// pair costs one LDS round trip and one barrier (an odd last stage runs alone).
// The butterflies and twiddles are those of the plain radix-2 form, in the same
// order.  LDS index i is stored at i + i / 32, spreading the bit-reversed writes
// over the banks.
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 5); }
__device__ __forceinline__ void butterfly(float2& u, float2& v, float2 w) {
  const float2 t = make_float2(w.x * v.x - w.y * v.y, w.x * v.y + w.y * v.x);
  const float2 a = u;
  u = make_float2(a.x + t.x, a.y + t.y);
  v = make_float2(a.x - t.x, a.y - t.y);
}
// Forward twiddles w_k = exp(-2 pi i k / n), k < n / 2 (computed once per handle).
__global__ void k_twiddles(float2* __restrict__ tw, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n / 2) return;
  float sn, cs;
  sincospif(2.f * (float)k / (float)n, &sn, &cs);
  tw[k] = make_float2(cs, -sn);
}

template <bool INV>
__global__ void __launch_bounds__(256) k_fft_rows(float2* __restrict__ data, const float2* __restrict__ twg, int n,
                                                  int logn) {
  extern __shared__ float2 sm[];
  float2* buf = sm;
  float2* tw = sm + n + (n >> 5);
  float2* row = data + (size_t)blockIdx.x * n;
  for (int i = threadIdx.x; i < n; i += 256) buf[lds_pad(__brev((unsigned)i) >> (32 - logn))] = row[i];
  for (int k = threadIdx.x; k < n / 2; k += 256) {
    const float2 w = twg[k];
    tw[k] = INV ? make_float2(w.x, -w.y) : w;
  }
  __syncthreads();
  int lh = 0;
  for (; lh + 1 < logn; lh += 2) {
    const int half = 1 << lh, s1 = n >> (lh + 1), s2 = n >> (lh + 2);
    for (int q = threadIdx.x; q < n / 4; q += 256) {
      const int pos = q & (half - 1), grp = q >> lh;
      const int i0 = (grp << (lh + 2)) + pos, i1 = i0 + half, i2 = i1 + half, i3 = i2 + half;
      float2 a0 = buf[lds_pad(i0)], a1 = buf[lds_pad(i1)], a2 = buf[lds_pad(i2)], a3 = buf[lds_pad(i3)];
      const float2 w1 = tw[pos * s1];
      butterfly(a0, a1, w1);  // stage lh: pairs at distance half
      butterfly(a2, a3, w1);
      butterfly(a0, a2, tw[pos * s2]);  // stage lh + 1: pairs at distance 2 half
      butterfly(a1, a3, tw[(pos + half) * s2]);
      buf[lds_pad(i0)] = a0;
      buf[lds_pad(i1)] = a1;
      buf[lds_pad(i2)] = a2;
      buf[lds_pad(i3)] = a3;
    }
    __syncthreads();
  }
  if (lh < logn) {
    const int half = 1 << lh, stride = n >> (lh + 1);
    for (int b = threadIdx.x; b < n / 2; b += 256) {
      const int pos = b & (half - 1), grp = b >> lh;
      const int i = (grp << (lh + 1)) + pos, j = i + half;
      float2 u = buf[lds_pad(i)], v = buf[lds_pad(j)];
      butterfly(u, v, tw[pos * stride]);
      buf[lds_pad(i)] = u;
      buf[lds_pad(j)] = v;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += 256) row[i] = buf[lds_pad(i)];
}

// out = in^T, 32 x 32 tiles through LDS (32 x 8 threads).
__global__ void k_transpose(const float2* __restrict__ in, float2* __restrict__ out, int n) {
  __shared__ float2 t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int j = threadIdx.y; j < 32; j += 8)
    if (by + j < n && bx + (int)threadIdx.x < n) t[j][threadIdx.x] = in[(size_t)(by + j) * n + bx + threadIdx.x];
  __syncthreads();
  for (int j = threadIdx.y; j < 32; j += 8)
    if (bx + j < n && by + (int)threadIdx.x < n) out[(size_t)(bx + j) * n + by + threadIdx.x] = t[threadIdx.x][j];
}

// From the transforms of za, zb, zc (natural layout): pE = |hat u_c|^2 / 2,
// pS = |hat phi|^2 (hat = FFT / n^2), and the inverse inputs
// w0 = (|hat du|^2, |hat dw|^2) (k = 0 removed: fluctuations), w1 = (|hat Q|^2, 0).
// With Z = FFT(a + i b) for real a, b: hat a = (Z(k) + conj Z(-k)) / 2,
// hat b = (Z(k) - conj Z(-k)) / 2i, |hat a|^2 + |hat b|^2 = (|Z(k)|^2 + |Z(-k)|^2) / 2.
__global__ void k_power(const float2* __restrict__ za, const float2* __restrict__ zb, const float2* __restrict__ zc,
                        int n, float inv_n4, float* __restrict__ pE, float* __restrict__ pS,
                        float2* __restrict__ w0, float2* __restrict__ w1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * n) return;
  const int a = i / n, b = i - a * n;
  const int m = ((n - a) & (n - 1)) * n + ((n - b) & (n - 1));
  const float2 A = za[i], Am = za[m];
  const float px = 0.5f * (A.x + Am.x), py = 0.5f * (A.y - Am.y);     // hat phi * n^2
  const float ox = 0.5f * (A.y + Am.y), oy = -0.5f * (A.x - Am.x);    // hat omega * n^2
  const float2 B = zb[i], Bm = zb[m], Cq = zc[i], Cm = zc[m];
  const float pu = 0.5f * ((B.x * B.x + B.y * B.y) + (Bm.x * Bm.x + Bm.y * Bm.y)) * inv_n4;
  const float pw = (ox * ox + oy * oy) * inv_n4;
  const float pq = 0.5f * ((Cq.x * Cq.x + Cq.y * Cq.y) + (Cm.x * Cm.x + Cm.y * Cm.y)) * inv_n4;
  pE[i] = 0.5f * pu;
  pS[i] = (px * px + py * py) * inv_n4;
  w0[i] = i == 0 ? make_float2(0.f, 0.f) : make_float2(pu, pw);
  w1[i] = make_float2(pq, 0.f);
}

// Largest integer r with r * r <= v (v >= 0), exactly.
__device__ __forceinline__ int isqrt_floor(int v) {
  int r = (int)sqrtf((float)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// Shell sums, one thread per (shell s, row j): the sites of row j in shell s are
// those with (s - 1/2)^2 <= fx^2 + fy^2 < (s + 1/2)^2, i.e. fx^2 in
// [s^2 - s + 1 - fy^2, s^2 + s - fy^2] (s = 0: fx = fy = 0), an interval of |fx|
// taken at +fx and -fx.  Each thread sums its sites in a fixed order; the block's
// 256 rows are then added by a fixed tree, and the block writes
// partial[c][s][b] (three inputs, element e at in_c[stride * e]) and the count
// (b = row block; n / 256 partials per shell instead of n).
__global__ void __launch_bounds__(256) k_shell_part(const float* __restrict__ in0, const float* __restrict__ in1,
                                                   const float* __restrict__ in2, int stride, int n, int ns,
                                                   double* __restrict__ partial, int* __restrict__ pcount) {
  __shared__ double red[4][256];
  const int t = threadIdx.x, j = blockIdx.x * 256 + t, s = blockIdx.y;
  const int fy = freq(j < n ? j : 0, n), f2 = j < n ? fy * fy : 0x7fffffff, half = n / 2;
  const int lo = s == 0 ? 0 : s * s - s + 1, hi = s == 0 ? 0 : s * s + s;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  int c = 0;
  if (f2 <= hi) {
    const int b2 = hi - f2, a2lim = lo > f2 ? lo - f2 : 0;
    int fa = isqrt_floor(a2lim);
    if (fa * fa < a2lim) ++fa;  // ceil
    int fb = isqrt_floor(b2);
    if (fb > half) fb = half;
    const size_t row = (size_t)j * n;
    for (int fx = fa; fx <= fb; ++fx) {
      for (int sign = 0; sign < 2; ++sign) {
        if (sign == 1 && (fx == 0 || fx == half)) continue;  // +fx and -fx are one bin
        const size_t e = (size_t)stride * (row + (sign ? n - fx : fx));
        if (in0) a0 += (double)in0[e];
        if (in1) a1 += (double)in1[e];
        if (in2) a2 += (double)in2[e];
        ++c;
      }
    }
  }
  red[0][t] = a0;
  red[1][t] = a1;
  red[2][t] = a2;
  red[3][t] = (double)c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int k = 0; k < 4; ++k) red[k][t] += red[k][t + w];
    __syncthreads();
  }
  if (t == 0) {
    const int nb = gridDim.x;
    const size_t plane = (size_t)ns * nb, o = (size_t)s * nb + blockIdx.x;
    partial[o] = red[0][0];
    partial[plane + o] = red[1][0];
    partial[2 * plane + o] = red[2][0];
    pcount[o] = (int)red[3][0];
  }
}

// Sum over the row blocks of every shell (one block per shell, fixed strided
// assignment and fixed tree); mean: divide by the value at the origin of the
// input and by the count (correlation maps).
__global__ void __launch_bounds__(256) k_shell_sum(const double* __restrict__ partial, const int* __restrict__ pcount,
                                                   int nb, int ns, const float* __restrict__ in0,
                                                   const float* __restrict__ in1, const float* __restrict__ in2,
                                                   int mean, double* __restrict__ out) {
  __shared__ double red[4][256];
  const int s = blockIdx.x, t = threadIdx.x;
  const size_t plane = (size_t)ns * nb, base = (size_t)s * nb;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, c = 0.0;
  for (int j = t; j < nb; j += 256) {
    a0 += partial[base + j];
    a1 += partial[plane + base + j];
    a2 += partial[2 * plane + base + j];
    c += (double)pcount[base + j];
  }
  red[0][t] = a0;
  red[1][t] = a1;
  red[2][t] = a2;
  red[3][t] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int k = 0; k < 4; ++k) red[k][t] += red[k][t + w];
    __syncthreads();
  }
  if (t == 0) {
    double v0 = red[0][0], v1 = red[1][0], v2 = red[2][0];
    const double cnt = red[3][0];
    if (mean) {
      v0 = in0 ? v0 / ((double)in0[0] * cnt) : 0.0;
      v1 = in1 ? v1 / ((double)in1[0] * cnt) : 0.0;
      v2 = in2 ? v2 / ((double)in2[0] * cnt) : 0.0;
    }
    out[s] = v0;
    out[ns + s] = v1;
    out[2 * ns + s] = v2;
    out[3 * ns + s] = cnt;
  }
}

// W(s) = k_s^2 E(s) and L from E = out[0..ns), S = out[ns..2ns); writes W into
// out[2ns..3ns) and L into out[4ns].  One block, fixed tree.
__global__ void __launch_bounds__(256) k_finish_spectra(double* __restrict__ out, int n, int ns) {
  __shared__ double red[2][256];
  const int t = threadIdx.x;
  const double two_pi = 2.0 * 3.14159265358979323846, two_pi_n = two_pi / (double)n;
  double num = 0.0, den = 0.0;
  for (int s = t; s < ns; s += 256) {
    const double k = two_pi_n * s;
    out[2 * ns + s] = k * k * out[s];
    if (s > 0) {
      num += out[ns + s];
      den += k * out[ns + s];
    }
  }
  red[0][t] = num;
  red[1][t] = den;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      red[0][t] += red[0][t + w];
      red[1][t] += red[1][t + w];
    }
    __syncthreads();
  }
  if (t == 0) out[4 * ns] = two_pi * red[0][0] / red[1][0];
}

// out[k] = scale * sum over blocks b of partial[b * cols + k]: one block per
// column, fixed strided assignment and fixed tree.
__global__ void __launch_bounds__(256) k_column_sum(const double* __restrict__ partial, int nblk, int cols,
                                                    double scale, double* __restrict__ out) {
  __shared__ double red[256];
  const int k = blockIdx.x, t = threadIdx.x;
  double a = 0.0;
  for (int b = t; b < nblk; b += 256) a += partial[(size_t)b * cols + k];
  red[t] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) out[k] = red[0] * scale;
}

constexpr int kRedThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Per-block sums of the six temporal-correlation products.
__global__ void __launch_bounds__(kRedThreads) k_overlaps(const float* __restrict__ s0, const float* __restrict__ s1,
                                                          int n, double* __restrict__ partial) {
  __shared__ double red[kRedThreads / 64];
  const size_t n2 = (size_t)n * n;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int i = blockIdx.x * kRedThreads + threadIdx.x; i < n * n; i += gridDim.x * kRedThreads) {
    const int y = i / n, x = i - y * n;
    const float2 ua = mixed(s0, n2, i), ub = mixed(s1, n2, i);
    const float wa = vort(s0, n, y, x), wb = vort(s1, n, y, x);
    acc[0] += (double)ua.x * ub.x + (double)ua.y * ub.y;
    acc[1] += (double)ua.x * ua.x + (double)ua.y * ua.y;
    acc[2] += (double)wa * wb;
    acc[3] += (double)wa * wa;
    acc[4] += 2.0 * ((double)s0[n2 + i] * s1[n2 + i] + (double)s0[2 * n2 + i] * s1[2 * n2 + i]);
    acc[5] += 2.0 * ((double)s0[n2 + i] * s0[n2 + i] + (double)s0[2 * n2 + i] * s0[2 * n2 + i]);
  }
  for (int k = 0; k < 6; ++k) {
    const double t = block_sum(acc[k], red);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * 6 + k] = t;
  }
}


// +-1/2 defects by winding number around every plaquette (float32 decisions).
__device__ __forceinline__ float wrap_half(float d) {
  const float hp = 1.57079632679489662f, pi = 3.14159265358979324f;
  d = d >= hp ? d - pi : d;
  return d < -hp ? d + pi : d;
}

__global__ void __launch_bounds__(kRedThreads) k_defects(const float* __restrict__ s, int n,
                                                         double* __restrict__ partial) {
  __shared__ double red[kRedThreads / 64];
  const size_t n2 = (size_t)n * n;
  double plus = 0.0, minus = 0.0;  // integer counts carried exactly in doubles (< 2^53)
  for (int i = blockIdx.x * kRedThreads + threadIdx.x; i < n * n; i += gridDim.x * kRedThreads) {
    const int y = i / n, x = i - y * n;
    const int x1 = wrapn(x + 1, n), y1 = wrapn(y + 1, n);
    const int i10 = y * n + x1, i11 = y1 * n + x1, i01 = y1 * n + x;
    const float t00 = 0.5f * atan2f(s[2 * n2 + i], s[n2 + i]);
    const float t10 = 0.5f * atan2f(s[2 * n2 + i10], s[n2 + i10]);
    const float t11 = 0.5f * atan2f(s[2 * n2 + i11], s[n2 + i11]);
    const float t01 = 0.5f * atan2f(s[2 * n2 + i01], s[n2 + i01]);
    const float w = ((wrap_half(t10 - t00) + wrap_half(t11 - t10)) + wrap_half(t01 - t11)) + wrap_half(t00 - t01);
    if (w > 1.57079632679489662f) plus += 1.0;
    if (w < -1.57079632679489662f) minus += 1.0;
  }
  const double p = block_sum(plus, red);
  const double m = block_sum(minus, red);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = p;
    partial[2 * blockIdx.x + 1] = m;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_pack(const float* s, int n, float2* za, float2* zb, float2* zc, hipStream_t st) {
  const int n2 = n * n;
  hipLaunchKernelGGL(k_pack, dim3((n2 + 255) / 256), dim3(256), 0, st, s, n, za, zb, zc);
  return hipGetLastError();
}

hipError_t launch_twiddles(float2* tw, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_twiddles, dim3((n / 2 + 255) / 256), dim3(256), 0, st, tw, n);
  return hipGetLastError();
}

hipError_t launch_fft2t(float2* in, float2* out, int n, int logn, bool inverse, const float2* tw, hipStream_t st) {
  const size_t lds = (size_t)(n + (n >> 5) + n / 2) * sizeof(float2);
  const dim3 tg((n + 31) / 32, (n + 31) / 32), tb(32, 8);
  if (inverse) hipLaunchKernelGGL(k_fft_rows<true>, dim3(n), dim3(256), lds, st, in, tw, n, logn);
  else hipLaunchKernelGGL(k_fft_rows<false>, dim3(n), dim3(256), lds, st, in, tw, n, logn);
  hipLaunchKernelGGL(k_transpose, tg, tb, 0, st, in, out, n);
  if (inverse) hipLaunchKernelGGL(k_fft_rows<true>, dim3(n), dim3(256), lds, st, out, tw, n, logn);
  else hipLaunchKernelGGL(k_fft_rows<false>, dim3(n), dim3(256), lds, st, out, tw, n, logn);
  return hipGetLastError();
}

hipError_t launch_power(const float2* za, const float2* zb, const float2* zc, int n, float* pE, float* pS,
                        float2* w0, float2* w1, hipStream_t st) {
  const double n4 = (double)n * n * (double)n * n;
  const int n2 = n * n;
  hipLaunchKernelGGL(k_power, dim3((n2 + 255) / 256), dim3(256), 0, st, za, zb, zc, n, (float)(1.0 / n4), pE, pS,
                     w0, w1);
  return hipGetLastError();
}

hipError_t launch_shells(const float* in0, const float* in1, const float* in2, int stride, int n, int ns, bool mean,
                         double* partial, int* pcount, double* out, hipStream_t st) {
  const int nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_shell_part, dim3(nb, ns), dim3(256), 0, st, in0, in1, in2, stride, n, ns, partial,
                     pcount);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_shell_sum, dim3(ns), dim3(256), 0, st, partial, pcount, nb, ns, in0, in1, in2, mean ? 1 : 0,
                     out);
  return hipGetLastError();
}

hipError_t launch_finish_spectra(double* out, int n, int ns, hipStream_t st) {
  hipLaunchKernelGGL(k_finish_spectra, dim3(1), dim3(256), 0, st, out, n, ns);
  return hipGetLastError();
}

int reduce_blocks(int n) {
  const int b = (n * n + kRedThreads - 1) / kRedThreads;
  return b < 1024 ? b : 1024;
}

hipError_t launch_overlaps(const float* s0, const float* s1, int n, double* partial, double* out, hipStream_t st) {
  const int nblk = reduce_blocks(n);
  hipLaunchKernelGGL(k_overlaps, dim3(nblk), dim3(kRedThreads), 0, st, s0, s1, n, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_column_sum, dim3(6), dim3(256), 0, st, partial, nblk, 6, 1.0 / ((double)n * n), out);
  return hipGetLastError();
}

hipError_t launch_defects(const float* s, int n, double* partial, double* out, hipStream_t st) {
  const int nblk = reduce_blocks(n);
  hipLaunchKernelGGL(k_defects, dim3(nblk), dim3(kRedThreads), 0, st, s, n, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_column_sum, dim3(2), dim3(256), 0, st, partial, nblk, 2, 1.0, out);
  return hipGetLastError();
}

}  // namespace tana
