// gfx950 kernels of the convolutional surrogate: periodic 3x3 convolutions as
// implicit GEMMs on bf16 matrix cores (v_mfma_f32_16x16x16_bf16, fp32
// accumulation), their weight gradients, the loss, Adam and data packing.
//
// Activations are stored channels-last (NHWC) in bfloat16 so that one k-block of
// 16 channels of a site is contiguous; pre-activations kept for the backward pass
// are fp32.  MFMA operand layout (16x16x16): lane l holds A[l%16][4(l/16)+v],
// B[4(l/16)+v][l%16] and D[4(l/16)+v][l%16], v = 0..3.
#include "cnn_internal.h"

#include <algorithm>

namespace tcnn {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Round to nearest even (NaN kept quiet): the __bf16 conversion, which gfx950
// executes as v_cvt_pk_bf16_f32 (two values per instruction).
__device__ __forceinline__ bf16 to_bf16(float x) { return __builtin_bit_cast(bf16, (__bf16)x); }
__device__ __forceinline__ float from_bf16(bf16 h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// ---------------------------------------------------------------------------
// Convolution.  A block computes a 16 x 16 tile of sites for all CO output
// channels as an implicit GEMM with the weights as the left operand: M = CO
// (16 channels per M-tile), N = 256 sites (wave w owns tile rows 4w..4w+3, one
// 16-site N-tile each), K = 9 taps x CI channels in tap-major order, 32 per
// v_mfma_f32_16x16x32_bf16 (a K remainder of 16 takes the 16x16x16 form).  A
// dot product does not depend on which k-slot of the instruction carries which
// k, so lane group g (lanes 16g..16g+15) takes the 8 consecutive k of its slot
// range: one 16-byte LDS read per fragment, never straddling a tap (taps are
// multiples of 16 channels).  The result D[4g+v][l%16] gives each lane four
// consecutive channels of one site, stored as one 8-byte (bf16) or 16-byte
// (fp32) access.  The input tile with a halo of 1 and the weights are staged in
// LDS with strides of 8 extra bf16, so the 16-byte reads of 8 lanes at a time
// fall in distinct banks.
// ---------------------------------------------------------------------------
constexpr int kHalo = kTile + 2;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// silu(z) = z sigmoid(z) and its derivative factor sigmoid(z) (1 + z (1 - sigmoid(z)));
// the reciprocal is the hardware one (1 ulp), far below the bf16 rounding that follows.
__device__ __forceinline__ float fast_sigmoid(float z) { return __builtin_amdgcn_rcpf(1.f + __expf(-z)); }

// Input tile of 16 x 16 sites with its periodic halo: this thread's 8-byte pieces.
template <int CI, int KP>
__device__ __forceinline__ void load_patch(const bf16* __restrict__ in, int t, int H, int W, uint2 (&pv)[KP]) {
  constexpr int GP = CI / 4, NP = kHalo * kHalo * GP;
  const int tiles_x = W / kTile, tiles_img = tiles_x * (H / kTile);
  const int b = t / tiles_img, tt = t - b * tiles_img;
  const int y0 = (tt / tiles_x) * kTile, x0 = (tt % tiles_x) * kTile;
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int i = min((int)threadIdx.x + 256 * k, NP - 1);
    const int pix = i / GP, g = i - pix * GP;
    const int py = pix / kHalo, px = pix - py * kHalo;
    const int gy = wrap(y0 + py - 1, H), gx = wrap(x0 + px - 1, W);
    pv[k] = *reinterpret_cast<const uint2*>(in + (((size_t)b * H + gy) * W + gx) * CI + 4 * g);
  }
}

// Persistent blocks: a block stages the layer's weights once and walks the tiles
// t = blockIdx.x, blockIdx.x + gridDim.x, ...; the next tile's input is loaded
// into registers while the matrix cores work on the current one.
template <int CI, int CO, int MODE>
__global__ void __launch_bounds__(256, 2) k_conv(const bf16* __restrict__ in, const bf16* __restrict__ w,
                                              const float* __restrict__ bias, const float* __restrict__ z_below,
                                              bf16* __restrict__ out_bf, float* __restrict__ out_f, int B, int H,
                                              int W) {
  constexpr int PS = CI + 8, WS = 9 * CI + 8, NT = CO / 16;
  constexpr int KTOT = 9 * CI, NC = KTOT / 32, REM = KTOT - 32 * NC;
  static_assert(CI % 16 == 0 && CO % 16 == 0 && (REM == 0 || REM == 16), "k-blocks of 16 channels");
  __shared__ __attribute__((aligned(16))) bf16 patch[kHalo * kHalo * PS];
  __shared__ __attribute__((aligned(16))) bf16 wts[CO * WS];
  const int tiles_x = W / kTile, tiles_img = tiles_x * (H / kTile), tiles = B * tiles_img;
  int t = blockIdx.x;
  if (t >= tiles) return;  // whole block, before any barrier
  const int tid = threadIdx.x;
  constexpr int GP = CI / 4, NP = kHalo * kHalo * GP, KP = (NP + 255) / 256;
  constexpr int GW = 9 * CI / 4, NWT = CO * GW, KW = (NWT + 255) / 256;
  // stage the weights and the first tile; all loads are issued before the first
  // LDS write, so the block waits for one memory latency
  uint2 pv[KP];
  {
    uint2 wv[KW];
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      const int i = min(tid + 256 * k, NWT - 1);
      const int o = i / GW, g = i - o * GW;
      wv[k] = *reinterpret_cast<const uint2*>(w + (size_t)o * 9 * CI + 4 * g);
    }
    load_patch<CI, KP>(in, t, H, W, pv);
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      const int i = tid + 256 * k;
      if (i < NWT) {
        const int o = i / GW, g = i - o * GW;
        *reinterpret_cast<uint2*>(&wts[o * WS + 4 * g]) = wv[k];
      }
    }
  }
  const int lane = tid & 63, wave = tid >> 6, li = lane & 15, lg = lane >> 4;
  float bias_c[NT][4];
#pragma unroll
  for (int n = 0; n < NT; ++n)
#pragma unroll
    for (int v = 0; v < 4; ++v) bias_c[n][v] = (MODE == kSilu || MODE == kLinear) ? bias[n * 16 + 4 * lg + v] : 0.f;
  // LDS offset of the patch pixel under site (row 4 wave + m, column li) at tap (0, 0)
  const int site0 = (4 * wave) * kHalo + li;
  for (;;) {
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int i = tid + 256 * k;
      if (i < NP) {
        const int pix = i / GP, g = i - pix * GP;
        *reinterpret_cast<uint2*>(&patch[pix * PS + 4 * g]) = pv[k];
      }
    }
    __syncthreads();
    const int tn = t + (int)gridDim.x;
    if (tn < tiles) load_patch<CI, KP>(in, tn, H, W, pv);
    f32x4 acc[NT][4];
#pragma unroll
    for (int n = 0; n < NT; ++n)
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[n][m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int k0 = 32 * j + 8 * lg;
      const int tap = k0 / CI, c0 = k0 - tap * CI;
      const int dy = tap / 3, dx = tap - 3 * dy;
      bf16x8 wa[NT], pb[4];
#pragma unroll
      for (int n = 0; n < NT; ++n) wa[n] = *reinterpret_cast<const bf16x8*>(&wts[(n * 16 + li) * WS + k0]);
#pragma unroll
      for (int m = 0; m < 4; ++m)
        pb[m] = *reinterpret_cast<const bf16x8*>(&patch[(site0 + (m + dy) * kHalo + dx) * PS + c0]);
#pragma unroll
      for (int n = 0; n < NT; ++n)
#pragma unroll
        for (int m = 0; m < 4; ++m)
          acc[n][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[n], pb[m], acc[n][m], 0, 0, 0);
    }
    if constexpr (REM == 16) {
      const int k0 = 32 * NC + 4 * lg;
      const int tap = k0 / CI, c0 = k0 - tap * CI;
      const int dy = tap / 3, dx = tap - 3 * dy;
      bf16x4 wa[NT], pb[4];
#pragma unroll
      for (int n = 0; n < NT; ++n) wa[n] = *reinterpret_cast<const bf16x4*>(&wts[(n * 16 + li) * WS + k0]);
#pragma unroll
      for (int m = 0; m < 4; ++m)
        pb[m] = *reinterpret_cast<const bf16x4*>(&patch[(site0 + (m + dy) * kHalo + dx) * PS + c0]);
#pragma unroll
      for (int n = 0; n < NT; ++n)
#pragma unroll
        for (int m = 0; m < 4; ++m)
          acc[n][m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[n], pb[m], acc[n][m], 0, 0, 0);
    }
    // epilogue: D[4 lg + v][li] of acc[n][m] -> channel n * 16 + 4 lg + v of site (row 4 wave + m, x li)
    const int b = t / tiles_img, tt = t - b * tiles_img;
    const int y0 = (tt / tiles_x) * kTile, x0 = (tt % tiles_x) * kTile;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const size_t site = ((size_t)b * H + y0 + 4 * wave + m) * W + x0 + li;
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const size_t o = site * CO + n * 16 + 4 * lg;
        if (MODE == kSilu) {
          f32x4 z;
          bf16x4 a;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            z[v] = acc[n][m][v] + bias_c[n][v];
            a[v] = (short)to_bf16(z[v] * fast_sigmoid(z[v]));
          }
          if (out_f) *reinterpret_cast<f32x4*>(out_f + o) = z;
          *reinterpret_cast<bf16x4*>(out_bf + o) = a;
        } else if (MODE == kLinear) {
          f32x4 y;
#pragma unroll
          for (int v = 0; v < 4; ++v) y[v] = acc[n][m][v] + bias_c[n][v];
          *reinterpret_cast<f32x4*>(out_f + o) = y;
        } else {
          const f32x4 z = *reinterpret_cast<const f32x4*>(z_below + o);
          bf16x4 a;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float sg = fast_sigmoid(z[v]);
            a[v] = (short)to_bf16(acc[n][m][v] * (sg * (1.f + z[v] * (1.f - sg))));
          }
          *reinterpret_cast<bf16x4*>(out_bf + o) = a;
        }
      }
    }
    if (tn >= tiles) break;
    t = tn;
    __syncthreads();  // every wave is done with this tile's patch
  }
}

// ---------------------------------------------------------------------------
// Weight gradient gW[co][tap][ci] = sum over sites p of g[p][co] a[p + off(tap)][ci]:
// a GEMM with M = CO, N = 9 CI and K = sites.  A block walks a range of 16 x 16
// tiles; per tile g is staged transposed ([co][site]) and the input tile with
// its halo channel-major ([ci][y][x]), and each MFMA takes the 16 sites of one
// tile row as its k-block.  The 9 * CI / 16 N-tiles are dealt round-robin to the
// 4 waves.  Bias gradient: row sums of the staged g.
// ---------------------------------------------------------------------------
constexpr int kDwBlocks = 256;
constexpr int GS = kTile * kTile + 4;  // site stride of the transposed gradient tile
constexpr int AS = kHalo + 2;          // row stride of the channel-major input tile

template <int CI, int CO>
__global__ void __launch_bounds__(256) k_weight_grad(const bf16* __restrict__ g, const bf16* __restrict__ a,
                                                     float* __restrict__ partial, float* __restrict__ partial_b,
                                                     int B, int H, int W) {
  constexpr int MT = CO / 16, NTT = 9 * CI / 16, NW = (NTT + 3) / 4;
  __shared__ __attribute__((aligned(16))) bf16 gT[CO * GS];
  __shared__ __attribute__((aligned(16))) bf16 aT[CI * kHalo * AS];
  __shared__ float bsum[4][CO];
  const int tiles_x = W / kTile, tiles_y = H / kTile, tiles = B * tiles_x * tiles_y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lg = lane >> 4;
  f32x4 acc[MT][NW];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int j = 0; j < NW; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;  // thread (co = tid % CO, part = tid / CO) sums sites part*64 .. +63
  const int bco = tid % CO, bpart = tid / CO;
  // 8-byte pieces (4 channels) of the gradient tile and of the input tile with its halo
  constexpr int GG = CO / 4, NG = kTile * kTile * GG, KG = (NG + 255) / 256;
  constexpr int GA = CI / 4, NA = kHalo * kHalo * GA, KA = (NA + 255) / 256;
  for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int b = t / (tiles_x * tiles_y), r = t % (tiles_x * tiles_y);
    const int y0 = (r / tiles_x) * kTile, x0 = (r % tiles_x) * kTile;
    // all loads of the tile are issued before the first LDS write
    uint2 gv[KG], av[KA];
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      const int i = min(tid + 256 * k, NG - 1);
      const int s = i / GG, c4 = i - s * GG;
      gv[k] = *reinterpret_cast<const uint2*>(g + (((size_t)b * H + y0 + s / kTile) * W + x0 + s % kTile) * CO + 4 * c4);
    }
#pragma unroll
    for (int k = 0; k < KA; ++k) {
      const int i = min(tid + 256 * k, NA - 1);
      const int pix = i / GA, c4 = i - pix * GA;
      const int py = pix / kHalo, px = pix - py * kHalo;
      av[k] = *reinterpret_cast<const uint2*>(
          a + (((size_t)b * H + wrap(y0 + py - 1, H)) * W + wrap(x0 + px - 1, W)) * CI + 4 * c4);
    }
    __syncthreads();  // previous tile's reads are done
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      const int i = tid + 256 * k;
      if (i < NG) {
        const int s = i / GG, c = 4 * (i - s * GG);
        gT[c * GS + s] = (bf16)(gv[k].x & 0xffffu);
        gT[(c + 1) * GS + s] = (bf16)(gv[k].x >> 16);
        gT[(c + 2) * GS + s] = (bf16)(gv[k].y & 0xffffu);
        gT[(c + 3) * GS + s] = (bf16)(gv[k].y >> 16);
      }
    }
#pragma unroll
    for (int k = 0; k < KA; ++k) {
      const int i = tid + 256 * k;
      if (i < NA) {
        const int pix = i / GA, c = 4 * (i - pix * GA);
        const int py = pix / kHalo, px = pix - py * kHalo;
        aT[(c * kHalo + py) * AS + px] = (bf16)(av[k].x & 0xffffu);
        aT[((c + 1) * kHalo + py) * AS + px] = (bf16)(av[k].x >> 16);
        aT[((c + 2) * kHalo + py) * AS + px] = (bf16)(av[k].y & 0xffffu);
        aT[((c + 3) * kHalo + py) * AS + px] = (bf16)(av[k].y >> 16);
      }
    }
    __syncthreads();
    if (bpart < 4) {
      for (int s = bpart * 64; s < bpart * 64 + 64; ++s) bacc += from_bf16(gT[bco * GS + s]);
    }
#pragma unroll 1
    for (int row = 0; row < kTile; ++row) {
      bf16x4 af[MT];
#pragma unroll
      for (int m = 0; m < MT; ++m)  // A[i][k]: co = m * 16 + li, site = (row, 4 lg + v)
        af[m] = *reinterpret_cast<const bf16x4*>(&gT[(m * 16 + li) * GS + row * kTile + 4 * lg]);
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        const int nt = wave + 4 * j;
        if (nt < NTT) {
          const int tap = nt / (CI / 16), kc = nt - tap * (CI / 16);
          const int dy = tap / 3, dx = tap - 3 * dy;
          // B[k][j]: site (row, 4 lg + v) shifted by the tap, channel kc * 16 + li
          const bf16* src = &aT[((kc * 16 + li) * kHalo + row + dy) * AS + 4 * lg + dx];
          bf16x4 bf;
          bf[0] = (short)src[0];
          bf[1] = (short)src[1];
          bf[2] = (short)src[2];
          bf[3] = (short)src[3];
#pragma unroll
          for (int m = 0; m < MT; ++m)
            acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[m], bf, acc[m][j], 0, 0, 0);
        }
      }
    }
  }
  // D[4 lg + v][li]: co = m * 16 + 4 lg + v, column (tap, kc * 16 + li)
  float* out = partial + (size_t)blockIdx.x * CO * 9 * CI;
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const int nt = wave + 4 * j;
    if (nt < NTT) {
      const int tap = nt / (CI / 16), kc = nt - tap * (CI / 16);
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[((m * 16 + 4 * lg + v) * 9 + tap) * CI + kc * 16 + li] = acc[m][j][v];
    }
  }
  if (bpart < 4) bsum[bpart][bco] = bacc;
  __syncthreads();
  if (tid < CO) partial_b[(size_t)blockIdx.x * CO + tid] = (bsum[0][tid] + bsum[1][tid]) + (bsum[2][tid] + bsum[3][tid]);
}

// Sum of the block partials into the natural layout of the real channels.  A
// block takes 32 columns (weight columns [co][9][ci], then the co bias entries);
// eight thread groups each sum every eighth block partial in ascending order,
// and the eight sums meet in a fixed tree, so the result is deterministic.
__global__ void __launch_bounds__(256) k_weight_grad_reduce(const float* __restrict__ partial,
                                                            const float* __restrict__ partial_b, int nblk, int ci,
                                                            int co, int ci_real, int co_real, float* __restrict__ gW,
                                                            float* __restrict__ gb) {
  __shared__ float red[8][32];
  const int lane = threadIdx.x & 31, grp = threadIdx.x >> 5;
  const int ncol = co * 9 * ci, ntot = ncol + co;
  const int col = blockIdx.x * 32 + lane;
  float s = 0.f;
  if (col < ntot) {
    const bool wcol = col < ncol;
    const float* src = wcol ? partial + col : partial_b + (col - ncol);
    const size_t stride = wcol ? (size_t)ncol : (size_t)co;
    for (int k = grp; k < nblk; k += 8) s += src[(size_t)k * stride];
  }
  red[grp][lane] = s;
  __syncthreads();
  if (grp != 0 || col >= ntot) return;
  const float t = ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane])) +
                  ((red[4][lane] + red[5][lane]) + (red[6][lane] + red[7][lane]));
  if (col < ncol) {
    const int o = col / (9 * ci), rem = col - o * 9 * ci, tap = rem / ci, c = rem - tap * ci;
    if (o < co_real && c < ci_real) gW[(o * ci_real + c) * 9 + tap] = t;
  } else if (col - ncol < co_real) {
    gb[col - ncol] = t;
  }
}

// ---------------------------------------------------------------------------
// Packing, loss, prediction, Adam, weight layouts, comparison.
// ---------------------------------------------------------------------------
__global__ void k_pack(const float* __restrict__ x, int64_t stride, const int* __restrict__ idx,
                       const float* __restrict__ inv_scale, bf16* __restrict__ a0, int B, int H, int W) {
  const int64_t hw = (int64_t)H * W;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= B * hw) return;
  const int b = (int)(p / hw);
  const int64_t s = p - b * hw;
  const float* xs = x + (int64_t)idx[b] * stride;
  bf16 v[kPadIO];
#pragma unroll
  for (int c = 0; c < kPadIO; ++c) v[c] = c < kChannels ? to_bf16(xs[c * hw + s] * inv_scale[c]) : (bf16)0;
  uint4* dst = reinterpret_cast<uint4*>(a0 + p * kPadIO);
  dst[0] = make_uint4(v[0] | (unsigned)v[1] << 16, v[2] | (unsigned)v[3] << 16, v[4] | (unsigned)v[5] << 16,
                      v[6] | (unsigned)v[7] << 16);
  dst[1] = make_uint4(v[8] | (unsigned)v[9] << 16, v[10] | (unsigned)v[11] << 16, v[12] | (unsigned)v[13] << 16,
                      v[14] | (unsigned)v[15] << 16);
}

constexpr int kLossThreads = 256;
__global__ void __launch_bounds__(kLossThreads) k_loss(const float* __restrict__ y, const float* __restrict__ x,
                                                       const float* __restrict__ target, int64_t stride,
                                                       const int* __restrict__ idx, const float* __restrict__ inv_scale,
                                                       bf16* __restrict__ g, double* __restrict__ partial, int B, int H,
                                                       int W) {
  const int64_t hw = (int64_t)H * W;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float scale_g = (float)(2.0 / ((double)B * hw * kChannels));
  double acc = 0.0;
  if (p < B * hw) {
    const int b = (int)(p / hw);
    const int64_t s = p - b * hw;
    const float* xs = x + (int64_t)idx[b] * stride;
    const float* ts = target + (int64_t)idx[b] * stride;
    bf16 v[kPadIO];
#pragma unroll
    for (int c = 0; c < kPadIO; ++c) {
      if (c < kChannels) {
        const float d = y[p * kPadIO + c] - (ts[c * hw + s] - xs[c * hw + s]) * inv_scale[c];
        acc += (double)d * (double)d;
        v[c] = to_bf16(scale_g * d);
      } else {
        v[c] = 0;
      }
    }
    uint4* dst = reinterpret_cast<uint4*>(g + p * kPadIO);
    dst[0] = make_uint4(v[0] | (unsigned)v[1] << 16, v[2] | (unsigned)v[3] << 16, v[4] | (unsigned)v[5] << 16,
                        v[6] | (unsigned)v[7] << 16);
    dst[1] = make_uint4(v[8] | (unsigned)v[9] << 16, v[10] | (unsigned)v[11] << 16, v[12] | (unsigned)v[13] << 16,
                        v[14] | (unsigned)v[15] << 16);
  }
  // block sum in a fixed order
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  __shared__ double red[kLossThreads / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_sum_partials(const double* __restrict__ partial, int n, double scale, double* __restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) acc += partial[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (threadIdx.x == 0) *out = acc * scale;
}

__global__ void k_unpack(const float* __restrict__ y, const float* __restrict__ x, const float* __restrict__ scale,
                         float* __restrict__ out, int B, int H, int W) {
  const int64_t hw = (int64_t)H * W;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= B * hw) return;
  const int b = (int)(p / hw);
  const int64_t s = p - b * hw;
#pragma unroll
  for (int c = 0; c < kChannels; ++c) {
    const int64_t o = ((int64_t)b * kChannels + c) * hw + s;
    out[o] = x[o] + scale[c] * y[p * kPadIO + c];
  }
}

// omb1 = 1 - beta1 and omb2 = 1 - beta2 come rounded from their exact values
// (1 - 0.999f is 0.00099998713 in fp32, not 0.001).
__global__ void k_adam(float* __restrict__ theta, const float* __restrict__ grad, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float omb1, float b2, float omb2,
                       float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = grad[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void k_pack_weights(const float* __restrict__ Wt, const float* __restrict__ bt, int ci_real, int co_real,
                               int ci, int co, bf16* __restrict__ wf, bf16* __restrict__ wb, float* __restrict__ bias) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // over co * 9 * ci
  if (i < co) bias[i] = i < co_real ? bt[i] : 0.f;
  if (i >= co * 9 * ci) return;
  const int o = i / (9 * ci), rem = i - o * 9 * ci, tap = rem / ci, c = rem - tap * ci;
  const float val = (o < co_real && c < ci_real) ? Wt[((size_t)o * ci_real + c) * 9 + tap] : 0.f;
  const bf16 h = to_bf16(val);
  wf[i] = h;
  wb[((size_t)c * 9 + (8 - tap)) * co + o] = h;
}

constexpr int kCmpThreads = 256;
__global__ void __launch_bounds__(kCmpThreads) k_compare(const float* __restrict__ a, const float* __restrict__ b,
                                                         int64_t plane, int B, double* __restrict__ partial) {
  // partial[block][14]: per channel sum (a - b)^2, sum b^2
  double s[2 * kChannels];
#pragma unroll
  for (int k = 0; k < 2 * kChannels; ++k) s[k] = 0.0;
  const int64_t total = (int64_t)B * plane;
  for (int64_t p = (int64_t)blockIdx.x * kCmpThreads + threadIdx.x; p < total; p += (int64_t)gridDim.x * kCmpThreads) {
    const int bb = (int)(p / plane);
    const int64_t q = p - bb * plane;
#pragma unroll
    for (int c = 0; c < kChannels; ++c) {
      const int64_t o = ((int64_t)bb * kChannels + c) * plane + q;
      const double d = (double)a[o] - (double)b[o], r = (double)b[o];
      s[2 * c] += d * d;
      s[2 * c + 1] += r * r;
    }
  }
  __shared__ double red[kCmpThreads / 64][2 * kChannels];
#pragma unroll
  for (int k = 0; k < 2 * kChannels; ++k) {
    double v = s[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 2 * kChannels)
    partial[(size_t)blockIdx.x * 2 * kChannels + threadIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// out[k] = sum over blocks of partial[block][k]: one block per k, fixed strided
// assignment and fixed tree.
__global__ void __launch_bounds__(256) k_compare_final(const double* __restrict__ partial, int nblk,
                                                       double* __restrict__ out) {
  __shared__ double red[256];
  const int k = blockIdx.x, t = threadIdx.x;
  double a = 0.0;
  for (int i = t; i < nblk; i += 256) a += partial[(size_t)i * 2 * kChannels + k];
  red[t] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) out[k] = red[0];
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_conv(int ci, int co, ConvMode mode, const bf16* in, const bf16* w, const float* bias,
                       const float* z_below, bf16* out_bf, float* out_f, int B, int H, int W, hipStream_t st) {
  // two resident blocks per compute unit (the LDS of one block is about 80 KB)
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || cus <= 0)
      cus = 256;
  }
  const int tiles = B * (H / kTile) * (W / kTile);
  const dim3 grid((unsigned)std::min(tiles, 2 * cus)), blk(256);
#define TCNN_CONV(CI_, CO_, M_) \
  hipLaunchKernelGGL((k_conv<CI_, CO_, M_>), grid, blk, 0, st, in, w, bias, z_below, out_bf, out_f, B, H, W)
  if (ci == kPadIO && co == kHidden && mode == kSilu) TCNN_CONV(kPadIO, kHidden, kSilu);
  else if (ci == kHidden && co == kHidden && mode == kSilu) TCNN_CONV(kHidden, kHidden, kSilu);
  else if (ci == kHidden && co == kPadIO && mode == kLinear) TCNN_CONV(kHidden, kPadIO, kLinear);
  else if (ci == kHidden && co == kHidden && mode == kBackward) TCNN_CONV(kHidden, kHidden, kBackward);
  else if (ci == kPadIO && co == kHidden && mode == kBackward) TCNN_CONV(kPadIO, kHidden, kBackward);
  else return hipErrorInvalidValue;
#undef TCNN_CONV
  return hipGetLastError();
}

int dw_blocks(int B, int H, int W) {
  const int tiles = B * (H / kTile) * (W / kTile);
  return tiles < kDwBlocks ? tiles : kDwBlocks;
}

hipError_t launch_weight_grad(int ci, int co, int ci_real, int co_real, const bf16* g, const bf16* a,
                              float* partial, float* partial_b, float* gW, float* gb, int B, int H, int W,
                              hipStream_t st) {
  const int nblk = dw_blocks(B, H, W);
  if (ci == kPadIO && co == kHidden)
    hipLaunchKernelGGL((k_weight_grad<kPadIO, kHidden>), dim3(nblk), dim3(256), 0, st, g, a, partial, partial_b, B, H, W);
  else if (ci == kHidden && co == kHidden)
    hipLaunchKernelGGL((k_weight_grad<kHidden, kHidden>), dim3(nblk), dim3(256), 0, st, g, a, partial, partial_b, B, H, W);
  else if (ci == kHidden && co == kPadIO)
    hipLaunchKernelGGL((k_weight_grad<kHidden, kPadIO>), dim3(nblk), dim3(256), 0, st, g, a, partial, partial_b, B, H, W);
  else
    return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = co * 9 * ci + co;  // padded weight columns, then the bias
  hipLaunchKernelGGL(k_weight_grad_reduce, dim3((n + 31) / 32), dim3(256), 0, st, partial, partial_b, nblk, ci, co,
                     ci_real, co_real, gW, gb);
  return hipGetLastError();
}

hipError_t launch_pack(const float* x, int64_t sample_stride, const int* idx, const float* inv_scale, bf16* a0,
                       int B, int H, int W, hipStream_t st) {
  const int64_t n = (int64_t)B * H * W;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, sample_stride, idx, inv_scale, a0,
                     B, H, W);
  return hipGetLastError();
}

int loss_blocks(int B, int H, int W) { return (int)(((int64_t)B * H * W + kLossThreads - 1) / kLossThreads); }

hipError_t launch_loss(const float* y, const float* x, const float* target, int64_t sample_stride, const int* idx,
                       const float* inv_scale, bf16* g, double* partial, double* loss, int B, int H, int W,
                       hipStream_t st) {
  const int nblk = loss_blocks(B, H, W);
  hipLaunchKernelGGL(k_loss, dim3(nblk), dim3(kLossThreads), 0, st, y, x, target, sample_stride, idx, inv_scale, g,
                     partial, B, H, W);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, st, partial, nblk, 1.0 / ((double)B * H * W * kChannels),
                     loss);
  return hipGetLastError();
}

hipError_t launch_unpack(const float* y, const float* x, const float* scale, float* out, int B, int H, int W,
                         hipStream_t st) {
  const int64_t n = (int64_t)B * H * W;
  hipLaunchKernelGGL(k_unpack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, y, x, scale, out, B, H, W);
  return hipGetLastError();
}

hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, int64_t n, float lr, double beta1,
                       double beta2, float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, theta, grad, m, v, n, lr,
                     (float)beta1, (float)(1.0 - beta1), (float)beta2, (float)(1.0 - beta2), eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_pack_weights(const float* W, const float* b, int ci_real, int co_real, int ci, int co, bf16* wf,
                               bf16* wb, float* bias, hipStream_t st) {
  const int n = co * 9 * ci;
  hipLaunchKernelGGL(k_pack_weights, dim3((n + 255) / 256), dim3(256), 0, st, W, b, ci_real, co_real, ci, co, wf, wb,
                     bias);
  return hipGetLastError();
}

int compare_blocks(int64_t plane, int B) {
  const int64_t n = (plane * B + kCmpThreads - 1) / kCmpThreads;
  return (int)(n < 1024 ? n : 1024);
}

hipError_t launch_compare(const float* a, const float* b, int64_t plane, int B, double* partial, double* out,
                          hipStream_t st) {
  const int nblk = compare_blocks(plane, B);
  hipLaunchKernelGGL(k_compare, dim3(nblk), dim3(kCmpThreads), 0, st, a, b, plane, B, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_compare_final, dim3(2 * kChannels), dim3(256), 0, st, partial, nblk, out);
  return hipGetLastError();
}

}  // namespace tcnn
