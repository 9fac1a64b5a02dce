// gfx950 kernels of the two-fluid active-nematic coupled step (arXiv 2511.00445,
// Model and Numerical Simulation sections).
//
// Storage: structure-of-arrays float32 planes [ny][nx], x fastest.  Populations
// are stored after collision and before streaming ("post-collision"), shifted by
// -w_i rho0 so that the small deviations from rest keep float32 precision; the
// next step streams them by pulling f_i(x) = f*_i(x - c_i).
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_ext.h>

#include <algorithm>

#include "tfan_internal.h"

namespace tfan {
namespace {

// D2Q9 velocities and weights (order: rest, +x, +y, -x, -y, +x+y, -x+y, -x-y, +x-y).
constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr float WT[9] = {4.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f,
                         1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};

// Population storage: float32, or IEEE binary16 of the same shifted values
// (arithmetic is float32 either way; the conversion rounds to nearest even).
// Populations are pulled with a non-temporal hint as well: each value is read by
// one site, and keeping the population stream out of the caches leaves phi, Q
// and the velocities resident (measured at 2048^2, float32: collision and
// sub-steps both 3.5% shorter; binary16: collision 3% shorter).
template <typename PT> __device__ __forceinline__ float pop_ld(const void* f, size_t i) {
  if constexpr (sizeof(PT) == 4) return __builtin_nontemporal_load(static_cast<const float*>(f) + i);
  else return (float)static_cast<const PT*>(f)[i];
}
// Populations are written with a non-temporal hint: they are not read again
// until the next step, and keeping them out of the caches leaves phi, Q and the
// frozen velocities resident for the sub-step passes that follow.
template <typename PT> __device__ __forceinline__ void pop_st(void* f, size_t i, float v) {
  __builtin_nontemporal_store((PT)v, static_cast<PT*>(f) + i);
}
// Element (fluid fl, direction i, site) of one population set, [9][n][2]: the two
// fluids of one direction and site side by side, so that a pull or a store of
// both fluids is one 8-byte (float32) or 4-byte (binary16) access, half the
// memory instructions of separate planes (collision at 2048^2: float32 127 ->
// 122 us, binary16 85 -> 82 us).
template <typename PT> __device__ __forceinline__ size_t pop_index(int fl, int i, size_t n, size_t site) {
  return (((size_t)i * n + site) << 1) + (size_t)fl;
}
typedef float f32x2_t __attribute__((ext_vector_type(2)));
// Both fluids' populations of direction i at a site.
template <typename PT>
__device__ __forceinline__ void pop_ld2(const void* f, int i, size_t n, size_t site, float& a, float& p) {
  if constexpr (sizeof(PT) == 4) {
    const f32x2_t v = __builtin_nontemporal_load(static_cast<const f32x2_t*>(f) + (size_t)i * n + site);
    a = v.x;
    p = v.y;
  } else {
    const unsigned v = __builtin_nontemporal_load(static_cast<const unsigned*>(f) + (size_t)i * n + site);
    a = (float)__builtin_bit_cast(_Float16, (unsigned short)(v & 0xffffu));
    p = (float)__builtin_bit_cast(_Float16, (unsigned short)(v >> 16));
  }
}
template <typename PT>
__device__ __forceinline__ void pop_st2(void* f, int i, size_t n, size_t site, float a, float p) {
  if constexpr (sizeof(PT) == 4) {
    f32x2_t v;
    v.x = a;
    v.y = p;
    __builtin_nontemporal_store(v, static_cast<f32x2_t*>(f) + (size_t)i * n + site);
  } else {
    const unsigned lo = __builtin_bit_cast(unsigned short, (_Float16)a);
    const unsigned hi = __builtin_bit_cast(unsigned short, (_Float16)p);
    __builtin_nontemporal_store(lo | (hi << 16), static_cast<unsigned*>(f) + (size_t)i * n + site);
  }
}

// Periodic index for offsets |d| <= n.
__device__ __forceinline__ int wrapi(int i, int n) {
  i = (i < 0) ? i + n : i;
  return (i >= n) ? i - n : i;
}

// Chemical potential mu = A (phi^3 - phi) - kappa lap(phi) at a point, given phi
// at the point and its four neighbours (Model, Eq. 2, order-parameter form).
__device__ __forceinline__ float chem_pot(float p, float pe, float pw, float pn, float ps,
                                          const DevParams& P) {
  return P.A_ch * (p * p * p - p) - P.kappa * ((pe + pw) + (pn + ps) - 4.f * p);
}

// Nematic stress at a point: Beris-Edwards elastic stress (Model, elastic stress
// display) plus the active stress -zeta c1 Q.  In two dimensions
// -lam (H.P + P.H) + 2 lam P (Q:H) = -lam H + 2 lam (Q:H) Q (P = Q + I/2), so the
// symmetric part is traceless apart from the Ericksen term.  Returned as
// sigma_xx, sigma_yy, the symmetric off-diagonal s and the antisymmetric a
// (sigma_xy = s + a, sigma_yx = s - a, a = (Q.H - H.Q)_xy).
struct Stress {
  float xx, yy, s, a;
};

__device__ __forceinline__ Stress nematic_stress(float qxx, float qxy, float qxxE, float qxyE,
                                                 float qxxW, float qxyW, float qxxN, float qxyN,
                                                 float qxxS, float qxyS, float c1,
                                                 const DevParams& P) {
  // molecular field H = -(A + (C/2) TrQ^2) Q + K lap Q (Model, Eqs. 7-8)
  const float lxx = (qxxE + qxxW) + (qxxN + qxxS) - 4.f * qxx;
  const float lxy = (qxyE + qxyW) + (qxyN + qxyS) - 4.f * qxy;
  const float b = P.A_ldg + P.halfC * (2.f * (qxx * qxx + qxy * qxy));
  const float hxx = P.K * lxx - b * qxx;
  const float hxy = P.K * lxy - b * qxy;
  const float qh = 2.f * (qxx * hxx + qxy * hxy);  // Q:H
  // central-difference gradients of Q
  const float axx = 0.5f * (qxxE - qxxW), bxx = 0.5f * (qxxN - qxxS);
  const float axy = 0.5f * (qxyE - qxyW), bxy = 0.5f * (qxyN - qxyS);
  const float twoK = 2.f * P.K;  // Ericksen: -K sum_kl d_i Q_kl d_j Q_kl
  const float lamxx = P.lam * (2.f * qh * qxx - hxx);
  const float lamxy = P.lam * (2.f * qh * qxy - hxy);
  const float zc = P.zeta * c1;
  Stress st;
  st.xx = lamxx - twoK * (axx * axx + axy * axy) - zc * qxx;
  st.yy = -lamxx - twoK * (bxx * bxx + bxy * bxy) + zc * qxx;
  st.s = lamxy - twoK * (axx * bxx + axy * bxy) - zc * qxy;
  st.a = 2.f * (qxx * hxy - qxy * hxx);
  return st;
}

// BGK collision with the Guo source for one fluid, written post-collision:
// f* = f + (f^eq - f)/tau + (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F,
// all populations shifted by -w_i rho0.
// The populations f are replaced by their post-collision values.
__device__ __forceinline__ void collide_fluid(float f[9], float dr, float ux, float uy, float Fx, float Fy,
                                              float om, float gk, float rho0) {
  const float rho = rho0 + dr;
  const float uu15 = 1.5f * (ux * ux + uy * uy);
  const float uF = ux * Fx + uy * Fy;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float cu = (float)CX[i] * ux + (float)CY[i] * uy;
    const float cF = (float)CX[i] * Fx + (float)CY[i] * Fy;
    const float feq = WT[i] * (dr + rho * (cu * (3.f + 4.5f * cu) - uu15));
    const float src = gk * WT[i] * (3.f * (cF - uF) + 9.f * cu * cF);
    f[i] = f[i] + om * (feq - f[i]) + src;
  }
}

// Stencil inputs of one site's update: the stress components, mu and phi at the
// four neighbours (E, W: x +- 1; N, S: y +- 1) and phi, mu at the site.
struct SiteStencil {
  float xxE, xxW, yyN, yyS, sE, sW, sN, sS, aE, aW, aN, aS, muE, muW, muN, muS, phi;
  float mu, phE, phW, phN, phS;
};

// Forces, Guo velocities with the drag implicit, and (COLLIDE) both collisions of
// one site, with fa, fp its pulled populations (replaced by post-collision values).
// uo receives (u_a,x, u_a,y, u_c,x, u_c,y) when colliding, else the density
// deviations and velocities (rho_a - rho0, rho_p - rho0, u_a,x, u_a,y, u_p,x, u_p,y).
// Non-drag forces on the two fluids at one site (the drag is implicit in the
// velocity solve) and the volume fractions c1 = (1 + phi)/2, c2 = (1 - phi)/2.
struct SiteForce {
  float ax, ay, px, py, c1, c2;
};
__device__ __forceinline__ SiteForce site_forces(const SiteStencil& t) {
  // F_i = d_j sigma_ij with sigma_xy = s + a, sigma_yx = s - a
  const float Fx = 0.5f * (t.xxE - t.xxW) + 0.5f * ((t.sN + t.aN) - (t.sS + t.aS));
  const float Fy = 0.5f * ((t.sE - t.aE) - (t.sW - t.aW)) + 0.5f * (t.yyN - t.yyS);
  const float pC = t.phi;
  const float c1 = 0.5f * (1.f + pC), c2 = 0.5f * (1.f - pC);
  // capillary force mu grad(phi) - grad(phi mu) with both gradients by central
  // differences (Model, capillary force), shared c1 : c2.  Term by term,
  // mu_C (phi_E - phi_W)/2 - (phi_E mu_E - phi_W mu_W)/2
  //   = (phi_E (mu_C - mu_E) - phi_W (mu_C - mu_W)) / 2,
  // the form evaluated here (the same value, fewer roundings).
  const float fchx = 0.5f * (t.phE * (t.mu - t.muE) - t.phW * (t.mu - t.muW));
  const float fchy = 0.5f * (t.phN * (t.mu - t.muN) - t.phS * (t.mu - t.muS));
  return SiteForce{Fx + c1 * fchx, Fy + c1 * fchy, c2 * fchx, c2 * fchy, c1, c2};
}

template <bool COLLIDE>
__device__ __forceinline__ void site_update(const DevParams& P, float fa[9], float fp[9], const SiteStencil& t,
                                            float uo[6]) {
  const SiteForce G = site_forces(t);
  const float c1 = G.c1, c2 = G.c2;
  const float Gax = G.ax, Gay = G.ay, Gpx = G.px, Gpy = G.py;
  float dra = 0.f, mxa = 0.f, mya = 0.f, drp = 0.f, mxp = 0.f, myp = 0.f;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    dra += fa[i];
    drp += fp[i];
    if (CX[i] != 0) { mxa += CX[i] * fa[i]; mxp += CX[i] * fp[i]; }
    if (CY[i] != 0) { mya += CY[i] * fa[i]; myp += CY[i] * fp[i]; }
  }
  const float rho_a = P.rho0 + dra, rho_p = P.rho0 + drp;
  // per component [[rho_a + g, -g], [-g, rho_p + g]] [u_a; u_p] = [m_a + G_a/2; m_p + G_p/2]
  const float g = 0.5f * P.gamma * c1 * c2;
  const float inv = 1.f / (rho_a * rho_p + g * (rho_a + rho_p));
  const float bax = mxa + 0.5f * Gax, bay = mya + 0.5f * Gay;
  const float bpx = mxp + 0.5f * Gpx, bpy = myp + 0.5f * Gpy;
  const float uax = ((rho_p + g) * bax + g * bpx) * inv;
  const float uay = ((rho_p + g) * bay + g * bpy) * inv;
  const float upx = (g * bax + (rho_a + g) * bpx) * inv;
  const float upy = (g * bay + (rho_a + g) * bpy) * inv;
  if (!COLLIDE) {
    uo[0] = dra;  // density deviations: rho0 is added in float64 by the reader
    uo[1] = drp;
    uo[2] = uax;
    uo[3] = uay;
    uo[4] = upx;
    uo[5] = upy;
  } else {
    const float fdx = 2.f * g * (upx - uax), fdy = 2.f * g * (upy - uay);
    collide_fluid(fa, dra, uax, uay, Gax + fdx, Gay + fdy, P.om_a, P.gk_a, P.rho0);
    collide_fluid(fp, drp, upx, upy, Gpx - fdx, Gpy - fdy, P.om_p, P.gk_p, P.rho0);
    uo[0] = uax;
    uo[1] = uay;
    uo[2] = c1 * uax + c2 * upx;
    uo[3] = c1 * uay + c2 * upy;
  }
}

// ---------------------------------------------------------------------------
// Collision kernel.  A block owns a tile of CollideTile<PT>::X x (ROWS * SITES)
// sites, SITES rows per thread.  phi and Q are staged with a halo of 2; mu and the nematic stress are
// evaluated once per site on the tile plus a halo of 1 and shared through LDS;
// a thread's staging loads and its 36 population pulls are all in flight before
// its first LDS write, so the pulls' latency hides behind the staging and the
// stress evaluation.  FIELDS = true evaluates the same velocities and densities and
// writes them out instead of colliding (get_fields / diagnostics).
// ---------------------------------------------------------------------------
//
// Tile shape per population type, measured at 2048^2 (two rows per thread).
// Pulls are non-temporal, so a cache line that x-shifted pulls share across a
// tile edge is fetched again by the neighbouring tile: float32 wants wide tiles
// (256 x 4 with 512 threads: 122 us; 128 x 4 with 256: 123 us; before the paired
// fluids, 64 x 8: 137 us).  Binary16: 128 x 4 with 256 threads (77 us; 64 x 8:
// 79 us; 256 x 4 with 512 threads: 85 us).
// NW (narrow): tiles of half that width with half the threads, for the autotuner.
// NT > 0: blocks of NT threads on 256-site-wide tiles (the persistent batch kernel).
template <typename PT, bool NW = false, int NT = 0> struct CollideTile {
  static constexpr bool F32 = sizeof(PT) == 4;
  static constexpr int X = NT ? 256 : (F32 ? 256 : 128) >> (NW ? 1 : 0), THREADS = NT ? NT : 2 * X;
  static constexpr int ROWS = THREADS / X;          // rows per pass of the block
  static constexpr int PX = X + 4, SX = X + 2;      // phi/Q staging halo 2, mu/stress halo 1
  // LDS of a tile of SITES rows per thread: phi, Qxx, Qxy with halo 2; mu and four
  // stress components with halo 1
  template <int SITES> static constexpr int lds_bytes() {
    return 4 * (3 * (ROWS * SITES + 4) * PX + 5 * (ROWS * SITES + 2) * SX);
  }
};

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Launching 8 * ceil(tiles / 8) workgroups and giving XCD k the contiguous tile
// range [k * per, (k + 1) * per) keeps spatial neighbours (which share the
// cache lines of their halos and of the shifted population pulls) in one L2.
// Returns the row-major tile index of this workgroup, or -1 for a spare one.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int tiles) {
  const int per = (tiles + kXcds - 1) / kXcds;
  const int t = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
  return t < tiles ? t : -1;
}
inline unsigned xcd_grid(int tiles) { return (unsigned)(kXcds * ((tiles + kXcds - 1) / kXcds)); }

// Periodic index for any offset (tiles of small grids wrap more than once).
__device__ __forceinline__ int wrap_any(int i, int n) {
  while (i < 0) i += n;
  while (i >= n) i -= n;
  return i;
}


// Raw buffer access to one float32 plane of n elements: a scalar resource plus
// a 32-bit byte offset per lane, so planes indexed alike share one offset
// register and small constant offsets fold into the instruction.
using Plane = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Plane plane(const float* p, int n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, n * 4, 0x00020000);
}
__device__ __forceinline__ float ldg(Plane r, unsigned idx) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, idx * 4u, 0, 0));
}
__device__ __forceinline__ void stg(Plane r, unsigned idx, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, idx * 4u, 0, 0);
}

// One forward-Euler Beris-Edwards update of (Qxx, Qxy) (Model, Eqs. 11-12) at a
// site: Q += h Proj[ -u_a.grad Q + S(W, Q) + Gamma H ], W_ij = d_j u_a,i by central
// differences of the four neighbouring velocities.  The symmetric traceless part
// of S(W, Q) in two dimensions is lam E_dev + lam tr(W) Q - 2 lam (Q:E) Q +
// (Om.Q - Q.Om).  With g_ij = 2 W_ij (the undivided differences):
// 4 E_dev = (g_xx - g_yy, g_xy + g_yx), 2 tr W = g_xx + g_yy, 4 Om_xy = g_xy - g_yx,
// and S_xx = lam E_xx + G Q_xx + 2 Om_xy Q_xy, S_xy = lam E_xy + G Q_xy - 2 Om_xy Q_xx
// with G = lam (tr W - 2 Q:E) (Q:E = 2 (Q_xx E_xx + Q_xy E_xy)).
__device__ __forceinline__ float2 be_update(float2 q, float2 qe, float2 qw, float2 qn, float2 qs, float2 u,
                                            float2 ue, float2 uw, float2 un, float2 us, float h,
                                            const DevParams& P) {
  const float gxx = ue.x - uw.x, gxy = un.x - us.x, gyx = ue.y - uw.y, gyy = un.y - us.y;
  const float exx4 = gxx - gyy, exy4 = gxy + gyx, tr2 = gxx + gyy, om2 = 0.5f * (gxy - gyx);
  const float b = P.A_ldg + (2.f * P.halfC) * (q.x * q.x + q.y * q.y);
  const float hxx = P.K * (((qe.x + qw.x) + (qn.x + qs.x)) - 4.f * q.x) - b * q.x;
  const float hxy = P.K * (((qe.y + qw.y) + (qn.y + qs.y)) - 4.f * q.y) - b * q.y;
  const float g = P.lam * (0.5f * tr2 - (q.x * exx4 + q.y * exy4));
  const float lq = 0.25f * P.lam;
  const float sxx = lq * exx4 + g * q.x + om2 * q.y;
  const float sxy = lq * exy4 + g * q.y - om2 * q.x;
  // twice the advection u_a . grad Q
  const float ax = u.x * (qe.x - qw.x) + u.y * (qn.x - qs.x);
  const float ay = u.x * (qe.y - qw.y) + u.y * (qn.y - qs.y);
  return make_float2(q.x + h * ((sxx + P.Gamma * hxx) - 0.5f * ax), q.y + h * ((sxy + P.Gamma * hxy) - 0.5f * ay));
}

// Tiles of the collision kernel: X x (ROWS * SITES) sites, SITES rows per thread.
template <typename PT, int SITES, bool NW = false, int NT = 0>
__host__ __device__ inline int collide_tiles(int nx, int ny) {
  using T = CollideTile<PT, NW, NT>;
  return ((nx + T::X - 1) / T::X) * ((ny + T::ROWS * SITES - 1) / (T::ROWS * SITES));
}

// lds: CollideTile<PT, NW, NT>::lds_bytes<CT_SITES>() bytes of the caller's shared memory.
template <bool FIELDS, typename PT, int CT_SITES, bool NW = false, int NT = 0>
__device__ __forceinline__ void collide_tile(const DevParams& P, const DevState& in, void* __restrict__ fout,
                                             float* __restrict__ uout, int tile, unsigned char* __restrict__ lds) {
  using T = CollideTile<PT, NW, NT>;
  constexpr int CT_X = T::X, CT_THREADS = T::THREADS, CT_ROWS_PER_PASS = T::ROWS, PX = T::PX, SX = T::SX;
  constexpr int CT_Y = CT_ROWS_PER_PASS * CT_SITES, PY = CT_Y + 4, SY = CT_Y + 2;
  using PRow = float[PX];
  using SRow = float[SX];
  PRow* sph = reinterpret_cast<PRow*>(lds);
  PRow* sqx = sph + PY;
  PRow* sqy = sqx + PY;
  SRow* smu = reinterpret_cast<SRow*>(sqy + PY);
  SRow* sxx = smu + SY;
  SRow* syy = sxx + SY;
  SRow* ssy = syy + SY;
  SRow* san = ssy + SY;
  const int nx = P.nx, ny = P.ny, n = P.n;
  const int gx = (nx + CT_X - 1) / CT_X;
  const int tx = threadIdx.x % CT_X, ty = threadIdx.x / CT_X;
  const int x0 = (tile % gx) * CT_X, y0 = (tile / gx) * CT_Y;

  // 1. phi, Qxx, Qxy of the tile with a halo of 2, loaded first: the LDS writes in
  //    step 3 then wait for these loads only, and the population pulls issued in
  //    step 2 stay in flight through the stress evaluation
  constexpr int NS = PX * PY, KS = (NS + CT_THREADS - 1) / CT_THREADS;
  float sv[KS][3];
  {
    const bool one_wrap = nx > CT_X && ny > PY;  // halo offsets need at most one periodic shift
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int c = min((int)threadIdx.x + k * CT_THREADS, NS - 1);
      const int cy = c / PX, cx = c - cy * PX;
      const int gy = y0 - 2 + cy, gxx = x0 - 2 + cx;
      const int g = (one_wrap ? wrapi(gy, ny) : wrap_any(gy, ny)) * nx +
                    (one_wrap ? wrapi(gxx, nx) : wrap_any(gxx, nx));
      sv[k][0] = in.phi[g];
      sv[k][1] = in.q[g];
      sv[k][2] = in.q[n + g];
    }
  }
  // 2. pull both population sets of this thread's sites: f_i(x) = f*_i(x - c_i)
  float fa[CT_SITES][9], fp[CT_SITES][9];
  const int x = x0 + tx;
  const bool xin = x < nx;
  const int xc = xin ? x : 0;
  const int xm1 = wrapi(xc - 1, nx), xp1 = wrapi(xc + 1, nx);
#pragma unroll
  for (int s = 0; s < CT_SITES; ++s) {
    const int y = y0 + ty + CT_ROWS_PER_PASS * s;
    const int yc = (y < ny) ? y : 0;
    const int r0 = yc * nx, rm1 = wrapi(yc - 1, ny) * nx, rp1 = wrapi(yc + 1, ny) * nx;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int sx = (CX[i] == 0) ? xc : (CX[i] > 0 ? xm1 : xp1);
      const int sy = (CY[i] == 0) ? r0 : (CY[i] > 0 ? rm1 : rp1);
      pop_ld2<PT>(in.f, i, (size_t)n, (size_t)(sy + sx), fa[s][i], fp[s][i]);
    }
  }
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int c = (int)threadIdx.x + k * CT_THREADS;
    if (c < NS) {
      const int cy = c / PX, cx = c - cy * PX;
      sph[cy][cx] = sv[k][0];
      sqx[cy][cx] = sv[k][1];
      sqy[cy][cx] = sv[k][2];
    }
  }
  __syncthreads();
  // 3. chemical potential and nematic stress on the tile plus a halo of 1
  for (int c = threadIdx.x; c < SX * SY; c += CT_THREADS) {
    const int sy = c / SX, sx = c - sy * SX;
    const int py = sy + 1, px = sx + 1;
    const float p = sph[py][px];
    smu[sy][sx] = chem_pot(p, sph[py][px + 1], sph[py][px - 1], sph[py + 1][px], sph[py - 1][px], P);
    const Stress st = nematic_stress(sqx[py][px], sqy[py][px], sqx[py][px + 1], sqy[py][px + 1],
                                     sqx[py][px - 1], sqy[py][px - 1], sqx[py + 1][px], sqy[py + 1][px],
                                     sqx[py - 1][px], sqy[py - 1][px], 0.5f * (1.f + p), P);
    sxx[sy][sx] = st.xx;
    syy[sy][sx] = st.yy;
    ssy[sy][sx] = st.s;
    san[sy][sx] = st.a;
  }
  __syncthreads();
  // 4. forces, Guo velocities with implicit drag, collision (or field output)
#pragma unroll
  for (int s = 0; s < CT_SITES; ++s) {
    const int ly = ty + CT_ROWS_PER_PASS * s;
    const int y = y0 + ly;
    if (!xin || y >= ny) continue;
    const int sy = ly + 1, sx = tx + 1;
    const SiteStencil t = {sxx[sy][sx + 1], sxx[sy][sx - 1], syy[sy + 1][sx], syy[sy - 1][sx],
                           ssy[sy][sx + 1], ssy[sy][sx - 1], ssy[sy + 1][sx], ssy[sy - 1][sx],
                           san[sy][sx + 1], san[sy][sx - 1], san[sy + 1][sx], san[sy - 1][sx],
                           smu[sy][sx + 1], smu[sy][sx - 1], smu[sy + 1][sx], smu[sy - 1][sx],
                           sph[ly + 2][tx + 2], smu[sy][sx],
                           sph[ly + 2][tx + 3], sph[ly + 2][tx + 1], sph[ly + 3][tx + 2], sph[ly + 1][tx + 2]};
    float uo[6];
    site_update<!FIELDS>(P, fa[s], fp[s], t, uo);
    const int idx = y * nx + x;
    if (FIELDS) {
#pragma unroll
      for (int c = 0; c < 6; ++c) uout[c * n + idx] = uo[c];
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        pop_st2<PT>(fout, i, (size_t)n, (size_t)idx, fa[s][i], fp[s][i]);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) uout[c * n + idx] = uo[c];
    }
  }
}

template <bool FIELDS, typename PT, int SITES, bool NW>
__global__ void __launch_bounds__((CollideTile<PT, NW>::THREADS)) k_collide(DevParams P, DevState in,
                                                                            void* __restrict__ fout,
                                                                            float* __restrict__ uout) {
  __shared__ __align__(16) unsigned char lds[CollideTile<PT, NW>::template lds_bytes<SITES>()];
  const int tile = xcd_tile(collide_tiles<PT, SITES, NW>(P.nx, P.ny));
  if (tile < 0) return;  // whole workgroup, before any barrier
  collide_tile<FIELDS, PT, SITES, NW>(P, in, fout, uout, tile, lds);
}

// Member of a batch whose tile index range starts at `first` (ascending array).
__device__ __forceinline__ int batch_member(const int* __restrict__ first, int count, int tile) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename PT, int SITES, bool NW>
__global__ void __launch_bounds__((CollideTile<PT, NW>::THREADS)) k_collide_batch(const BatchMember* __restrict__ mem,
                                                                    const int* __restrict__ first, int count,
                                                                    int tiles, int cur) {
  __shared__ __align__(16) unsigned char lds[CollideTile<PT, NW>::template lds_bytes<SITES>()];
  const int tile = xcd_tile(tiles);
  if (tile < 0) return;
  const int m = batch_member(first, count, tile);
  const DevParams P = mem[m].P;
  const DevState in = mem[m].st[cur];
  collide_tile<false, PT, SITES, NW>(P, in, mem[m].st[1 - cur].f, mem[m].U, tile - first[m], lds);
}

// ---------------------------------------------------------------------------
// One forward-Euler sub-step of the Cahn-Hilliard (Model, Eq. 1) and
// Beris-Edwards (Model, Eqs. 11-12) equations with u_a and u_c frozen.  Each
// thread updates R consecutive rows of one column, so the stencils of
// neighbouring rows share their loads and their chemical-potential values.
// ---------------------------------------------------------------------------
constexpr int FD_TX = 64, FD_TY = 4;
template <int R> __host__ __device__ inline int fd_tiles(int nx, int ny) {
  return ((nx + FD_TX - 1) / FD_TX) * ((ny + FD_TY * R - 1) / (FD_TY * R));
}

template <int R>
__device__ __forceinline__ void fd_tile(const DevParams& P, const DevState& in, const DevState& out,
                                        const float* __restrict__ U, int tile) {
  const int nx = P.nx, ny = P.ny, n = P.n;
  const int gx = (nx + FD_TX - 1) / FD_TX;
  const int x = (tile % gx) * FD_TX + threadIdx.x;
  const int y0 = ((tile / gx) * FD_TY + threadIdx.y) * R;
  if (x >= nx || y0 >= ny) return;
  const unsigned xc = x, xm1 = wrapi(x - 1, nx), xp1 = wrapi(x + 1, nx);
  const unsigned xm2 = wrapi(x - 2, nx), xp2 = wrapi(x + 2, nx);
  unsigned row[R + 4];  // rows y0 - 2 .. y0 + R + 1 (offsets below n: n >= 8 > R + 1)
#pragma unroll
  for (int j = 0; j < R + 4; ++j) row[j] = (unsigned)wrapi(y0 - 2 + j, ny) * (unsigned)nx;
  const Plane ph = plane(in.phi, n), ophi = plane(out.phi, n);
  // ---- Cahn-Hilliard: phi += h [ -div(phi u_c) + M lap(mu) ]
  float pc[R + 4], pe[R + 2], pw[R + 2], pee[R], pww[R];
#pragma unroll
  for (int j = 0; j < R + 4; ++j) pc[j] = ldg(ph, row[j] + xc);        // rows y0-2+j
#pragma unroll
  for (int j = 0; j < R + 2; ++j) {                                     // rows y0-1+j
    pe[j] = ldg(ph, row[j + 1] + xp1);
    pw[j] = ldg(ph, row[j + 1] + xm1);
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {                                         // rows y0+j
    pee[j] = ldg(ph, row[j + 2] + xp2);
    pww[j] = ldg(ph, row[j + 2] + xm2);
  }
  float mc[R + 2], me[R], mw[R];
#pragma unroll
  for (int j = 0; j < R + 2; ++j) mc[j] = chem_pot(pc[j + 1], pe[j], pw[j], pc[j + 2], pc[j], P);
#pragma unroll
  for (int j = 0; j < R; ++j) {
    me[j] = chem_pot(pe[j + 1], pee[j], pc[j + 2], pe[j + 2], pe[j], P);
    mw[j] = chem_pot(pw[j + 1], pc[j + 2], pww[j], pw[j + 2], pw[j], P);
  }
  const Plane ucx = plane(U + 2 * n, n), ucy = plane(U + 3 * n, n);
  float cy[R + 2];
#pragma unroll
  for (int j = 0; j < R + 2; ++j) cy[j] = ldg(ucy, row[j + 1] + xc);  // rows y0-1+j
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if (y0 + j >= ny) break;
    const float cxe = ldg(ucx, row[j + 2] + xp1), cxw = ldg(ucx, row[j + 2] + xm1);
    const float div = 0.5f * (pe[j + 1] * cxe - pw[j + 1] * cxw) + 0.5f * (pc[j + 3] * cy[j + 2] - pc[j + 1] * cy[j]);
    const float lapmu = (me[j] + mw[j]) + (mc[j + 2] + mc[j]) - 4.f * mc[j + 1];
    stg(ophi, row[j + 2] + xc, pc[j + 2] + P.h * (P.M * lapmu - div));
  }
  // ---- Beris-Edwards: Q += h Proj[ -u_a.grad Q + S(W, Q) + Gamma H ]
  const Plane qx = plane(in.q, n), qy = plane(in.q + n, n), oqx = plane(out.q, n), oqy = plane(out.q + n, n);
  const Plane ax = plane(U, n), ay = plane(U + n, n);
  float2 qc[R + 2], ac[R + 2];                                          // rows y0-1+j
#pragma unroll
  for (int j = 0; j < R + 2; ++j) {
    const unsigned o = row[j + 1] + xc;
    qc[j] = make_float2(ldg(qx, o), ldg(qy, o));
    ac[j] = make_float2(ldg(ax, o), ldg(ay, o));
  }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if (y0 + j >= ny) break;
    const unsigned oe = row[j + 2] + xp1, ow = row[j + 2] + xm1;
    const float2 qe = make_float2(ldg(qx, oe), ldg(qy, oe)), qw = make_float2(ldg(qx, ow), ldg(qy, ow));
    const float2 ue = make_float2(ldg(ax, oe), ldg(ay, oe)), uw = make_float2(ldg(ax, ow), ldg(ay, ow));
    const float2 nq = be_update(qc[j + 1], qe, qw, qc[j + 2], qc[j], ac[j + 1], ue, uw, ac[j + 2], ac[j], P.h, P);
    const unsigned o = row[j + 2] + xc;
    stg(oqx, o, nq.x);
    stg(oqy, o, nq.y);
  }
}

template <int R>
__global__ void __launch_bounds__(FD_TX * FD_TY) k_fd(DevParams P, DevState in, DevState out,
                                                       const float* __restrict__ U) {
  const int tile = xcd_tile(fd_tiles<R>(P.nx, P.ny));
  if (tile < 0) return;
  fd_tile<R>(P, in, out, U, tile);
}

template <int R>
__global__ void __launch_bounds__(FD_TX * FD_TY) k_fd_batch(const BatchMember* __restrict__ mem,
                                                             const int* __restrict__ first, int count,
                                                             int tiles, int src) {
  const int tile = xcd_tile(tiles);
  if (tile < 0) return;
  const int m = batch_member(first, count, tile);
  const DevParams P = mem[m].P;
  fd_tile<R>(P, mem[m].st[src], mem[m].st[1 - src], mem[m].U, tile - first[m]);
}

// ---------------------------------------------------------------------------
// Several finite-difference sub-steps in one launch (temporal blocking in LDS).
// The Cahn-Hilliard and Beris-Edwards sub-steps do not depend on each other, so
// the two fields grow their halos separately: phi needs phi at distance 2 per
// sub-step (through mu), Q needs Q at distance 1.  For up to MS sub-steps a
// block stages, for a 64 x TH tile, phi and u_c with a halo of 2 MS and Q and
// u_a with a halo of MS, then runs the sub-steps on boxes that shrink by 2 (phi)
// and 1 (Q) per sub-step, and writes only the final phi and Q of its tile.  The
// arithmetic of each site update is that of fd_tile, term for term, so every
// blocking gives the same bits.  Deeper blocking reads the fields fewer times
// but recomputes more halo sites (MS = 5 on 64 x 16 tiles: 1.6x the sub-step
// work; MS = 2: 1.2x).
// ---------------------------------------------------------------------------
constexpr int FF_X = 64;
template <int TH, int MS> struct Fused {
  static constexpr int HA = 2 * MS, HB = MS;  // halos of the phi / mu / u_c and Q / u_a frames
  static constexpr int AW = FF_X + 2 * HA, AH = TH + 2 * HA;
  static constexpr int BW = FF_X + 2 * HB, BH = TH + 2 * HB;
  static constexpr int NT = TH >= 32 ? 1024 : 512;
  static constexpr int KA = (AW * AH + NT - 1) / NT, KB = (BW * BH + NT - 1) / NT;
  // largest boxes updated into registers: phi with halo 2 MS - 2, Q with MS - 1
  static constexpr int KP = ((FF_X + 4 * MS - 4) * (TH + 4 * MS - 4) + NT - 1) / NT;
  static constexpr int KQ = ((FF_X + 2 * MS - 2) * (TH + 2 * MS - 2) + NT - 1) / NT;
  // largest mu box: halo 2 MS - 1
  static constexpr int KM = ((FF_X + 4 * MS - 2) * (TH + 4 * MS - 2) + NT - 1) / NT;
};
template <int TH> __host__ __device__ inline int fused_tiles(int nx, int ny) {
  return ((nx + FF_X - 1) / FF_X) * ((ny + TH - 1) / TH);
}

// Row of entry c of a box w entries wide (c < 2^13, 64 <= w < 2^10): (c + 0.5) / w
// is at least 0.5 / w away from an integer, while the product with the hardware
// reciprocal (relative error below 2^-21 with the rounding of the product) is off by
// less than 2^13 / 64 * 2^-21 = 6e-5 < 0.5 / w: the truncation is exact.  The
// reciprocal is one instruction where an IEEE division takes about a dozen.
__device__ __forceinline__ float box_inv(int w) { return __builtin_amdgcn_rcpf((float)w); }
__device__ __forceinline__ int box_row(int c, float inv_w) { return (int)(((float)c + 0.5f) * inv_w); }

// Frame offset of entry c (row cy) of a box whose rows are `gap` entries
// narrower than the frame and whose first entry sits at frame offset `base`:
// (cy + o) * FW + (c - cy * w + o) = c + cy * (FW - w) + o * (FW + 1).  All
// factors are below 2^13, so a 24-bit product is exact.
__device__ __forceinline__ int frame_offset(int c, int cy, int gap, int base) {
  return c + __mul24(cy, gap) + base;
}

// S (1 <= S <= MS) sub-steps from state `in` to state `out`.
template <int TH, int MS>
__device__ __forceinline__ void fd_fused_tile(const DevParams& P, const DevState& in, const DevState& out,
                                              const float* __restrict__ U, int tile, int S) {
  using F = Fused<TH, MS>;
  constexpr int AW = F::AW, AH = F::AH, BW = F::BW, BH = F::BH, NT = F::NT;
  constexpr int FF_HA = F::HA, FF_HB = F::HB;
  // pairs that are always read together live interleaved (one 8-byte LDS read)
  __shared__ float sphi[AH * AW], smu[AH * AW];
  __shared__ float2 suc[AH * AW];  // (u_c,x, u_c,y)
  __shared__ float2 sq[BH * BW];   // (Qxx, Qxy)
  __shared__ float2 sua[BH * BW];  // (u_a,x, u_a,y)
  __shared__ unsigned scol[AW], srow[AH];
  const int nx = P.nx, ny = P.ny, n = P.n;
  const int gx = (nx + FF_X - 1) / FF_X;
  const int x0 = (tile % gx) * FF_X, y0 = (tile / gx) * TH;
  const int tid = threadIdx.x;
  // periodic source column / row offset of every frame entry (small grids wrap
  // more than once)
  for (int i = tid; i < AW + AH; i += NT) {
    if (i < AW) {
      const int g = (x0 - FF_HA + i) % nx;
      scol[i] = (unsigned)(g < 0 ? g + nx : g);
    } else {
      const int g = (y0 - FF_HA + (i - AW)) % ny;
      srow[i - AW] = (unsigned)(g < 0 ? g + ny : g) * (unsigned)nx;
    }
  }
  __syncthreads();
  // stage the frames; every load is issued before the first LDS store
  {
    const Plane ph = plane(in.phi, n), qx = plane(in.q, n), qy = plane(in.q + n, n);
    const Plane uax = plane(U, n), uay = plane(U + n, n), ucx = plane(U + 2 * n, n), ucy = plane(U + 3 * n, n);
    float va[F::KA][3], vb[F::KB][4];
#pragma unroll
    for (int k = 0; k < F::KA; ++k) {
      const int c = min(tid + k * NT, AW * AH - 1);
      const int cy = c / AW, cx = c - cy * AW;
      const unsigned g = srow[cy] + scol[cx];
      va[k][0] = ldg(ph, g);
      va[k][1] = ldg(ucx, g);
      va[k][2] = ldg(ucy, g);
    }
#pragma unroll
    for (int k = 0; k < F::KB; ++k) {
      const int c = min(tid + k * NT, BW * BH - 1);
      const int cy = c / BW, cx = c - cy * BW;
      const unsigned g = srow[cy + FF_HA - FF_HB] + scol[cx + FF_HA - FF_HB];
      vb[k][0] = ldg(qx, g);
      vb[k][1] = ldg(qy, g);
      vb[k][2] = ldg(uax, g);
      vb[k][3] = ldg(uay, g);
    }
#pragma unroll
    for (int k = 0; k < F::KA; ++k) {
      const int c = tid + k * NT;
      if (c < AW * AH) {
        sphi[c] = va[k][0];
        suc[c] = make_float2(va[k][1], va[k][2]);
      }
    }
#pragma unroll
    for (int k = 0; k < F::KB; ++k) {
      const int c = tid + k * NT;
      if (c < BW * BH) {
        sq[c] = make_float2(vb[k][0], vb[k][1]);
        sua[c] = make_float2(vb[k][2], vb[k][3]);
      }
    }
  }
  __syncthreads();
  const Plane ophi = plane(out.phi, n), oqx = plane(out.q, n), oqy = plane(out.q + n, n);
  constexpr int KP = F::KP, KQ = F::KQ, KM = F::KM;
  float pn[KP], qn[KQ][2];
  int pp[KP], pq[KQ];  // LDS offsets of this thread's points (reused by the write-back)
  for (int m = 1; m <= S; ++m) {
    const int r = 2 * (S - m), s = S - m;  // halos of the boxes updated in this sub-step
    // (1) mu on the phi box of halo r + 1
    {
      const int w = FF_X + 2 * (r + 1), cnt = w * (TH + 2 * (r + 1)), off = FF_HA - (r + 1);
      const float inv = box_inv(w);
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        const int c = tid + k * NT;
        if (c < cnt) {
          const int p = frame_offset(c, box_row(c, inv), AW - w, off * (AW + 1));
          smu[p] = chem_pot(sphi[p], sphi[p + 1], sphi[p - 1], sphi[p + AW], sphi[p - AW], P);
        }
      }
    }
    // (2) Beris-Edwards update on the Q box of halo s, into registers
    const int wq = FF_X + 2 * s, cq = wq * (TH + 2 * s), oq = FF_HB - s;
    const float invq = box_inv(wq);
#pragma unroll
    for (int k = 0; k < KQ; ++k) {
      const int c = tid + k * NT;
      if (c < cq) {
        const int p = frame_offset(c, box_row(c, invq), BW - wq, oq * (BW + 1));
        pq[k] = p;
        const float2 nq = be_update(sq[p], sq[p + 1], sq[p - 1], sq[p + BW], sq[p - BW], sua[p], sua[p + 1],
                                    sua[p - 1], sua[p + BW], sua[p - BW], P.h, P);
        qn[k][0] = nq.x;
        qn[k][1] = nq.y;
      }
    }
    __syncthreads();
    // (3) Cahn-Hilliard update on the phi box of halo r, into registers
    const int wp = FF_X + 2 * r, cp = wp * (TH + 2 * r), op = FF_HA - r;
    const float invp = box_inv(wp);
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int c = tid + k * NT;
      if (c < cp) {
        const int p = frame_offset(c, box_row(c, invp), AW - wp, op * (AW + 1));
        pp[k] = p;
        const float div = 0.5f * (sphi[p + 1] * suc[p + 1].x - sphi[p - 1] * suc[p - 1].x) +
                          0.5f * (sphi[p + AW] * suc[p + AW].y - sphi[p - AW] * suc[p - AW].y);
        const float lapmu = (smu[p + 1] + smu[p - 1]) + (smu[p + AW] + smu[p - AW]) - 4.f * smu[p];
        pn[k] = sphi[p] + P.h * (P.M * lapmu - div);
      }
    }
    __syncthreads();  // every read of this sub-step's frames done
    // (4) write back: into the frames, or the tile to the output after the last sub-step
    if (m < S) {
#pragma unroll
      for (int k = 0; k < KP; ++k)
        if (tid + k * NT < cp) sphi[pp[k]] = pn[k];
#pragma unroll
      for (int k = 0; k < KQ; ++k)
        if (tid + k * NT < cq) sq[pq[k]] = make_float2(qn[k][0], qn[k][1]);
      __syncthreads();
    } else {
      // r = s = 0: both boxes are the tile, entry c = cy * 64 + cx
#pragma unroll
      for (int k = 0; k < KQ; ++k) {
        const int c = tid + k * NT;
        const int cy = c / FF_X, cx = c - cy * FF_X;
        if (c < FF_X * TH && x0 + cx < nx && y0 + cy < ny) {
          const unsigned o = (unsigned)(y0 + cy) * (unsigned)nx + (unsigned)(x0 + cx);
          stg(oqx, o, qn[k][0]);
          stg(oqy, o, qn[k][1]);
        }
      }
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        const int c = tid + k * NT;
        const int cy = c / FF_X, cx = c - cy * FF_X;
        if (c < FF_X * TH && x0 + cx < nx && y0 + cy < ny)
          stg(ophi, (unsigned)(y0 + cy) * (unsigned)nx + (unsigned)(x0 + cx), pn[k]);
      }
    }
  }
}

template <int TH, int MS>
__global__ void __launch_bounds__((Fused<TH, MS>::NT)) k_fd_fused(DevParams P, DevState in, DevState out,
                                                                 const float* __restrict__ U, int subs) {
  const int tile = xcd_tile(fused_tiles<TH>(P.nx, P.ny));
  if (tile < 0) return;
  fd_fused_tile<TH, MS>(P, in, out, U, tile, subs);
}

template <int TH, int MS>
__global__ void __launch_bounds__((Fused<TH, MS>::NT)) k_fd_fused_batch(const BatchMember* __restrict__ mem,
                                                                       const int* __restrict__ first, int count,
                                                                       int tiles, int src, int subs) {
  const int tile = xcd_tile(tiles);
  if (tile < 0) return;
  const int m = batch_member(first, count, tile);
  const DevParams P = mem[m].P;
  fd_fused_tile<TH, MS>(P, mem[m].st[src], mem[m].st[1 - src], mem[m].U, tile - first[m], subs);
}

// ---------------------------------------------------------------------------
// The same temporal blocking with the two fields in separate thread blocks (the
// sub-steps of phi and Q are independent with u_a and u_c frozen), so that each
// block holds only its own frames in LDS.  Threads update strips of R vertically
// consecutive sites of one column: the north/south stencil values of a strip are
// read once from LDS and shared through registers.  Site arithmetic is that of
// fd_tile, term for term.  On 64 x 40 tiles with five sub-steps the phi block
// recomputes 1.46x (mu) and 1.36x (phi) the sites of its tile, the Q block 1.17x
// (64 x 32: 1.53x, 1.42x, 1.20x and 3% longer; 64 x 40 is the tallest tile whose
// phi frames, 81 KB, still let two blocks share a compute unit's 160 KB of LDS).
// ---------------------------------------------------------------------------
template <int TH, int MS> struct PhiBlock {
  static constexpr int H = 2 * MS;                           // frame halo
  static constexpr int W = FF_X + 2 * H, HT = TH + 2 * H;    // frame width, height
  static constexpr int NT = 1024;
  static constexpr int RM = 2, RP = 4;                       // strip heights: mu, phi
  static constexpr int KS = (W * HT + NT - 1) / NT;
  // largest boxes: mu with halo 2 MS - 1, phi with halo 2 MS - 2
  static constexpr int KM = ((FF_X + 4 * MS - 2) * ((TH + 4 * MS - 2) / RM) + NT - 1) / NT;
  static constexpr int KP = ((FF_X + 4 * MS - 4) * ((TH + 4 * MS - 4) / RP) + NT - 1) / NT;
  static constexpr int LDS = 4 * HT * W * 4 + (W + HT) * 4;  // phi, mu, u_c,x, u_c,y, sources
  static_assert(TH % RP == 0, "box heights must be whole strips");
};
template <int TH, int MS> struct QBlock {
  static constexpr int H = MS;
  static constexpr int W = FF_X + 2 * H, HT = TH + 2 * H;
  static constexpr int NT = 1024;
  static constexpr int R = 2;
  static constexpr int KS = (W * HT + NT - 1) / NT;
  static constexpr int KQ = ((FF_X + 2 * MS - 2) * ((TH + 2 * MS - 2) / R) + NT - 1) / NT;
  static constexpr int LDS = 2 * HT * W * 8 + (W + HT) * 4;  // Q, u_a, sources
  static_assert(TH % R == 0, "box heights must be whole strips");
};

// Periodic source offsets of the columns and rows of a frame with halo h.
__device__ __forceinline__ void frame_sources(unsigned* scol, unsigned* srow, int w, int ht, int x0, int y0,
                                              int h, int nx, int ny, int nt) {
  for (int i = threadIdx.x; i < w + ht; i += nt) {
    if (i < w) {
      const int g = (x0 - h + i) % nx;
      scol[i] = (unsigned)(g < 0 ? g + nx : g);
    } else {
      const int g = (y0 - h + (i - w)) % ny;
      srow[i - w] = (unsigned)(g < 0 ? g + ny : g) * (unsigned)nx;
    }
  }
}

// S (1 <= S <= MS) Cahn-Hilliard sub-steps of phi from `in` to `out`.
template <int TH, int MS>
__device__ __forceinline__ void phi_block_tile(const DevParams& P, const DevState& in, const DevState& out,
                                               const float* __restrict__ U, int tile, int S,
                                               unsigned char* __restrict__ lds) {
  using B = PhiBlock<TH, MS>;
  constexpr int W = B::W, HT = B::HT, NT = B::NT, H = B::H;
  float* sphi = reinterpret_cast<float*>(lds);
  float* smu = sphi + HT * W;
  float* sux = smu + HT * W;
  float* suy = sux + HT * W;
  unsigned* scol = reinterpret_cast<unsigned*>(suy + HT * W);
  unsigned* srow = scol + W;
  const int nx = P.nx, ny = P.ny, n = P.n;
  const int gx = (nx + FF_X - 1) / FF_X;
  const int x0 = (tile % gx) * FF_X, y0 = (tile / gx) * TH;
  const int tid = threadIdx.x;
  frame_sources(scol, srow, W, HT, x0, y0, H, nx, ny, NT);
  __syncthreads();
  {
    const Plane ph = plane(in.phi, n), ucx = plane(U + 2 * n, n), ucy = plane(U + 3 * n, n);
    float v[B::KS][3];
#pragma unroll
    for (int k = 0; k < B::KS; ++k) {
      const int c = min(tid + k * NT, W * HT - 1);
      const int cy = c / W, cx = c - cy * W;
      const unsigned g = srow[cy] + scol[cx];
      v[k][0] = ldg(ph, g);
      v[k][1] = ldg(ucx, g);
      v[k][2] = ldg(ucy, g);
    }
#pragma unroll
    for (int k = 0; k < B::KS; ++k) {
      const int c = tid + k * NT;
      if (c < W * HT) {
        sphi[c] = v[k][0];
        sux[c] = v[k][1];
        suy[c] = v[k][2];
      }
    }
  }
  __syncthreads();
  constexpr int RP = B::RP;
  float pn[B::KP][RP];
  int pp[B::KP];
  for (int m = 1; m <= S; ++m) {
    const int r = 2 * (S - m);  // halo of the phi box of this sub-step
    // (1) mu on the box of halo r + 1, two rows per strip
    {
      const int w = FF_X + 2 * (r + 1), cnt = w * ((TH + 2 * (r + 1)) / 2), o = H - (r + 1);
      const float inv = box_inv(w);
#pragma unroll
      for (int k = 0; k < B::KM; ++k) {
        const int c = tid + k * NT;
        if (c < cnt) {
          const int p = frame_offset(c, box_row(c, inv), 2 * W - w, o * (W + 1));
          const float a0 = sphi[p - W], a1 = sphi[p], a2 = sphi[p + W], a3 = sphi[p + 2 * W];
          smu[p] = chem_pot(a1, sphi[p + 1], sphi[p - 1], a2, a0, P);
          smu[p + W] = chem_pot(a2, sphi[p + W + 1], sphi[p + W - 1], a3, a1, P);
        }
      }
    }
    __syncthreads();
    // (2) phi on the box of halo r, RP rows per strip, into registers
    const int w = FF_X + 2 * r, cnt = w * ((TH + 2 * r) / RP), o = H - r;
    const float inv = box_inv(w);
#pragma unroll
    for (int k = 0; k < B::KP; ++k) {
      const int c = tid + k * NT;
      if (c < cnt) {
        const int p = frame_offset(c, box_row(c, inv), RP * W - w, o * (W + 1));
        pp[k] = p;
        float ph[RP + 2], uy[RP + 2], mu[RP + 2];
#pragma unroll
        for (int j = 0; j < RP + 2; ++j) {
          const int q = p + (j - 1) * W;
          ph[j] = sphi[q];
          uy[j] = suy[q];
          mu[j] = smu[q];
        }
#pragma unroll
        for (int j = 0; j < RP; ++j) {
          const int q = p + j * W;
          const float div = 0.5f * (sphi[q + 1] * sux[q + 1] - sphi[q - 1] * sux[q - 1]) +
                            0.5f * (ph[j + 2] * uy[j + 2] - ph[j] * uy[j]);
          const float lapmu = (smu[q + 1] + smu[q - 1]) + (mu[j + 2] + mu[j]) - 4.f * mu[j + 1];
          pn[k][j] = ph[j + 1] + P.h * (P.M * lapmu - div);
        }
      }
    }
    __syncthreads();
    // (3) write back into the frame, or the tile to the output after the last sub-step
    if (m < S) {
#pragma unroll
      for (int k = 0; k < B::KP; ++k)
        if (tid + k * NT < cnt) {
#pragma unroll
          for (int j = 0; j < RP; ++j) sphi[pp[k] + j * W] = pn[k][j];
        }
      __syncthreads();
    } else {
      // r = 0: strip c covers rows RP * (c / 64) .. + RP - 1 of column c % 64
      const Plane ophi = plane(out.phi, n);
#pragma unroll
      for (int k = 0; k < B::KP; ++k) {
        const int c = tid + k * NT;
        const int sy = c / FF_X, cx = c - sy * FF_X;
        if (c < cnt && x0 + cx < nx) {
#pragma unroll
          for (int j = 0; j < RP; ++j) {
            const int y = y0 + RP * sy + j;
            if (y < ny) stg(ophi, (unsigned)y * (unsigned)nx + (unsigned)(x0 + cx), pn[k][j]);
          }
        }
      }
    }
  }
}

// S (1 <= S <= MS) Beris-Edwards sub-steps of Q from `in` to `out`.
template <int TH, int MS>
__device__ __forceinline__ void q_block_tile(const DevParams& P, const DevState& in, const DevState& out,
                                             const float* __restrict__ U, int tile, int S,
                                             unsigned char* __restrict__ lds) {
  using B = QBlock<TH, MS>;
  constexpr int W = B::W, HT = B::HT, NT = B::NT, H = B::H, R = B::R;
  float2* sq = reinterpret_cast<float2*>(lds);  // (Qxx, Qxy)
  float2* sua = sq + HT * W;                    // (u_a,x, u_a,y)
  unsigned* scol = reinterpret_cast<unsigned*>(sua + HT * W);
  unsigned* srow = scol + W;
  const int nx = P.nx, ny = P.ny, n = P.n;
  const int gx = (nx + FF_X - 1) / FF_X;
  const int x0 = (tile % gx) * FF_X, y0 = (tile / gx) * TH;
  const int tid = threadIdx.x;
  frame_sources(scol, srow, W, HT, x0, y0, H, nx, ny, NT);
  __syncthreads();
  {
    const Plane qx = plane(in.q, n), qy = plane(in.q + n, n), uax = plane(U, n), uay = plane(U + n, n);
    float v[B::KS][4];
#pragma unroll
    for (int k = 0; k < B::KS; ++k) {
      const int c = min(tid + k * NT, W * HT - 1);
      const int cy = c / W, cx = c - cy * W;
      const unsigned g = srow[cy] + scol[cx];
      v[k][0] = ldg(qx, g);
      v[k][1] = ldg(qy, g);
      v[k][2] = ldg(uax, g);
      v[k][3] = ldg(uay, g);
    }
#pragma unroll
    for (int k = 0; k < B::KS; ++k) {
      const int c = tid + k * NT;
      if (c < W * HT) {
        sq[c] = make_float2(v[k][0], v[k][1]);
        sua[c] = make_float2(v[k][2], v[k][3]);
      }
    }
  }
  __syncthreads();
  float2 qn[B::KQ][R];
  int pq[B::KQ];
  for (int m = 1; m <= S; ++m) {
    const int s = S - m;  // halo of the Q box of this sub-step
    const int w = FF_X + 2 * s, cnt = w * ((TH + 2 * s) / R), o = H - s;
    const float inv = box_inv(w);
#pragma unroll
    for (int k = 0; k < B::KQ; ++k) {
      const int c = tid + k * NT;
      if (c < cnt) {
        const int p = frame_offset(c, box_row(c, inv), R * W - w, o * (W + 1));
        pq[k] = p;
        float2 qc[R + 2], ac[R + 2];
#pragma unroll
        for (int j = 0; j < R + 2; ++j) {
          qc[j] = sq[p + (j - 1) * W];
          ac[j] = sua[p + (j - 1) * W];
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const int q = p + j * W;
          qn[k][j] = be_update(qc[j + 1], sq[q + 1], sq[q - 1], qc[j + 2], qc[j], ac[j + 1], sua[q + 1], sua[q - 1],
                               ac[j + 2], ac[j], P.h, P);
        }
      }
    }
    __syncthreads();
    if (m < S) {
#pragma unroll
      for (int k = 0; k < B::KQ; ++k)
        if (tid + k * NT < cnt) {
#pragma unroll
          for (int j = 0; j < R; ++j) sq[pq[k] + j * W] = qn[k][j];
        }
      __syncthreads();
    } else {
      const Plane oqx = plane(out.q, n), oqy = plane(out.q + n, n);
#pragma unroll
      for (int k = 0; k < B::KQ; ++k) {
        const int c = tid + k * NT;
        const int sy = c / FF_X, cx = c - sy * FF_X;
        if (c < cnt && x0 + cx < nx) {
#pragma unroll
          for (int j = 0; j < R; ++j) {
            const int y = y0 + R * sy + j;
            if (y < ny) {
              const unsigned g = (unsigned)y * (unsigned)nx + (unsigned)(x0 + cx);
              stg(oqx, g, qn[k][j].x);
              stg(oqy, g, qn[k][j].y);
            }
          }
        }
      }
    }
  }
}

// phi and Q tiles in one grid that shares one LDS allocation, so that the
// LDS-latency-bound phi blocks and the VALU-bound Q blocks run side by side on
// the compute units.  Work item t of the XCD-ordered grid belongs to group
// g = t / kPairGroup; even groups are phi tiles and odd groups Q tiles, the
// group pair g / 2 covering tiles [(g / 2) kPairGroup, (g / 2 + 1) kPairGroup).
// With kPairGroup = 64 (the block slots of one XCD) the blocks resident on a
// compute unit are mostly one of each kind.
constexpr int kPairGroup = 64;
template <int TH, int MS> struct PairBlock {
  static constexpr int NT = PhiBlock<TH, MS>::NT;
  static constexpr int LDS = PhiBlock<TH, MS>::LDS > QBlock<TH, MS>::LDS ? PhiBlock<TH, MS>::LDS : QBlock<TH, MS>::LDS;
  static_assert(PhiBlock<TH, MS>::NT == QBlock<TH, MS>::NT, "one block size for both fields");
};
__host__ __device__ inline int pair_items(int tiles) {
  return 2 * ((tiles + kPairGroup - 1) / kPairGroup) * kPairGroup;
}
// Tile of work item t and whether it advances phi (else Q); -1 for a spare item.
__device__ __forceinline__ int pair_tile(int t, int tiles, bool& phi) {
  const int g = t / kPairGroup;
  const int tile = (g >> 1) * kPairGroup + (t - g * kPairGroup);
  phi = (g & 1) == 0;
  return tile < tiles ? tile : -1;
}

template <int TH, int MS>
__global__ void __launch_bounds__((PairBlock<TH, MS>::NT), 8) k_fd_pair(DevParams P, DevState in, DevState out,
                                                                      const float* __restrict__ U, int subs) {
  __shared__ __align__(16) unsigned char lds[PairBlock<TH, MS>::LDS];
  const int tiles = fused_tiles<TH>(P.nx, P.ny);
  const int t = xcd_tile(pair_items(tiles));
  if (t < 0) return;
  bool phi;
  const int tile = pair_tile(t, tiles, phi);
  if (tile < 0) return;
  if (phi) phi_block_tile<TH, MS>(P, in, out, U, tile, subs, lds);
  else q_block_tile<TH, MS>(P, in, out, U, tile, subs, lds);
}

template <int TH, int MS>
__global__ void __launch_bounds__((PairBlock<TH, MS>::NT), 8) k_fd_pair_batch(const BatchMember* __restrict__ mem,
                                                                            const int* __restrict__ first, int count,
                                                                            int tiles, int src, int subs) {
  __shared__ __align__(16) unsigned char lds[PairBlock<TH, MS>::LDS];
  const int t = xcd_tile(pair_items(tiles));
  if (t < 0) return;
  bool phi;
  const int tile = pair_tile(t, tiles, phi);
  if (tile < 0) return;
  const int m = batch_member(first, count, tile);
  const DevParams P = mem[m].P;
  if (phi) phi_block_tile<TH, MS>(P, mem[m].st[src], mem[m].st[1 - src], mem[m].U, tile - first[m], subs, lds);
  else q_block_tile<TH, MS>(P, mem[m].st[src], mem[m].st[1 - src], mem[m].U, tile - first[m], subs, lds);
}

// ---------------------------------------------------------------------------
// One persistent launch for every member of a batch and every step: blocks of
// 1024 threads (two per compute unit) loop over the steps; in each step they
// take the collision tiles of all members (256 x 4 sites, one site per thread),
// meet at a grid-wide barrier, take the split phi / Q sub-step tiles of all
// members (64 x 40, all sub-steps of the step), and meet again.  The launch is
// cooperative, so every block is resident and every block reaches every
// barrier (the work loops may be empty, the barriers are not).  Each block owns
// a contiguous range of tiles, ranges ordered so that the blocks of one XCD hold
// neighbouring tiles.
// ---------------------------------------------------------------------------
constexpr int kPersistThreads = 1024;
template <typename PT> struct Persist {
  using CT = CollideTile<PT, false, kPersistThreads>;
  static constexpr int CLDS = CT::template lds_bytes<1>();
  static constexpr int FLDS = PairBlock<kSplitTile, kFusedMaxSub>::LDS;
  static constexpr int LDS = CLDS > FLDS ? CLDS : FLDS;
  static_assert(PairBlock<kSplitTile, kFusedMaxSub>::NT == kPersistThreads, "one block size for both phases");
};

__device__ __forceinline__ void persist_range(int items, int& lo, int& hi) {
  const int G = (int)gridDim.x, b = (int)blockIdx.x;
  const int logical = (b % kXcds) * (G / kXcds) + b / kXcds;  // G is a multiple of kXcds
  const int per = (items + G - 1) / G;
  lo = min(items, logical * per);
  hi = min(items, lo + per);
}

// One block per compute unit (124 VGPRs, 4 waves per SIMD): forcing two blocks
// (64 VGPRs) spills ~50 registers and was slower (sweep 0.66 against 0.57 ms per step).
template <typename PT>
__global__ void __launch_bounds__(kPersistThreads, 4) k_batch_persistent(const BatchMember* __restrict__ mem,
                                                                         const int* __restrict__ first_c,
                                                                         const int* __restrict__ first_f, int count,
                                                                         int tiles_c, int tiles_f, int nsteps, int cur,
                                                                         int subs) {
  __shared__ __align__(16) unsigned char lds[Persist<PT>::LDS];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  int c0, c1, f0, f1;
  persist_range(tiles_c, c0, c1);
  persist_range(pair_items(tiles_f), f0, f1);
  for (int step = 0; step < nsteps; ++step) {
    for (int t = c0; t < c1; ++t) {
      const int m = batch_member(first_c, count, t);
      const DevParams P = mem[m].P;
      collide_tile<false, PT, 1, false, kPersistThreads>(P, mem[m].st[cur], mem[m].st[1 - cur].f, mem[m].U,
                                                         t - first_c[m], lds);
      __syncthreads();
    }
    grid.sync();
    for (int it = f0; it < f1; ++it) {
      bool phi;
      const int tile = pair_tile(it, tiles_f, phi);
      if (tile >= 0) {
        const int m = batch_member(first_f, count, tile);
        const DevParams P = mem[m].P;
        if (phi)
          phi_block_tile<kSplitTile, kFusedMaxSub>(P, mem[m].st[cur], mem[m].st[1 - cur], mem[m].U,
                                                   tile - first_f[m], subs, lds);
        else
          q_block_tile<kSplitTile, kFusedMaxSub>(P, mem[m].st[cur], mem[m].st[1 - cur], mem[m].U, tile - first_f[m],
                                                 subs, lds);
      }
      __syncthreads();
    }
    grid.sync();
    cur = 1 - cur;
  }
}

// Post-collision populations whose pull gives f^eq(rho0, u) at every site:
// stored f*_i(x) = f^eq_i(u(x + c_i)) - w_i rho0.
template <typename PT>
__global__ void __launch_bounds__(256) k_init(DevParams P, const float* __restrict__ aux,
                                              void* __restrict__ f) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= P.nx || y >= P.ny) return;
  const int nx = P.nx, ny = P.ny, n = P.n;
  const int idx = y * nx + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int src = wrapi(y + CY[i], ny) * nx + wrapi(x + CX[i], nx);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const float ux = aux[(2 * s) * n + src], uy = aux[(2 * s + 1) * n + src];
      const float cu = (float)CX[i] * ux + (float)CY[i] * uy;
      pop_st<PT>(f, pop_index<PT>(s, i, (size_t)n, (size_t)idx),
                 WT[i] * P.rho0 * (cu * (3.f + 4.5f * cu) - 1.5f * (ux * ux + uy * uy)));
    }
  }
}

// Populations that reproduce a given macroscopic state at the next step.  For
// every site: the densities are the given deviations drho ([2][n]) or else those of
// the current populations f_old (pulled as the next step would pull them), the
// forces those of the given phi and Q, and the
// momenta m solve the velocity equations of the step for the given velocities,
// m_a = (rho_a + g) u_a - g u_p - G_a / 2 and m_p = (rho_p + g) u_p - g u_a - G_p / 2,
// so that the next step's Guo velocities equal u.  The pull of site x then sees
// f^eq(rho, m / rho): stored f*_i(x - c_i) = f^eq_i(x) - w_i rho0 in f_out (which
// must not alias f_old).  Neither drho nor f_old: densities rho0.  One thread per
// site; stencils read from global memory.
template <typename PT>
__global__ void __launch_bounds__(256) k_import(DevParams P, const void* __restrict__ f_old,
                                                const float* __restrict__ phi, const float* __restrict__ q,
                                                const float* __restrict__ u_in, const float* __restrict__ drho,
                                                void* __restrict__ f_out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= P.nx || y >= P.ny) return;
  const int nx = P.nx, ny = P.ny, n = P.n;
  auto at = [&](int dx, int dy) { return wrap_any(y + dy, ny) * nx + wrap_any(x + dx, nx); };
  auto mu_at = [&](int dx, int dy) {
    return chem_pot(phi[at(dx, dy)], phi[at(dx + 1, dy)], phi[at(dx - 1, dy)], phi[at(dx, dy + 1)],
                    phi[at(dx, dy - 1)], P);
  };
  auto stress_at = [&](int dx, int dy) {
    const int c = at(dx, dy), e = at(dx + 1, dy), w = at(dx - 1, dy), nn = at(dx, dy + 1), ss = at(dx, dy - 1);
    return nematic_stress(q[c], q[n + c], q[e], q[n + e], q[w], q[n + w], q[nn], q[n + nn], q[ss], q[n + ss],
                          0.5f * (1.f + phi[c]), P);
  };
  const Stress sE = stress_at(1, 0), sW = stress_at(-1, 0), sN = stress_at(0, 1), sS = stress_at(0, -1);
  const SiteStencil t = {sE.xx, sW.xx, sN.yy, sS.yy, sE.s, sW.s, sN.s, sS.s, sE.a, sW.a, sN.a, sS.a,
                         mu_at(1, 0), mu_at(-1, 0), mu_at(0, 1), mu_at(0, -1), phi[at(0, 0)],
                         mu_at(0, 0), phi[at(1, 0)], phi[at(-1, 0)], phi[at(0, 1)], phi[at(0, -1)]};
  const SiteForce G = site_forces(t);
  const int idx = y * nx + x;
  float dra = 0.f, drp = 0.f;  // rho0 without densities given or populations to keep
  if (drho) {
    dra = drho[idx];
    drp = drho[n + idx];
  } else if (f_old) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      float a, b;
      pop_ld2<PT>(f_old, i, (size_t)n, (size_t)at(-CX[i], -CY[i]), a, b);
      dra += a;
      drp += b;
    }
  }
  const float rho_a = P.rho0 + dra, rho_p = P.rho0 + drp;
  const float g = 0.5f * P.gamma * G.c1 * G.c2;
  const float uax = u_in[idx], uay = u_in[n + idx], upx = u_in[2 * n + idx], upy = u_in[3 * n + idx];
  const float vax = ((rho_a + g) * uax - g * upx - 0.5f * G.ax) / rho_a;
  const float vay = ((rho_a + g) * uay - g * upy - 0.5f * G.ay) / rho_a;
  const float vpx = ((rho_p + g) * upx - g * uax - 0.5f * G.px) / rho_p;
  const float vpy = ((rho_p + g) * upy - g * uay - 0.5f * G.py) / rho_p;
  const float ua15 = 1.5f * (vax * vax + vay * vay), up15 = 1.5f * (vpx * vpx + vpy * vpy);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float ca = (float)CX[i] * vax + (float)CY[i] * vay;
    const float cp = (float)CX[i] * vpx + (float)CY[i] * vpy;
    pop_st2<PT>(f_out, i, (size_t)n, (size_t)at(-CX[i], -CY[i]), WT[i] * (dra + rho_a * (ca * (3.f + 4.5f * ca) - ua15)),
                WT[i] * (drp + rho_p * (cp * (3.f + 4.5f * cp) - up15)));
  }
}

// State exchange layout [planes][n], planes 7 or 9: phi, Qxx, Qxy, u_a,x, u_a,y,
// u_p,x, u_p,y, then (9) rho_a - rho0, rho_p - rho0.  Pack reads the velocities and
// densities from aux as the fields kernel leaves it, [drho_a, drho_p, u_a (2), u_p (2)];
// unpack writes the velocities to aux planes 0..3 and the densities to planes 4..5.
__global__ void __launch_bounds__(256) k_pack_state(int n, int planes, const float* __restrict__ phi,
                                                    const float* __restrict__ q, const float* __restrict__ aux,
                                                    float* __restrict__ out) {
  const size_t total = (size_t)planes * n;
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (size_t)gridDim.x * blockDim.x) {
    const size_t plane = j / (size_t)n, i = j - plane * (size_t)n;
    const float v = plane == 0  ? phi[i]
                    : plane < 3 ? q[(plane - 1) * (size_t)n + i]
                    : plane < 7 ? aux[(plane - 1) * (size_t)n + i]
                                : aux[(plane - 7) * (size_t)n + i];
    out[j] = v;
  }
}

__global__ void __launch_bounds__(256) k_unpack_state(int n, int planes, const float* __restrict__ in,
                                                      float* __restrict__ phi, float* __restrict__ q,
                                                      float* __restrict__ aux) {
  const size_t total = (size_t)planes * n;
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (size_t)gridDim.x * blockDim.x) {
    const size_t plane = j / (size_t)n, i = j - plane * (size_t)n;
    const float v = in[j];
    if (plane == 0) phi[i] = v;
    else if (plane < 3) q[(plane - 1) * (size_t)n + i] = v;
    else aux[(plane - 3) * (size_t)n + i] = v;
  }
}

// ---------------------------------------------------------------------------
// Diagnostics: per-site float64 contributions, wavefront shuffle reduction,
// one record per block, then a single-block pass.  Deterministic for a given
// grid (fixed block count and fixed site-to-thread assignment).
// ---------------------------------------------------------------------------
constexpr int kDiagThreads = 256;
constexpr int kDiagMaxBlocks = 1024;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ void block_reduce_store(double acc[kDiagSlots], double* __restrict__ dst) {
  __shared__ double red[kDiagThreads / 64][kDiagSlots];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kDiagSlots; ++k) {
    const double v = diag_is_max(k) ? wave_max(acc[k]) : wave_sum(acc[k]);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kDiagSlots) {
    const int k = threadIdx.x;
    double v = red[0][k];
    for (int w = 1; w < kDiagThreads / 64; ++w) v = diag_is_max(k) ? fmax(v, red[w][k]) : v + red[w][k];
    dst[k] = v;
  }
}

__device__ __forceinline__ int is_bad(float v) { return (isfinite(v) ? 0 : 1); }

template <typename PT>
__global__ void __launch_bounds__(kDiagThreads) k_diag(DevParams P, DevState in,
                                                      const float* __restrict__ aux,
                                                      double* __restrict__ partials) {
  double acc[kDiagSlots];
#pragma unroll
  for (int k = 0; k < kDiagSlots; ++k) acc[k] = 0.0;
  const int nx = P.nx, ny = P.ny, n = P.n;
  const float* drho_a = aux;
  const float* drho_p = aux + n;
  const float* uax = aux + 2 * n;
  const float* uay = aux + 3 * n;
  const float* upx = aux + 4 * n;
  const float* upy = aux + 5 * n;
  const float* qx = in.q;
  const float* qy = in.q + n;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += gridDim.x * blockDim.x) {
    const int y = idx / nx, x = idx - y * nx;
    const int e = y * nx + wrapi(x + 1, nx), w = y * nx + wrapi(x - 1, nx);
    const int no = wrapi(y + 1, ny) * nx + x, so = wrapi(y - 1, ny) * nx + x;
    const double ph = in.phi[idx];
    acc[D_PHI] += ph;
    acc[D_PHI2] += ph * ph;
    acc[D_PHIMAX] = fmax(acc[D_PHIMAX], fabs(ph));
    const double ra = P.rho0_d + (double)drho_a[idx], rp = P.rho0_d + (double)drho_p[idx];
    acc[D_MASS_A] += ra;
    acc[D_MASS_P] += rp;
    const double ax = uax[idx], ay = uay[idx], px = upx[idx], py = upy[idx];
    const double c1 = 0.5 * (1.0 + ph), c2 = 0.5 * (1.0 - ph);
    const double cx = c1 * ax + c2 * px, cy = c1 * ay + c2 * py;
    const double ua2 = ax * ax + ay * ay, up2 = px * px + py * py, uc2 = cx * cx + cy * cy;
    acc[D_KE_A] += 0.5 * ra * ua2;
    acc[D_KE_P] += 0.5 * rp * up2;
    acc[D_KE_C] += 0.5 * uc2;
    acc[D_UA2] += ua2;
    acc[D_UC2] += uc2;
    acc[D_UMAX] = fmax(acc[D_UMAX], sqrt(fmax(ua2, up2)));
    // vorticities d_x u_y - d_y u_x
    const double wa = 0.5 * ((double)uay[e] - uay[w]) - 0.5 * ((double)uax[no] - uax[so]);
    auto ucomp = [&](int j, const float* ua_, const float* up_) {
      const double c = 0.5 * (1.0 + (double)in.phi[j]);
      return c * ua_[j] + (1.0 - c) * up_[j];
    };
    const double wc = 0.5 * (ucomp(e, uay, upy) - ucomp(w, uay, upy)) -
                      0.5 * (ucomp(no, uax, upx) - ucomp(so, uax, upx));
    acc[D_ENS_A] += wa * wa;
    acc[D_ENS_C] += wc * wc;
    const double gxx = 0.5 * ((double)qx[e] - qx[w]), gxy = 0.5 * ((double)qx[no] - qx[so]);
    const double hxx = 0.5 * ((double)qy[e] - qy[w]), hxy = 0.5 * ((double)qy[no] - qy[so]);
    acc[D_ELASTIC] += P.K * (gxx * gxx + gxy * gxy + hxx * hxx + hxy * hxy);  // (K/2) * 2 (...)
    const double q1 = qx[idx], q2 = qy[idx];
    acc[D_S] += sqrt(q1 * q1 + q2 * q2);
    int bad = is_bad(in.phi[idx]) + is_bad(qx[idx]) + is_bad(qy[idx]);
#pragma unroll
    for (int i = 0; i < 18; ++i) bad += is_bad(pop_ld<PT>(in.f, pop_index<PT>(i / 9, i % 9, (size_t)n, (size_t)idx)));
    acc[D_NONFINITE] += (double)bad;
  }
  block_reduce_store(acc, partials + (size_t)blockIdx.x * kDiagSlots);
}

__global__ void __launch_bounds__(kDiagThreads) k_diag_final(const double* __restrict__ partials,
                                                            int nblocks, double* __restrict__ out) {
  double acc[kDiagSlots];
#pragma unroll
  for (int k = 0; k < kDiagSlots; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < kDiagSlots; ++k) {
      const double v = partials[(size_t)b * kDiagSlots + k];
      acc[k] = diag_is_max(k) ? fmax(acc[k], v) : acc[k] + v;
    }
  }
  block_reduce_store(acc, out);
}

inline dim3 grid2d(const DevParams& P, dim3 blk) {
  return dim3((P.nx + blk.x - 1) / blk.x, (P.ny + blk.y - 1) / blk.y);
}

}  // namespace

int diag_blocks(const DevParams& P) {
  const int b = (P.n + kDiagThreads - 1) / kDiagThreads;
  return b < kDiagMaxBlocks ? b : kDiagMaxBlocks;
}

hipError_t launch_import(const DevParams& P, const void* f_old, DevState out, const float* u_in, const float* drho,
                         hipStream_t st) {
  const dim3 blk(64, 4);
  if (P.pop16)
    hipLaunchKernelGGL(k_import<_Float16>, grid2d(P, blk), blk, 0, st, P, f_old, out.phi, out.q, u_in, drho, out.f);
  else
    hipLaunchKernelGGL(k_import<float>, grid2d(P, blk), blk, 0, st, P, f_old, out.phi, out.q, u_in, drho, out.f);
  return hipGetLastError();
}

hipError_t launch_init(const DevParams& P, const float* aux_u, DevState out, hipStream_t st) {
  const dim3 blk(64, 4);
  if (P.pop16)
    hipLaunchKernelGGL(k_init<_Float16>, grid2d(P, blk), blk, 0, st, P, aux_u, out.f);
  else
    hipLaunchKernelGGL(k_init<float>, grid2d(P, blk), blk, 0, st, P, aux_u, out.f);
  return hipGetLastError();
}

// Launch on st; with timing events, they travel in the kernel's own dispatch (the
// recorded interval is the kernel's execution, without the gaps around it).
template <typename K, typename... A>
inline void launch_timed(K kernel, dim3 grid, dim3 block, hipStream_t st, hipEvent_t e0, hipEvent_t e1, A... args) {
  if (e0)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

template <bool FIELDS, typename PT, int SITES, bool NW = false>
void launch_collide_tiles(const DevParams& P, DevState in, void* f_out, float* u_out, hipStream_t st,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  const dim3 grid(xcd_grid(collide_tiles<PT, SITES, NW>(P.nx, P.ny)));
  launch_timed(k_collide<FIELDS, PT, SITES, NW>, grid, dim3(CollideTile<PT, NW>::THREADS), st, e0, e1, P, in, f_out,
               u_out);
}

template <typename PT, int SITES, bool NW>
inline int batch_collide_tiles(const DevParams& P) { return collide_tiles<PT, SITES, NW>(P.nx, P.ny); }

hipError_t launch_collide(const DevParams& P, DevState in, void* f_out, float* u_out, Tuning tn,
                          hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
#define TFAN_COLLIDE(R_, NW_)                                                                       \
  (P.pop16 ? launch_collide_tiles<false, _Float16, R_, NW_>(P, in, f_out, u_out, st, e0, e1)        \
           : launch_collide_tiles<false, float, R_, NW_>(P, in, f_out, u_out, st, e0, e1))
  const bool nw = collide_narrow(tn);
  if (collide_site_rows(tn) == 1) {
    if (nw) TFAN_COLLIDE(1, true); else TFAN_COLLIDE(1, false);
  } else {
    if (nw) TFAN_COLLIDE(2, true); else TFAN_COLLIDE(2, false);
  }
#undef TFAN_COLLIDE
  return hipGetLastError();
}

hipError_t launch_fd(const DevParams& P, DevState in, DevState out, const float* u, Tuning tn, int subs,
                     hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const int block = fd_block(tn, P.n_sub);
  if (block > 1 && fd_split(tn)) {
    if (fd_pair_rows(tn) == kSplitTile) {
      const dim3 grid(xcd_grid(pair_items(fused_tiles<kSplitTile>(P.nx, P.ny))));
      launch_timed(k_fd_pair<kSplitTile, kFusedMaxSub>, grid, dim3(PairBlock<kSplitTile, kFusedMaxSub>::NT), st, e0,
                   e1, P, in, out, u, subs);
    } else {
      const dim3 grid(xcd_grid(pair_items(fused_tiles<kSplitTileShort>(P.nx, P.ny))));
      launch_timed(k_fd_pair<kSplitTileShort, kFusedMaxSub>, grid, dim3(PairBlock<kSplitTileShort, kFusedMaxSub>::NT),
                   st, e0, e1, P, in, out, u, subs);
    }
    return hipGetLastError();
  }
  if (e0) (void)hipEventRecord(e0, st);  // other shapes: events around the launch
  if (block > 1) {
    const int th = fd_tile_rows(tn);
#define TFAN_FUSED(TH_, MS_)                                                                                  \
  hipLaunchKernelGGL((k_fd_fused<TH_, MS_>), dim3(xcd_grid(fused_tiles<TH_>(P.nx, P.ny))),                    \
                     dim3(Fused<TH_, MS_>::NT), 0, st, P, in, out, u, subs)
    if (block == 2) TFAN_FUSED(16, 2);
    else if (block == 3) TFAN_FUSED(16, 3);
    else if (th == 16) TFAN_FUSED(16, 5);
    else TFAN_FUSED(32, 5);
#undef TFAN_FUSED
    if (e1) (void)hipEventRecord(e1, st);
    return hipGetLastError();
  }
  switch (tn.fd_shape) {
    case 1: hipLaunchKernelGGL(k_fd<1>, dim3(xcd_grid(fd_tiles<1>(P.nx, P.ny))), dim3(FD_TX, FD_TY), 0, st, P, in, out, u); break;
    case 2: hipLaunchKernelGGL(k_fd<2>, dim3(xcd_grid(fd_tiles<2>(P.nx, P.ny))), dim3(FD_TX, FD_TY), 0, st, P, in, out, u); break;
    default: hipLaunchKernelGGL(k_fd<4>, dim3(xcd_grid(fd_tiles<4>(P.nx, P.ny))), dim3(FD_TX, FD_TY), 0, st, P, in, out, u); break;
  }
  if (e1) (void)hipEventRecord(e1, st);
  return hipGetLastError();
}

int batch_tiles(const DevParams& P, Tuning tn, bool collide) {
  if (collide) {
    const bool one = collide_site_rows(tn) == 1, nw = collide_narrow(tn);
    if (P.pop16)
      return one ? (nw ? batch_collide_tiles<_Float16, 1, true>(P) : batch_collide_tiles<_Float16, 1, false>(P))
                 : (nw ? batch_collide_tiles<_Float16, 2, true>(P) : batch_collide_tiles<_Float16, 2, false>(P));
    return one ? (nw ? batch_collide_tiles<float, 1, true>(P) : batch_collide_tiles<float, 1, false>(P))
               : (nw ? batch_collide_tiles<float, 2, true>(P) : batch_collide_tiles<float, 2, false>(P));
  }
  if (fd_block(tn, P.n_sub) > 1) {
    if (fd_split(tn))
      return fd_pair_rows(tn) == kSplitTile ? fused_tiles<kSplitTile>(P.nx, P.ny) : fused_tiles<kSplitTileShort>(P.nx, P.ny);
    return fd_tile_rows(tn) == 16 ? fused_tiles<16>(P.nx, P.ny) : fused_tiles<32>(P.nx, P.ny);
  }
  return tn.fd_shape == 1 ? fd_tiles<1>(P.nx, P.ny) : tn.fd_shape == 2 ? fd_tiles<2>(P.nx, P.ny) : fd_tiles<4>(P.nx, P.ny);
}

hipError_t launch_collide_batch(const BatchMember* mem, const int* first, int count, int tiles, int cur, bool pop16,
                                Tuning tn, hipStream_t st) {
  const dim3 grid(xcd_grid(tiles));
#define TFAN_COLLIDE_B(PT_, R_, NW_)                                                                          \
  hipLaunchKernelGGL((k_collide_batch<PT_, R_, NW_>), grid, dim3(CollideTile<PT_, NW_>::THREADS), 0, st, mem, \
                     first, count, tiles, cur)
  const bool one = collide_site_rows(tn) == 1, nw = collide_narrow(tn);
  if (pop16) {
    if (one) { if (nw) TFAN_COLLIDE_B(_Float16, 1, true); else TFAN_COLLIDE_B(_Float16, 1, false); }
    else { if (nw) TFAN_COLLIDE_B(_Float16, 2, true); else TFAN_COLLIDE_B(_Float16, 2, false); }
  } else {
    if (one) { if (nw) TFAN_COLLIDE_B(float, 1, true); else TFAN_COLLIDE_B(float, 1, false); }
    else { if (nw) TFAN_COLLIDE_B(float, 2, true); else TFAN_COLLIDE_B(float, 2, false); }
  }
#undef TFAN_COLLIDE_B
  return hipGetLastError();
}

hipError_t launch_fd_batch(const BatchMember* mem, const int* first, int count, int tiles, int src, Tuning tn,
                           int n_sub, int subs, hipStream_t st) {
  const dim3 grid(xcd_grid(tiles)), blk(FD_TX, FD_TY);
  const int block = fd_block(tn, n_sub);
  if (block > 1 && fd_split(tn)) {
    if (fd_pair_rows(tn) == kSplitTile)
      hipLaunchKernelGGL((k_fd_pair_batch<kSplitTile, kFusedMaxSub>), dim3(xcd_grid(pair_items(tiles))),
                         dim3(PairBlock<kSplitTile, kFusedMaxSub>::NT), 0, st, mem, first, count, tiles, src, subs);
    else
      hipLaunchKernelGGL((k_fd_pair_batch<kSplitTileShort, kFusedMaxSub>), dim3(xcd_grid(pair_items(tiles))),
                         dim3(PairBlock<kSplitTileShort, kFusedMaxSub>::NT), 0, st, mem, first, count, tiles, src, subs);
    return hipGetLastError();
  }
  if (block > 1) {
#define TFAN_FUSED_B(TH_, MS_) \
  hipLaunchKernelGGL((k_fd_fused_batch<TH_, MS_>), grid, dim3(Fused<TH_, MS_>::NT), 0, st, mem, first, count, tiles, src, subs)
    if (block == 2) TFAN_FUSED_B(16, 2);
    else if (block == 3) TFAN_FUSED_B(16, 3);
    else if (fd_tile_rows(tn) == 16) TFAN_FUSED_B(16, 5);
    else TFAN_FUSED_B(32, 5);
#undef TFAN_FUSED_B
    return hipGetLastError();
  }
  switch (tn.fd_shape) {
    case 1: hipLaunchKernelGGL(k_fd_batch<1>, grid, blk, 0, st, mem, first, count, tiles, src); break;
    case 2: hipLaunchKernelGGL(k_fd_batch<2>, grid, blk, 0, st, mem, first, count, tiles, src); break;
    default: hipLaunchKernelGGL(k_fd_batch<4>, grid, blk, 0, st, mem, first, count, tiles, src); break;
  }
  return hipGetLastError();
}

hipError_t launch_fields(const DevParams& P, DevState in, float* aux, hipStream_t st) {
  if (P.pop16) launch_collide_tiles<true, _Float16, 2, false>(P, in, nullptr, aux, st);
  else launch_collide_tiles<true, float, 2, false>(P, in, nullptr, aux, st);
  return hipGetLastError();
}

int persist_collide_tiles(const DevParams& P) { return collide_tiles<float, 1, false, kPersistThreads>(P.nx, P.ny); }
int persist_fd_tiles(const DevParams& P) { return fused_tiles<kSplitTile>(P.nx, P.ny); }

hipError_t launch_batch_persistent(const BatchMember* mem, const int* first_c, const int* first_f, int count,
                                   int tiles_c, int tiles_f, int nsteps, int cur, int subs, bool pop16, int* grid_out,
                                   hipStream_t st) {
  const void* fn = pop16 ? reinterpret_cast<const void*>(&k_batch_persistent<_Float16>)
                         : reinterpret_cast<const void*>(&k_batch_persistent<float>);
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kPersistThreads, 0);
  if (e != hipSuccess) return e;
  const int grid = (per_cu * cus) / kXcds * kXcds;
  if (grid < kXcds) return hipErrorInvalidConfiguration;
  if (grid_out) *grid_out = grid;
  void* args[] = {(void*)&mem, (void*)&first_c, (void*)&first_f, (void*)&count, (void*)&tiles_c,
                  (void*)&tiles_f, (void*)&nsteps, (void*)&cur, (void*)&subs};
  e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kPersistThreads), args, 0, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_pack_state(int n, int planes, const float* phi, const float* q, const float* aux, float* out,
                             hipStream_t st) {
  const size_t total = (size_t)planes * n;
  const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_pack_state, dim3(blocks), dim3(256), 0, st, n, planes, phi, q, aux, out);
  return hipGetLastError();
}

hipError_t launch_unpack_state(int n, int planes, const float* in, float* phi, float* q, float* aux, hipStream_t st) {
  const size_t total = (size_t)planes * n;
  const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_unpack_state, dim3(blocks), dim3(256), 0, st, n, planes, in, phi, q, aux);
  return hipGetLastError();
}

hipError_t launch_diag(const DevParams& P, DevState in, const float* aux, double* partials,
                       int nblocks, double* result, hipStream_t st) {
  if (P.pop16)
    hipLaunchKernelGGL(k_diag<_Float16>, dim3(nblocks), dim3(kDiagThreads), 0, st, P, in, aux, partials);
  else
    hipLaunchKernelGGL(k_diag<float>, dim3(nblocks), dim3(kDiagThreads), 0, st, P, in, aux, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagThreads), 0, st, partials, nblocks, result);
  return hipGetLastError();
}

}  // namespace tfan
