// gfx950 kernels of the two-fluid active-nematic coupled step (arXiv 2511.00445,
// Model and Numerical Simulation sections).
//
// Storage: structure-of-arrays float32 planes [ny][nx], x fastest.  Populations
// are stored after collision and before streaming ("post-collision"), shifted by
// -w_i rho0 so that the small deviations from rest keep float32 precision; the
// next step streams them by pulling f_i(x) = f*_i(x - c_i).
#include "tfan_internal.h"

namespace tfan {
namespace {

// D2Q9 velocities and weights (order: rest, +x, +y, -x, -y, +x+y, -x+y, -x-y, +x-y).
constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr float WT[9] = {4.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f,
                         1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};

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

// Everything one site needs before collision: pulled populations, densities,
// half-force velocities and total forces of both fluids.
struct Site {
  float fa[9], fp[9];
  float dra, drp;        // rho - rho0
  float uax, uay, upx, upy;
  float Fax, Fay, Fpx, Fpy;
  float c1, c2;
};

__device__ __forceinline__ void site_macroscopic(const DevParams& P, const DevState& in, int x,
                                                 int y, Site& S) {
  const int nx = P.nx, ny = P.ny, n = P.n;
  const int xm1 = wrapi(x - 1, nx), xp1 = wrapi(x + 1, nx);
  const int xm2 = wrapi(x - 2, nx), xp2 = wrapi(x + 2, nx);
  const int r0 = y * nx, rm1 = wrapi(y - 1, ny) * nx, rp1 = wrapi(y + 1, ny) * nx;
  const int rm2 = wrapi(y - 2, ny) * nx, rp2 = wrapi(y + 2, ny) * nx;
  const float* __restrict__ ph = in.phi;
  const float* __restrict__ qx = in.q;
  const float* __restrict__ qy = in.q + n;
#define TFAN_LD3(name, off)                                                  \
  const float p##name = ph[off], x##name = qx[off], y##name = qy[off];
  TFAN_LD3(C, r0 + x)
  TFAN_LD3(E, r0 + xp1)
  TFAN_LD3(W, r0 + xm1)
  TFAN_LD3(N, rp1 + x)
  TFAN_LD3(S, rm1 + x)
  TFAN_LD3(EE, r0 + xp2)
  TFAN_LD3(WW, r0 + xm2)
  TFAN_LD3(NN, rp2 + x)
  TFAN_LD3(SS, rm2 + x)
  TFAN_LD3(NE, rp1 + xp1)
  TFAN_LD3(NW, rp1 + xm1)
  TFAN_LD3(SE, rm1 + xp1)
  TFAN_LD3(SW, rm1 + xm1)
#undef TFAN_LD3
  // chemical potential and stress at the four neighbours
  const float muE = chem_pot(pE, pEE, pC, pNE, pSE, P);
  const float muW = chem_pot(pW, pC, pWW, pNW, pSW, P);
  const float muN = chem_pot(pN, pNE, pNW, pNN, pC, P);
  const float muS = chem_pot(pS, pSE, pSW, pC, pSS, P);
  const Stress sE = nematic_stress(xE, yE, xEE, yEE, xC, yC, xNE, yNE, xSE, ySE, 0.5f * (1.f + pE), P);
  const Stress sW = nematic_stress(xW, yW, xC, yC, xWW, yWW, xNW, yNW, xSW, ySW, 0.5f * (1.f + pW), P);
  const Stress sN = nematic_stress(xN, yN, xNE, yNE, xNW, yNW, xNN, yNN, xC, yC, 0.5f * (1.f + pN), P);
  const Stress sS = nematic_stress(xS, yS, xSE, ySE, xSW, ySW, xC, yC, xSS, ySS, 0.5f * (1.f + pS), P);
  // F_i = d_j sigma_ij
  const float Fx = 0.5f * (sE.xx - sW.xx) + 0.5f * ((sN.s + sN.a) - (sS.s + sS.a));
  const float Fy = 0.5f * ((sE.s - sE.a) - (sW.s - sW.a)) + 0.5f * (sN.yy - sS.yy);
  const float c1 = 0.5f * (1.f + pC), c2 = 0.5f * (1.f - pC);
  // capillary force -phi grad(mu), shared c1 : c2
  const float fchx = -pC * 0.5f * (muE - muW);
  const float fchy = -pC * 0.5f * (muN - muS);
  const float Gax = Fx + c1 * fchx, Gay = Fy + c1 * fchy;
  const float Gpx = c2 * fchx, Gpy = c2 * fchy;

  // pull both population sets and take moments
  float dra = 0.f, mxa = 0.f, mya = 0.f, drp = 0.f, mxp = 0.f, myp = 0.f;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int sx = (CX[i] == 0) ? x : (CX[i] > 0 ? xm1 : xp1);
    const int sy = (CY[i] == 0) ? r0 : (CY[i] > 0 ? rm1 : rp1);
    const float a = in.f[(size_t)i * n + sy + sx];
    const float p = in.f[(size_t)(9 + i) * n + sy + sx];
    S.fa[i] = a;
    S.fp[i] = p;
    dra += a;
    drp += p;
    if (CX[i] != 0) { mxa += CX[i] * a; mxp += CX[i] * p; }
    if (CY[i] != 0) { mya += CY[i] * a; myp += CY[i] * p; }
  }
  const float rho_a = P.rho0 + dra, rho_p = P.rho0 + drp;
  // Guo half-force velocities with the drag implicit: per component
  // [[rho_a + g, -g], [-g, rho_p + g]] [u_a; u_p] = [m_a + G_a/2; m_p + G_p/2]
  const float g = 0.5f * P.gamma * c1 * c2;
  const float inv = 1.f / (rho_a * rho_p + g * (rho_a + rho_p));
  const float bax = mxa + 0.5f * Gax, bay = mya + 0.5f * Gay;
  const float bpx = mxp + 0.5f * Gpx, bpy = myp + 0.5f * Gpy;
  S.uax = ((rho_p + g) * bax + g * bpx) * inv;
  S.uay = ((rho_p + g) * bay + g * bpy) * inv;
  S.upx = (g * bax + (rho_a + g) * bpx) * inv;
  S.upy = (g * bay + (rho_a + g) * bpy) * inv;
  const float fdx = 2.f * g * (S.upx - S.uax), fdy = 2.f * g * (S.upy - S.uay);
  S.Fax = Gax + fdx;
  S.Fay = Gay + fdy;
  S.Fpx = Gpx - fdx;
  S.Fpy = Gpy - fdy;
  S.dra = dra;
  S.drp = drp;
  S.c1 = c1;
  S.c2 = c2;
}

// BGK collision with the Guo source for one fluid, written post-collision:
// f* = f + (f^eq - f)/tau + (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F,
// all populations shifted by -w_i rho0.
__device__ __forceinline__ void collide_fluid(const float f[9], float dr, float ux, float uy,
                                              float Fx, float Fy, float om, float gk, float rho0,
                                              float* __restrict__ out, int n, int idx) {
  const float rho = rho0 + dr;
  const float uu15 = 1.5f * (ux * ux + uy * uy);
  const float uF = ux * Fx + uy * Fy;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float cu = (float)CX[i] * ux + (float)CY[i] * uy;
    const float cF = (float)CX[i] * Fx + (float)CY[i] * Fy;
    const float feq = WT[i] * (dr + rho * (cu * (3.f + 4.5f * cu) - uu15));
    const float src = gk * WT[i] * (3.f * (cF - uF) + 9.f * cu * cF);
    out[(size_t)i * n + idx] = f[i] + om * (feq - f[i]) + src;
  }
}

__global__ void __launch_bounds__(256) k_collide(DevParams P, DevState in, float* __restrict__ fout,
                                                 float* __restrict__ uout) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= P.nx || y >= P.ny) return;
  Site S;
  site_macroscopic(P, in, x, y, S);
  const int idx = y * P.nx + x, n = P.n;
  collide_fluid(S.fa, S.dra, S.uax, S.uay, S.Fax, S.Fay, P.om_a, P.gk_a, P.rho0, fout, n, idx);
  collide_fluid(S.fp, S.drp, S.upx, S.upy, S.Fpx, S.Fpy, P.om_p, P.gk_p, P.rho0, fout + (size_t)9 * n,
                n, idx);
  uout[idx] = S.uax;
  uout[n + idx] = S.uay;
  uout[2 * n + idx] = S.c1 * S.uax + S.c2 * S.upx;
  uout[3 * n + idx] = S.c1 * S.uay + S.c2 * S.upy;
}

__global__ void __launch_bounds__(256) k_fields(DevParams P, DevState in, float* __restrict__ aux) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= P.nx || y >= P.ny) return;
  Site S;
  site_macroscopic(P, in, x, y, S);
  const int idx = y * P.nx + x, n = P.n;
  aux[idx] = S.dra;  // density deviations: rho0 is added in float64 by the reader
  aux[n + idx] = S.drp;
  aux[2 * n + idx] = S.uax;
  aux[3 * n + idx] = S.uay;
  aux[4 * n + idx] = S.upx;
  aux[5 * n + idx] = S.upy;
}

// One forward-Euler sub-step of the Cahn-Hilliard (Model, Eq. 1) and
// Beris-Edwards (Model, Eqs. 11-12) equations with frozen u_a, u_c.
__global__ void __launch_bounds__(256) k_fd(DevParams P, DevState in, DevState out,
                                            const float* __restrict__ U) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= P.nx || y >= P.ny) return;
  const int nx = P.nx, ny = P.ny, n = P.n;
  const int xm1 = wrapi(x - 1, nx), xp1 = wrapi(x + 1, nx);
  const int xm2 = wrapi(x - 2, nx), xp2 = wrapi(x + 2, nx);
  const int r0 = y * nx, rm1 = wrapi(y - 1, ny) * nx, rp1 = wrapi(y + 1, ny) * nx;
  const int rm2 = wrapi(y - 2, ny) * nx, rp2 = wrapi(y + 2, ny) * nx;
  const float* __restrict__ ph = in.phi;
  // --- Cahn-Hilliard: phi += h [ -div(phi u_c) + M lap(mu) ]
  const float pC = ph[r0 + x], pE = ph[r0 + xp1], pW = ph[r0 + xm1], pN = ph[rp1 + x], pS = ph[rm1 + x];
  const float pEE = ph[r0 + xp2], pWW = ph[r0 + xm2], pNN = ph[rp2 + x], pSS = ph[rm2 + x];
  const float pNE = ph[rp1 + xp1], pNW = ph[rp1 + xm1], pSE = ph[rm1 + xp1], pSW = ph[rm1 + xm1];
  const float muC = chem_pot(pC, pE, pW, pN, pS, P);
  const float muE = chem_pot(pE, pEE, pC, pNE, pSE, P);
  const float muW = chem_pot(pW, pC, pWW, pNW, pSW, P);
  const float muN = chem_pot(pN, pNE, pNW, pNN, pC, P);
  const float muS = chem_pot(pS, pSE, pSW, pC, pSS, P);
  const float* __restrict__ ucx = U + 2 * n;
  const float* __restrict__ ucy = U + 3 * n;
  const float div = 0.5f * (pE * ucx[r0 + xp1] - pW * ucx[r0 + xm1]) +
                    0.5f * (pN * ucy[rp1 + x] - pS * ucy[rm1 + x]);
  const float lapmu = (muE + muW) + (muN + muS) - 4.f * muC;
  out.phi[r0 + x] = pC + P.h * (P.M * lapmu - div);

  // --- Beris-Edwards: Q += h Proj[ -u_a.grad Q + S(W, Q) + Gamma H ]
  const float* __restrict__ qx = in.q;
  const float* __restrict__ qy = in.q + n;
  const float xC = qx[r0 + x], xE = qx[r0 + xp1], xW = qx[r0 + xm1], xN = qx[rp1 + x], xS = qx[rm1 + x];
  const float yC = qy[r0 + x], yE = qy[r0 + xp1], yW = qy[r0 + xm1], yN = qy[rp1 + x], yS = qy[rm1 + x];
  const float* __restrict__ uax = U;
  const float* __restrict__ uay = U + n;
  const float ux = uax[r0 + x], uy = uay[r0 + x];
  // W_ij = d_j u_a,i
  const float wxx = 0.5f * (uax[r0 + xp1] - uax[r0 + xm1]);
  const float wxy = 0.5f * (uax[rp1 + x] - uax[rm1 + x]);
  const float wyx = 0.5f * (uay[r0 + xp1] - uay[r0 + xm1]);
  const float wyy = 0.5f * (uay[rp1 + x] - uay[rm1 + x]);
  const float d = 0.5f * (wxx - wyy), e = 0.5f * (wxy + wyx), tr = wxx + wyy;
  const float om = 0.5f * (wxy - wyx);
  const float b = P.A_ldg + P.halfC * (2.f * (xC * xC + yC * yC));
  const float hxx = P.K * ((xE + xW) + (xN + xS) - 4.f * xC) - b * xC;
  const float hxy = P.K * ((yE + yW) + (yN + yS) - 4.f * yC) - b * yC;
  // symmetric traceless part of S(W, Q): lam E_dev + lam tr(W) Q - 2 lam (Q:E) Q + (Om.Q - Q.Om)
  const float g = P.lam * (tr - 4.f * (xC * d + yC * e));
  const float sxx = P.lam * d + g * xC + 2.f * om * yC;
  const float sxy = P.lam * e + g * yC - 2.f * om * xC;
  const float advx = -(ux * 0.5f * (xE - xW) + uy * 0.5f * (xN - xS));
  const float advy = -(ux * 0.5f * (yE - yW) + uy * 0.5f * (yN - yS));
  out.q[r0 + x] = xC + P.h * (advx + sxx + P.Gamma * hxx);
  out.q[n + r0 + x] = yC + P.h * (advy + sxy + P.Gamma * hxy);
}

// Post-collision populations whose pull gives f^eq(rho0, u) at every site:
// stored f*_i(x) = f^eq_i(u(x + c_i)) - w_i rho0.
__global__ void __launch_bounds__(256) k_init(DevParams P, const float* __restrict__ aux,
                                              float* __restrict__ f) {
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
      f[(size_t)(9 * s + i) * n + idx] =
          WT[i] * P.rho0 * (cu * (3.f + 4.5f * cu) - 1.5f * (ux * ux + uy * uy));
    }
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
    const double v = (k == D_UMAX) ? wave_max(acc[k]) : wave_sum(acc[k]);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kDiagSlots) {
    const int k = threadIdx.x;
    double v = red[0][k];
    for (int w = 1; w < kDiagThreads / 64; ++w) v = (k == D_UMAX) ? fmax(v, red[w][k]) : v + red[w][k];
    dst[k] = v;
  }
}

__device__ __forceinline__ int is_bad(float v) { return (isfinite(v) ? 0 : 1); }

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
    for (int i = 0; i < 18; ++i) bad += is_bad(in.f[(size_t)i * n + idx]);
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
      acc[k] = (k == D_UMAX) ? fmax(acc[k], v) : acc[k] + v;
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

hipError_t launch_init(const DevParams& P, const float* aux_u, DevState out, hipStream_t st) {
  const dim3 blk(64, 4);
  hipLaunchKernelGGL(k_init, grid2d(P, blk), blk, 0, st, P, aux_u, out.f);
  return hipGetLastError();
}

hipError_t launch_collide(const DevParams& P, DevState in, float* f_out, float* u_out, hipStream_t st) {
  const dim3 blk(64, 4);
  hipLaunchKernelGGL(k_collide, grid2d(P, blk), blk, 0, st, P, in, f_out, u_out);
  return hipGetLastError();
}

hipError_t launch_fd(const DevParams& P, DevState in, DevState out, const float* u, hipStream_t st) {
  const dim3 blk(64, 4);
  hipLaunchKernelGGL(k_fd, grid2d(P, blk), blk, 0, st, P, in, out, u);
  return hipGetLastError();
}

hipError_t launch_fields(const DevParams& P, DevState in, float* aux, hipStream_t st) {
  const dim3 blk(64, 4);
  hipLaunchKernelGGL(k_fields, grid2d(P, blk), blk, 0, st, P, in, aux);
  return hipGetLastError();
}

hipError_t launch_diag(const DevParams& P, DevState in, const float* aux, double* partials,
                       int nblocks, double* result, hipStream_t st) {
  hipLaunchKernelGGL(k_diag, dim3(nblocks), dim3(kDiagThreads), 0, st, P, in, aux, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagThreads), 0, st, partials, nblocks, result);
  return hipGetLastError();
}

}  // namespace tfan
