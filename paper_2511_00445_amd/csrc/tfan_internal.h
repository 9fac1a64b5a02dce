// Internal declarations shared by the host library (tfan.cpp) and the gfx950
// kernels (tfan_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace tfan {

// Parameters in the form the kernels use (float32 arithmetic).
struct DevParams {
  int nx, ny;          // grid
  int n;               // nx * ny
  int n_sub;           // sub-steps per step
  float rho0;
  float om_a, om_p;    // 1/tau
  float gk_a, gk_p;    // Guo prefactor 1 - 1/(2 tau)
  float gamma;         // drag
  float A_ch, kappa, M;
  float A_ldg, halfC;  // H_bulk = -(A + (C/2) TrQ^2) Q
  float K, lam, Gamma, zeta;
  float h;             // 1 / n_sub
  double rho0_d;       // rho0 for float64 reductions
  int pop16;           // populations stored as binary16 (else float32)
};

// Number of float64 slots in one diagnostics record.
constexpr int kDiagSlots = 16;
// Slot order of the diagnostics record (the last two are maxima, the rest sums).
enum DiagSlot {
  D_PHI = 0, D_PHI2, D_MASS_A, D_MASS_P, D_KE_A, D_KE_P, D_KE_C, D_UA2, D_UC2,
  D_ENS_A, D_ENS_C, D_ELASTIC, D_S, D_NONFINITE, D_PHIMAX, D_UMAX
};
constexpr bool diag_is_max(int k) { return k >= D_PHIMAX; }

// Device buffers of one solver (all float32, each [ny][nx] plane n floats).
struct DevState {
  void* f;         // populations, shifted by -w_i rho0: [2 fluids][9][n], float32 or binary16
  float* phi;      // [n]
  float* q;        // [2][n] (Qxx, Qxy)
};

// Launch shape of the hot kernels (results do not depend on it):
// collide_rows in {1, 2} rows of sites per thread; fd_shape in {1, 2, 4}: one
// launch per finite-difference sub-step with that many rows per thread;
// {16, 32}: all sub-steps of a step in one launch on 64 x fd_shape tiles (n_sub
// <= kFusedMaxSub, else one launch per sub-step with 4 rows per thread);
// {162, 163}: blocks of 2 or 3 sub-steps per launch on 64 x 16 tiles;
// 165: blocks of up to kFusedMaxSub sub-steps on 64 x kSplitTile tiles, with
// separate thread blocks for phi and Q in one launch.
// 166: as 165 on 64 x kSplitTileShort tiles.
// collide_rows: 1, 2 rows of sites per thread on the default tile width (256
// sites float32, 128 binary16); 11, 12: the same on tiles of half that width.
constexpr int kFusedMaxSub = 5, kSplitTile = 40, kSplitTileShort = 32;
struct Tuning {
  int collide_rows = 2;
  int fd_shape = 165;
};
inline int collide_site_rows(const Tuning& tn) { return tn.collide_rows % 10; }
inline bool collide_narrow(const Tuning& tn) { return tn.collide_rows > 10; }
// Default launch shape of one simulation by grid size (measured, both storages):
// below 2^21 sites one row of sites per collision thread gives twice the blocks
// and is faster (64^2-256^2: 16 against 18 us per step; 1024^2: 63.5 against 64.4
// us), from 2^21 sites two rows are (2048^2: 215 against 217 us).
inline Tuning default_tuning(int nx, int ny) {
  Tuning t;
  t.collide_rows = (long long)nx * ny < (1LL << 21) ? 1 : 2;
  return t;
}
// Sub-steps per finite-difference launch (1: the per-sub-step kernel).
inline int fd_block(const Tuning& tn, int n_sub) {
  if (tn.fd_shape == 162) return n_sub >= 2 ? 2 : 1;
  if (tn.fd_shape == 163) return n_sub >= 3 ? 3 : (n_sub == 2 ? 2 : 1);
  if (tn.fd_shape == 16 || tn.fd_shape == 32) return (n_sub >= 2 && n_sub <= kFusedMaxSub) ? n_sub : 1;
  if (tn.fd_shape == 165 || tn.fd_shape == 166) return n_sub >= 2 ? (n_sub < kFusedMaxSub ? n_sub : kFusedMaxSub) : 1;
  return 1;
}
// Tile rows of the blocked sub-step kernel.
inline int fd_tile_rows(const Tuning& tn) { return tn.fd_shape == 32 ? 32 : 16; }
// phi and Q advanced by separate thread blocks.
inline bool fd_split(const Tuning& tn) { return tn.fd_shape == 165 || tn.fd_shape == 166; }
// Tile rows of the split (phi / Q blocks) kernel.
inline int fd_pair_rows(const Tuning& tn) { return tn.fd_shape == 166 ? kSplitTileShort : kSplitTile; }

// One member of a batch of independent simulations (device-resident table).
struct BatchMember {
  DevParams P;
  DevState st[2];  // ping-pong states
  float* U;        // frozen velocities [4][n]
};

// Kernel ids for timing.
enum KernelId { K_COLLIDE = 0, K_FD, K_INIT, K_FIELDS, K_DIAG, K_FDN, K_COUNT };

// Launchers (return hipGetLastError() after the launch).
hipError_t launch_init(const DevParams& P, const float* aux_u /*[4][n]*/, DevState out,
                       hipStream_t st);
// Populations of out.f reproducing the velocities u_in ([4][n]: u_a,x, u_a,y, u_p,x,
// u_p,y) at the next step, with the forces of out.phi, out.q, and the density
// deviations drho ([2][n]) or else those of f_old (neither: rho0).  out.f must not
// alias f_old.
hipError_t launch_import(const DevParams& P, const void* f_old, DevState out, const float* u_in, const float* drho,
                         hipStream_t st);
// e0, e1 (optional): timing events recorded at the kernel's start and end.
hipError_t launch_collide(const DevParams& P, DevState in, void* f_out, float* u_out /*[4][n]*/,
                          Tuning tn, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// `subs` finite-difference sub-steps in one launch: subs = 1 with the
// per-sub-step kernel when fd_block(tn, n_sub) == 1, else 1 <= subs <= fd_block.
hipError_t launch_fd(const DevParams& P, DevState in, DevState out, const float* u /*[4][n]*/,
                     Tuning tn, int subs, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Tiles of one member for the collision (collide = true) or sub-step kernel.
int batch_tiles(const DevParams& P, Tuning tn, bool collide);
// Batched launches over the tiles of all members; first[m] = first tile of member m.
hipError_t launch_collide_batch(const BatchMember* mem, const int* first, int count, int tiles, int cur,
                                bool pop16, Tuning tn, hipStream_t st);
// (all members share n_sub)
hipError_t launch_fd_batch(const BatchMember* mem, const int* first, int count, int tiles, int src,
                           Tuning tn, int n_sub, int subs, hipStream_t st);
hipError_t launch_fields(const DevParams& P, DevState in, float* aux /*[6][n]: drho_a, drho_p, u_a, u_p*/,
                         hipStream_t st);
hipError_t launch_diag(const DevParams& P, DevState in, const float* aux /*[6][n]*/,
                       double* partials, int nblocks, double* result, hipStream_t st);
int diag_blocks(const DevParams& P);
// The persistent batch launch: tiles of one member for its collision phase (256 x 4)
// and its sub-step phase (split phi / Q kernel, 64 x 40 tiles); one cooperative
// launch of nsteps steps over all members, buffers `cur` -> 1 - cur -> ...,
// `subs` (1..kFusedMaxSub) sub-steps per step.  *grid_out receives the block count.
int persist_collide_tiles(const DevParams& P);
int persist_fd_tiles(const DevParams& P);
hipError_t launch_batch_persistent(const BatchMember* mem, const int* first_c, const int* first_f, int count,
                                   int tiles_c, int tiles_f, int nsteps, int cur, int subs, bool pop16, int* grid_out,
                                   hipStream_t st);
// State exchange [planes][n], planes 7 (phi, Qxx, Qxy, u_a, u_p) or 9 (and the density
// deviations of both fluids).  Pack from phi, q [2][n] and aux as the fields kernel
// leaves it ([drho_a, drho_p, u_a (2), u_p (2)]); unpack to phi, q, the velocities in
// aux planes 0..3 and the density deviations in aux planes 4..5.
hipError_t launch_pack_state(int n, int planes, const float* phi, const float* q, const float* aux, float* out,
                             hipStream_t st);
hipError_t launch_unpack_state(int n, int planes, const float* in, float* phi, float* q, float* aux, hipStream_t st);

}  // namespace tfan
