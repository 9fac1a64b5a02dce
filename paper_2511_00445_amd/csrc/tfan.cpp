// Host side of the C ABI declared in include/tfan.h: parameter validation,
// workspace layout, kernel launches, host<->device conversion, checkpoints and
// event-based kernel timing.
#include "tfan.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "tfan_internal.h"

using tfan::DevParams;
using tfan::DevState;

struct tfan_sim {
  tfan_params p{};
  DevParams dp{};
  hipStream_t stream = nullptr;
  int device = 0;
  // workspace carve-up
  void* f[2] = {nullptr, nullptr};     // [18][n] each, float32 or binary16
  size_t pop_bytes = 4;                // bytes per stored population
  float* phi[2] = {nullptr, nullptr};  // [n]
  float* q[2] = {nullptr, nullptr};    // [2][n]
  float* U = nullptr;                  // [4][n]: u_a, u_c of the current step
  float* aux = nullptr;                // [7][n]: fields / staging
  double* partials = nullptr;          // [diag blocks][kDiagSlots]
  double* result = nullptr;            // [kDiagSlots]
  int cur = 0;                         // index of the buffers holding the state
  bool has_state = false;              // set by init_fields, set_state and import_state
  tfan::Tuning tune;                   // launch shape of the hot kernels
  int64_t step = 0;
  std::string err;
  // kernel timing
  std::vector<hipEvent_t> ev;          // 2 per recorded launch
  std::vector<int> ev_kernel;
  int64_t ev_cap = 0, ev_used = 0;
  double ms_total[tfan::K_COUNT] = {};
  int64_t launches[tfan::K_COUNT] = {};
};

namespace {

std::string g_err;  // failures without a handle

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int fail(tfan_sim* s, int code, const std::string& msg) {
  if (s) s->err = msg; else g_err = msg;
  return code;
}

int hip_fail(tfan_sim* s, hipError_t e, const char* where) {
  return fail(s, TFAN_EHIP, std::string(where) + ": " + hipGetErrorName(e) + " (" +
                                hipGetErrorString(e) + ")");
}

std::string check(const tfan_params* p) {
  if (!p) return "params is NULL";
  if (p->nx < 8 || p->ny < 8 || p->nx > 32768 || p->ny > 32768) return "nx, ny must be in [8, 32768]";
  if ((int64_t)p->nx * p->ny > (int64_t(1) << 28)) return "nx * ny must not exceed 2^28";
  if (p->n_sub < 1 || p->n_sub > 8) return "n_sub must be in [1, 8]";
  if (p->storage != TFAN_STORAGE_F32 && p->storage != TFAN_STORAGE_F16) return "unsupported storage format";
  const double r[] = {p->rho0, p->tau_a, p->tau_p, p->gamma, p->A_ch, p->kappa, p->M,
                      p->A0, p->gamma_ldg, p->K, p->lam, p->Gamma, p->zeta};
  for (double v : r)
    if (!std::isfinite(v)) return "parameters must be finite";
  if (!(p->rho0 > 0)) return "rho0 must be positive";
  if (!(p->tau_a > 0.5) || !(p->tau_p > 0.5)) return "tau_a and tau_p must exceed 1/2";
  if (p->gamma < 0 || p->kappa < 0 || p->M < 0 || p->K < 0 || p->Gamma < 0)
    return "gamma, kappa, M, K and Gamma must be non-negative";
  return "";
}

struct Layout {
  size_t f[2], phi[2], q[2], U, aux, partials, result, total;
};

Layout layout(const tfan_params* p) {
  const size_t n = (size_t)p->nx * p->ny;
  DevParams dp{};
  dp.n = (int)n;
  const size_t nb = (size_t)tfan::diag_blocks(dp);
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  const size_t pb = p->storage == TFAN_STORAGE_F16 ? 2 : 4;
  for (int k = 0; k < 2; ++k) L.f[k] = take(18 * n * pb);
  for (int k = 0; k < 2; ++k) L.phi[k] = take(n * sizeof(float));
  for (int k = 0; k < 2; ++k) L.q[k] = take(2 * n * sizeof(float));
  L.U = take(4 * n * sizeof(float));
  L.aux = take(7 * n * sizeof(float));
  L.partials = take(nb * tfan::kDiagSlots * sizeof(double));
  L.result = take(tfan::kDiagSlots * sizeof(double));
  L.total = off;
  return L;
}

double ldg_A(const tfan_params* p) { return p->A0 * (1.0 - p->gamma_ldg / 3.0); }
double ldg_C(const tfan_params* p) { return 2.0 * p->A0 * p->gamma_ldg; }

DevParams dev_params(const tfan_params* p) {
  DevParams d{};
  d.nx = p->nx;
  d.ny = p->ny;
  d.n = p->nx * p->ny;
  d.n_sub = p->n_sub;
  d.rho0 = (float)p->rho0;
  d.om_a = (float)(1.0 / p->tau_a);
  d.om_p = (float)(1.0 / p->tau_p);
  d.gk_a = (float)(1.0 - 0.5 / p->tau_a);
  d.gk_p = (float)(1.0 - 0.5 / p->tau_p);
  d.gamma = (float)p->gamma;
  d.A_ch = (float)p->A_ch;
  d.kappa = (float)p->kappa;
  d.M = (float)p->M;
  // Landau-de Gennes bulk energy in the (A0, gamma) form,
  // (A0/2)(1 - gamma/3) TrQ^2 - (A0 gamma/3) TrQ^3 + (A0 gamma/4)(TrQ^2)^2, written in the
  // Model section's form (A/2)TrQ^2 + (B/3)TrQ^3 + (C/4)TrQ^4 (Eq. 8): A = A0 (1 - gamma/3),
  // and C = 2 A0 gamma since TrQ^4 = (TrQ^2)^2 / 2 for a 2x2 traceless Q.  The cubic term
  // adds only a multiple of I to dF/dQ and drops out of the traceless molecular field.
  const double A_ldg = ldg_A(p), C_ldg = ldg_C(p);
  d.A_ldg = (float)A_ldg;
  d.halfC = (float)(0.5 * C_ldg);
  d.K = (float)p->K;
  d.lam = (float)p->lam;
  d.Gamma = (float)p->Gamma;
  d.zeta = (float)p->zeta;
  d.h = (float)(1.0 / p->n_sub);
  d.rho0_d = p->rho0;
  d.pop16 = p->storage == TFAN_STORAGE_F16;
  return d;
}

DevState state_of(tfan_sim* s, int k) { return DevState{s->f[k], s->phi[k], s->q[k]}; }

// Event bracketing of one launch when timing is on.
struct TimedLaunch {
  tfan_sim* s;
  int kernel;
  int64_t slot = -1;
  bool in_dispatch;  // the launcher places the events in the kernel's own dispatch
  TimedLaunch(tfan_sim* s_, int k, bool in_dispatch_ = false) : s(s_), kernel(k), in_dispatch(in_dispatch_) {
    if (s->ev_used < s->ev_cap) {
      slot = s->ev_used++;
      s->ev_kernel[slot] = kernel;
      if (!in_dispatch) (void)hipEventRecord(s->ev[2 * slot], s->stream);
    }
  }
  hipEvent_t start() const { return slot >= 0 ? s->ev[2 * slot] : nullptr; }
  hipEvent_t stop() const { return slot >= 0 ? s->ev[2 * slot + 1] : nullptr; }
  ~TimedLaunch() {
    if (slot >= 0 && !in_dispatch) (void)hipEventRecord(s->ev[2 * slot + 1], s->stream);
  }
};

void harvest(tfan_sim* s) {
  for (int64_t k = 0; k < s->ev_used; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->ev[2 * k], s->ev[2 * k + 1]) == hipSuccess) {
      s->ms_total[s->ev_kernel[k]] += ms;
      s->launches[s->ev_kernel[k]] += 1;
    }
  }
  s->ev_used = 0;
}

void free_events(tfan_sim* s) {
  for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
  s->ev.clear();
  s->ev_kernel.clear();
  s->ev_cap = s->ev_used = 0;
}

int sync_stream(tfan_sim* s, const char* where) {
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, where);
  return TFAN_OK;
}

// Host float64 -> device float32 through a pinned-free staging copy.
int upload(tfan_sim* s, float* dst, const double* src, size_t count, std::vector<float>& tmp) {
  tmp.resize(count);
  for (size_t i = 0; i < count; ++i) tmp[i] = (float)src[i];
  hipError_t e = hipMemcpyAsync(dst, tmp.data(), count * sizeof(float), hipMemcpyHostToDevice, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "upload");
  e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "upload");
  return TFAN_OK;
}

int download(tfan_sim* s, double* dst, const float* src, size_t count, std::vector<float>& tmp,
             double offset = 0.0) {
  tmp.resize(count);
  hipError_t e = hipMemcpyAsync(tmp.data(), src, count * sizeof(float), hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "download");
  e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "download");
  for (size_t i = 0; i < count; ++i) dst[i] = offset + (double)tmp[i];
  return TFAN_OK;
}

}  // namespace

static const int kFdShapes[] = {1, 2, 4, 16, 32, 162, 163, 165, 166};
static const int kCollideShapes[] = {1, 2, 11, 12};
static bool valid_shape(int32_t collide_rows, int32_t fd_shape) {
  bool ok = false;
  for (int c : kCollideShapes) ok = ok || c == collide_rows;
  if (!ok) return false;
  for (int f : kFdShapes)
    if (f == fd_shape) return true;
  return false;
}
static const char* kShapeMsg =
    "collide_rows must be 1, 2, 11 or 12 and fd_shape 1, 2, 4, 16, 32, 162, 163, 165 or 166";
// Shapes the autotuners try: every collide_rows with every fd_shape, skipping
// blocked shapes that n_sub turns into the per-sub-step launch.
static std::vector<tfan::Tuning> tuning_candidates(int n_sub) {
  std::vector<tfan::Tuning> out;
  for (int c : kCollideShapes)
    for (int f : kFdShapes) {
      tfan::Tuning t;
      t.collide_rows = c;
      t.fd_shape = f;
      if (f < 16 || tfan::fd_block(t, n_sub) > 1) out.push_back(t);
    }
  return out;
}

extern "C" {

int tfan_check_params(const tfan_params* p) {
  const std::string m = check(p);
  return m.empty() ? TFAN_OK : fail(nullptr, TFAN_EINVAL, m);
}

size_t tfan_workspace_bytes(const tfan_params* p) {
  if (!check(p).empty()) return 0;
  return layout(p).total;
}

int tfan_create(const tfan_params* p, void* ws, size_t bytes, void* stream, tfan_sim** out) {
  if (!out) return fail(nullptr, TFAN_EINVAL, "out is NULL");
  *out = nullptr;
  const std::string m = check(p);
  if (!m.empty()) return fail(nullptr, TFAN_EINVAL, m);
  if (!ws) return fail(nullptr, TFAN_EINVAL, "workspace is NULL");
  if (((uintptr_t)ws) % kAlign) return fail(nullptr, TFAN_EINVAL, "workspace must be 256-byte aligned");
  const Layout L = layout(p);
  if (bytes < L.total)
    return fail(nullptr, TFAN_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
  tfan_sim* s = new tfan_sim();
  s->p = *p;
  s->dp = dev_params(p);
  s->tune = tfan::default_tuning(p->nx, p->ny);
  s->pop_bytes = p->storage == TFAN_STORAGE_F16 ? 2 : 4;
  s->stream = (hipStream_t)stream;
  (void)hipGetDevice(&s->device);
  char* base = (char*)ws;
  for (int k = 0; k < 2; ++k) {
    s->f[k] = (void*)(base + L.f[k]);
    s->phi[k] = (float*)(base + L.phi[k]);
    s->q[k] = (float*)(base + L.q[k]);
  }
  s->U = (float*)(base + L.U);
  s->aux = (float*)(base + L.aux);
  s->partials = (double*)(base + L.partials);
  s->result = (double*)(base + L.result);
  *out = s;
  return TFAN_OK;
}

int tfan_init_fields(tfan_sim* s, const double* phi, const double* qxx, const double* qxy,
                     const double* u_a, const double* u_p) {
  if (!s) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!phi || !qxx || !qxy) return fail(s, TFAN_EINVAL, "phi, qxx and qxy are required");
  const size_t n = (size_t)s->dp.n;
  for (const double* a : {phi, qxx, qxy})
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(a[i])) return fail(s, TFAN_EINVAL, "initial fields must be finite");
  for (const double* a : {u_a, u_p})
    if (a)
      for (size_t i = 0; i < 2 * n; ++i)
        if (!std::isfinite(a[i])) return fail(s, TFAN_EINVAL, "initial velocities must be finite");
  std::vector<float> tmp;
  s->cur = 0;
  int rc;
  if ((rc = upload(s, s->phi[0], phi, n, tmp))) return rc;
  if ((rc = upload(s, s->q[0], qxx, n, tmp))) return rc;
  if ((rc = upload(s, s->q[0] + n, qxy, n, tmp))) return rc;
  std::vector<double> zero;
  if (!u_a || !u_p) zero.assign(2 * n, 0.0);
  if ((rc = upload(s, s->aux, u_a ? u_a : zero.data(), 2 * n, tmp))) return rc;
  if ((rc = upload(s, s->aux + 2 * n, u_p ? u_p : zero.data(), 2 * n, tmp))) return rc;
  {
    TimedLaunch t(s, tfan::K_INIT);
    hipError_t e = tfan::launch_init(s->dp, s->aux, state_of(s, 0), s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "init kernel launch");
  }
  s->step = 0;
  s->has_state = true;
  return sync_stream(s, "init_fields");
}

int tfan_step(tfan_sim* s, int64_t nsteps) {
  if (!s) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(s, TFAN_EINVAL, "step count must be >= 0");
  for (int64_t k = 0; k < nsteps; ++k) {
    const int a = s->cur, b = 1 - s->cur;
    {
      TimedLaunch t(s, tfan::K_COLLIDE, true);
      hipError_t e = tfan::launch_collide(s->dp, state_of(s, a), s->f[b], s->U, s->tune, s->stream, t.start(), t.stop());
      if (e != hipSuccess) return hip_fail(s, e, "collide kernel launch");
    }
    // finite-difference launches alternate the phi/Q buffers; the collision above
    // already read state a
    int src = a;
    const int block = tfan::fd_block(s->tune, s->dp.n_sub);
    for (int done = 0; done < s->dp.n_sub;) {
      const int subs = std::min(block, s->dp.n_sub - done);
      TimedLaunch t(s, block > 1 ? tfan::K_FDN : tfan::K_FD, true);
      hipError_t e = tfan::launch_fd(s->dp, state_of(s, src), state_of(s, 1 - src), s->U, s->tune, subs, s->stream,
                                     t.start(), t.stop());
      if (e != hipSuccess) return hip_fail(s, e, "sub-step kernel launch");
      src = 1 - src;
      done += subs;
    }
    // keep the new populations and fields under one index
    if (src != b) {
      hipError_t e = hipMemcpyAsync(s->phi[b], s->phi[src], (size_t)s->dp.n * sizeof(float),
                                    hipMemcpyDeviceToDevice, s->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(s->q[b], s->q[src], (size_t)2 * s->dp.n * sizeof(float),
                           hipMemcpyDeviceToDevice, s->stream);
      if (e != hipSuccess) return hip_fail(s, e, "field copy");
    }
    s->cur = b;
    s->step += 1;
  }
  return TFAN_OK;
}

int tfan_get_fields(tfan_sim* s, double* phi, double* qxx, double* qxy, double* u_a, double* u_p,
                    double* rho_a, double* rho_p) {
  if (!s) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  const size_t n = (size_t)s->dp.n;
  std::vector<float> tmp;
  int rc;
  if (u_a || u_p || rho_a || rho_p) {
    TimedLaunch t(s, tfan::K_FIELDS);
    hipError_t e = tfan::launch_fields(s->dp, state_of(s, s->cur), s->aux, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "fields kernel launch");
  }
  if (phi && (rc = download(s, phi, s->phi[s->cur], n, tmp))) return rc;
  if (qxx && (rc = download(s, qxx, s->q[s->cur], n, tmp))) return rc;
  if (qxy && (rc = download(s, qxy, s->q[s->cur] + n, n, tmp))) return rc;
  if (rho_a && (rc = download(s, rho_a, s->aux, n, tmp, s->p.rho0))) return rc;
  if (rho_p && (rc = download(s, rho_p, s->aux + n, n, tmp, s->p.rho0))) return rc;
  if (u_a && (rc = download(s, u_a, s->aux + 2 * n, 2 * n, tmp))) return rc;
  if (u_p && (rc = download(s, u_p, s->aux + 4 * n, 2 * n, tmp))) return rc;
  return sync_stream(s, "get_fields");
}

int tfan_diagnostics(tfan_sim* s, tfan_diag* out) {
  if (!s) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!out) return fail(s, TFAN_EINVAL, "out is NULL");
  {
    TimedLaunch t(s, tfan::K_FIELDS);
    hipError_t e = tfan::launch_fields(s->dp, state_of(s, s->cur), s->aux, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "fields kernel launch");
  }
  {
    TimedLaunch t(s, tfan::K_DIAG);
    hipError_t e = tfan::launch_diag(s->dp, state_of(s, s->cur), s->aux, s->partials,
                                     tfan::diag_blocks(s->dp), s->result, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "diagnostics kernel launch");
  }
  double r[tfan::kDiagSlots];
  hipError_t e = hipMemcpyAsync(r, s->result, sizeof(r), hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "diagnostics copy");
  int rc = sync_stream(s, "diagnostics");
  if (rc) return rc;
  out->step = s->step;
  out->nonfinite = (int64_t)r[tfan::D_NONFINITE];
  out->phi_sum = r[tfan::D_PHI];
  out->phi_sq_sum = r[tfan::D_PHI2];
  out->mass_a = r[tfan::D_MASS_A];
  out->mass_p = r[tfan::D_MASS_P];
  out->ke_a = r[tfan::D_KE_A];
  out->ke_p = r[tfan::D_KE_P];
  out->ke_c = r[tfan::D_KE_C];
  out->ua_sq = r[tfan::D_UA2];
  out->uc_sq = r[tfan::D_UC2];
  out->enstrophy_a = r[tfan::D_ENS_A];
  out->enstrophy_c = r[tfan::D_ENS_C];
  out->elastic = r[tfan::D_ELASTIC];
  out->s_mean = r[tfan::D_S] / (double)s->dp.n;
  out->umax = r[tfan::D_UMAX];
  out->phi_absmax = r[tfan::D_PHIMAX];
  if (out->nonfinite > 0) return fail(s, TFAN_ENONFINITE, "state holds non-finite values");
  if (out->umax > 0.3) return fail(s, TFAN_EUNSTABLE, "max |u| exceeds 0.3");
  return TFAN_OK;
}

size_t tfan_state_bytes(const tfan_sim* s) {
  if (!s) return 0;
  return sizeof(int64_t) + (size_t)s->dp.n * (18 * s->pop_bytes + 3 * sizeof(float));
}

int tfan_get_state(tfan_sim* s, void* host, size_t bytes) {
  if (!s) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!host) return fail(s, TFAN_EINVAL, "host buffer is NULL");
  if (bytes < tfan_state_bytes(s)) return fail(s, TFAN_ENOMEM, "host buffer too small");
  const size_t n = (size_t)s->dp.n;
  char* h = (char*)host;
  std::memcpy(h, &s->step, sizeof(int64_t));
  h += sizeof(int64_t);
  const size_t fb = 18 * n * s->pop_bytes;
  hipError_t e = hipMemcpyAsync(h, s->f[s->cur], fb, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h + fb, s->phi[s->cur], n * sizeof(float), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h + fb + n * sizeof(float), s->q[s->cur], 2 * n * sizeof(float),
                       hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "get_state");
  return sync_stream(s, "get_state");
}

int tfan_set_state(tfan_sim* s, const void* host, size_t bytes) {
  if (!s) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!host) return fail(s, TFAN_EINVAL, "host buffer is NULL");
  if (bytes != tfan_state_bytes(s)) return fail(s, TFAN_EINVAL, "state size does not match this grid");
  const size_t n = (size_t)s->dp.n;
  const char* h = (const char*)host;
  int64_t step;
  std::memcpy(&step, h, sizeof(int64_t));
  if (step < 0) return fail(s, TFAN_EINVAL, "negative step counter in state");
  h += sizeof(int64_t);
  s->cur = 0;
  const size_t fb = 18 * n * s->pop_bytes;
  hipError_t e = hipMemcpyAsync(s->f[0], h, fb, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->phi[0], h + fb, n * sizeof(float), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->q[0], h + fb + n * sizeof(float), 2 * n * sizeof(float), hipMemcpyHostToDevice,
                       s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "set_state");
  s->has_state = true;
  s->step = step;
  return sync_stream(s, "set_state");
}

int tfan_sync(tfan_sim* s) {
  if (!s) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  return sync_stream(s, "sync");
}

int64_t tfan_step_count(const tfan_sim* s) { return s ? s->step : -1; }

// A caller's device array must be device memory of this handle's GPU that holds
// `bytes` bytes from ptr on.  An address the HIP runtime does not know as a device
// allocation (host memory, a stale or foreign pointer) is rejected here: passed to a
// runtime copy it would be copied on the CPU, and passed to a kernel it would fault.
static int check_device_range(tfan_sim* s, const void* ptr, size_t bytes, const char* what) {
  hipPointerAttribute_t at{};
  hipError_t e = hipPointerGetAttributes(&at, ptr);
  if (e != hipSuccess || at.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(s, TFAN_EINVAL, std::string(what) + " is not device memory");
  }
  if (at.device != s->device) return fail(s, TFAN_EINVAL, std::string(what) + " is on another device");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(s, TFAN_EINVAL, std::string(what) + ": allocation range unknown");
  }
  if ((const char*)ptr + bytes > (const char*)base + size)
    return fail(s, TFAN_ENOMEM, std::string(what) + " extends past the end of its allocation");
  return TFAN_OK;
}

size_t tfan_exchange_bytes(const tfan_sim* s, int32_t planes) {
  return s && (planes == 7 || planes == 9) ? (size_t)planes * (size_t)s->dp.n * sizeof(float) : 0;
}

int tfan_export_state(tfan_sim* s, float* out, size_t bytes, int32_t planes) {
  if (!s) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (planes != 7 && planes != 9) return fail(s, TFAN_EINVAL, "planes must be 7 or 9");
  if (!out) return fail(s, TFAN_EINVAL, "output array is NULL");
  const size_t need = tfan_exchange_bytes(s, planes);
  if (bytes < need) return fail(s, TFAN_ENOMEM, "output array smaller than `planes` planes of the grid");
  if (int rc = check_device_range(s, out, need, "output array")) return rc;
  const int n = s->dp.n;
  {
    TimedLaunch t(s, tfan::K_FIELDS);
    hipError_t e = tfan::launch_fields(s->dp, state_of(s, s->cur), s->aux, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "fields kernel launch");
  }
  hipError_t e = tfan::launch_pack_state(n, planes, s->phi[s->cur], s->q[s->cur], s->aux, out, s->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(s, e, "state export launch");
}

int tfan_import_state(tfan_sim* s, const float* in, size_t bytes, int32_t planes, int64_t step) {
  if (!s) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (planes != 7 && planes != 9) return fail(s, TFAN_EINVAL, "planes must be 7 or 9");
  if (!in) return fail(s, TFAN_EINVAL, "input array is NULL");
  if (step < 0) return fail(s, TFAN_EINVAL, "step must be >= 0");
  const size_t need = tfan_exchange_bytes(s, planes);
  if (bytes < need) return fail(s, TFAN_ENOMEM, "input array smaller than `planes` planes of the grid");
  if (int rc = check_device_range(s, in, need, "input array")) return rc;
  const int n = s->dp.n;
  // phi, Q go to the spare buffers, the velocities (and densities) to aux; the
  // populations are rebuilt in the spare buffer, which becomes the current state
  const int nxt = s->cur ^ 1;
  hipError_t e = tfan::launch_unpack_state(n, planes, in, s->phi[nxt], s->q[nxt], s->aux, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "state import launch");
  {
    TimedLaunch t(s, tfan::K_INIT);
    const void* keep = planes == 7 && s->has_state ? s->f[s->cur] : nullptr;
    const float* drho = planes == 9 ? s->aux + 4 * (size_t)n : nullptr;
    e = tfan::launch_import(s->dp, keep, state_of(s, nxt), s->aux, drho, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "import kernel launch");
  }
  s->cur = nxt;
  s->step = step;
  s->has_state = true;
  return TFAN_OK;
}

int tfan_kernel_timing(tfan_sim* s, int64_t cap) {
  if (!s) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (cap < 0 || cap > (int64_t(1) << 20)) return fail(s, TFAN_EINVAL, "cap must be in [0, 2^20]");
  int rc = sync_stream(s, "kernel_timing");
  if (rc) return rc;
  free_events(s);
  for (int k = 0; k < tfan::K_COUNT; ++k) { s->ms_total[k] = 0; s->launches[k] = 0; }
  if (cap == 0) return TFAN_OK;
  s->ev.resize(2 * cap);
  s->ev_kernel.resize(cap);
  for (size_t i = 0; i < s->ev.size(); ++i) {
    hipError_t e = hipEventCreate(&s->ev[i]);
    if (e != hipSuccess) {
      s->ev.resize(i);
      free_events(s);
      return hip_fail(s, e, "hipEventCreate");
    }
  }
  s->ev_cap = cap;
  return TFAN_OK;
}

int tfan_kernel_times(tfan_sim* s, double* ms_total, int64_t* launches, int n) {
  if (!s) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (n < 0 || n > tfan::K_COUNT || (n > 0 && (!ms_total || !launches)))
    return fail(s, TFAN_EINVAL, "bad output arrays");
  int rc = sync_stream(s, "kernel_times");
  if (rc) return rc;
  harvest(s);
  for (int k = 0; k < n; ++k) {
    ms_total[k] = s->ms_total[k];
    launches[k] = s->launches[k];
  }
  return TFAN_OK;
}

int tfan_set_tuning(tfan_sim* s, int32_t collide_rows, int32_t fd_shape) {
  if (!s) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!valid_shape(collide_rows, fd_shape)) return fail(s, TFAN_EINVAL, kShapeMsg);
  s->tune.collide_rows = collide_rows;
  s->tune.fd_shape = fd_shape;
  return TFAN_OK;
}

int tfan_get_tuning(const tfan_sim* s, int32_t* collide_rows, int32_t* fd_shape) {
  if (!s || !collide_rows || !fd_shape) return fail(nullptr, TFAN_EINVAL, "NULL argument");
  *collide_rows = s->tune.collide_rows;
  *fd_shape = s->tune.fd_shape;
  return TFAN_OK;
}

int tfan_autotune(tfan_sim* s, int32_t steps, double* best_ms_per_step) {
  if (!s) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (steps < 1 || steps > 100000) return fail(s, TFAN_EINVAL, "steps must be in [1, 100000]");
  std::vector<unsigned char> ck(tfan_state_bytes(s));
  int rc = tfan_get_state(s, ck.data(), ck.size());
  if (rc) return rc;
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(s, e, "autotune events");
  tfan::Tuning best = s->tune;
  float best_ms = -1.f;
  for (const tfan::Tuning& cand : tuning_candidates(s->dp.n_sub)) {
      s->tune = cand;
      if ((rc = tfan_step(s, 1))) break;  // warm-up
      (void)hipEventRecord(e0, s->stream);
      if ((rc = tfan_step(s, steps))) break;
      (void)hipEventRecord(e1, s->stream);
      if ((rc = sync_stream(s, "autotune"))) break;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (best_ms < 0.f || ms < best_ms) {
        best_ms = ms;
        best = s->tune;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  s->tune = best;
  const int rc2 = tfan_set_state(s, ck.data(), ck.size());
  if (rc) return rc;
  if (rc2) return rc2;
  if (best_ms_per_step) *best_ms_per_step = best_ms / steps;
  return TFAN_OK;
}

int tfan_kernel_count(void) { return tfan::K_COUNT; }

const char* tfan_kernel_name(int id) {
  static const char* names[tfan::K_COUNT] = {"collide", "substep", "init", "fields", "diagnostics", "substeps"};
  return (id >= 0 && id < tfan::K_COUNT) ? names[id] : "";
}

void tfan_destroy(tfan_sim* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  free_events(s);
  delete s;
}

const char* tfan_last_error(const tfan_sim* s) { return s ? s->err.c_str() : g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: independent members with their own grids and parameters (equal
// n_sub and storage), advanced together by one collision launch and one launch
// per sub-step over the tiles of all members.
// ---------------------------------------------------------------------------
struct tfan_batch {
  std::vector<tfan_sim*> m;
  hipStream_t stream = nullptr;
  tfan::BatchMember* table = nullptr;  // device
  int* first_c = nullptr;              // device [count]
  int* first_f = nullptr;              // device [count]
  int tiles_c = 0, tiles_f = 0;
  int* first_pc = nullptr;             // device [count]: tiles of the persistent launch's phases
  int* first_pf = nullptr;
  int tiles_pc = 0, tiles_pf = 0;
  int persist_grid = 0;                // blocks of the last persistent launch
  int cur = 0;
  int64_t step = 0;
  tfan::Tuning tune;
  bool pop16 = false;
  int n_sub = 0;
  std::string err;
};

namespace {

int bfail(tfan_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg; else g_err = msg;
  return code;
}

size_t batch_table_bytes(int count) {
  return align_up(count * sizeof(tfan::BatchMember)) + 4 * align_up(count * sizeof(int));
}

int upload_first(tfan_batch* b) {
  std::vector<int> fc(b->m.size()), ff(b->m.size());
  int tc = 0, tf = 0;
  for (size_t i = 0; i < b->m.size(); ++i) {
    fc[i] = tc;
    ff[i] = tf;
    tc += tfan::batch_tiles(b->m[i]->dp, b->tune, true);
    tf += tfan::batch_tiles(b->m[i]->dp, b->tune, false);
  }
  b->tiles_c = tc;
  b->tiles_f = tf;
  std::vector<int> pc(b->m.size()), pf(b->m.size());
  int tpc = 0, tpf = 0;
  for (size_t i = 0; i < b->m.size(); ++i) {
    pc[i] = tpc;
    pf[i] = tpf;
    tpc += tfan::persist_collide_tiles(b->m[i]->dp);
    tpf += tfan::persist_fd_tiles(b->m[i]->dp);
  }
  b->tiles_pc = tpc;
  b->tiles_pf = tpf;
  hipError_t e = hipMemcpyAsync(b->first_c, fc.data(), fc.size() * sizeof(int), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->first_f, ff.data(), ff.size() * sizeof(int), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->first_pc, pc.data(), pc.size() * sizeof(int), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->first_pf, pf.data(), pf.size() * sizeof(int), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, TFAN_EHIP, std::string("batch tables: ") + hipGetErrorString(e));
  return TFAN_OK;
}

int member_check(tfan_batch* b, int32_t member) {
  if (!b) return bfail(nullptr, TFAN_EINVAL, "batch is NULL");
  if (member < 0 || member >= (int32_t)b->m.size()) return bfail(b, TFAN_EINVAL, "member out of range");
  return TFAN_OK;
}

// A member re-initialised (state in buffer 0) while the batch holds its state in
// buffer 1: copy it across so that all members share one ping-pong index.
int align_member(tfan_batch* b, tfan_sim* s) {
  if (s->cur == b->cur) return TFAN_OK;
  const size_t n = (size_t)s->dp.n;
  hipError_t e = hipMemcpyAsync(s->f[b->cur], s->f[s->cur], 18 * n * s->pop_bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->phi[b->cur], s->phi[s->cur], n * sizeof(float), hipMemcpyDeviceToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->q[b->cur], s->q[s->cur], 2 * n * sizeof(float), hipMemcpyDeviceToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, TFAN_EHIP, std::string("batch align: ") + hipGetErrorString(e));
  s->cur = b->cur;
  return TFAN_OK;
}

}  // namespace

extern "C" {

size_t tfan_batch_workspace_bytes(const tfan_params* p, int32_t count) {
  if (!p || count < 1 || count > 4096) return 0;
  size_t total = batch_table_bytes(count);
  for (int i = 0; i < count; ++i) {
    const size_t w = tfan_workspace_bytes(p + i);
    if (!w) return 0;
    total += align_up(w);
  }
  return total;
}

int tfan_batch_create(const tfan_params* p, int32_t count, void* ws, size_t bytes, void* stream,
                      tfan_batch** out) {
  if (!out) return bfail(nullptr, TFAN_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p || count < 1 || count > 4096) return bfail(nullptr, TFAN_EINVAL, "count must be in [1, 4096]");
  for (int i = 0; i < count; ++i) {
    const std::string m = check(p + i);
    if (!m.empty()) return bfail(nullptr, TFAN_EINVAL, "member " + std::to_string(i) + ": " + m);
    if (p[i].n_sub != p[0].n_sub || p[i].storage != p[0].storage)
      return bfail(nullptr, TFAN_EINVAL, "all members need the same n_sub and storage");
  }
  const size_t need = tfan_batch_workspace_bytes(p, count);
  if (!ws) return bfail(nullptr, TFAN_EINVAL, "workspace is NULL");
  if (((uintptr_t)ws) % kAlign) return bfail(nullptr, TFAN_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < need) return bfail(nullptr, TFAN_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  tfan_batch* b = new tfan_batch();
  b->stream = (hipStream_t)stream;
  char* base = (char*)ws;
  b->table = (tfan::BatchMember*)base;
  b->first_c = (int*)(base + align_up(count * sizeof(tfan::BatchMember)));
  b->first_f = (int*)((char*)b->first_c + align_up(count * sizeof(int)));
  b->first_pc = (int*)((char*)b->first_f + align_up(count * sizeof(int)));
  b->first_pf = (int*)((char*)b->first_pc + align_up(count * sizeof(int)));
  size_t off = batch_table_bytes(count);
  std::vector<tfan::BatchMember> host(count);
  for (int i = 0; i < count; ++i) {
    const size_t w = tfan_workspace_bytes(p + i);
    tfan_sim* s = nullptr;
    int rc = tfan_create(p + i, base + off, w, stream, &s);
    if (rc) {
      for (tfan_sim* t : b->m) tfan_destroy(t);
      delete b;
      return rc;
    }
    off += align_up(w);
    b->m.push_back(s);
    host[i].P = s->dp;
    host[i].st[0] = state_of(s, 0);
    host[i].st[1] = state_of(s, 1);
    host[i].U = s->U;
  }
  b->pop16 = p[0].storage == TFAN_STORAGE_F16;
  b->n_sub = p[0].n_sub;
  hipError_t e = hipMemcpyAsync(b->table, host.data(), count * sizeof(tfan::BatchMember), hipMemcpyHostToDevice,
                                b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  int rc = e == hipSuccess ? upload_first(b) : bfail(b, TFAN_EHIP, hipGetErrorString(e));
  if (rc) {
    g_err = b->err;
    for (tfan_sim* t : b->m) tfan_destroy(t);
    delete b;
    return rc;
  }
  *out = b;
  return TFAN_OK;
}

int tfan_batch_count(const tfan_batch* b) { return b ? (int)b->m.size() : -1; }

int tfan_batch_init_fields(tfan_batch* b, int32_t member, const double* phi, const double* qxx,
                           const double* qxy, const double* u_a, const double* u_p) {
  int rc = member_check(b, member);
  if (rc) return rc;
  tfan_sim* s = b->m[member];
  rc = tfan_init_fields(s, phi, qxx, qxy, u_a, u_p);
  if (rc) return bfail(b, rc, s->err);
  return align_member(b, s);
}

int tfan_batch_step(tfan_batch* b, int64_t nsteps) {
  if (!b) return bfail(nullptr, TFAN_EINVAL, "batch is NULL");
  if (nsteps < 0) return bfail(b, TFAN_EINVAL, "step count must be >= 0");
  const int count = (int)b->m.size();
  for (int64_t k = 0; k < nsteps; ++k) {
    hipError_t e = tfan::launch_collide_batch(b->table, b->first_c, count, b->tiles_c, b->cur, b->pop16, b->tune,
                                              b->stream);
    if (e != hipSuccess) return bfail(b, TFAN_EHIP, std::string("batch collide launch: ") + hipGetErrorString(e));
    int src = b->cur;
    const int block = tfan::fd_block(b->tune, b->n_sub);
    for (int done = 0; done < b->n_sub;) {
      const int subs = std::min(block, b->n_sub - done);
      e = tfan::launch_fd_batch(b->table, b->first_f, count, b->tiles_f, src, b->tune, b->n_sub, subs, b->stream);
      if (e != hipSuccess) return bfail(b, TFAN_EHIP, std::string("batch sub-step launch: ") + hipGetErrorString(e));
      src = 1 - src;
      done += subs;
    }
    const int nb = 1 - b->cur;
    if (src != nb) {
      for (tfan_sim* s : b->m) {
        const size_t n = (size_t)s->dp.n;
        e = hipMemcpyAsync(s->phi[nb], s->phi[src], n * sizeof(float), hipMemcpyDeviceToDevice, b->stream);
        if (e == hipSuccess)
          e = hipMemcpyAsync(s->q[nb], s->q[src], 2 * n * sizeof(float), hipMemcpyDeviceToDevice, b->stream);
        if (e != hipSuccess) return bfail(b, TFAN_EHIP, std::string("batch field copy: ") + hipGetErrorString(e));
      }
    }
    b->cur = nb;
    b->step += 1;
    for (tfan_sim* s : b->m) {
      s->cur = nb;
      s->step += 1;
    }
  }
  return TFAN_OK;
}

int tfan_batch_step_persistent(tfan_batch* b, int64_t nsteps) {
  if (!b) return bfail(nullptr, TFAN_EINVAL, "batch is NULL");
  if (nsteps < 0 || nsteps > INT32_MAX) return bfail(b, TFAN_EINVAL, "step count must be in [0, 2^31)");
  if (b->n_sub > tfan::kFusedMaxSub)
    return bfail(b, TFAN_EINVAL, "the persistent launch takes n_sub <= 5 (all sub-steps of a step in one phase)");
  if (nsteps == 0) return TFAN_OK;
  hipError_t e = tfan::launch_batch_persistent(b->table, b->first_pc, b->first_pf, (int)b->m.size(), b->tiles_pc,
                                               b->tiles_pf, (int)nsteps, b->cur, b->n_sub, b->pop16, &b->persist_grid,
                                               b->stream);
  if (e != hipSuccess) return bfail(b, TFAN_EHIP, std::string("persistent batch launch: ") + hipGetErrorString(e));
  // one sub-step phase per step: the fields alternate with the populations
  const int nb = (int)((b->cur + nsteps) % 2);
  b->cur = nb;
  b->step += nsteps;
  for (tfan_sim* s : b->m) {
    s->cur = nb;
    s->step += nsteps;
  }
  return TFAN_OK;
}

int tfan_batch_get_fields(tfan_batch* b, int32_t member, double* phi, double* qxx, double* qxy, double* u_a,
                          double* u_p, double* rho_a, double* rho_p) {
  int rc = member_check(b, member);
  if (rc) return rc;
  rc = tfan_get_fields(b->m[member], phi, qxx, qxy, u_a, u_p, rho_a, rho_p);
  return rc ? bfail(b, rc, b->m[member]->err) : TFAN_OK;
}

int tfan_batch_diagnostics(tfan_batch* b, int32_t member, tfan_diag* out) {
  int rc = member_check(b, member);
  if (rc) return rc;
  rc = tfan_diagnostics(b->m[member], out);
  if (rc) b->err = b->m[member]->err;
  return rc;
}

int tfan_batch_set_tuning(tfan_batch* b, int32_t collide_rows, int32_t fd_shape) {
  if (!b) return bfail(nullptr, TFAN_EINVAL, "batch is NULL");
  if (!valid_shape(collide_rows, fd_shape)) return bfail(b, TFAN_EINVAL, kShapeMsg);
  b->tune.collide_rows = collide_rows;
  b->tune.fd_shape = fd_shape;
  return upload_first(b);
}

int tfan_batch_get_tuning(const tfan_batch* b, int32_t* collide_rows, int32_t* fd_shape) {
  if (!b || !collide_rows || !fd_shape) return bfail(nullptr, TFAN_EINVAL, "NULL argument");
  *collide_rows = b->tune.collide_rows;
  *fd_shape = b->tune.fd_shape;
  return TFAN_OK;
}

int tfan_batch_autotune(tfan_batch* b, int32_t steps, double* best_ms_per_step) {
  if (!b) return bfail(nullptr, TFAN_EINVAL, "batch is NULL");
  if (steps < 1 || steps > 100000) return bfail(b, TFAN_EINVAL, "steps must be in [1, 100000]");
  std::vector<std::vector<unsigned char>> ck(b->m.size());
  for (size_t i = 0; i < b->m.size(); ++i) {
    ck[i].resize(tfan_state_bytes(b->m[i]));
    int rc = tfan_get_state(b->m[i], ck[i].data(), ck[i].size());
    if (rc) return bfail(b, rc, b->m[i]->err);
  }
  const int64_t step0 = b->step;
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return bfail(b, TFAN_EHIP, "autotune events");
  tfan::Tuning best = b->tune;
  float best_ms = -1.f;
  int rc = TFAN_OK;
  for (const tfan::Tuning& cand : tuning_candidates(b->n_sub)) {
      if ((rc = tfan_batch_set_tuning(b, cand.collide_rows, cand.fd_shape))) break;
      if ((rc = tfan_batch_step(b, 1))) break;
      (void)hipEventRecord(e0, b->stream);
      if ((rc = tfan_batch_step(b, steps))) break;
      (void)hipEventRecord(e1, b->stream);
      if (hipStreamSynchronize(b->stream) != hipSuccess) { rc = bfail(b, TFAN_EHIP, "autotune sync"); break; }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (best_ms < 0.f || ms < best_ms) {
        best_ms = ms;
        best = b->tune;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // restore: every member back to its checkpoint, in buffer 0
  for (size_t i = 0; i < b->m.size(); ++i) {
    const int r2 = tfan_set_state(b->m[i], ck[i].data(), ck[i].size());
    if (r2 && !rc) rc = bfail(b, r2, b->m[i]->err);
  }
  b->cur = 0;
  b->step = step0;
  const int r3 = tfan_batch_set_tuning(b, best.collide_rows, best.fd_shape);
  if (rc) return rc;
  if (r3) return r3;
  if (best_ms_per_step) *best_ms_per_step = best_ms / steps;
  return TFAN_OK;
}

int tfan_batch_sync(tfan_batch* b) {
  if (!b) return bfail(nullptr, TFAN_EINVAL, "batch is NULL");
  hipError_t e = hipStreamSynchronize(b->stream);
  return e == hipSuccess ? TFAN_OK : bfail(b, TFAN_EHIP, std::string("batch sync: ") + hipGetErrorString(e));
}

void tfan_batch_destroy(tfan_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  for (tfan_sim* s : b->m) tfan_destroy(s);
  delete b;
}

const char* tfan_batch_last_error(const tfan_batch* b) { return b ? b->err.c_str() : g_err.c_str(); }

}  // extern "C"

extern "C" int tfan_batch_persistent_blocks(const tfan_batch* b) { return b ? b->persist_grid : 0; }
