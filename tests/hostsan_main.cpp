// Host-side validation paths of libtfan (tfan.h, tfan_cnn.h, tfan_analysis.h),
// built with AddressSanitizer and UndefinedBehaviorSanitizer on the host code by
// tests/test_host_sanitize.py.  Every call here returns before any device work:
// parameter checks, workspace sizes, handle set-up on a host stand-in buffer
// that the library never dereferences, argument checks on NULL handles, and the
// host-array scans of tfan_init_fields.  Exit code 0 when every result is the
// documented one; sanitizer reports abort the run.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "tfan.h"
#include "tfan_analysis.h"
#include "tfan_cnn.h"

static int g_fail = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::fprintf(stderr, "line %d: expected %s\n", __LINE__, #cond); \
      ++g_fail;                                                        \
    }                                                                  \
  } while (0)

static tfan_params valid(int nx, int ny) {
  tfan_params p{};
  p.nx = nx;
  p.ny = ny;
  p.n_sub = 5;
  p.storage = TFAN_STORAGE_F32;
  p.rho0 = 1.0;
  p.tau_a = p.tau_p = 1.0;
  p.gamma = 0.01;
  p.A_ch = 0.04;
  p.kappa = 0.04;
  p.M = 0.1;
  p.A0 = 0.1;
  p.gamma_ldg = 3.0;
  p.K = 0.04;
  p.lam = 0.7;
  p.Gamma = 0.34;
  p.zeta = 0.005;
  return p;
}

static void params_checks() {
  EXPECT(tfan_check_params(nullptr) == TFAN_EINVAL);
  EXPECT(std::strlen(tfan_last_error(nullptr)) > 0);
  tfan_params p = valid(64, 48);
  EXPECT(tfan_check_params(&p) == TFAN_OK);
  struct Bad { void (*apply)(tfan_params*); } bad[] = {
      {[](tfan_params* q) { q->nx = 7; }},         {[](tfan_params* q) { q->ny = 32769; }},
      {[](tfan_params* q) { q->nx = 32768; q->ny = 16384; }},
      {[](tfan_params* q) { q->n_sub = 0; }},      {[](tfan_params* q) { q->n_sub = 9; }},
      {[](tfan_params* q) { q->storage = 2; }},    {[](tfan_params* q) { q->rho0 = 0.0; }},
      {[](tfan_params* q) { q->tau_a = 0.5; }},    {[](tfan_params* q) { q->tau_p = 0.2; }},
      {[](tfan_params* q) { q->gamma = -1e-3; }},  {[](tfan_params* q) { q->kappa = -1.0; }},
      {[](tfan_params* q) { q->M = -0.1; }},       {[](tfan_params* q) { q->K = -0.04; }},
      {[](tfan_params* q) { q->Gamma = -1.0; }},   {[](tfan_params* q) { q->zeta = NAN; }},
      {[](tfan_params* q) { q->A0 = INFINITY; }},  {[](tfan_params* q) { q->gamma_ldg = NAN; }},
      {[](tfan_params* q) { q->lam = -INFINITY; }}, {[](tfan_params* q) { q->A_ch = NAN; }},
  };
  for (const Bad& b : bad) {
    tfan_params q = valid(64, 48);
    b.apply(&q);
    EXPECT(tfan_check_params(&q) == TFAN_EINVAL);
    EXPECT(tfan_workspace_bytes(&q) == 0);
  }
  // sizes: the 8 x 8 minimum and the 2^28-site maximum, both storage formats
  tfan_params lo = valid(8, 8), hi = valid(32768, 8192);
  EXPECT(tfan_workspace_bytes(&lo) > 0);
  const size_t w32 = tfan_workspace_bytes(&hi);
  hi.storage = TFAN_STORAGE_F16;
  const size_t w16 = tfan_workspace_bytes(&hi);
  EXPECT(w32 > w16 && w16 > ((size_t)1 << 28) * 36);
}

static void handle_checks() {
  tfan_params p = valid(40, 24);
  const size_t need = tfan_workspace_bytes(&p);
  tfan_sim* s = nullptr;
  EXPECT(tfan_create(&p, nullptr, need, nullptr, nullptr) == TFAN_EINVAL);
  EXPECT(tfan_create(&p, nullptr, need, nullptr, &s) == TFAN_EINVAL && s == nullptr);
  // host stand-in for the device workspace: create only records the address
  void* ws = std::aligned_alloc(256, need + 256);
  EXPECT(tfan_create(&p, (char*)ws + 16, need, nullptr, &s) == TFAN_EINVAL);
  EXPECT(tfan_create(&p, ws, need - 1, nullptr, &s) == TFAN_ENOMEM);
  tfan_params badp = valid(40, 24);
  badp.tau_a = 0.4;
  EXPECT(tfan_create(&badp, ws, need, nullptr, &s) == TFAN_EINVAL);
  EXPECT(tfan_create(&p, ws, need, nullptr, &s) == TFAN_OK && s != nullptr);
  const size_t n = 40 * 24;
  std::vector<double> f(n, 0.0), v(2 * n, 0.0);
  EXPECT(tfan_init_fields(s, nullptr, f.data(), f.data(), nullptr, nullptr) == TFAN_EINVAL);
  f[n - 1] = NAN;  // the last element: the scan covers every site
  EXPECT(tfan_init_fields(s, f.data(), f.data(), f.data(), nullptr, nullptr) == TFAN_EINVAL);
  f[n - 1] = 0.0;
  v[2 * n - 1] = INFINITY;
  EXPECT(tfan_init_fields(s, f.data(), f.data(), f.data(), v.data(), nullptr) == TFAN_EINVAL);
  EXPECT(tfan_init_fields(s, f.data(), f.data(), f.data(), nullptr, v.data()) == TFAN_EINVAL);
  EXPECT(std::strlen(tfan_last_error(s)) > 0);
  EXPECT(tfan_step(s, -1) == TFAN_EINVAL);
  EXPECT(tfan_set_tuning(s, 3, 165) == TFAN_EINVAL);
  EXPECT(tfan_set_tuning(s, 1, 17) == TFAN_EINVAL);
  EXPECT(tfan_set_tuning(s, 2, 32) == TFAN_OK);
  int32_t cr = 0, fs = 0;
  EXPECT(tfan_get_tuning(s, &cr, &fs) == TFAN_OK && cr == 2 && fs == 32);
  EXPECT(tfan_get_tuning(s, nullptr, &fs) == TFAN_EINVAL);
  EXPECT(tfan_autotune(s, 0, nullptr) == TFAN_EINVAL);
  const size_t sb = tfan_state_bytes(s);
  EXPECT(sb == sizeof(int64_t) + n * (18 * 4 + 12));
  std::vector<unsigned char> st(sb, 0);
  EXPECT(tfan_get_state(s, st.data(), sb - 1) == TFAN_ENOMEM);
  EXPECT(tfan_get_state(s, nullptr, sb) == TFAN_EINVAL);
  EXPECT(tfan_set_state(s, st.data(), sb + 1) == TFAN_EINVAL);
  const int64_t neg = -5;
  std::memcpy(st.data(), &neg, sizeof neg);
  EXPECT(tfan_set_state(s, st.data(), sb) == TFAN_EINVAL);
  EXPECT(tfan_exchange_bytes(s, 7) == 7 * n * 4);
  EXPECT(tfan_exchange_bytes(s, 9) == 9 * n * 4);
  EXPECT(tfan_exchange_bytes(s, 8) == 0);
  EXPECT(tfan_export_state(s, nullptr, 7 * n * 4, 7) == TFAN_EINVAL);
  std::vector<float> xs(9 * n);
  EXPECT(tfan_export_state(s, xs.data(), 9 * n * 4, 8) == TFAN_EINVAL);
  EXPECT(tfan_export_state(s, xs.data(), 7 * n * 4 - 4, 7) == TFAN_ENOMEM);
  EXPECT(tfan_export_state(s, xs.data(), 7 * n * 4, 9) == TFAN_ENOMEM);
  EXPECT(tfan_import_state(s, xs.data(), 7 * n * 4, 7, -1) == TFAN_EINVAL);
  EXPECT(tfan_import_state(s, xs.data(), 9 * n * 4, 0, 0) == TFAN_EINVAL);
  EXPECT(tfan_import_state(s, xs.data(), 3, 7, 0) == TFAN_ENOMEM);
  EXPECT(tfan_kernel_timing(s, -1) == TFAN_EINVAL);
  EXPECT(tfan_kernel_timing(s, (int64_t(1) << 20) + 1) == TFAN_EINVAL);
  EXPECT(tfan_step_count(s) == 0);
  tfan_destroy(s);
  std::free(ws);
}

static void null_handles() {
  double d = 0;
  tfan_diag dg;
  EXPECT(tfan_step(nullptr, 1) == TFAN_EINVAL);
  EXPECT(tfan_init_fields(nullptr, &d, &d, &d, nullptr, nullptr) == TFAN_EINVAL);
  EXPECT(tfan_get_fields(nullptr, &d, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == TFAN_EINVAL);
  EXPECT(tfan_diagnostics(nullptr, &dg) == TFAN_EINVAL);
  EXPECT(tfan_sync(nullptr) == TFAN_EINVAL);
  EXPECT(tfan_state_bytes(nullptr) == 0 && tfan_exchange_bytes(nullptr, 7) == 0);
  EXPECT(tfan_step_count(nullptr) == -1);
  EXPECT(tfan_set_tuning(nullptr, 1, 165) == TFAN_EINVAL);
  EXPECT(tfan_export_state(nullptr, nullptr, 0, 7) == TFAN_EINVAL);
  EXPECT(tfan_import_state(nullptr, nullptr, 0, 7, 0) == TFAN_EINVAL);
  tfan_destroy(nullptr);
  EXPECT(tfan_kernel_count() > 0);
  for (int k = -1; k <= tfan_kernel_count(); ++k) {
    const char* nm = tfan_kernel_name(k);
    EXPECT(nm != nullptr);
    EXPECT((k >= 0 && k < tfan_kernel_count()) == (nm && nm[0] != 0));
  }
}

static void batch_checks() {
  std::vector<tfan_params> p = {valid(128, 128), valid(256, 256), valid(64, 96)};
  EXPECT(tfan_batch_workspace_bytes(p.data(), 0) == 0);
  EXPECT(tfan_batch_workspace_bytes(p.data(), 4097) == 0);
  EXPECT(tfan_batch_workspace_bytes(nullptr, 2) == 0);
  size_t sum = 0;
  for (auto& q : p) sum += tfan_workspace_bytes(&q);
  EXPECT(tfan_batch_workspace_bytes(p.data(), 3) >= sum);
  tfan_batch* b = nullptr;
  EXPECT(tfan_batch_create(p.data(), 3, nullptr, 0, nullptr, nullptr) == TFAN_EINVAL);
  p[2].n_sub = 4;
  EXPECT(tfan_batch_create(p.data(), 3, nullptr, 0, nullptr, &b) == TFAN_EINVAL && b == nullptr);
  p[2].n_sub = 5;
  p[1].storage = TFAN_STORAGE_F16;
  EXPECT(tfan_batch_create(p.data(), 3, nullptr, 0, nullptr, &b) == TFAN_EINVAL);
  p[1].storage = TFAN_STORAGE_F32;
  p[0].nx = 4;
  EXPECT(tfan_batch_create(p.data(), 3, nullptr, 0, nullptr, &b) == TFAN_EINVAL);
  p[0].nx = 128;
  EXPECT(tfan_batch_create(p.data(), 3, nullptr, 1 << 20, nullptr, &b) == TFAN_EINVAL);
  EXPECT(std::strlen(tfan_batch_last_error(nullptr)) > 0);
  EXPECT(tfan_batch_step(nullptr, 1) == TFAN_EINVAL);
  tfan_batch_destroy(nullptr);
}

static void cnn_checks() {
  EXPECT(tfan_cnn_param_count() == 89239);
  EXPECT(tfan_cnn_workspace_bytes(0, 64, 64, 0) == 0);
  EXPECT(tfan_cnn_workspace_bytes(1, 63, 64, 0) == 0);
  EXPECT(tfan_cnn_workspace_bytes(1, 64, 40, 1) == 0);
  const size_t inf = tfan_cnn_workspace_bytes(2, 64, 48, 0), tr = tfan_cnn_workspace_bytes(2, 64, 48, 1);
  EXPECT(inf > 0 && tr > inf);
  tfan_cnn* c = nullptr;
  EXPECT(tfan_cnn_create(1, 64, 64, 0, nullptr, 0, nullptr, nullptr) == TFAN_EINVAL);
  EXPECT(tfan_cnn_create(1, 60, 64, 0, nullptr, 0, nullptr, &c) == TFAN_EINVAL && c == nullptr);
  void* ws = std::aligned_alloc(256, 4096);
  EXPECT(tfan_cnn_create(1, 64, 64, 0, ws, 4096, nullptr, &c) == TFAN_ENOMEM);
  std::free(ws);
  tfan_cnn_destroy(nullptr);
}

static void analysis_checks() {
  for (int n : {0, 4, 7, 12, 8192, -8}) {
    EXPECT(tfan_analysis_shells(n) == 0);
    EXPECT(tfan_analysis_workspace_bytes(n) == 0);
  }
  for (int n = 8; n <= 4096; n *= 2) {
    // the largest shell index is the integer nearest to (n/2) sqrt(2)
    const int expect = (int)std::floor(0.5 * n * std::sqrt(2.0) + 0.5) + 1;
    EXPECT(tfan_analysis_shells(n) == expect);
    EXPECT(tfan_analysis_workspace_bytes(n) > (size_t)n * n * 8);
  }
  tfan_analysis* a = nullptr;
  EXPECT(tfan_analysis_create(12, nullptr, 0, nullptr, &a) == TFAN_EINVAL && a == nullptr);
  EXPECT(tfan_analysis_create(64, nullptr, 0, nullptr, nullptr) == TFAN_EINVAL);
  void* ws = std::aligned_alloc(256, 4096);
  EXPECT(tfan_analysis_create(64, ws, 4096, nullptr, &a) == TFAN_ENOMEM);
  std::free(ws);
  tfan_analysis_destroy(nullptr);
  double out[6];
  float dummy[8];
  for (int n : {7, 12, 4, 8192})
    EXPECT(tfan_analysis_overlaps_noalloc(n, dummy, dummy, out, nullptr) == TFAN_EINVAL);
  EXPECT(tfan_analysis_overlaps_noalloc(64, nullptr, dummy, out, nullptr) == TFAN_EINVAL);
  EXPECT(tfan_analysis_overlaps_noalloc(64, dummy, dummy, nullptr, nullptr) == TFAN_EINVAL);
  EXPECT(std::strlen(tfan_analysis_noalloc_last_error()) > 0);
}

int main() {
  params_checks();
  handle_checks();
  null_handles();
  batch_checks();
  cnn_checks();
  analysis_checks();
  if (g_fail) {
    std::fprintf(stderr, "%d host checks failed\n", g_fail);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
