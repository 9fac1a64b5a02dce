// Host side of the observables' C ABI (include/tfan_analysis.h): workspace layout
// and the kernel sequences of the spectra, correlations, overlaps and defects.
#include "tfan_analysis.h"

#include <cstring>
#include <string>
#include <vector>

#include "analysis_internal.h"

namespace {

std::string g_err;
constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int log2_exact(int32_t n) {
  if (n < 8 || n > 4096 || (n & (n - 1))) return -1;
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Nearest integer to sqrt(m2), exactly.
int shell_of(long long m2) {
  long long s = 0;
  while ((s + 1) * (s + 1) <= m2) ++s;
  return (int)((m2 >= s * s + s + 1) ? s + 1 : s);
}

struct Plan {
  size_t z[3], scratch, w[2], pE, pS, partial, pcount, out, red, dpart, res, tw, total;
};

Plan plan(int n, int ns) {
  Plan p{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align_up(bytes);
    return at;
  };
  const size_t c = (size_t)n * n * 8, r = (size_t)n * n * 4;
  for (auto& z : p.z) z = take(c);
  p.scratch = take(c);
  p.w[0] = take(c);
  p.w[1] = take(c);
  p.pE = take(r);
  p.pS = take(r);
  const size_t nb = (size_t)(n + 255) / 256;  // row blocks of the shell sums
  p.partial = take(3 * nb * ns * 8);
  p.pcount = take(nb * ns * 4);
  p.out = take(6 * 8);  // overlaps
  p.red = take((size_t)tana::reduce_blocks(n) * 6 * 8 + 64);
  p.dpart = take((size_t)tana::reduce_blocks(n) * 2 * 8);
  p.res = take((size_t)(8 * ns + 3) * 8);
  p.tw = take((size_t)(n / 2) * 8);
  p.total = o;
  return p;
}

}  // namespace

struct tfan_analysis {
  int n = 0, logn = 0, ns = 0;
  hipStream_t stream = nullptr;
  char* base = nullptr;
  Plan p{};
  std::string err;
  std::vector<double> host;  // staging of the result block
  template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
  const float2* twiddles() const { return at<float2>(p.tw); }
  // Result block on the device: spectra E, S, W, count, L (4 ns + 1), then the
  // correlations Cuu, Cww, CQQ, count (4 ns), then the defect counts (2), so that
  // any call reads its results back in one copy.
  size_t corr_at() const { return (size_t)4 * ns + 1; }
  size_t def_at() const { return (size_t)8 * ns + 1; }
  double* res(size_t at_) const { return at<double>(p.res) + at_; }
};

namespace {

int fail(tfan_analysis* a, int code, const std::string& msg) {
  if (a) a->err = msg; else g_err = msg;
  return code;
}
int hip_fail(tfan_analysis* a, hipError_t e, const char* where) {
  return fail(a, TFAN_EHIP, std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}
int copy_out(tfan_analysis* a, double* dst, const double* src, size_t count) {
  if (!dst) return TFAN_OK;
  hipError_t e = hipMemcpyAsync(dst, src, count * 8, hipMemcpyDeviceToHost, a->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(a, e, "read-back");
}
int finish(tfan_analysis* a) {
  hipError_t e = hipStreamSynchronize(a->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(a, e, "analysis");
}

// Pack and forward-transform the three complex fields; the transforms land
// transposed in scratch, z[0] and z[1], and the powers (pE, pS, w0, w1) keep that
// layout (every later use is symmetric in the two axes).  z[2] is free afterwards.
int transforms(tfan_analysis* a, const float* s) {
  float2* z[3] = {a->at<float2>(a->p.z[0]), a->at<float2>(a->p.z[1]), a->at<float2>(a->p.z[2])};
  float2* scratch = a->at<float2>(a->p.scratch);
  hipError_t e = tana::launch_pack(s, a->n, z[0], z[1], z[2], a->stream);
  if (e == hipSuccess) e = tana::launch_fft2t(z[0], scratch, a->n, a->logn, false, a->twiddles(), a->stream);
  if (e == hipSuccess) e = tana::launch_fft2t(z[1], z[0], a->n, a->logn, false, a->twiddles(), a->stream);
  if (e == hipSuccess) e = tana::launch_fft2t(z[2], z[1], a->n, a->logn, false, a->twiddles(), a->stream);
  if (e == hipSuccess)
    e = tana::launch_power(scratch, z[0], z[1], a->n, a->at<float>(a->p.pE), a->at<float>(a->p.pS),
                           a->at<float2>(a->p.w[0]), a->at<float2>(a->p.w[1]), a->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(a, e, "transforms");
}

// Shell sums of the spectra and L from the transforms, into the result block.
int spectra_enqueue(tfan_analysis* a) {
  double* out = a->res(0);
  hipError_t e = tana::launch_shells(a->at<float>(a->p.pE), a->at<float>(a->p.pS), nullptr, 1, a->n, a->ns, false,
                                     a->at<double>(a->p.partial), a->at<int>(a->p.pcount), out, a->stream);
  if (e == hipSuccess) e = tana::launch_finish_spectra(out, a->n, a->ns, a->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(a, e, "spectra");
}

// Inverse transforms of the (transposed) powers, which come out in natural
// layout, and their shell means, into the result block.
int correlations_enqueue(tfan_analysis* a) {
  float2* c0 = a->at<float2>(a->p.z[2]);
  float2* c1 = a->at<float2>(a->p.scratch);
  hipError_t e = tana::launch_fft2t(a->at<float2>(a->p.w[0]), c0, a->n, a->logn, true, a->twiddles(), a->stream);
  if (e == hipSuccess) e = tana::launch_fft2t(a->at<float2>(a->p.w[1]), c1, a->n, a->logn, true, a->twiddles(), a->stream);
  if (e == hipSuccess)
    e = tana::launch_shells(reinterpret_cast<const float*>(c0), reinterpret_cast<const float*>(c0) + 1,
                            reinterpret_cast<const float*>(c1), 2, a->n, a->ns, true, a->at<double>(a->p.partial),
                            a->at<int>(a->p.pcount), a->res(a->corr_at()), a->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(a, e, "correlations");
}

// Defect counts into the result block.
int defects_enqueue(tfan_analysis* a, const float* s) {
  hipError_t e = tana::launch_defects(s, a->n, a->at<double>(a->p.dpart), a->res(a->def_at()), a->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(a, e, "defects");
}

// One read-back of result-block entries [from, from + count), then synchronise.
int fetch(tfan_analysis* a, size_t from, size_t count) {
  hipError_t e = hipMemcpyAsync(a->host.data() + from, a->res(from), count * 8, hipMemcpyDeviceToHost, a->stream);
  if (e != hipSuccess) return hip_fail(a, e, "read-back");
  return finish(a);
}
void put(double* dst, const double* src, size_t count) {
  if (dst) std::memcpy(dst, src, count * 8);
}
void put_spectra(const tfan_analysis* a, double* E, double* W, double* S, double* count, double* L) {
  const double* h = a->host.data();
  const size_t ns = (size_t)a->ns;
  put(E, h, ns);
  put(S, h + ns, ns);
  put(W, h + 2 * ns, ns);
  put(count, h + 3 * ns, ns);
  put(L, h + 4 * ns, 1);
}
void put_correlations(const tfan_analysis* a, double* Cuu, double* Cww, double* CQQ, double* count) {
  const double* h = a->host.data() + a->corr_at();
  const size_t ns = (size_t)a->ns;
  put(Cuu, h, ns);
  put(Cww, h + ns, ns);
  put(CQQ, h + 2 * ns, ns);
  put(count, h + 3 * ns, ns);
}

}  // namespace

extern "C" {

int32_t tfan_analysis_shells(int32_t n) {
  if (log2_exact(n) < 0) return 0;
  return shell_of(2LL * (n / 2) * (n / 2)) + 1;
}

size_t tfan_analysis_workspace_bytes(int32_t n) {
  if (log2_exact(n) < 0) return 0;
  return plan(n, tfan_analysis_shells(n)).total;
}

int tfan_analysis_create(int32_t n, void* ws, size_t bytes, void* stream, tfan_analysis** out) {
  if (!out) return fail(nullptr, TFAN_EINVAL, "out is NULL");
  *out = nullptr;
  if (log2_exact(n) < 0) return fail(nullptr, TFAN_EINVAL, "n must be a power of two in [8, 4096]");
  if (!ws || ((uintptr_t)ws % kAlign) != 0) return fail(nullptr, TFAN_EINVAL, "workspace must be 256-byte aligned");
  const int ns = tfan_analysis_shells(n);
  const Plan p = plan(n, ns);
  if (bytes < p.total) return fail(nullptr, TFAN_ENOMEM, "workspace too small");
  tfan_analysis* a = new tfan_analysis();
  a->n = n;
  a->logn = log2_exact(n);
  a->ns = ns;
  a->stream = (hipStream_t)stream;
  a->base = (char*)ws;
  a->p = p;
  a->host.assign((size_t)8 * ns + 3, 0.0);
  // the FFT twiddle table, enqueued on the handle's stream ahead of every later call
  hipError_t e = tana::launch_twiddles(a->at<float2>(p.tw), n, a->stream);
  if (e != hipSuccess) {
    delete a;
    return fail(nullptr, TFAN_EHIP, std::string("twiddle table: ") + hipGetErrorName(e));
  }
  *out = a;
  return TFAN_OK;
}

int tfan_analysis_spectra(tfan_analysis* a, const float* s, double* E, double* W, double* S, double* count,
                          double* L) {
  if (!a) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!s) return fail(a, TFAN_EINVAL, "state is NULL");
  int rc;
  if ((rc = transforms(a, s)) || (rc = spectra_enqueue(a)) || (rc = fetch(a, 0, a->corr_at()))) return rc;
  put_spectra(a, E, W, S, count, L);
  return TFAN_OK;
}

int tfan_analysis_correlations(tfan_analysis* a, const float* s, double* Cuu, double* Cww, double* CQQ,
                               double* count) {
  if (!a) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!s) return fail(a, TFAN_EINVAL, "state is NULL");
  int rc;
  if ((rc = transforms(a, s)) || (rc = correlations_enqueue(a)) || (rc = fetch(a, a->corr_at(), (size_t)4 * a->ns)))
    return rc;
  put_correlations(a, Cuu, Cww, CQQ, count);
  return TFAN_OK;
}

int tfan_analysis_overlaps(tfan_analysis* a, const float* s0, const float* s1, double* out) {
  if (!a) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!s0 || !s1 || !out) return fail(a, TFAN_EINVAL, "NULL argument");
  double* d = a->at<double>(a->p.out);
  hipError_t e = tana::launch_overlaps(s0, s1, a->n, a->at<double>(a->p.red), d, a->stream);
  if (e != hipSuccess) return hip_fail(a, e, "overlaps");
  int rc = copy_out(a, out, d, 6);
  return rc ? rc : finish(a);
}

int tfan_analysis_defects(tfan_analysis* a, const float* s, int64_t* plus, int64_t* minus) {
  if (!a) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!s || !plus || !minus) return fail(a, TFAN_EINVAL, "NULL argument");
  int rc;
  if ((rc = defects_enqueue(a, s)) || (rc = fetch(a, a->def_at(), 2))) return rc;
  *plus = (int64_t)a->host[a->def_at()];
  *minus = (int64_t)a->host[a->def_at() + 1];
  return TFAN_OK;
}

int tfan_analysis_all(tfan_analysis* a, const float* s, double* E, double* W, double* S, double* L, double* Cuu,
                      double* Cww, double* CQQ, double* count, int64_t* plus, int64_t* minus) {
  if (!a) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!s) return fail(a, TFAN_EINVAL, "state is NULL");
  int rc;
  if ((rc = transforms(a, s)) || (rc = spectra_enqueue(a)) || (rc = correlations_enqueue(a)) ||
      (rc = defects_enqueue(a, s)) || (rc = fetch(a, 0, a->def_at() + 2)))
    return rc;
  put_spectra(a, E, W, S, count, L);
  put_correlations(a, Cuu, Cww, CQQ, nullptr);
  if (plus) *plus = (int64_t)a->host[a->def_at()];
  if (minus) *minus = (int64_t)a->host[a->def_at() + 1];
  return TFAN_OK;
}

int tfan_analysis_sync(tfan_analysis* a) {
  if (!a) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  return finish(a);
}

void tfan_analysis_destroy(tfan_analysis* a) {
  if (!a) return;
  (void)hipStreamSynchronize(a->stream);
  delete a;
}

const char* tfan_analysis_last_error(const tfan_analysis* a) { return a ? a->err.c_str() : g_err.c_str(); }

}  // extern "C"
