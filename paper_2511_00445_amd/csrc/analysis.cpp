// Host side of the observables' C ABI (include/tfan_analysis.h): workspace layout
// and the kernel sequences of the spectra, correlations, overlaps and defects.
#include "tfan_analysis.h"

#include <string>

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
  size_t z[3], scratch, w[2], pE, pS, partial, pcount, out, red, dpart, dout, tw, total;
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
  p.partial = take((size_t)3 * n * ns * 8);
  p.pcount = take((size_t)n * ns * 4);
  p.out = take((size_t)(4 * ns + 1) * 8);
  p.red = take((size_t)tana::reduce_blocks(n) * 6 * 8 + 64);
  p.dpart = take((size_t)tana::reduce_blocks(n) * 2 * 8);
  p.dout = take(2 * 8);
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
  template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
  const float2* twiddles() const { return at<float2>(p.tw); }
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

// Shell sums of the spectra and L from the transforms; results copied out
// (stream-ordered, before any later kernel reuses the output buffer).
int spectra_from_transforms(tfan_analysis* a, double* E, double* W, double* S, double* count, double* L) {
  const int ns = a->ns;
  double* out = a->at<double>(a->p.out);
  hipError_t e = tana::launch_shells(a->at<float>(a->p.pE), a->at<float>(a->p.pS), nullptr, 1, a->n, ns, false,
                                     a->at<double>(a->p.partial), a->at<int>(a->p.pcount), out, a->stream);
  if (e == hipSuccess) e = tana::launch_finish_spectra(out, a->n, ns, a->stream);
  if (e != hipSuccess) return hip_fail(a, e, "spectra");
  int rc;
  if ((rc = copy_out(a, E, out, ns)) || (rc = copy_out(a, S, out + ns, ns)) || (rc = copy_out(a, W, out + 2 * ns, ns)) ||
      (rc = copy_out(a, count, out + 3 * ns, ns)) || (rc = copy_out(a, L, out + 4 * ns, 1)))
    return rc;
  return TFAN_OK;
}

// Inverse transforms of the (transposed) powers, which come out in natural
// layout, and their shell means; results copied out.
int correlations_from_transforms(tfan_analysis* a, double* Cuu, double* Cww, double* CQQ, double* count) {
  float2* c0 = a->at<float2>(a->p.z[2]);
  float2* c1 = a->at<float2>(a->p.scratch);
  hipError_t e = tana::launch_fft2t(a->at<float2>(a->p.w[0]), c0, a->n, a->logn, true, a->twiddles(), a->stream);
  if (e == hipSuccess) e = tana::launch_fft2t(a->at<float2>(a->p.w[1]), c1, a->n, a->logn, true, a->twiddles(), a->stream);
  const int ns = a->ns;
  double* out = a->at<double>(a->p.out);
  if (e == hipSuccess)
    e = tana::launch_shells(reinterpret_cast<const float*>(c0), reinterpret_cast<const float*>(c0) + 1,
                            reinterpret_cast<const float*>(c1), 2, a->n, ns, true, a->at<double>(a->p.partial),
                            a->at<int>(a->p.pcount), out, a->stream);
  if (e != hipSuccess) return hip_fail(a, e, "correlations");
  int rc;
  if ((rc = copy_out(a, Cuu, out, ns)) || (rc = copy_out(a, Cww, out + ns, ns)) ||
      (rc = copy_out(a, CQQ, out + 2 * ns, ns)) || (rc = copy_out(a, count, out + 3 * ns, ns)))
    return rc;
  return TFAN_OK;
}

// Defect counts into the host pair (stream-ordered copy; the caller synchronises).
int defects_enqueue(tfan_analysis* a, const float* s, double* host2) {
  double* d = a->at<double>(a->p.dout);
  hipError_t e = tana::launch_defects(s, a->n, a->at<double>(a->p.dpart), d, a->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(host2, d, 16, hipMemcpyDeviceToHost, a->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(a, e, "defects");
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
  int rc = transforms(a, s);
  if (rc) return rc;
  rc = spectra_from_transforms(a, E, W, S, count, L);
  return rc ? rc : finish(a);
}

int tfan_analysis_correlations(tfan_analysis* a, const float* s, double* Cuu, double* Cww, double* CQQ,
                               double* count) {
  if (!a) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!s) return fail(a, TFAN_EINVAL, "state is NULL");
  int rc = transforms(a, s);
  if (rc) return rc;
  rc = correlations_from_transforms(a, Cuu, Cww, CQQ, count);
  return rc ? rc : finish(a);
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
  double h[2] = {0, 0};
  int rc = defects_enqueue(a, s, h);
  if (rc) return rc;
  if ((rc = finish(a))) return rc;
  *plus = (int64_t)h[0];
  *minus = (int64_t)h[1];
  return TFAN_OK;
}

int tfan_analysis_all(tfan_analysis* a, const float* s, double* E, double* W, double* S, double* L, double* Cuu,
                      double* Cww, double* CQQ, double* count, int64_t* plus, int64_t* minus) {
  if (!a) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!s) return fail(a, TFAN_EINVAL, "state is NULL");
  int rc = transforms(a, s);
  if (rc) return rc;
  if ((rc = spectra_from_transforms(a, E, W, S, count, L))) return rc;
  if ((rc = correlations_from_transforms(a, Cuu, Cww, CQQ, nullptr))) return rc;
  double h[2] = {0, 0};
  if ((rc = defects_enqueue(a, s, h))) return rc;
  if ((rc = finish(a))) return rc;
  if (plus) *plus = (int64_t)h[0];
  if (minus) *minus = (int64_t)h[1];
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
