// Host side of the surrogate network's C ABI (include/tfan_cnn.h): workspace
// layout, the layer sequence of the forward and backward passes, Adam.
#include "tfan_cnn.h"

#include <cmath>
#include <string>
#include <vector>

#include "cnn_internal.h"

using tcnn::bf16;

namespace {

struct LayerDims {
  int ci_real, co_real, ci, co;  // real and padded channel counts
};
constexpr LayerDims kDims[tcnn::kLayers] = {{7, 48, 16, 48},  {48, 48, 48, 48}, {48, 48, 48, 48},
                                            {48, 48, 48, 48}, {48, 48, 48, 48}, {48, 7, 48, 16}};

int64_t layer_params(int l) { return (int64_t)kDims[l].co_real * kDims[l].ci_real * 9 + kDims[l].co_real; }
int64_t param_count() {
  int64_t s = 0;
  for (int l = 0; l < tcnn::kLayers; ++l) s += layer_params(l);
  return s;
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

std::string g_err;

// Offsets of every device buffer in the workspace.
struct Plan {
  size_t theta, grad, m, v, wf[tcnn::kLayers], wb[tcnn::kLayers], bias[tcnn::kLayers], idx_id, idx_b;
  size_t inv_in, out_scale, inv_out;
  size_t act[tcnn::kLayers], z[tcnn::kLayers - 1], y, g[2], part, part_b, loss_part, loss, cmp_part, cmp;
  size_t total;
};

bool valid_sizes(int32_t B, int32_t ny, int32_t nx) {
  return B >= 1 && ny >= 16 && nx >= 16 && ny % 16 == 0 && nx % 16 == 0 &&
         (int64_t)B * ny * nx <= ((int64_t)1 << 28);
}

Plan plan(int32_t B, int32_t ny, int32_t nx, bool train) {
  Plan p{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align_up(bytes);
    return at;
  };
  const size_t P = (size_t)param_count(), sites = (size_t)B * ny * nx;
  p.theta = take(P * 4);
  p.grad = take(P * 4);
  p.m = take(P * 4);
  p.v = take(P * 4);
  for (int l = 0; l < tcnn::kLayers; ++l) {
    const size_t nw = (size_t)kDims[l].co * 9 * kDims[l].ci;
    p.wf[l] = take(nw * 2);
    p.wb[l] = take(nw * 2);
    p.bias[l] = take((size_t)kDims[l].co * 4);
  }
  p.idx_id = take((size_t)B * 4);
  p.idx_b = take((size_t)B * 4);
  p.inv_in = take(16 * 4);
  p.out_scale = take(16 * 4);
  p.inv_out = take(16 * 4);
  // activations: a_0 (16 channels) and a_1..a_5 (48); inference keeps two hidden buffers
  p.act[0] = take(sites * tcnn::kPadIO * 2);
  for (int l = 1; l < tcnn::kLayers; ++l)
    p.act[l] = (train || l <= 2) ? take(sites * tcnn::kHidden * 2) : p.act[l - 2];
  for (int l = 0; l < tcnn::kLayers - 1; ++l) p.z[l] = train ? take(sites * tcnn::kHidden * 4) : 0;
  p.y = take(sites * tcnn::kPadIO * 4);
  p.g[0] = train ? take(sites * tcnn::kHidden * 2) : 0;
  p.g[1] = train ? take(sites * tcnn::kHidden * 2) : 0;
  const int nblk = tcnn::dw_blocks(B, ny, nx);
  p.part = train ? take((size_t)nblk * tcnn::kHidden * 9 * tcnn::kHidden * 4) : 0;
  p.part_b = train ? take((size_t)nblk * tcnn::kHidden * 4) : 0;
  p.loss_part = take((size_t)tcnn::loss_blocks(B, ny, nx) * 8);
  p.loss = take(8);
  p.cmp_part = take((size_t)tcnn::compare_blocks((int64_t)ny * nx, B) * 2 * tcnn::kChannels * 8);
  p.cmp = take(2 * tcnn::kChannels * 8);
  p.total = o;
  return p;
}

}  // namespace

struct tfan_cnn {
  int B = 0, H = 0, W = 0;
  bool train = false;
  hipStream_t stream = nullptr;
  char* base = nullptr;
  Plan p{};
  int64_t adam_t = 0;
  std::string err;
  template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
};

namespace {

int fail(tfan_cnn* c, int code, const std::string& msg) {
  if (c) c->err = msg; else g_err = msg;
  return code;
}
int hip_fail(tfan_cnn* c, hipError_t e, const char* where) {
  return fail(c, TFAN_EHIP, std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}
int64_t theta_off(int l, bool bias) {
  int64_t o = 0;
  for (int k = 0; k < l; ++k) o += layer_params(k);
  return bias ? o + (int64_t)kDims[l].co_real * kDims[l].ci_real * 9 : o;
}

int pack_weights(tfan_cnn* c) {
  for (int l = 0; l < tcnn::kLayers; ++l) {
    const float* th = c->at<float>(c->p.theta);
    hipError_t e = tcnn::launch_pack_weights(th + theta_off(l, false), th + theta_off(l, true), kDims[l].ci_real,
                                             kDims[l].co_real, kDims[l].ci, kDims[l].co, c->at<bf16>(c->p.wf[l]),
                                             c->at<bf16>(c->p.wb[l]), c->at<float>(c->p.bias[l]), c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "weight packing");
  }
  return TFAN_OK;
}

// Forward pass of the batch (samples idx of the stack x); train keeps z.
int forward(tfan_cnn* c, const float* x, const int* idx_dev) {
  const int B = c->B, H = c->H, W = c->W;
  hipError_t e = tcnn::launch_pack(x, (int64_t)tcnn::kChannels * H * W, idx_dev, c->at<float>(c->p.inv_in),
                                   c->at<bf16>(c->p.act[0]), B, H, W, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "input packing");
  for (int l = 0; l < tcnn::kLayers; ++l) {
    const bool last = l == tcnn::kLayers - 1;
    e = tcnn::launch_conv(kDims[l].ci, kDims[l].co, last ? tcnn::kLinear : tcnn::kSilu, c->at<bf16>(c->p.act[l]),
                          c->at<bf16>(c->p.wf[l]), c->at<float>(c->p.bias[l]), nullptr,
                          last ? nullptr : c->at<bf16>(c->p.act[l + 1]),
                          last ? c->at<float>(c->p.y) : (c->train ? c->at<float>(c->p.z[l]) : nullptr), B, H, W,
                          c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "convolution");
  }
  return TFAN_OK;
}

int check_batch(tfan_cnn* c, const float* x, const float* t, int64_t samples, const int32_t* idx) {
  if (!c->train) return fail(c, TFAN_EINVAL, "network was created without training buffers");
  if (!x || !t || !idx) return fail(c, TFAN_EINVAL, "x, target and idx are required");
  for (int b = 0; b < c->B; ++b)
    if (idx[b] < 0 || idx[b] >= samples) return fail(c, TFAN_EINVAL, "sample index out of range");
  hipError_t e = hipMemcpyAsync(c->at<int>(c->p.idx_b), idx, (size_t)c->B * 4, hipMemcpyHostToDevice, c->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(c, e, "index upload");
}

// Loss and gradient of the batch already uploaded to idx_b.
int backward(tfan_cnn* c, const float* x, const float* t) {
  const int B = c->B, H = c->H, W = c->W;
  int rc = forward(c, x, c->at<int>(c->p.idx_b));
  if (rc) return rc;
  bf16* g[2] = {c->at<bf16>(c->p.g[0]), c->at<bf16>(c->p.g[1])};
  hipError_t e = tcnn::launch_loss(c->at<float>(c->p.y), x, t, (int64_t)tcnn::kChannels * H * W, c->at<int>(c->p.idx_b),
                                   c->at<float>(c->p.inv_out), g[0], c->at<double>(c->p.loss_part),
                                   c->at<double>(c->p.loss), B, H, W, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "loss");
  int cur = 0;
  float* grad = c->at<float>(c->p.grad);
  for (int l = tcnn::kLayers - 1; l >= 0; --l) {
    e = tcnn::launch_weight_grad(kDims[l].ci, kDims[l].co, kDims[l].ci_real, kDims[l].co_real, g[cur],
                                 c->at<bf16>(c->p.act[l]), c->at<float>(c->p.part), c->at<float>(c->p.part_b),
                                 grad + theta_off(l, false), grad + theta_off(l, true), B, H, W, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "weight gradient");
    if (l > 0) {
      e = tcnn::launch_conv(kDims[l].co, kDims[l].ci, tcnn::kBackward, g[cur], c->at<bf16>(c->p.wb[l]), nullptr,
                            c->at<float>(c->p.z[l - 1]), g[1 - cur], nullptr, B, H, W, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "input gradient");
      cur = 1 - cur;
    }
  }
  return TFAN_OK;
}

int read_loss(tfan_cnn* c, double* loss) {
  if (!loss) return TFAN_OK;
  hipError_t e = hipMemcpyAsync(loss, c->at<double>(c->p.loss), 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(c, e, "loss read-back");
}

}  // namespace

extern "C" {

int64_t tfan_cnn_param_count(void) { return param_count(); }

size_t tfan_cnn_workspace_bytes(int32_t batch, int32_t ny, int32_t nx, int32_t train) {
  if (!valid_sizes(batch, ny, nx)) return 0;
  return plan(batch, ny, nx, train != 0).total;
}

int tfan_cnn_create(int32_t batch, int32_t ny, int32_t nx, int32_t train, void* ws, size_t bytes, void* stream,
                    tfan_cnn** out) {
  if (!out) return fail(nullptr, TFAN_EINVAL, "out is NULL");
  *out = nullptr;
  if (!valid_sizes(batch, ny, nx))
    return fail(nullptr, TFAN_EINVAL, "batch >= 1 and ny, nx positive multiples of 16 (<= 2^28 sites) required");
  if (!ws || ((uintptr_t)ws % kAlign) != 0) return fail(nullptr, TFAN_EINVAL, "workspace must be 256-byte aligned");
  const Plan p = plan(batch, ny, nx, train != 0);
  if (bytes < p.total) return fail(nullptr, TFAN_ENOMEM, "workspace too small");
  tfan_cnn* c = new tfan_cnn();
  c->B = batch;
  c->H = ny;
  c->W = nx;
  c->train = train != 0;
  c->stream = (hipStream_t)stream;
  c->base = (char*)ws;
  c->p = p;
  std::vector<int> id(batch);
  for (int b = 0; b < batch; ++b) id[b] = b;
  const float ones[16] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
  const size_t P = (size_t)param_count();
  hipError_t e = hipMemsetAsync(c->at<float>(p.theta), 0, P * 4, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->at<float>(p.m), 0, P * 4, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->at<float>(p.v), 0, P * 4, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->at<int>(p.idx_id), id.data(), batch * 4, hipMemcpyHostToDevice, c->stream);
  for (size_t off : {p.inv_in, p.out_scale, p.inv_out})
    if (e == hipSuccess) e = hipMemcpyAsync(c->at<float>(off), ones, 64, hipMemcpyHostToDevice, c->stream);
  int rc = e == hipSuccess ? pack_weights(c) : hip_fail(c, e, "workspace initialisation");
  if (!rc) {
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = hip_fail(c, e, "create");
  }
  if (rc) {
    g_err = c->err;
    delete c;
    return rc;
  }
  *out = c;
  return TFAN_OK;
}

int tfan_cnn_set_params(tfan_cnn* c, const float* params) {
  if (!c) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!params) return fail(c, TFAN_EINVAL, "params is NULL");
  const size_t P = (size_t)param_count();
  for (size_t i = 0; i < P; ++i)
    if (!std::isfinite(params[i])) return fail(c, TFAN_EINVAL, "parameters must be finite");
  hipError_t e = hipMemcpyAsync(c->at<float>(c->p.theta), params, P * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->at<float>(c->p.m), 0, P * 4, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->at<float>(c->p.v), 0, P * 4, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "parameter upload");
  c->adam_t = 0;
  int rc = pack_weights(c);
  if (rc) return rc;
  e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(c, e, "parameter upload");
}

int tfan_cnn_get_params(tfan_cnn* c, float* params) {
  if (!c) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!params) return fail(c, TFAN_EINVAL, "params is NULL");
  hipError_t e = hipMemcpyAsync(params, c->at<float>(c->p.theta), (size_t)param_count() * 4, hipMemcpyDeviceToHost,
                                c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(c, e, "parameter read-back");
}

int tfan_cnn_set_scales(tfan_cnn* c, const float* s_in, const float* s_out) {
  if (!c) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!s_in || !s_out) return fail(c, TFAN_EINVAL, "scales are NULL");
  // host copies must outlive the asynchronous uploads: synchronise below
  float inv_in[16], so[16], inv_out[16];
  for (int k = 0; k < 16; ++k) {
    const float a = k < tcnn::kChannels ? s_in[k] : 1.f, b = k < tcnn::kChannels ? s_out[k] : 1.f;
    if (!(std::isfinite(a) && a > 0.f && std::isfinite(b) && b > 0.f))
      return fail(c, TFAN_EINVAL, "scales must be finite and positive");
    inv_in[k] = 1.f / a;
    so[k] = b;
    inv_out[k] = 1.f / b;
  }
  hipError_t e = hipMemcpyAsync(c->at<float>(c->p.inv_in), inv_in, 64, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->at<float>(c->p.out_scale), so, 64, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->at<float>(c->p.inv_out), inv_out, 64, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(c, e, "scale upload");
}

int tfan_cnn_forward(tfan_cnn* c, const float* x, float* out) {
  if (!c) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!x || !out || x == out) return fail(c, TFAN_EINVAL, "x and out must be distinct device arrays");
  int rc = forward(c, x, c->at<int>(c->p.idx_id));
  if (rc) return rc;
  hipError_t e = tcnn::launch_unpack(c->at<float>(c->p.y), x, c->at<float>(c->p.out_scale), out, c->B, c->H, c->W,
                                     c->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(c, e, "prediction");
}

int tfan_cnn_gradients(tfan_cnn* c, const float* x, const float* t, int64_t samples, const int32_t* idx, float* grads,
                       double* loss) {
  if (!c) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  int rc = check_batch(c, x, t, samples, idx);
  if (!rc) rc = backward(c, x, t);
  if (rc) return rc;
  if (grads) {
    hipError_t e = hipMemcpyAsync(grads, c->at<float>(c->p.grad), (size_t)param_count() * 4, hipMemcpyDeviceToHost,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "gradient read-back");
  }
  return read_loss(c, loss);
}

int tfan_cnn_train_step(tfan_cnn* c, const float* x, const float* t, int64_t samples, const int32_t* idx, float lr,
                        double* loss) {
  if (!c) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!(std::isfinite(lr) && lr > 0.f)) return fail(c, TFAN_EINVAL, "learning rate must be positive");
  int rc = check_batch(c, x, t, samples, idx);
  if (!rc) rc = backward(c, x, t);
  if (rc) return rc;
  c->adam_t += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)c->adam_t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)c->adam_t)));
  hipError_t e = tcnn::launch_adam(c->at<float>(c->p.theta), c->at<float>(c->p.grad), c->at<float>(c->p.m),
                                   c->at<float>(c->p.v), param_count(), lr, b1, b2, 1e-8f, c1, c2,
                                   c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "adam");
  if ((rc = pack_weights(c))) return rc;
  return read_loss(c, loss);
}

int tfan_cnn_compare(tfan_cnn* c, const float* a, const float* b, double* out) {
  if (!c) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  if (!a || !b || !out) return fail(c, TFAN_EINVAL, "NULL argument");
  hipError_t e = tcnn::launch_compare(a, b, (int64_t)c->H * c->W, c->B, c->at<double>(c->p.cmp_part),
                                      c->at<double>(c->p.cmp), c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, c->at<double>(c->p.cmp), 2 * tcnn::kChannels * 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(c, e, "compare");
}

int tfan_cnn_sync(tfan_cnn* c) {
  if (!c) return fail(nullptr, TFAN_EINVAL, "handle is NULL");
  hipError_t e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? TFAN_OK : hip_fail(c, e, "sync");
}

void tfan_cnn_destroy(tfan_cnn* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

const char* tfan_cnn_last_error(const tfan_cnn* c) { return c ? c->err.c_str() : g_err.c_str(); }

}  // extern "C"
