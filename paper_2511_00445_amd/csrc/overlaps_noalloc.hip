// tfan_analysis_overlaps_noalloc: the temporal-correlation overlaps of
// tfan_analysis_overlaps without a handle or workspace, for callers that cannot
// allocate device memory.  The block partials live in a fixed device array of
// this library (one copy per GPU, held until the process ends); host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device, never through the array's name.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "analysis_internal.h"
#include "tfan_analysis.h"

namespace {

// Block partials of the overlap reduction (at most 1024 blocks x 6 sums) and the
// six results: 6,150 doubles, 49,200 bytes.
constexpr int kMaxBlocks = 1024;
constexpr size_t kScratchDoubles = (size_t)kMaxBlocks * 6 + 6;
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};  // device address of `scratch` per device, set once
std::string g_err;

int set_error(int code, const std::string& msg) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_err = msg;
  return code;
}

// Address of this device's copy of `scratch`, looked up once per device with that
// device current (each GPU holds its own copy at its own address).
int scratch_for_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(TFAN_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(TFAN_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      g_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return TFAN_EHIP;
    }
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return TFAN_OK;
}

bool power_of_two_in_range(int n) { return n >= 8 && n <= 4096 && (n & (n - 1)) == 0; }

}  // namespace

extern "C" {

int tfan_analysis_overlaps_noalloc(int32_t n, const float* s0, const float* s1, double* out, void* hip_stream) {
  if (!power_of_two_in_range(n)) return set_error(TFAN_EINVAL, "n must be a power of two in [8, 4096]");
  if (!s0 || !s1 || !out) return set_error(TFAN_EINVAL, "NULL argument");
  if (tana::reduce_blocks(n) > kMaxBlocks) return set_error(TFAN_EINVAL, "grid exceeds the fixed scratch array");
  double* ptr = nullptr;
  if (int rc = scratch_for_current_device(&ptr)) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  double* partial = ptr;
  double* res = ptr + (size_t)kMaxBlocks * 6;
  // every block writes all six of its partials and the column sums write all six
  // results, so nothing has to start at zero
  hipError_t e = tana::launch_overlaps(s0, s1, n, partial, res, st);
  if (e == hipSuccess) e = hipMemcpyAsync(out, res, 6 * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return set_error(TFAN_EHIP, std::string("overlaps: ") + hipGetErrorString(e));
  return TFAN_OK;
}

const char* tfan_analysis_noalloc_last_error(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_err.c_str();
}

}  // extern "C"
