// The latent step with a library-owned workspace, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).  The workspace is a file-scope
// device array; each GPU the library runs on holds its own copy for the
// life of the process.  Its address is taken once per device with that
// device current (hipGetSymbolAddress) and only that address is handed to
// the kernels: in host code the array's name is not a device address.
//
// Every call on one GPU shares that GPU's array, which keeps the contents
// of the last call; the step's set-up kernel initialises every word the
// step reads before writing it, so nothing has to be cleared between
// calls.  Calls that overlap on one GPU (two streams or two host threads at
// once) race on the array and must be serialised by the caller.
#include <mutex>

#include "common.hpp"

namespace crom {

constexpr size_t STATIC_WS_BYTES = size_t(64) << 20;  // 64 MiB per device
constexpr int STATIC_WS_DEVICES = 64;

static __device__ __align__(256) char scratch[STATIC_WS_BYTES];

static void* g_scratch_ptr[STATIC_WS_DEVICES];
static hipError_t g_scratch_err[STATIC_WS_DEVICES];
static std::once_flag g_scratch_once[STATIC_WS_DEVICES];

// Device address of the current device's copy of `scratch` (resolved on the
// first call made on that device).
static crom_status scratch_of_current_device(void** out) {
  int dev = 0;
  crom_status s = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (s != CROM_OK) return s;
  if (dev < 0 || dev >= STATIC_WS_DEVICES) return fail(CROM_ERR_UNSUPPORTED, "device index beyond 63");
  std::call_once(g_scratch_once[dev], [dev]() {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? p : nullptr;
  });
  if (g_scratch_err[dev] != hipSuccess) return hip_check(g_scratch_err[dev], "hipGetSymbolAddress(scratch)");
  if (!g_scratch_ptr[dev]) return fail(CROM_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
  *out = g_scratch_ptr[dev];
  return CROM_OK;
}

}  // namespace crom

using namespace crom;

extern "C" {

size_t crom_step_static_capacity(void) { return STATIC_WS_BYTES; }

crom_status crom_step_static(const crom_net* net, const crom_pde* pde, int32_t n_inst, const int64_t* offsets,
                             int64_t total_samples, const float* y, const uint8_t* clamp, const double* q_prev,
                             const double* q_n, double* q_next, const crom_gn_opts* opts, crom_step_info* info,
                             void* stream) {
  size_t need = 0;
  crom_status s = crom_step_workspace(net, n_inst, total_samples, &need);
  if (s != CROM_OK) return s;
  if (need > STATIC_WS_BYTES) {
    set_error("crom_step_static: the step needs %zu workspace bytes, the static workspace holds %zu (use crom_step "
              "with a caller workspace)",
              need, STATIC_WS_BYTES);
    return CROM_ERR_WORKSPACE;
  }
  void* ws = nullptr;
  if ((s = scratch_of_current_device(&ws)) != CROM_OK) return s;
  return crom_step(net, pde, n_inst, offsets, total_samples, y, clamp, q_prev, q_n, q_next, opts, info, ws,
                   STATIC_WS_BYTES, stream);
}

}  // extern "C"
