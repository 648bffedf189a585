// Allocation-free variant of tdgemm_plan followed by tdgemm_gemm(fused = 1):
// the plan's workspace (block statistics, pair records, budgets, calibration
// table and, with a split l-sum, the group partial results) lives in a
// file-scope device array instead of caller memory, for callers that cannot
// allocate. The kernels are those of the two entry points it replaces.
#include <mutex>

#include "api_internal.h"

// One copy per GPU, kept until the process ends. Host code never passes this
// name to a kernel or a copy: it is a host-side stand-in; the device address
// comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) char scratch[TDGEMM_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch[kMaxDevices];   // device address of `scratch` per device, once looked up

// Device address of the current device's copy of `scratch`, looked up on the
// first call on that device with the device current.
hipError_t scratch_of_current_device(char **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = static_cast<char *>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" tdgemm_status tdgemm_matmul_noalloc(const tdgemm_desc *desc, const void *A,
                                               const void *B, const tdgemm_calib *calib,
                                               void *C, void *stream) {
  tdgemm_status s = tdg::validate_desc(desc);
  if (s != TDGEMM_OK) return s;
  // a tile map needs a host-to-device copy and a synchronisation; the
  // block-scaled forms need byte operand buffers of their own
  if (desc->tile_target || tdg::is_block_scaled(desc->prec)) return TDGEMM_E_UNSUPPORTED;
  const tdg::Layout ly = tdg::layout_of(*desc);
  if (ly.total > TDGEMM_NOALLOC_MAX_BYTES) return TDGEMM_E_WORKSPACE;
  s = tdg::check_plan_inputs(*desc, A, B, calib);
  if (s != TDGEMM_OK) return s;
  if (desc->M == 0 || desc->N == 0) return TDGEMM_OK;
  if (!C) return TDGEMM_E_ARG;
  char *ws = nullptr;
  if (scratch_of_current_device(&ws) != hipSuccess) return TDGEMM_E_HIP;
  tdgemm_plan_s p;
  p.desc = *desc;
  p.desc.tile_target = nullptr;
  p.tile_map = false;
  p.ly = ly;
  p.ws = ws;
  p.stream = static_cast<hipStream_t>(stream);
  if (tdg::enqueue_plan(p, A, B, calib, nullptr) != hipSuccess) return TDGEMM_E_HIP;
  if (tdg::enqueue_fused(p, A, B, C) != hipSuccess) return TDGEMM_E_HIP;
  return TDGEMM_OK;
}
