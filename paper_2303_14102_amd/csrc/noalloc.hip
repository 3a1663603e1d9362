// The forward without a caller workspace: a file-scope device array serves as the workspace.
//
// `scratch` is a static __device__ array, so every GPU the library runs on holds its own copy,
// at its own address, until the process ends.  Host code never passes the array's name to a
// kernel or a copy (on the host that name is only a stand-in, not a device address): the first
// call on each device, with that device current, asks the runtime for the device address
// (hipGetSymbolAddress) and keeps it, and every launch takes that address.  Nothing on this path
// allocates: the phases are the same kernels as the workspace entry point's, and the statistics
// pass clears, with a fill kernel, the header, counters and sums that must start at zero.
#include <mutex>

#include "sil_internal.h"

namespace sil {

constexpr size_t kScratchBytes = SIL_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SIL_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SIL_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SIL_OK;
}

__global__ void k_status_out(const int32_t* __restrict__ hdr, int32_t* __restrict__ out) {
  if (threadIdx.x == 0) *out = hdr[0];
}

}  // namespace
}  // namespace sil

using namespace sil;

extern "C" int silhouette_sqeuclid_noalloc(const void* X, int32_t dtype, const float* col_scale,
                                           const int32_t* labels, int64_t N, int32_t D,
                                           int32_t K, int32_t products, int32_t flags, float* s,
                                           double* S, int32_t* status, void* stream) {
  if (!shape_ok(N, D, K)) return SIL_E_ARG;
  if (flags & SIL_FLAG_SAVE_FOR_GRAD) return SIL_E_ARG;
  if (dtype != SIL_F32 && dtype != SIL_BF16 && dtype != SIL_FP8_E4M3) return SIL_E_DTYPE;
  if (make_layout(N, D, K, SIL_SQEUCLID, dtype, flags).total > kScratchBytes) return SIL_E_SCRATCH;
  void* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  rc = run_forward(SIL_SQEUCLID, X, dtype, col_scale, labels, N, D, K, products, flags, s, S, ws,
                   kScratchBytes, stream);
  if (rc) return rc;
  if (status) {
    // the header's first word is the status (the workspace layout's first region)
    k_status_out<<<1, 64, 0, static_cast<hipStream_t>(stream)>>>(static_cast<const int32_t*>(ws),
                                                                  status);
    if (hipGetLastError() != hipSuccess) return SIL_E_HIP;
  }
  return SIL_OK;
}
