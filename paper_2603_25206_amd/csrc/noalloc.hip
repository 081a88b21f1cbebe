// noalloc.hip -- hsz_op_fused_noalloc: hsz_op_fused with its workspace taken
// from a fixed device array owned by the library, for callers that cannot
// allocate device memory (code under stream capture, serving loops that must
// not call the allocator).
//
// The array lives in this translation unit.  Its host-side name is only a
// stand-in for the device symbol, so host code never passes it to a kernel
// or a copy: the first call on each device resolves the symbol's device
// address with hipGetSymbolAddress (with that device current) and every
// later call on the device uses that address.  Each device holds its own
// copy of the array until the process ends.
#include <mutex>

#include "abi_util.hpp"

namespace {

using namespace hsz_abi;

constexpr uint64_t kScratchBytes = HSZ_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// device address of this device's copy of 'scratch' (resolved once per device)
int scratch_of_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev < 0 || dev >= kMaxDevices) return HSZ_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if (!p) return HSZ_ERR_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return HSZ_OK;
}

__global__ void k_copy_status(const int* __restrict__ from, int* __restrict__ to) {
  if (threadIdx.x == 0) *to = *from;
}

}  // namespace

extern "C" int hsz_op_fused_noalloc(const void* d_c, const hsz_header* h, int via, int op, int axis,
                                    const hsz_box* h_box, void* d_result, uint64_t cap, int* d_status,
                                    void* stream) {
  int rc = check_header(h);
  if (rc) return rc;
  uint64_t need = 0;
  if ((rc = hsz_op_workspace(h, op, &need))) return rc;
  if (need > kScratchBytes) return HSZ_ERR_CAPACITY;
  if (d_status && ((uintptr_t)d_status & 3u)) return HSZ_ERR_INVALID_ARG;
  void* ws = nullptr;
  if ((rc = scratch_of_current_device(&ws))) return rc;
  // the operation resets the status word at the start of ws with a kernel
  // (no memset node, so the sequence can be captured) and clears everything
  // else it reads before reading it
  rc = hsz_op_fused(d_c, h, via, op, axis, h_box, d_result, cap, ws, need, stream);
  if (rc) return rc;
  if (d_status) {
    hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, (hipStream_t)stream, (const int*)ws, d_status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e);
  }
  return HSZ_OK;
}
