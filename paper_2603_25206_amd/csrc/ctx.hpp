// ctx.hpp -- the context object (include/hsz.h, "contexts") as the C-ABI
// units that issue work through it see it.
#pragma once

#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "abi_util.hpp"

// events of the out-of-core pipeline, by index
enum { kOocH2d = 0, kOocUsed = 3, kOocOutReady = 6, kOocOutDone = 8, kOocFinal = 10, kOocEvents = 11 };

struct hsz_ctx {
  int device = 0;
  uint8_t* d_scratch = nullptr;
  uint64_t scratch_bytes = 0;
  uint8_t* h_ring = nullptr;  // pinned staging for work tables
  uint64_t ring_bytes = 0, ring_head = 0;
  struct Seg {
    uint64_t begin, end;
    hipEvent_t ev;  // the copy that reads [begin, end) has completed
  };
  std::deque<Seg> inflight;
  std::vector<hipEvent_t> spare;
  hipStream_t copy = nullptr;  // out-of-core host <-> device copies
  hipEvent_t ooc[kOocEvents] = {};
  hipEvent_t last = nullptr;  // end of the last call issued through the context
  bool last_set = false;
  std::map<std::string, hsz_tuning> tunings;
  std::mutex mu;  // one call at a time per context on the host side
};

namespace hsz_ctx_util {

// The calling thread's current device is the context's.
int check_device(const hsz_ctx* c);
// 's' waits (on the device) for the context's previous call.
hipError_t order_after_last(hsz_ctx* c, hipStream_t s);
// The context's last call ends with the work enqueued on 's' so far.
hipError_t mark_last(hsz_ctx* c, hipStream_t s);
// Copy 'bytes' from host 'src' through the pinned ring to d_dst on 's'.
int stage_copy(hsz_ctx* c, const void* src, uint64_t bytes, void* d_dst, hipStream_t s);

}  // namespace hsz_ctx_util
