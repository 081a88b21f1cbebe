// ctx.cpp -- contexts: a device scratch buffer, a pinned staging ring, the
// out-of-core copy stream and events, and stored launch shapes, created once
// so that the calls issued through a context neither allocate nor wait on
// the host (Sec. III-A's pipeline run many times over resident streams).
#include "ctx.hpp"

using namespace hsz_abi;

namespace hsz_ctx_util {

int check_device(const hsz_ctx* c) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device) return HSZ_ERR_INVALID_ARG;
  return HSZ_OK;
}

hipError_t order_after_last(hsz_ctx* c, hipStream_t s) {
  return c->last_set ? hipStreamWaitEvent(s, c->last, 0) : hipSuccess;
}

hipError_t mark_last(hsz_ctx* c, hipStream_t s) {
  hipError_t e = hipEventRecord(c->last, s);
  if (e == hipSuccess) c->last_set = true;
  return e;
}

int stage_copy(hsz_ctx* c, const void* src, uint64_t bytes, void* d_dst, hipStream_t s) {
  if (bytes > c->ring_bytes) return HSZ_ERR_CAPACITY;
  uint64_t start = (c->ring_head + 255) / 256 * 256;
  if (start + bytes > c->ring_bytes) start = 0;
  const uint64_t end = start + bytes;
  // retire the segments whose copies have completed, then wait for any
  // still in flight over the region (only when the ring is exhausted)
  for (auto it = c->inflight.begin(); it != c->inflight.end();) {
    const bool overlap = it->begin < end && start < it->end;
    hipError_t q = hipEventQuery(it->ev);
    if (q == hipErrorNotReady && overlap) q = hipEventSynchronize(it->ev);
    if (q == hipSuccess) {
      c->spare.push_back(it->ev);
      it = c->inflight.erase(it);
    } else if (q == hipErrorNotReady) {
      ++it;
    } else {
      return hip_fail(q);
    }
  }
  memcpy(c->h_ring + start, src, bytes);
  hipError_t e = hipMemcpyAsync(d_dst, c->h_ring + start, bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e);
  hipEvent_t ev = nullptr;
  if (!c->spare.empty()) {
    ev = c->spare.back();
    c->spare.pop_back();
  } else if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) {
    return hip_fail(e);
  }
  if ((e = hipEventRecord(ev, s)) != hipSuccess) {
    c->spare.push_back(ev);
    return hip_fail(e);
  }
  c->inflight.push_back({start, end, ev});
  c->ring_head = end;
  return HSZ_OK;
}

}  // namespace hsz_ctx_util

namespace {

void release(hsz_ctx* c) {
  if (c->last_set) (void)hipEventSynchronize(c->last);
  if (c->copy) (void)hipStreamSynchronize(c->copy);
  for (auto& g : c->inflight) {
    (void)hipEventSynchronize(g.ev);
    (void)hipEventDestroy(g.ev);
  }
  for (hipEvent_t e : c->spare) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ooc)
    if (e) (void)hipEventDestroy(e);
  if (c->last) (void)hipEventDestroy(c->last);
  if (c->copy) (void)hipStreamDestroy(c->copy);
  if (c->d_scratch) (void)hipFree(c->d_scratch);
  if (c->h_ring) (void)hipHostFree(c->h_ring);
  delete c;
}

uint64_t round_mib(uint64_t v) { return (v + (1ull << 20) - 1) >> 20 << 20; }

}  // namespace

extern "C" {

int hsz_ctx_create(uint64_t scratch_bytes, uint64_t host_bytes, hsz_ctx** out) {
  if (!out) return HSZ_ERR_INVALID_ARG;
  *out = nullptr;
  hsz_ctx* c = new hsz_ctx();
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess && scratch_bytes) {
    c->scratch_bytes = round_mib(scratch_bytes);
    e = hipMalloc((void**)&c->d_scratch, c->scratch_bytes);
  }
  if (e == hipSuccess && host_bytes) {
    c->ring_bytes = host_bytes;
    e = hipHostMalloc((void**)&c->h_ring, host_bytes, hipHostMallocDefault);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->copy, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->last, hipEventDisableTiming);
  for (int i = 0; i < kOocEvents && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&c->ooc[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    if (!c->d_scratch) c->scratch_bytes = 0;
    if (!c->h_ring) c->ring_bytes = 0;
    release(c);
    return hip_fail(e);
  }
  *out = c;
  return HSZ_OK;
}

void hsz_ctx_destroy(hsz_ctx* c) {
  if (c) release(c);
}

int hsz_ctx_reserve(hsz_ctx* c, uint64_t bytes) {
  if (!c) return HSZ_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(c->mu);
  if (bytes <= c->scratch_bytes) return HSZ_OK;
  hipError_t e = c->last_set ? hipEventSynchronize(c->last) : hipSuccess;
  if (e != hipSuccess) return hip_fail(e);
  if (c->d_scratch && (e = hipFree(c->d_scratch)) != hipSuccess) return hip_fail(e);
  c->d_scratch = nullptr;
  c->scratch_bytes = 0;
  const uint64_t want = round_mib(bytes);
  if ((e = hipMalloc((void**)&c->d_scratch, want)) != hipSuccess) {
    c->d_scratch = nullptr;
    return hip_fail(e);
  }
  c->scratch_bytes = want;
  return HSZ_OK;
}

int hsz_ctx_scratch(hsz_ctx* c, void** d_scratch, uint64_t* bytes) {
  if (!c || !d_scratch || !bytes) return HSZ_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(c->mu);
  *d_scratch = c->d_scratch;
  *bytes = c->scratch_bytes;
  return HSZ_OK;
}

int hsz_ctx_set_tuning(hsz_ctx* c, const char* key, const hsz_tuning* t) {
  if (!c || !key || !t || strnlen(key, 1024) >= 1024) return HSZ_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(c->mu);
  c->tunings[key] = *t;
  return HSZ_OK;
}

int hsz_ctx_get_tuning(hsz_ctx* c, const char* key, hsz_tuning* t) {
  if (!c || !key || !t || strnlen(key, 1024) >= 1024) return HSZ_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(c->mu);
  auto it = c->tunings.find(key);
  if (it == c->tunings.end()) return HSZ_ERR_INVALID_ARG;
  *t = it->second;
  return HSZ_OK;
}

}  // extern "C"
