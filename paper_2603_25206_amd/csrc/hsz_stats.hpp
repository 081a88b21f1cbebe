// hsz_stats.hpp -- finishing the statistics of Sec. V-A (mean) and Alg. 4
// (variance) from exact integer sums: the record a job writes, the closed
// forms, and the batch's finish (one wave per job over the accumulator's
// stripes), shared by the finalize kernel and the gradient kernel that
// finishes its own batch.
#pragma once

#include "hsz_device.hpp"
#include "hsz_launch.hpp"

namespace hsz {

// hsz_stats as the device writes it
struct StatsOut {
  int64_t n, s1;
  uint64_t s2lo;
  int64_t s2hi;
  double mean, var;
};

__device__ __forceinline__ double u128_to_f64(unsigned __int128 v) {
  return (double)(uint64_t)(v >> 64) * 18446744073709551616.0 + (double)(uint64_t)v;
}

// mean = s1 Delta / n; var = (n s2 - s1^2) / (n (n - 1)) Delta^2 with the
// numerator exact in 128 bits (n < 2^34, |q| < 2^29), one rounding each
__device__ __forceinline__ StatsOut stats_from_sums(int64_t n, int64_t s1, uint64_t s2lo, uint64_t s2hi, int op,
                                                    double quantum) {
  StatsOut r{};
  r.n = n;
  r.s1 = s1;
  r.mean = (double)s1 * quantum / (double)n;
  if (op == 2) {
    const unsigned __int128 S2 = ((unsigned __int128)s2hi << 64) | s2lo;
    r.s2lo = s2lo;
    r.s2hi = (int64_t)s2hi;
    const unsigned __int128 a = (unsigned __int128)(uint64_t)n * S2;
    const uint64_t m = (uint64_t)(s1 < 0 ? -s1 : s1);
    const unsigned __int128 b = (unsigned __int128)m * m;
    const double num = u128_to_f64(a - b);
    r.var = n > 1 ? num / ((double)n * (double)(n - 1)) * (quantum * quantum) : __builtin_nan("");
  } else {
    r.var = __builtin_nan("");
  }
  return r;
}

// One wave finishes job J from its accumulator slot: lane k takes stripe k,
// the wave adds them exactly (sum q^2 = hi * 2^32 + lo in 128 bits), lane 0
// writes the record.  ATOMIC reads the stripes with device-scope atomic
// loads (the slot was filled by other workgroups of the same launch).
template <bool ATOMIC>
__device__ __forceinline__ void finish_stats_job(const StatsJob& J, const BatchAcc* slot) {
  const BatchAcc* p = slot + lane_id();
  BatchAcc a;
  if constexpr (ATOMIC) {
    a.s1 = __hip_atomic_load(&p->s1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.cnt = __hip_atomic_load(&p->cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.s2lo = __hip_atomic_load(&p->s2lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.s2hi = __hip_atomic_load(&p->s2hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    a = *p;
  }
  const int64_t s1 = wave_sum64(a.s1), cnt = wave_sum64(a.cnt);
  U128 lo = {a.s2lo, 0}, hi = {a.s2hi, 0};
  for (int m = 32; m >= 1; m >>= 1) {
    U128 o;
    o.lo = __shfl_xor(lo.lo, m);
    o.hi = __shfl_xor(lo.hi, m);
    add_u128(lo, o);
    o.lo = __shfl_xor(hi.lo, m);
    o.hi = __shfl_xor(hi.hi, m);
    add_u128(hi, o);
  }
  if (lane_id() == 0) {
    const unsigned __int128 s2 = ((((unsigned __int128)hi.hi << 64) | hi.lo) << 32) +
                                 (((unsigned __int128)lo.hi << 64) | lo.lo);
    *(StatsOut*)J.out = stats_from_sums(cnt, s1, (uint64_t)s2, (uint64_t)(s2 >> 64), J.op, J.v.quantum);
  }
}

// The finish of a batch whose every statistic is summed inside one
// kernel's workgroups, done by that kernel's last workgroup: each
// workgroup, after its last accumulator atomics, counts itself done; the
// one that completes the count finishes every job, zeroes the
// accumulators, publishes the launch's status word (errors are recorded in
// 'live' during the launch) and re-arms 'live' and the count for the next
// launch.  Accumulators, 'live' and the count start at zero (a reset
// before the first launch).
struct BatchTail {
  const StatsJob* jobs[2];
  const int64_t* counts[2];  // counts[c][0]: jobs of class c in the table
  BatchAcc* acc[2];          // each class's slots (n[c] of them)
  int n[2];
  unsigned* done;
  int* live;
  int* status_out;
};

// Ordering: the accumulators and the status words are only ever changed
// by device-scope atomics during a pass, which are performed at the point
// of coherence; the barrier's wait makes every wave's atomics complete
// before thread 0 (which issued the workgroup's accumulator atomics itself)
// counts the workgroup, and the last workgroup reads them with device-scope
// atomic loads after its count returned.  No cache writeback is needed (a
// device-scope fence per workgroup would write back the L2 each time).
__device__ __forceinline__ void batch_tail(const BatchTail& T, int* flag) {
  __syncthreads();  // every wave's accumulator atomics and status records completed
  if (threadIdx.x == 0) *flag = atomicAdd(T.done, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!*flag) return;
  const int nw = blockDim.x / kWave, w = (int)(threadIdx.x / kWave);
  for (int k = w; k < T.n[0] + T.n[1]; k += nw) {
    const int c = k < T.n[0] ? 0 : 1, i = c ? k - T.n[0] : k;
    if (i >= (int)T.counts[c][0]) continue;
    const StatsJob J = load_job(T.jobs[c], i);
    finish_stats_job<true>(J, T.acc[c] + (int64_t)J.acc * kAccStripes);
  }
  __syncthreads();  // every stripe read before it is zeroed
  for (int c = 0; c < 2; ++c)
    for (int e = threadIdx.x; e < T.n[c] * kAccStripes; e += blockDim.x) T.acc[c][e] = BatchAcc{0, 0, 0, 0};
  if (threadIdx.x == 0) {
    *T.status_out = __hip_atomic_load(T.live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *T.live = 0;
    *T.done = 0u;
  }
}

}  // namespace hsz
