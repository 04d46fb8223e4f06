// Counter barrier of a set of workgroups of one persistent launch (the
// workgroups of one instance of a batched launch, or a whole grid).
#pragma once

#include "pass_device.h"

namespace ggdt {
namespace dev {

// Every workgroup adds one to *counter and waits until it reaches `target`
// (the arrivals expected so far; the counter only grows).  The workgroup's
// threads first meet at a workgroup barrier, which orders their earlier memory
// accesses before thread 0's at workgroup scope; thread 0 alone then releases
// at agent scope, arrives, polls, and acquires at agent scope; a second
// workgroup barrier passes the acquisition on to the other threads.  So each
// workgroup issues one agent-scope fence pair per barrier rather than one per
// wave (each such fence writes back or invalidates the L2 of its XCD), and the
// polls are relaxed loads.  The wait is bounded: it gives up, setting the
// watchdog word, after `limit` polls, or when another wait has given up.
// Returns false if it gave up.
template <typename CT>
__device__ bool counter_barrier(CT* counter, CT target, unsigned* words, unsigned long long limit) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(counter, (CT)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    unsigned long long polls = 0;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (ld_relaxed(words + kWordAbort) != 0u) {
        ok = 0;
        break;
      }
      if (++polls > limit) {
        __hip_atomic_fetch_or(words + kWordAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

}  // namespace dev
}  // namespace ggdt
