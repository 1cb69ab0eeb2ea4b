// Device side of the persistent task-graph executor, shared by every
// executor kernel (the QR tile kernels, the Cholesky-inversion tile
// kernels): the ready queue, the dependency counts and the memory ordering
// between a task and its successors.
#pragma once
#include <hip/hip_runtime.h>

#include "tqr_types.h"

namespace tqr {

__device__ __forceinline__ Task load_task(const Task *p) {
  Task t = *p;
  t.kind = __builtin_amdgcn_readfirstlane(t.kind);
  t.i = __builtin_amdgcn_readfirstlane(t.i);
  t.piv = __builtin_amdgcn_readfirstlane(t.piv);
  t.k = __builtin_amdgcn_readfirstlane(t.k);
  t.j = __builtin_amdgcn_readfirstlane(t.j);
  t.stripe = __builtin_amdgcn_readfirstlane(t.stripe);
  t.prob = __builtin_amdgcn_readfirstlane(t.prob);
  return t;
}

__device__ __forceinline__ int ld_relaxed(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(int32_t *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Resets the executor state: dependency counts, queue (initially ready
// tasks first, the rest empty = -1) and control block.
__device__ __forceinline__ void executor_reset(const ExecArgs &a) {
  if (a.skip && *a.skip) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < a.ntasks; x += stride) {
    a.indeg[x] = a.indeg0[x];
    a.queue[x] = (x < a.nready0) ? a.ready0[x] : -1;
  }
  if (a.probs)
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < a.nprob; x += stride)
      *a.probs[x].singular = 0x7fffffff;
  if (blockIdx.x == 0 && threadIdx.x < 16) {
    int32_t *c = reinterpret_cast<int32_t *>(a.ctl);
    c[threadIdx.x] = 0;
    if (threadIdx.x == 1) c[1] = a.nready0;  // tail
    if (threadIdx.x == 5) c[5] = 0x7fffffff; // smallest 1-based index of a zero R(j,j)
  }
}

// The persistent loop: every workgroup pops queue slots in order, waits for
// the slot to be filled and its task's predecessors to be finished, runs
// the task (run(task), every thread of the workgroup), then releases its
// successors; a successor whose count reaches zero is pushed, unless the
// reset filled the whole queue with a precomputed order (static_order,
// where every task follows all its predecessors, so the earliest unfinished
// slot can always start).  Every task is in the queue exactly once, so a
// workgroup that pops slot h >= ntasks exits.  A spin that exceeds
// spin_limit sets abort/error and every workgroup exits.  Memory ordering costs whole-L2
// operations on this chip (an agent-scope release writes back the XCD's
// L2, an acquire invalidates it), so each task pays exactly one of each: no
// acquire while polling, none on push.  `slot` is an int in LDS.
template <class Run>
__device__ __forceinline__ void executor_loop(const ExecArgs &a, int *slot, Run run) {
  ExecCtl *ctl = a.ctl;
  for (;;) {
    // Every iteration starts with all threads past their last use of LDS.
    __syncthreads();
    if (threadIdx.x == 0) {
      int task = -1;
      const int h = __hip_atomic_fetch_add(&ctl->head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (h < a.ntasks) {
        const int64_t t0 = wall_clock64();
        for (;;) {
          // Relaxed polling (an acquire here would invalidate this XCD's L2
          // at every poll, under every other workgroup's feet).  A popped
          // task synchronises with all its predecessors at once: each
          // released its results and then decremented indeg[task], so
          // reading the final count of zero (the end of that chain of
          // read-modify-writes) and then fencing acquires every one of them.
          const int t = ld_relaxed(&a.queue[h]);
          if (t >= 0 && ld_relaxed(&a.indeg[t]) == 0) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            task = t;
            break;
          }
          if (ld_relaxed(&ctl->abort)) break;
          if (wall_clock64() - t0 > a.spin_limit) {
            __hip_atomic_store(&ctl->error, -1000, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            st_release(&ctl->abort, 1);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      *slot = task;
    }
    __syncthreads();
    // The task id is wave-uniform; reading it as a scalar makes the loop exit
    // a scalar branch, so no lane can leave the loop while others stay in it.
    const int tid = __builtin_amdgcn_readfirstlane(*slot);
    if (tid < 0) break;
    // (thread 0's acquire before the barrier invalidated the caches this
    // CU reads through; the barrier orders every wave's loads after it)
    const int64_t tstart = a.trace ? (int64_t)wall_clock64() : 0;
    run(load_task(a.tasks + tid));
    // Every wave's stores reach L2 before the barrier (a workgroup barrier
    // alone does not wait for them); thread 0 then releases the task's
    // results to the device with one L2 write-back.
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (a.trace && tid < a.trace_cap) {
        int64_t *tr = a.trace + 4 * (int64_t)tid;
        tr[0] = tstart;
        tr[1] = (int64_t)wall_clock64();
        tr[2] = blockIdx.x;
        tr[3] = (int64_t)__smid();
      }
      for (int e = a.succ_off[tid]; e < a.succ_off[tid + 1]; e++) {
        const int s = a.succ[e];
        if (__hip_atomic_fetch_add(&a.indeg[s], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1 &&
            !a.static_order) {
          const int q = __hip_atomic_fetch_add(&ctl->tail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          // every task is pushed at most once, so q < ntasks unless the
          // launch's queue was filled up front without static_order set; a
          // push past the end is dropped (the watchdog then reports it)
          // rather than written over the dependency counts
          if (q < a.ntasks) __hip_atomic_store(&a.queue[q], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      __hip_atomic_fetch_add(&ctl->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace tqr
