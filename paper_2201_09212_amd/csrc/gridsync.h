// Grid-wide barriers for the persistent kernels (cooperative launch: every
// workgroup is resident).  One counter + generation word pair in device
// memory; agent-scope acquire/release atomics make the other XCDs' writes
// visible (on gfx950 they emit the L2 write-back / invalidate).
#pragma once

#include "common.h"

namespace vfpi {

// Residual reduction + convergence test of Alg. 1 (theta < tol or l = l_max).
// Every thread of every workgroup calls.  `th2` and `cnt` are this
// workgroup's totals, valid in thread 0.  The last workgroup to arrive sums
// all partials in workgroup-index order (deterministic: the result does not
// depend on which workgroup arrives last), writes the stats when stopping,
// and releases the others.  Returns the common stop decision.
VFPI_DEV bool grid_residual_step(uint32_t* sync, double* red, int32_t* ired, int G, int lb, double th2,
                                 const int cnt[3], int l, int max_iters, int fixed, double tol, vfpi_stats* stats,
                                 double* s_red, int* s_ired) {
  __shared__ int s_last;
  __shared__ unsigned s_gen;
  __shared__ int s_stop;
  auto decide = [&](double tot, int o, int s, int sl) {
    const double theta = sqrt(tot);
    const bool conv = !fixed && theta < tol;
    const bool stop = conv || l >= max_iters;
    if (stop) {
      stats->iters = l;
      stats->status = conv ? VFPI_S_CONVERGED : VFPI_S_MAXITER;
      stats->theta = theta;
      stats->n_open = o;
      stats->n_stick = s;
      stats->n_slip = sl;
      stats->reserved = 0;
    }
    return stop;
  };
  if (G == 1) {
    if (threadIdx.x == 0) s_stop = decide(th2, cnt[0], cnt[1], cnt[2]);
  } else {
    if (threadIdx.x == 0) {
      red[lb] = th2;
      ired[3 * lb] = cnt[0];
      ired[3 * lb + 1] = cnt[1];
      ired[3 * lb + 2] = cnt[2];
      const unsigned gen = __hip_atomic_load(sync + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned old = __hip_atomic_fetch_add(sync, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      s_gen = gen;
      s_last = (old == (unsigned)G - 1u);
    }
    __syncthreads();
    if (s_last) {
      double acc = 0.0;
      int io = 0, is = 0, il = 0;
      for (int k = threadIdx.x; k < G; k += blockDim.x) {
        acc += __hip_atomic_load(red + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        io += __hip_atomic_load(ired + 3 * k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        is += __hip_atomic_load(ired + 3 * k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        il += __hip_atomic_load(ired + 3 * k + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      acc = block_sum(acc, s_red);
      io = block_sum_int(io, s_ired);
      is = block_sum_int(is, s_ired);
      il = block_sum_int(il, s_ired);
      if (threadIdx.x == 0) {
        const bool stop = decide(acc, io, is, il);
        s_stop = stop;
        __hip_atomic_store(red + G, stop ? 1.0 : 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(sync, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(sync + 1, s_gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    } else if (threadIdx.x == 0) {
      while (__hip_atomic_load(sync + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == s_gen)
        __builtin_amdgcn_s_sleep(1);
      s_stop = __hip_atomic_load(red + G, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0.0;
    }
  }
  __syncthreads();
  const bool stop = s_stop != 0;
  __syncthreads();
  return stop;
}

// Plain grid barrier (all writes before it visible to all workgroups after it).
VFPI_DEV void grid_barrier(uint32_t* sync, int G) {
  __shared__ unsigned s_gen2;
  __syncthreads();
  if (G > 1 && threadIdx.x == 0) {
    const unsigned gen = __hip_atomic_load(sync + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned old = __hip_atomic_fetch_add(sync, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_gen2 = gen;
    if (old == (unsigned)G - 1u) {
      __hip_atomic_store(sync, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(sync + 1, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      while (__hip_atomic_load(sync + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == s_gen2)
        __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
}

// Workgroup numbering that gives each XCD one contiguous range of work
// (workgroups are dealt round-robin to the 8 XCDs).
VFPI_DEV int xcd_logical_block(int b, int G) { return (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b; }

}  // namespace vfpi
