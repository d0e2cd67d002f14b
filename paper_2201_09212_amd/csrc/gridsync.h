// Grid-wide synchronization for the persistent kernels (cooperative launch,
// at most one workgroup per CU, so every workgroup is resident).
//
// Everything that crosses workgroups (the iterate, the partial sums) moves
// through agent-scope relaxed atomics, which are coherent across the XCDs'
// separate L2 caches by themselves; no cache write-back or invalidation is
// issued, so the read-only A stays cached between sweeps.
//
// Barrier + residual reduction without read-modify-write atomics: for its
// k-th synchronization a workgroup first drains its own stores, then
// publishes its partial sum in slot[k & 1][lb] (one slot per 256 bytes),
// tagged with a number derived from k (publish below: the whole FP64 value
// and the tag in two words).  Every workgroup polls all G slots of that
// parity (one slot per thread, in parallel) until each carries the tag, and
// sums them in slot order: every workgroup gets the same bits, hence the same
// convergence decision, without a broadcast step.  Double-buffering by parity is enough: a workgroup can
// only overwrite a slot of parity k & 1 at synchronization k + 2, after every
// workgroup has published for k + 1, i.e. finished polling for k.  Slots
// start at tag 0, which no synchronization uses.
#pragma once

#include "common.h"

namespace vfpi {

template <class T>
VFPI_DEV T ld_relaxed(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
VFPI_DEV void st_relaxed(T* p, T x) {
  __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Drain this thread's outstanding memory operations (vector and scalar).
VFPI_DEV void drain() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
}

VFPI_DEV unsigned sync_tag(int seq) { return (unsigned)(seq % 255) + 1u; }

// A partial travels as two tagged 8-byte words: the double's upper 56 bits
// with the tag in the low byte, and its low byte moved up by 8 bits with the
// same tag.  Each word is a single-copy atomic store, so a reader that finds
// the tag in both words holds the whole FP64 value of one publication.
VFPI_DEV void publish(uint64_t* p, double x, unsigned tag) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  st_relaxed<uint64_t>(p, (b & ~0xffull) | tag);
  st_relaxed<uint64_t>(p + 1, ((b & 0xffull) << 8) | tag);
}
VFPI_DEV bool tagged_both(uint64_t w0, uint64_t w1, unsigned tag) {
  return ((w0 & 0xffull) == tag) & ((w1 & 0xffull) == tag);
}
VFPI_DEV double joined(uint64_t w0, uint64_t w1) {
  return __builtin_bit_cast(double, (w0 & ~0xffull) | ((w1 >> 8) & 0xffull));
}
// Poll one slot (both words) until it carries `tag`; the words in w0, w1.
VFPI_DEV void poll_slot(const uint64_t* p, unsigned tag, uint64_t& w0, uint64_t& w1) {
  for (;;) {
    w0 = ld_relaxed(p);
    w1 = ld_relaxed(p + 1);
    if (tagged_both(w0, w1, tag)) return;
    __builtin_amdgcn_s_sleep(1);
  }
}

// Sum over the workgroup of the polled slots with one workgroup barrier:
// wave sums (DPP) go to red[0, nw) and every thread adds them in wave order,
// the same arithmetic as block_sum.  No trailing barrier is needed: red is
// written again only by the next grid_sum / grid_sum3, after its own
// pre-publication barrier, which every thread reaches after reading here.
VFPI_DEV double poll_sum(double acc, double* red) {
  acc = wave_sum(acc);
  const int nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// Synchronization number `seq` (1, 2, ... in the same order in every
// workgroup).  `x` is this workgroup's partial (valid in thread 0).  Returns
// the fixed-order sum of all workgroups' partials in every thread.  s_poll
// (LDS, 3 doubles per wave, apart from the callers' block_sum buffer) takes
// the wave sums of the polled slots.
VFPI_DEV double grid_sum(uint64_t* slots, int G, int lb, int seq, double x, double* s_poll) {
  const unsigned tag = sync_tag(seq);
  uint64_t* sl = slots + (seq & 1) * (int64_t)kMaxGridSlots * kSlotPad;
  drain();
  __syncthreads();
  if (threadIdx.x == 0) publish(sl + (int64_t)lb * kSlotPad, x, tag);
  double acc = 0.0;
  for (int k = threadIdx.x; k < G; k += blockDim.x) {
    uint64_t w0, w1;
    poll_slot(sl + (int64_t)k * kSlotPad, tag, w0, w1);
    acc += joined(w0, w1);
  }
  return poll_sum(acc, s_poll);
}

// Three partials at once (valid in every thread of the workgroup), in the slot
// region `reg` = [2][3][kMaxGridSlots] slots of two words with its own
// sequence numbers; the same tagging and double-buffering argument as
// grid_sum applies per region.
// Returns the fixed-order sums in x, in every thread.
VFPI_DEV void grid_sum3(uint64_t* reg, int G, int lb, int seq, double x[3], double* s_red, double* s_poll) {
  if (G == 1) {
#pragma unroll
    for (int q = 0; q < 3; ++q) x[q] = block_sum(x[q], s_red);
    return;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) x[q] = block_sum(x[q], s_red);
  const unsigned tag = sync_tag(seq);
  uint64_t* sl = reg + (seq & 1) * 6 * (int64_t)kMaxGridSlots;
  drain();
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) publish(sl + 2 * ((int64_t)q * kMaxGridSlots + lb), x[q], tag);
  }
  double acc[3] = {0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < G; k += blockDim.x) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      uint64_t w0, w1;
      poll_slot(sl + 2 * ((int64_t)q * kMaxGridSlots + k), tag, w0, w1);
      acc[q] += joined(w0, w1);
    }
  }
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int q = 0; q < 3; ++q) acc[q] = wave_sum(acc[q]);
  double* red = s_poll;  // 3 nw doubles, one barrier for the three sums (see poll_sum)
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) red[q * nw + (threadIdx.x >> 6)] = acc[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += red[q * nw + i];
    x[q] = t;
  }
}

// Residual reduction + convergence test of Alg. 1 (theta < tol or l = l_max).
// Every thread of every workgroup calls with the same seq.  `th2` is this
// workgroup's partial (valid in thread 0).  Workgroup 0 writes iters,
// status and theta of the stopping sweep.
VFPI_DEV bool grid_residual_step(uint64_t* slots, int G, int lb, int seq, double th2, int l, int max_iters,
                                 int fixed, double tol, vfpi_stats* stats, double* s_poll,
                                 double* theta_out = nullptr) {
  const double tot = (G == 1) ? th2 : grid_sum(slots, G, lb, seq, th2, s_poll);
  const double theta = sqrt(tot);
  if (theta_out) *theta_out = theta;
  const bool conv = !fixed && theta < tol;
  const bool stop = conv || l >= max_iters;
  if (stop && lb == 0 && threadIdx.x == 0) {
    stats->iters = l;
    stats->status = conv ? VFPI_S_CONVERGED : VFPI_S_MAXITER;
    stats->theta = theta;
  }
  return stop;
}

// ---- lagged residual and neighbour barrier --------------------------------
// Without Chebyshev acceleration the stop test of sweep l can wait: after
// publishing sweep l's partial, a workgroup waits only for the workgroups
// that own columns of its rows (its neighbours, a symmetric relation since A
// is symmetric) to have published sweep l, which is all that sweep l + 1's
// gathers need, and for every workgroup's partial of sweep l - 1, which is
// the stop test of sweep l - 1, taken one sweep late.  When it stops, sweep
// l - 1's results are still at hand: v^l is the buffer sweep l read, the
// contact results are double-buffered by sweep parity.  Sweep l + 1 of
// workgroup X overwrites v^l only after X's neighbours, the only readers of
// X's nodes, have published sweep l.  Slots form a ring of four: a
// workgroup publishes sweep l + 4 only after every workgroup has published
// l + 2, which each does only after it has read all partials of sweep l (with
// three, a workgroup that is not X's neighbour could overwrite the slot of
// sweep l while X still reads it).  Every wait is bounded (kSpinLimit polls);
// a workgroup that gives up sets VFPI_S_SYNC_TIMEOUT and leaves the loop, so
// the kernel ends even if the protocol were broken.
constexpr int kSpinLimit = 1 << 21;

VFPI_DEV uint64_t* ring_slot(uint64_t* slots, int l, int k) {
  return slots + ((int64_t)(l & (kSlotRings - 1)) * kMaxGridSlots + k) * kSlotPad;
}

// Poll one slot until it carries `tag` (both words, or only the first when
// the value is not wanted); false on timeout.
VFPI_DEV bool spin_tag(const uint64_t* p, unsigned tag, uint64_t& w0, uint64_t& w1, bool both) {
  for (int n = 0; n < kSpinLimit; ++n) {
    w0 = ld_relaxed(p);
    w1 = both ? ld_relaxed(p + 1) : (uint64_t)tag;
    if (tagged_both(w0, w1, tag)) return true;
    __builtin_amdgcn_s_sleep(1);
  }
  return false;
}

struct LagResult {
  int stop;      // sweep at which Alg. 1 stops (0: go on)
  int status;    // VFPI_S_CONVERGED / VFPI_S_MAXITER (/ VFPI_S_SYNC_TIMEOUT)
  double theta;  // residual of the stopping sweep
};

// End of sweep l (every thread calls; th2 = this workgroup's partial, valid
// in every thread).  nbm: bitmap of the neighbour workgroups (LDS).  s_poll:
// 3 doubles per wave, s_flag: one int (LDS).
VFPI_DEV LagResult lag_sync(uint64_t* slots, int G, int lb, int l, double th2, int max_iters, int fixed, double tol,
                            const uint32_t* nbm, double* s_poll, int* s_flag) {
  const unsigned tag_l = sync_tag(l), tag_p = sync_tag(l - 1);
  // the flag's readers of the previous call have all passed the sweep's
  // barriers since, and its writers below come after the next one
  if (threadIdx.x == 0) *s_flag = 0;
  drain();
  __syncthreads();
  if (threadIdx.x == 0) publish(ring_slot(slots, l, lb), th2, tag_l);
  const bool last = l >= max_iters;
  const bool prev = !fixed && l >= 2;
  double acc_p = 0.0, acc_l = 0.0;
  bool ok = true;
  for (int k = threadIdx.x; k < G && ok; k += blockDim.x) {
    // both slots' loads in flight together; a slot not yet tagged is then
    // polled on its own
    const bool want_l = last || ((nbm[k >> 5] >> (k & 31)) & 1u);
    const uint64_t* pp = ring_slot(slots, l - 1, k);
    const uint64_t* pl = ring_slot(slots, l, k);
    // (a neighbour's slot of sweep l is only waited for, its value unused
    // before the last sweep: its first word, which carries the tag, suffices)
    uint64_t bp0 = prev ? ld_relaxed(pp) : 0ull, bp1 = prev ? ld_relaxed(pp + 1) : 0ull;
    uint64_t bl0 = want_l ? ld_relaxed(pl) : 0ull, bl1 = last ? ld_relaxed(pl + 1) : tag_l;
    if (prev && !tagged_both(bp0, bp1, tag_p)) ok = spin_tag(pp, tag_p, bp0, bp1, true);
    if (ok && want_l && !tagged_both(bl0, bl1, tag_l)) ok = spin_tag(pl, tag_l, bl0, bl1, last);
    acc_p += prev ? joined(bp0, bp1) : 0.0;
    acc_l += last ? joined(bl0, bl1) : 0.0;
  }
  if (!ok) atomicOr(s_flag, 1);  // read after poll_sum's barrier
  acc_p = prev ? poll_sum(acc_p, s_poll) : 0.0;
  __syncthreads();
  acc_l = last ? poll_sum(acc_l, s_poll) : 0.0;
  LagResult r = {0, VFPI_S_MAXITER, 0.0};
  if (*s_flag) {
    r.stop = l;
    r.status = VFPI_S_SYNC_TIMEOUT;
    r.theta = INFINITY;
    return r;
  }
  if (prev && sqrt(acc_p) < tol) {
    r.stop = l - 1;
    r.status = VFPI_S_CONVERGED;
    r.theta = sqrt(acc_p);
  } else if (last) {
    r.stop = l;
    r.theta = sqrt(acc_l);
    r.status = (!fixed && r.theta < tol) ? VFPI_S_CONVERGED : VFPI_S_MAXITER;
  }
  return r;
}

// D-contact phase of sweep l in the lagged kernel: after draining its
// stores of v* (its D-contact nodes'), a workgroup tags its slot of ring
// l & 1 and waits for its partner workgroups (the owners of the other nodes
// of its D-contacts, bitmap pbm in LDS; a symmetric relation) to have tagged
// theirs.  A ring of two suffices: a workgroup tags its slot for sweep l + 2
// only after its partners tagged l + 1, which each did after reading what
// sweep l published.  The v* buffer is double-buffered by the same parity.
// Bounded: returns false in every thread of the workgroup on a timeout.
// s_pflag: one int (LDS), for this call only.
VFPI_DEV bool pair_sync(uint64_t* slots, int G, int lb, int l, const uint32_t* pbm, int* s_pflag) {
  const unsigned tag = sync_tag(l);
  uint64_t* ring = slots + kDSlotOffset + (int64_t)(l & 1) * kMaxGridSlots * kSlotPad;
  // the flag's readers of the previous call have passed the sweep's barriers
  if (threadIdx.x == 0) *s_pflag = 0;
  drain();
  __syncthreads();
  if (threadIdx.x == 0) st_relaxed<uint64_t>(ring + (int64_t)lb * kSlotPad, (uint64_t)tag);
  bool ok = true;
  for (int k = threadIdx.x; k < G && ok; k += blockDim.x) {
    if ((pbm[k >> 5] >> (k & 31)) & 1u) {
      uint64_t w0, w1;
      ok = spin_tag(ring + (int64_t)k * kSlotPad, tag, w0, w1, false);
    }
  }
  if (!ok) atomicOr(s_pflag, 1);
  __syncthreads();
  return *s_pflag == 0;
}

// Plain grid barrier: every write before it is visible to every workgroup
// after it (through coherent loads).
VFPI_DEV void grid_barrier(uint64_t* slots, int G, int lb, int seq, double* s_poll) {
  if (G == 1) {
    __syncthreads();
    return;
  }
  (void)grid_sum(slots, G, lb, seq, 0.0, s_poll);
}

// Branch counts of the final sweep: integer atomics, so the totals do not
// depend on the order (the counters are zeroed before the launch).
VFPI_DEV void add_counts(vfpi_stats* st, int o, int s, int sl) {
  if (threadIdx.x == 0) {
    if (o) atomicAdd(&st->n_open, o);
    if (s) atomicAdd(&st->n_stick, s);
    if (sl) atomicAdd(&st->n_slip, sl);
  }
}

// Chebyshev acceleration state (Alg. 3), identical in every workgroup because
// it only depends on the reduced residuals.
struct Cheby {
  int ls = 0;            // 0: off
  double u = 1.0;
  double nu = 1.0, rho = 0.0, theta_prev = 0.0;
  // nu_{l+1} used by sweep l
  VFPI_DEV double next_nu(int l) {
    if (ls == 0) return nu = 1.0;  // off: plain V-FPI, no divisions
    if (l < ls) nu = 1.0;
    else if (l == ls) nu = 2.0 / (2.0 - rho * rho);
    else nu = 4.0 / (4.0 - rho * rho * nu);
    return nu;
  }
  // after the stop test of sweep l (eq. varrho from the two latest residuals)
  VFPI_DEV void observe(double theta) {
    rho = theta_prev > 0.0 ? fmin(theta / theta_prev, 1.0) : 0.0;
    theta_prev = theta;
  }
};

// Workgroup numbering that gives each XCD one contiguous range of work
// (workgroups are dealt round-robin to the 8 XCDs).
VFPI_DEV int xcd_logical_block(int b, int G) { return (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b; }

}  // namespace vfpi
