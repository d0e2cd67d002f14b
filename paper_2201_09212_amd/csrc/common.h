// Device building blocks shared by the V-FPI kernels (gfx950, wave64).
//
// Layout of A inside the library ("chunk-interleaved" block rows):
// nodes are grouped in chunks of up to 64 consecutive nodes, one chunk per
// wavefront, lane t <-> node n0 + t.  A chunk's blocks occupy the same block
// range [row_ptr[n0], row_ptr[n0+cnt]) as in the caller's block-row layout,
// but permuted by "level": level k holds block k of every lane whose row has
// more than k blocks, packed in lane order, and within a level the 9 entries
// are stored entry-major (all lanes' entry 0, then entry 1, ...).  A lane finds
// its slot with a wave ballot + popcount, so the copy has exactly nnzb blocks
// (no padding), and every entry load of a level is one contiguous,
// fully coalesced run across the active lanes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vfpi.h"

#define VFPI_DEV __device__ __forceinline__

namespace vfpi {

enum { BR_OPEN = 0, BR_STICK = 1, BR_SLIP = 2 };

constexpr int kWave = 64;
constexpr int kPack = 12;  // per-contact record: R (9), phi, mu, gamma

VFPI_DEV uint64_t ballot(bool p) { return __ballot(p); }

VFPI_DEV int lanes_below(uint64_t mask, int lane) {
  (void)lane;
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

VFPI_DEV void set_flag(int32_t* flags, int32_t bit) { atomicOr(flags, bit); }

template <class T>
VFPI_DEV bool finite(T x) { return __builtin_isfinite(x); }

// ---- ProjectFC (eq. operator) ------------------------------------------
// In: lambda* = (n, t1, t2); out: lambda.  Returns the branch.
// Strict: lambda_n = max(n, 0), lambda_t = projection of t onto the disk of
// radius mu * lambda_n.  n <= 0 gives lambda = 0 (open); |t| <= mu lambda_n is
// stick; no division when |t| = 0.
template <class T>
VFPI_DEV int project_strict(T& n, T& t1, T& t2, T mu) {
  if (!(n > T(0))) {
    n = t1 = t2 = T(0);
    return BR_OPEN;
  }
  T s = sqrt(t1 * t1 + t2 * t2);
  T rad = mu * n;
  if (s <= rad) return BR_STICK;
  T sc = rad / s;
  t1 *= sc;
  t2 *= sc;
  return BR_SLIP;
}

// Proximal: Euclidean projection onto {lambda_n >= 0, |lambda_t| <= mu lambda_n}.
template <class T>
VFPI_DEV int project_proximal(T& n, T& t1, T& t2, T mu) {
  T s = sqrt(t1 * t1 + t2 * t2);
  if (s <= mu * n && n >= T(0)) return BR_STICK;
  if (mu * s <= -n) {
    n = t1 = t2 = T(0);
    return BR_OPEN;
  }
  T nn = (n + mu * s) / (T(1) + mu * mu);
  T sc = mu * nn / (s > T(0) ? s : T(1));
  n = nn;
  t1 *= sc;
  t2 *= sc;
  return BR_SLIP;
}

template <class T>
VFPI_DEV int project(int mode, T& n, T& t1, T& t2, T mu) {
  return mode == VFPI_PROJ_PROXIMAL ? project_proximal(n, t1, t2, mu) : project_strict(n, t1, t2, mu);
}

// ---- chunk-interleaved copy of one chunk's block rows ------------------
// Whole wave calls; lanes with t >= cnt pass nk = 0.  src: caller's
// row-major blocks of this lane's row starting at block `rp`.
template <class T, class Fn>
VFPI_DEV void for_each_level(int nk, int lane, Fn&& fn) {
  int64_t off = 0;
  for (int k = 0;; ++k) {
    uint64_t mask = ballot(k < nk);
    if (mask == 0) break;
    int cnt = __popcll(mask);
    if (k < nk) fn(k, off, cnt, lanes_below(mask, lane));
    off += cnt;
  }
}

// y_r = sum_blocks A_block[r][:] . x[col]  for r = 0..2  (one lane = one node)
template <class T>
VFPI_DEV void spmv_rows3(const int32_t* __restrict__ scol, const T* __restrict__ sval,
                         const T* __restrict__ x, int64_t base, int nk, int lane, T acc[3]) {
  acc[0] = acc[1] = acc[2] = T(0);
  int64_t off = 0;
  for (int k = 0;; ++k) {
    uint64_t mask = ballot(k < nk);
    if (mask == 0) break;
    int cnt = __popcll(mask);
    if (k < nk) {
      int pos = lanes_below(mask, lane);
      int64_t q = base + off;
      int c = scol[q + pos];
      const T* a = sval + 9 * q + pos;
      T x0 = x[3 * (int64_t)c], x1 = x[3 * (int64_t)c + 1], x2 = x[3 * (int64_t)c + 2];
      T a0 = a[0], a1 = a[cnt], a2 = a[2 * cnt];
      T a3 = a[3 * cnt], a4 = a[4 * cnt], a5 = a[5 * cnt];
      T a6 = a[6 * cnt], a7 = a[7 * cnt], a8 = a[8 * cnt];
      acc[0] += a0 * x0 + a1 * x1 + a2 * x2;
      acc[1] += a3 * x0 + a4 * x1 + a5 * x2;
      acc[2] += a6 * x0 + a7 * x1 + a8 * x2;
    }
    off += cnt;
  }
}

// y = sum_blocks A_block[r][:] . x[col] for one row r (one lane = one node row)
template <class T>
VFPI_DEV T spmv_row1(const int32_t* __restrict__ scol, const T* __restrict__ sval,
                     const T* __restrict__ x, int64_t base, int nk, int lane, int r) {
  T acc = T(0);
  int64_t off = 0;
  for (int k = 0;; ++k) {
    uint64_t mask = ballot(k < nk);
    if (mask == 0) break;
    int cnt = __popcll(mask);
    if (k < nk) {
      int pos = lanes_below(mask, lane);
      int64_t q = base + off;
      int c = scol[q + pos];
      const T* a = sval + 9 * q + 3 * r * cnt + pos;
      T x0 = x[3 * (int64_t)c], x1 = x[3 * (int64_t)c + 1], x2 = x[3 * (int64_t)c + 2];
      acc += a[0] * x0 + a[cnt] * x1 + a[2 * cnt] * x2;
    }
    off += cnt;
  }
  return acc;
}

// ---- reductions ---------------------------------------------------------
// Fixed-order sum over a workgroup (deterministic): wave butterfly, then the
// per-wave totals summed in wave order by thread 0.  Result valid in all
// threads.  `red` is __shared__ scratch of >= blockDim/64 doubles.
VFPI_DEV double block_sum(double x, double* red) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  int wv = threadIdx.x >> 6;
  int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wv] = x;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

VFPI_DEV int block_sum_int(int x, int* red) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  int wv = threadIdx.x >> 6;
  int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wv] = x;
  __syncthreads();
  int s = 0;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

}  // namespace vfpi
