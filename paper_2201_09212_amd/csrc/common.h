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
constexpr int kPack = 13;  // per-contact record: R (9), phi, mu, gamma, mu2
constexpr int kMaxGridSlots = 1024;  // workgroups of a persistent launch (slots per parity)
// Slot memory of the grid reductions: region 0 = [4][kMaxGridSlots] slots for
// the residual / barrier (rings 0-1 for the synchronous reduction, 0-3 for the
// lagged one), each slot alone in kSlotPad words (256 bytes) so that the
// workgroups polling one slot do not contend with those polling its
// neighbours; region 1 = [2][3][kMaxGridSlots] slots of two words for the
// three dot products of the Barzilai-Borwein step size; region 2 =
// [2][kMaxGridSlots] tag slots (padded like region 0) for the lagged
// kernel's D-contact phase.  A slot's value takes two words (see publish in
// gridsync.h).
constexpr int kSlotPad = 32;
constexpr int kSlotRings = 4;
constexpr int kBBSlotOffset = kSlotRings * kMaxGridSlots * kSlotPad;
constexpr int kDSlotOffset = kBBSlotOffset + 12 * kMaxGridSlots;
constexpr int kSlotWords = kDSlotOffset + 2 * kMaxGridSlots * kSlotPad;

VFPI_DEV uint64_t ballot(bool p) { return __ballot(p); }

VFPI_DEV int lanes_below(uint64_t mask, int lane) {
  (void)lane;
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

VFPI_DEV void set_flag(int32_t* flags, int32_t bit) { atomicOr(flags, bit); }

// Loads / stores of the V-FPI iterate v.  COH = true: agent-scope relaxed
// atomics, coherent across the XCDs' separate L2 caches without any cache
// write-back or invalidation, so the persistent kernel's grid barrier needs
// no fences and the read-only A stays cached between sweeps.
template <bool COH, class T>
VFPI_DEV T ldv(const T* p) {
  if constexpr (COH)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *p;
}

template <bool COH, class T>
VFPI_DEV void stv(T* p, T x) {
  if constexpr (COH)
    __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = x;
}

// One row of a 3x3 block times x.  FP64: in a fixed rounding order, with
// explicit fused multiply-adds, fma(a2, x2, fma(a1, x1, a0 x0)), so that
// every kernel and instance rounds the product alike, whatever the compiler
// would contract on its own (which can depend on how the operands were
// produced).  FP32 (the batched form): as the compiler contracts it.
template <class T>
VFPI_DEV T dot3(T a0, T a1, T a2, T x0, T x1, T x2) {
  return a0 * x0 + a1 * x1 + a2 * x2;
}
template <>
VFPI_DEV double dot3<double>(double a0, double a1, double a2, double x0, double x1, double x2) {
  return __builtin_fma(a2, x2, __builtin_fma(a1, x1, a0 * x0));
}

// Chunk-interleaved copy of A: the blocks of level k of a chunk (ck of them,
// one per row that has a k-th block, in lane order) sit at block offset q.
// Position of entry e (row-major, 0..8) of the block of lane position pos.
// FP64 (80 bytes a block, so every level starts 16-byte aligned): entries
// (0,1), (2,3), (4,5), (6,7) as 16-byte pairs, each pair for all ck lanes in
// lane order, then for all lanes a 16-byte record of entry 8 and the block's
// column (the low 32 bits of the record's second word), so that a lane reads
// its block and column with five 16-byte loads (each load instruction
// reading one contiguous run over the lanes).  FP32 (36 bytes a block):
// entry-major (entry e for all lanes, then e + 1); its columns are in scol.
constexpr int kSvalWords64 = 10;
template <class T>
VFPI_DEV int64_t sval_at(int64_t q, int ck, int pos, int e) {
  if constexpr (sizeof(T) == 8)
    return kSvalWords64 * q + 2 * ((int64_t)ck * (e >> 1) + pos) + (e & 1);  // e = 8: the record
  else
    return 9 * q + (int64_t)e * ck + pos;
}

typedef double vfpi_d2 __attribute__((ext_vector_type(2)));

// Entries 0..7 of a block of the FP64 interleaved copy (see sval_at).
VFPI_DEV void load_spairs(const double* __restrict__ sval, int64_t q, int ck, int pos, double a[9]) {
  const double* bp = sval + kSvalWords64 * q + 2 * pos;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const vfpi_d2 t = *reinterpret_cast<const vfpi_d2*>(bp + 2 * (int64_t)ck * p);
    a[2 * p] = t.x;
    a[2 * p + 1] = t.y;
  }
}
// Entry 8 and the column of a block of the FP64 interleaved copy.
VFPI_DEV int load_srec(const double* __restrict__ sval, int64_t q, int ck, int pos, double& a8) {
  const vfpi_d2 t = *reinterpret_cast<const vfpi_d2*>(sval + kSvalWords64 * q + 8 * (int64_t)ck + 2 * pos);
  a8 = t.x;
  // (through a scalar: this compiler's __builtin_bit_cast of a vector
  // element reads element 0, whichever element is named)
  const double cw = t.y;
  return (int)(uint32_t)__builtin_bit_cast(uint64_t, cw);
}

// One block of the interleaved copy into registers (see sval_at).
VFPI_DEV void load_sblock(const double* __restrict__ sval, int64_t q, int ck, int pos, double a[9]) {
  load_spairs(sval, q, ck, pos, a);
  a[8] = sval[sval_at<double>(q, ck, pos, 8)];
}
VFPI_DEV void load_sblock(const float* __restrict__ sval, int64_t q, int ck, int pos, float a[9]) {
  const float* ap = sval + 9 * q + pos;
#pragma unroll
  for (int e = 0; e < 9; ++e) a[e] = ap[(int64_t)e * ck];
}

// The three components of node c of an FP64 iterate x (24 bytes) in two
// loads of 16 and 8 bytes instead of three.  COH: with the agent-coherent
// cache policy (the bit the relaxed agent-scope atomic loads set), through a
// raw buffer resource over x; no atomicity is needed, since the values were
// published before the barrier that precedes the gather.
typedef unsigned int vfpi_u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int vfpi_u32x2 __attribute__((ext_vector_type(2)));
template <bool COH>
VFPI_DEV void ldv3(const double* __restrict__ x, int64_t c, double out[3]) {
  if constexpr (COH) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(x), 0, 0x7fffffff, 0x00020000);
    const uint32_t off = 24u * (uint32_t)c;
    const vfpi_u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 1 << 4);
    const vfpi_u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(rs, off + 16u, 0, 1 << 4);
    out[0] = __builtin_bit_cast(double, (uint64_t)a[0] | ((uint64_t)a[1] << 32));
    out[1] = __builtin_bit_cast(double, (uint64_t)a[2] | ((uint64_t)a[3] << 32));
    out[2] = __builtin_bit_cast(double, b);
  } else {
    out[0] = x[3 * c];
    out[1] = x[3 * c + 1];
    out[2] = x[3 * c + 2];
  }
}

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

// Lagrange multiplier s > 0 of the closest point a_i^2 t_i / (a_i^2 + s) to
// (t1, t2) outside the ellipse of semi-axes a, b > 0: the root of
// F(s) = sum_i a_i^2 t_i^2 / (a_i^2 + s)^2 - 1, which is convex and falling
// for s >= 0.  Each term of F + 1 is at most 1 at the root, so
// s >= a |t1| - a^2 and s >= b |t2| - b^2: Newton starts at that lower bound
// (left of the root) and climbs monotonically until it stops gaining.
template <class T>
VFPI_DEV T ellipse_multiplier(T a, T b, T t1, T t2) {
  const T a2 = a * a, b2 = b * b, c1 = a2 * t1 * t1, c2 = b2 * t2 * t2;
  T s = fmax(T(0), fmax(a * fabs(t1) - a2, b * fabs(t2) - b2));
  for (int it = 0; it < 200; ++it) {
    const T r1 = T(1) / (a2 + s), r2 = T(1) / (b2 + s);
    const T f1 = c1 * r1 * r1, f2 = c2 * r2 * r2;
    const T F = f1 + f2 - T(1);
    const T dF = T(-2) * (f1 * r1 + f2 * r2);
    const T sn = s - F / dF;
    if (!(sn > s)) break;
    s = sn;
  }
  return s;
}

// Strict operator on the elliptic cone t1^2/mu1^2 + t2^2/mu2^2 <= lambda_n^2
// (anisotropic friction, Sec. III-E): lambda_t = the closest point to t in the
// ellipse of semi-axes a = mu1 lambda_n, b = mu2 lambda_n, which is the
// maximal-dissipation answer (Prop. 6).  Outside it, x_i = a_i^2 t_i / (a_i^2
// + s) with s from ellipse_multiplier.  A zero semi-axis makes the ellipse a
// segment (clamp).
template <class T>
VFPI_DEV int project_ellipse(T& n, T& t1, T& t2, T mu1, T mu2) {
  if (!(n > T(0))) {
    n = t1 = t2 = T(0);
    return BR_OPEN;
  }
  const T a = mu1 * n, b = mu2 * n;
  if (a == T(0) || b == T(0)) {
    const T x1 = fmin(fmax(t1, -a), a), x2 = fmin(fmax(t2, -b), b);
    const bool in = (x1 == t1) && (x2 == t2);
    t1 = x1;
    t2 = x2;
    return in ? BR_STICK : BR_SLIP;
  }
  const T tb = t1 * b, ta = t2 * a, ab = a * b;
  if (tb * tb + ta * ta <= ab * ab) return BR_STICK;
  const T a2 = a * a, b2 = b * b;
  const T s = ellipse_multiplier(a, b, t1, t2);
  t1 = a2 * t1 / (a2 + s);
  t2 = b2 * t2 / (b2 + s);
  return BR_SLIP;
}

// mu2 != mu selects the anisotropic strict operator (the caller refuses it
// with the proximal operator).
template <class T>
VFPI_DEV int project(int mode, T& n, T& t1, T& t2, T mu, T mu2) {
  if (mode == VFPI_PROJ_PROXIMAL) return project_proximal(n, t1, t2, mu);
  return (mu2 != mu) ? project_ellipse(n, t1, t2, mu, mu2) : project_strict(n, t1, t2, mu);
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

// Level masks of a group of U levels starting at k0: mask, active count and
// the level's offset inside the chunk's block range.
template <int U>
VFPI_DEV bool level_group(int k0, int nk, int64_t& off, uint64_t m[U], int cnt[U], int64_t offk[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    m[u] = ballot(k0 + u < nk);
    cnt[u] = __popcll(m[u]);
    offk[u] = off;
    off += cnt[u];
  }
  return m[0] != 0;
}

// y_r += sum_blocks A_block[r][:] . x[col]  for r = 0..2  (one lane = one node),
// over the levels k >= k_start (whose blocks start at offset off_start of the
// chunk's block range).  Levels are processed in groups of U: all column
// indices and block entries of the group are loaded first, then all gathers
// of x, then the products, so the group's memory latencies overlap instead of
// chaining level by level.  The accumulation order is level by level.
//
// BF (default for FP64, whose kernels are latency-bound): the group's loads
// are issued by every lane as one straight-line block.  The FP32 batched
// kernel is bandwidth-bound and keeps the form where only lanes with the
// level load.
template <class T, bool COH = false, int U = 4, bool BF = (sizeof(T) == 8)>
VFPI_DEV void spmv_rows3_from(const int32_t* __restrict__ scol, const T* __restrict__ sval,
                              const T* __restrict__ x, int64_t base, int nk, int lane, int k_start,
                              int64_t off_start, T acc[3]) {
  int64_t off = off_start;
  for (int k0 = k_start;; k0 += U) {
    uint64_t m[U];
    int cnt[U];
    int64_t offk[U];
    if (!level_group<U>(k0, nk, off, m, cnt, offk)) break;
    if constexpr (BF) {
      // Every lane loads, so that the group's loads form one straight-line
      // block: behind a divergent branch each level's gather would wait for all
      // earlier loads (the wait counters are merged at the branch's join).  A
      // lane without level k0 + u reads a block inside that level's range (or
      // level k0's, when no lane has k0 + u) and drops it in the select below.
      // The group's column indices are issued before its block entries, so
      // that each gather waits only for the columns (loads return in issue
      // order) while the entries are still in flight.
      // (FP64: each column comes with its block's entry 8, in one load.)
      int c[U], cu[U], pos[U];
      int64_t q[U];
      T a[U][9];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool any = cnt[u] > 0;  // the same in every lane; cnt[0] > 0
        cu[u] = any ? cnt[u] : cnt[0];
        q[u] = base + (any ? offk[u] : offk[0]);
        pos[u] = min(lanes_below(any ? m[u] : m[0], lane), cu[u] - 1);
        if constexpr (sizeof(T) == 8)
          c[u] = load_srec(sval, q[u], cu[u], pos[u], a[u][8]);
        else
          c[u] = scol[q[u] + pos[u]];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if constexpr (sizeof(T) == 8)
          load_spairs(sval, q[u], cu[u], pos[u], a[u]);
        else
          load_sblock(sval, q[u], cu[u], pos[u], a[u]);
      }
      T xs[U][3];
#pragma unroll
      for (int u = 0; u < U; ++u) ldv3<COH>(x, c[u], xs[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool has = k0 + u < nk;
        const T y0 = acc[0] + dot3(a[u][0], a[u][1], a[u][2], xs[u][0], xs[u][1], xs[u][2]);
        const T y1 = acc[1] + dot3(a[u][3], a[u][4], a[u][5], xs[u][0], xs[u][1], xs[u][2]);
        const T y2 = acc[2] + dot3(a[u][6], a[u][7], a[u][8], xs[u][0], xs[u][1], xs[u][2]);
        acc[0] = has ? y0 : acc[0];
        acc[1] = has ? y1 : acc[1];
        acc[2] = has ? y2 : acc[2];
      }
    } else {
      // streaming form (bandwidth-bound callers): only lanes with the level load
      int c[U];
      T a[U][9];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        c[u] = 0;
        if (k0 + u < nk) {
          const int pos = lanes_below(m[u], lane);
          const int64_t q = base + offk[u];
          c[u] = scol[q + pos];
          load_sblock(sval, q, cnt[u], pos, a[u]);
        }
      }
      T xs[U][3];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (k0 + u < nk) {
          const T* xp = x + 3 * (int64_t)c[u];
          xs[u][0] = ldv<COH>(xp);
          xs[u][1] = ldv<COH>(xp + 1);
          xs[u][2] = ldv<COH>(xp + 2);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (k0 + u < nk) {
          acc[0] += a[u][0] * xs[u][0] + a[u][1] * xs[u][1] + a[u][2] * xs[u][2];
          acc[1] += a[u][3] * xs[u][0] + a[u][4] * xs[u][1] + a[u][5] * xs[u][2];
          acc[2] += a[u][6] * xs[u][0] + a[u][7] * xs[u][1] + a[u][8] * xs[u][2];
        }
      }
    }
  }
}

template <class T, bool COH = false, int U = 4>
VFPI_DEV void spmv_rows3(const int32_t* __restrict__ scol, const T* __restrict__ sval,
                         const T* __restrict__ x, int64_t base, int nk, int lane, T acc[3]) {
  acc[0] = acc[1] = acc[2] = T(0);
  spmv_rows3_from<T, COH, U>(scol, sval, x, base, nk, lane, 0, 0, acc);
}

// y = sum_blocks A_block[r][:] . x[col] for one row r (one lane = one node row),
// with the same grouped issue order.
template <class T, bool COH = false, int U = 8>
VFPI_DEV T spmv_row1(const int32_t* __restrict__ scol, const T* __restrict__ sval,
                     const T* __restrict__ x, int64_t base, int nk, int lane, int r) {
  T acc = T(0);
  int64_t off = 0;
  for (int k0 = 0;; k0 += U) {
    uint64_t m[U];
    int cnt[U];
    int64_t offk[U];
    if (!level_group<U>(k0, nk, off, m, cnt, offk)) break;
    int c[U];
    T a[U][3];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = 0;
      if (k0 + u < nk) {
        const int pos = lanes_below(m[u], lane);
        const int64_t q = base + offk[u];
        c[u] = scol[q + pos];
#pragma unroll
        for (int j = 0; j < 3; ++j) a[u][j] = sval[sval_at<T>(q, cnt[u], pos, 3 * r + j)];
      }
    }
    T xs[U][3];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (k0 + u < nk) {
        const T* xp = x + 3 * (int64_t)c[u];
        xs[u][0] = ldv<COH>(xp);
        xs[u][1] = ldv<COH>(xp + 1);
        xs[u][2] = ldv<COH>(xp + 2);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k0 + u < nk) acc += dot3(a[u][0], a[u][1], a[u][2], xs[u][0], xs[u][1], xs[u][2]);
  }
  return acc;
}

// ---- reductions ---------------------------------------------------------
// Fixed-order sum of one double and three ints over a workgroup in one pass.
VFPI_DEV void block_sum4(double& x, int& a, int& b, int& c, double* red, int* ired) {
  for (int o = 32; o > 0; o >>= 1) {
    x += __shfl_xor(x, o, 64);
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  const int wv = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[wv] = x;
    ired[3 * wv] = a;
    ired[3 * wv + 1] = b;
    ired[3 * wv + 2] = c;
  }
  __syncthreads();
  x = 0.0;
  a = b = c = 0;
  for (int i = 0; i < nw; ++i) {
    x += red[i];
    a += ired[3 * i];
    b += ired[3 * i + 1];
    c += ired[3 * i + 2];
  }
  __syncthreads();
}

// Workgroup sum of three ints (order-independent), result in every thread.
VFPI_DEV void block_sum4_int(int& a, int& b, int& c, int* ired) {
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  const int wv = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    ired[3 * wv] = a;
    ired[3 * wv + 1] = b;
    ired[3 * wv + 2] = c;
  }
  __syncthreads();
  a = b = c = 0;
  for (int i = 0; i < nw; ++i) {
    a += ired[3 * i];
    b += ired[3 * i + 1];
    c += ired[3 * i + 2];
  }
  __syncthreads();
}

// Fixed-order sum over a workgroup (deterministic): wave butterfly, then the
// per-wave totals summed in wave order by thread 0.  Result valid in all
// threads.  `red` is __shared__ scratch of >= blockDim/64 doubles.
// One DPP move of a double (two 32-bit halves); lanes whose source lies
// outside the pattern, or whose row is masked off, read 0.
template <int CTRL, int ROW_MASK>
VFPI_DEV double dpp_f64(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 64 lanes of a full wave, returned in every lane: an inclusive
// scan inside each row of 16 lanes (row_shr 1, 2, 4, 8), then the row totals
// carried forward by row_bcast 15 (into rows 1, 3) and row_bcast 31 (into
// rows 2, 3), so lane 63 holds the total, read back as a scalar.  Register
// moves only, where a shuffle butterfly goes through LDS six times.
VFPI_DEV double wave_sum(double x) {
  x += dpp_f64<0x111, 0xf>(x);
  x += dpp_f64<0x112, 0xf>(x);
  x += dpp_f64<0x114, 0xf>(x);
  x += dpp_f64<0x118, 0xf>(x);
  x += dpp_f64<0x142, 0xa>(x);
  x += dpp_f64<0x143, 0xc>(x);
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Workgroup sum (every thread calls; full waves), the same bits in every
// thread.
VFPI_DEV double block_sum(double x, double* red) {
  x = wave_sum(x);
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
