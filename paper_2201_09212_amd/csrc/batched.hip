// (compiled as part of vfpi_lib.hip)
// Batched V-FPI: many independent environments of uneven size in one
// persistent launch.  Each workgroup takes environments from an atomic work
// queue (in the caller's env_order), builds that environment's setup (contact
// map, chunk-interleaved A, W, gamma) and runs its whole V-FPI loop with
// workgroup barriers only: FP32 arithmetic, residual accumulated and tested
// in FP64, per-environment exit.  No grid-wide synchronization, so the launch
// can be captured in a HIP graph.
#include <math.h>

#include "internal.h"
#include "setup.h"
#include "sweep.h"
#include "gridsync.h"

namespace vfpi {

struct BatchArgs {
  int32_t n_env, n_nodes, n_contacts;
  const int32_t* env_node_off;
  const int32_t* env_con_off;
  const int32_t* env_order;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const float* val;
  int32_t nnzb;
  const float* b;
  const int32_t* crp;
  const int32_t* ccol;
  const float* cval;
  const float* phi;
  const float* mu;
  const float* mu2;    // nullable: anisotropic friction
  int32_t nnzb_c;
  int32_t* scol;
  float* sval;
  double* diag;
  double* rn2;
  float* w;
  int32_t* cmap;
  float* cpack;
  int32_t* cpair;      // contact nodes (D-contacts)
  int32_t has_d;       // some J_c row has two blocks
  float* v_user;
  float* v_alt;
  float* lambda;
  int32_t max_iters, fixed;
  double tol;
  int proj;
  RowsArgs ra;
  vfpi_stats* stats;
  uint32_t* queue;
  float* vprev;        // Chebyshev v^{l-1} buffer
  int32_t cheby_ls;    // 0: off
  double cheby_u;
};

__global__ void k_reset_queue(uint32_t* q) { *q = 0u; }

// Node and contact ranges of one environment.
struct EnvRange {
  int e;
  int64_t n_lo, n_hi, m_lo, m_hi;
};

// Per-environment setup (a0), every thread of the workgroup calls: validates
// the offsets, builds the contact map and records, the chunk-interleaved copy
// of A, W and gamma.  Returns false when the environment is done (bad
// offsets, a device-detected data error, or max_iters <= 0): its stats and
// lambda are then written here.
template <int NWAVES>
VFPI_DEV bool env_setup(const BatchArgs& a, const EnvRange& r, int* s_flag) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool bad_off = r.n_lo < 0 || r.n_hi < r.n_lo || r.n_hi > a.n_nodes || r.m_lo < 0 || r.m_hi < r.m_lo ||
                       r.m_hi > a.n_contacts || r.m_hi - r.m_lo > r.n_hi - r.n_lo;
  if (bad_off) {
    if (threadIdx.x == 0) {
      vfpi_stats* st = a.stats + r.e;
      st->iters = 0;
      st->status = VFPI_S_BAD_PATTERN;
      st->theta = INFINITY;
      st->n_open = st->n_stick = st->n_slip = st->reserved = 0;
    }
    __syncthreads();
    return false;
  }
  for (int64_t i = r.n_lo + threadIdx.x; i < r.n_hi; i += blockDim.x) a.cmap[i] = -1;
  __syncthreads();
  for (int64_t m = r.m_lo + threadIdx.x; m < r.m_hi; m += blockDim.x)
    contact_setup<float>(m, a.nnzb_c, a.crp, a.ccol, a.cval, a.phi, a.mu, a.mu2, r.n_lo, r.n_hi, a.cmap, a.cpack,
                         a.cpair, s_flag, 1e-5);
  __syncthreads();
  const int64_t nch = (r.n_hi - r.n_lo + 63) / 64;
  for (int64_t c = wave; c < nch; c += NWAVES) {
    const int64_t n0 = r.n_lo + 64 * c;
    rows_chunk<float>(n0, (int)min<int64_t>(64, r.n_hi - n0), lane, a.row_ptr, a.col_idx, a.val, a.scol, a.sval,
                      r.n_lo, r.n_hi, a.diag, a.rn2, a.ra, nullptr, a.cmap, a.cpack, a.w, nullptr, a.b, a.v_user,
                      s_flag);
  }
  __syncthreads();
  if (a.has_d) {
    for (int64_t m = r.m_lo + threadIdx.x; m < r.m_hi; m += blockDim.x)
      pair_setup<float>(m, a.cpair, a.diag, a.rn2, a.ra, a.w, nullptr, a.cpack, s_flag);
    __syncthreads();
  }
  const int flag = *s_flag;
  if (flag != 0 || a.max_iters <= 0) {
    for (int64_t k = 3 * r.m_lo + threadIdx.x; k < 3 * r.m_hi; k += blockDim.x) a.lambda[k] = 0.0f;
    if (threadIdx.x == 0) {
      vfpi_stats* st = a.stats + r.e;
      st->iters = 0;
      st->status = flag ? flag : VFPI_S_MAXITER;
      st->theta = INFINITY;
      st->n_open = st->n_stick = st->n_slip = st->reserved = 0;
    }
    __syncthreads();
    return false;
  }
  return true;
}

// Takes the next environment from the work queue (every thread calls).
// Returns false when the queue is empty; r.e < 0 for an entry of env_order
// that is not a valid index (nothing safe to touch, skipped).
VFPI_DEV bool env_next(const BatchArgs& a, EnvRange& r, int* s_env, int* s_flag) {
  if (threadIdx.x == 0) {
    *s_env = (int)atomicAdd(a.queue, 1u);
    *s_flag = 0;
  }
  __syncthreads();
  int e = *s_env;
  if (e >= a.n_env) return false;
  if (a.env_order) e = a.env_order[e];
  r.e = (e < 0 || e >= a.n_env) ? -1 : e;
  if (r.e >= 0) {
    r.n_lo = a.env_node_off[e];
    r.n_hi = a.env_node_off[e + 1];
    r.m_lo = a.env_con_off[e];
    r.m_hi = a.env_con_off[e + 1];
  }
  return true;
}

// The V-FPI loop (a1-a5) of one environment with the iterate in global memory
// (workgroup barriers only): FP32 arithmetic, FP64 residual, its own exit.
template <int TPN, int NW, int MW>
VFPI_DEV void env_solve_global(const BatchArgs& a, const EnvRange& r, float (*s_vs)[TPN == 3 ? NW : 1][3][64],
                               double* s_red, int* s_ired, int* s_stop) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = wave / TPN, rr = (TPN == 3) ? wave % 3 : 0;
  const int64_t n_lo = r.n_lo, n_hi = r.n_hi;
  const int64_t nch = (n_hi - n_lo + 63) / 64;
  SweepData<float> d;
  d.row_ptr = a.row_ptr;
  d.scol = a.scol;
  d.sval = a.sval;
  d.b = a.b;
  d.w = a.w;
  d.cmap = a.cmap;
  d.cpack = a.cpack;
  d.lambda = a.lambda;
  d.tape_lamstar = nullptr;
  d.tape_branch = nullptr;
  d.proj = a.proj;
  d.col_idx = a.col_idx;
  d.val = a.val;
  d.cpair = a.has_d ? a.cpair : nullptr;
  Cheby ch;
  ch.ls = a.cheby_ls;
  ch.u = a.cheby_u;
  d.vprev = ch.ls ? a.vprev : nullptr;
  d.u = ch.u;
  float* vcur = a.v_user;
  float* vnext = a.v_alt;
  const int passes = (int)((nch + NW - 1) / NW);
  int l = 0;
  for (;;) {
    ++l;
    double th2 = 0.0;
    int cb[3] = {0, 0, 0};
    d.nu = ch.next_nu(l);
    d.first = (l == 1);
    for (int p = 0; p < passes; ++p) {
      const int64_t c = (int64_t)p * NW + slot;
      const int64_t n0 = n_lo + 64 * c;
      const int cnt = (c < nch) ? (int)min<int64_t>(64, n_hi - n0) : 0;
      if (TPN == 3) {
        sweep_chunk_row<float>(d, vcur, vnext, n0, cnt, lane, rr, s_vs[p & 1][TPN == 3 ? slot : 0], th2, cb);
      } else {
        // levels streamed in groups of 4 with two workgroups per CU, of 2 with one
        // (fewer registers, and measured faster on the 2048-environment mix)
        sweep_chunk_node<float, false, (MW == 1 ? 2 : 4)>(d, vcur, vnext, n0, cnt, lane, th2, cb);
      }
    }
    block_sum4(th2, cb[0], cb[1], cb[2], s_red, s_ired);
    const int o = cb[0], s = cb[1], sl = cb[2];
    if (threadIdx.x == 0) {
      const double theta = sqrt(th2);
      const bool conv = !a.fixed && theta < a.tol;
      const bool stop = conv || l >= a.max_iters;
      if (stop) {
        vfpi_stats* st = a.stats + r.e;
        st->iters = l;
        st->status = conv ? VFPI_S_CONVERGED : VFPI_S_MAXITER;
        st->theta = theta;
        st->n_open = o;
        st->n_stick = s;
        st->n_slip = sl;
        st->reserved = 0;
      }
      *s_stop = stop;
    }
    __syncthreads();
    const bool stop = *s_stop != 0;
    if (!stop) ch.observe(sqrt(th2));
    float* t = vcur;
    vcur = vnext;
    vnext = t;
    __syncthreads();
    if (stop) break;
  }
  if (vcur != a.v_user) {
    for (int64_t k = 3 * n_lo + threadIdx.x; k < 3 * n_hi; k += blockDim.x) a.v_user[k] = vcur[k];
  }
  __syncthreads();
}

// MW: minimum waves per SIMD the registers must allow (4 lets two 8-wave
// workgroups share a CU, so two environments are in flight per CU).
template <int TPN, int NW, int MW = 1>
__global__ void __launch_bounds__(64 * TPN * NW, MW) k_vfpi_batched(BatchArgs a) {
  __shared__ float s_vs[2][TPN == 3 ? NW : 1][3][64];
  __shared__ double s_red[TPN * NW];
  __shared__ int s_ired[3 * TPN * NW];
  __shared__ int s_env;
  __shared__ int s_flag;
  __shared__ int s_stop;
  EnvRange r;
  while (env_next(a, r, &s_env, &s_flag)) {
    if (r.e < 0) {
      __syncthreads();
      continue;
    }
    if (!env_setup<TPN * NW>(a, r, &s_flag)) continue;
    env_solve_global<TPN, NW, MW>(a, r, s_vs, s_red, s_ired, &s_stop);
  }
}

// ---- environments with the iterate in LDS --------------------------------
// y += A_x v over the levels k >= k_start of the lanes' rows (blocks from
// offset off_start of the chunk's range), streamed in groups of U; the
// gathers read the environment's iterate from LDS (local node index =
// column - n_lo; the setup has checked that every column lies inside the
// environment).  The accumulation order is level by level.
template <int U>
VFPI_DEV void spmv_rows3_lds(const int32_t* __restrict__ scol, const float* __restrict__ sval,
                             const float* __restrict__ xl, int64_t n_lo, int64_t base, int nk, int lane,
                             int k_start, int64_t off_start, float acc[3]) {
  int64_t off = off_start;
  for (int k0 = k_start;; k0 += U) {
    uint64_t m[U];
    int cnt[U];
    int64_t offk[U];
    if (!level_group<U>(k0, nk, off, m, cnt, offk)) break;
    int c[U];
    float av[U][9];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = 0;
      if (k0 + u < nk) {
        const int pos = lanes_below(m[u], lane);
        const int64_t q = base + offk[u];
        c[u] = scol[q + pos] - (int32_t)n_lo;
        const float* ap = sval + 9 * q + pos;
#pragma unroll
        for (int e = 0; e < 9; ++e) av[u][e] = ap[(int64_t)e * cnt[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (k0 + u < nk) {
        const float* xp = xl + 3 * c[u];
        const float x0 = xp[0], x1 = xp[1], x2 = xp[2];
        acc[0] += av[u][0] * x0 + av[u][1] * x1 + av[u][2] * x2;
        acc[1] += av[u][3] * x0 + av[u][4] * x1 + av[u][5] * x2;
        acc[2] += av[u][6] * x0 + av[u][7] * x1 + av[u][8] * x2;
      }
    }
  }
}

// One node's sweep after A v (eq. pgd1, Alg. 2, eq. vup, Alg. 3): v*, then
// for an S-contact the contact step and the update, written to the next
// iterate; a D-contact node only stages v* (finished after the barrier).
// bw = b (3), W (3); returns the squared change of the node's iterate.
VFPI_DEV double lds_node_update(const BatchArgs& a, int64_t i, int il, int m, const float Av[3], const float bw[6],
                                const float* vc, float* vnx, float* s_st, unsigned char* s_br, bool cheb, int l,
                                float nu, float uu) {
  float vo[3], vs[3], vn[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    vo[q] = vc[3 * il + q];
    vs[q] = vo[q] - bw[3 + q] * (Av[q] - bw[q]);
    vn[q] = vs[q];
  }
  if (m >= 0 && a.has_d && a.cpair[2 * (int64_t)m + 1] >= 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) s_st[3 * il + q] = vs[q];
    return 0.0;
  }
  if (m >= 0) {
    const float* pk = a.cpack + kPack * (int64_t)m;
    float lam[3], ls[3];
    s_br[il] = (unsigned char)contact_step<float>(pk, vs[0], vs[1], vs[2], a.proj, lam, ls);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float F = pk[q] * lam[0] + pk[3 + q] * lam[1] + pk[6 + q] * lam[2];
      vn[q] = vs[q] + bw[3 + q] * F;
      a.lambda[3 * (int64_t)m + q] = lam[q];
    }
  }
  double th2 = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (cheb) {  // v^{l-1} in the global buffer (v^0 = v^1)
      const float pv = (l == 1) ? vo[q] : a.vprev[3 * i + q];
      a.vprev[3 * i + q] = vo[q];
      vn[q] = nu * (uu * (vn[q] - vo[q]) + vo[q] - pv) + pv;
    }
    vnx[3 * il + q] = vn[q];
    const double dd = (double)(vn[q] - vo[q]);
    th2 += dd * dd;
  }
  return th2;
}

// Batched V-FPI with each environment's iterate in LDS (two buffers, plus a
// third that stages v* of D-contact nodes): the sweep's neighbour gathers
// and its scatter stay inside the CU.  One workgroup of NW waves per
// environment.  Chunks 0 .. RP * NW - 1 ("register passes", wave w owning
// chunks w, w + NW, ...) keep their first KC block levels of A, the column
// indices and the contact index in registers for the whole step, loaded once
// after the setup (a level a row lacks is a zero block on local column 0, so
// the sweep runs them without branches, adding exact zeros); their longer
// rows and every further chunk stream A from L2 in groups of U levels.  One
// workgroup barrier per sweep (two with D-contacts): the residual's wave
// sums are double-buffered by sweep parity and every thread adds them in
// wave order, so all threads take the same stop decision.  Environments of
// more than MAXN nodes run the global-memory loop.
template <int NW, int RP, int KC, int MAXN, int U>
__global__ void __launch_bounds__(64 * NW) k_vfpi_batched_lds(BatchArgs a) {
  __shared__ float s_v[2][3 * MAXN];
  __shared__ float s_st[3 * MAXN];
  __shared__ unsigned char s_br[MAXN];
  __shared__ float s_vs[2][1][3][64];
  __shared__ double s_red[2][NW];
  __shared__ int s_ired[3 * NW];
  __shared__ int s_env;
  __shared__ int s_flag;
  __shared__ int s_stop;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  EnvRange r;
  while (env_next(a, r, &s_env, &s_flag)) {
    if (r.e < 0) {
      __syncthreads();
      continue;
    }
    if (!env_setup<NW>(a, r, &s_flag)) continue;
    const int64_t n_lo = r.n_lo, n_hi = r.n_hi;
    const int64_t nn = n_hi - n_lo;
    if (nn > MAXN) {
      env_solve_global<1, NW, 1>(a, r, s_vs, &s_red[0][0], s_ired, &s_stop);
      continue;
    }
    const int nch = (int)((nn + 63) / 64);
    for (int il = threadIdx.x; il < nn; il += blockDim.x) {
#pragma unroll
      for (int q = 0; q < 3; ++q) s_v[0][3 * il + q] = a.v_user[3 * (n_lo + il) + q];
      s_br[il] = BR_OPEN;
    }
    // register passes: A's first KC levels, their columns, the node's contact
    constexpr int RA = RP > 0 ? RP : 1;
    int rcol[RA][KC];
    float rav[RA][KC][9];
    int rm[RA], rnk[RA], rbase[RA], roff[RA];
#pragma unroll
    for (int p = 0; p < RP; ++p) {
      const int c = p * NW + wave;
      const int64_t n0 = n_lo + 64 * (int64_t)c;
      const int cnt = (c < nch) ? (int)min<int64_t>(64, n_hi - n0) : 0;
      const int64_t i = n0 + lane;
      const bool act = lane < cnt;
      rbase[p] = cnt > 0 ? a.row_ptr[n0] : 0;
      rnk[p] = act ? a.row_ptr[i + 1] - a.row_ptr[i] : 0;
      rm[p] = act ? a.cmap[i] : -1;
      int off = 0;
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const uint64_t msk = ballot(k < rnk[p]);
        const int ck = __popcll(msk);
        rcol[p][k] = 0;
#pragma unroll
        for (int e = 0; e < 9; ++e) rav[p][k][e] = 0.0f;
        if (k < rnk[p]) {
          const int pos = lanes_below(msk, lane);
          const int64_t q = rbase[p] + off;
          rcol[p][k] = a.scol[q + pos] - (int32_t)n_lo;
#pragma unroll
          for (int e = 0; e < 9; ++e) rav[p][k][e] = a.sval[9 * q + (int64_t)e * ck + pos];
        }
        off += ck;
      }
      roff[p] = off;
    }
    __syncthreads();
    Cheby ch;
    ch.ls = a.cheby_ls;
    ch.u = a.cheby_u;
    const bool cheb = ch.ls != 0;
    int cur = 0;
    int l = 0;
    for (;;) {
      ++l;
      const float nu = (float)ch.next_nu(l);
      const float uu = (float)ch.u;
      const float* vc = s_v[cur];
      float* vnx = s_v[cur ^ 1];
      double th2 = 0.0;
#pragma unroll
      for (int p = 0; p < RP; ++p) {
        const int c = p * NW + wave;
        if (c < nch) {  // wave-uniform
          const int il = 64 * c + lane;
          const int64_t i = n_lo + il;
          const bool act = il < nn;
          float bw[6];
          if (act) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              bw[q] = a.b[3 * i + q];
              bw[3 + q] = a.w[3 * i + q];
            }
          }
          float Av[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int k = 0; k < KC; ++k) {
            const float* xp = vc + 3 * rcol[p][k];
            const float x0 = xp[0], x1 = xp[1], x2 = xp[2];
            Av[0] += rav[p][k][0] * x0 + rav[p][k][1] * x1 + rav[p][k][2] * x2;
            Av[1] += rav[p][k][3] * x0 + rav[p][k][4] * x1 + rav[p][k][5] * x2;
            Av[2] += rav[p][k][6] * x0 + rav[p][k][7] * x1 + rav[p][k][8] * x2;
          }
          spmv_rows3_lds<U>(a.scol, a.sval, vc, n_lo, rbase[p], rnk[p], lane, KC, roff[p], Av);
          if (act) th2 += lds_node_update(a, i, il, rm[p], Av, bw, vc, vnx, s_st, s_br, cheb, l, nu, uu);
        }
      }
#pragma unroll 1
      for (int c = RP * NW + wave; c < nch; c += NW) {  // wave-uniform
        const int il = 64 * c + lane;
        const int64_t i = n_lo + il;
        const bool act = il < nn;
        const int base = a.row_ptr[n_lo + 64 * c];
        const int nk = act ? a.row_ptr[i + 1] - a.row_ptr[i] : 0;
        const int m = act ? a.cmap[i] : -1;
        float bw[6];
        if (act) {
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            bw[q] = a.b[3 * i + q];
            bw[3 + q] = a.w[3 * i + q];
          }
        }
        float Av[3] = {0.0f, 0.0f, 0.0f};
        spmv_rows3_lds<U>(a.scol, a.sval, vc, n_lo, base, nk, lane, 0, 0, Av);
        if (act) th2 += lds_node_update(a, i, il, m, Av, bw, vc, vnx, s_st, s_br, cheb, l, nu, uu);
      }
      if (a.has_d) {
        // D-contacts: both nodes of a pair read the same two staged v*, so
        // they form the same lambda (eq. jcnode, Alg. 2)
        __syncthreads();
#pragma unroll 1
        for (int il = threadIdx.x; il < nn; il += blockDim.x) {
          const int64_t i = n_lo + il;
          const int m = a.cmap[i];
          if (m >= 0 && a.cpair[2 * (int64_t)m + 1] >= 0) {
            const int64_t pi = a.cpair[2 * (int64_t)m], pj = a.cpair[2 * (int64_t)m + 1];
            const bool owner = pi == i;
            const int oth = (int)((owner ? pj : pi) - n_lo);
            const float* pk = a.cpack + kPack * (int64_t)m;
            float vo[3], vs[3], vn[3], eta[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              vo[q] = vc[3 * il + q];
              vs[q] = s_st[3 * il + q];
              const float vx = s_st[3 * oth + q];
              eta[q] = owner ? vs[q] - vx : vx - vs[q];  // v*_i - v*_j
            }
            float lam[3], ls[3];
            const int b_ = contact_step<float>(pk, eta[0], eta[1], eta[2], a.proj, lam, ls);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              const float F = pk[q] * lam[0] + pk[3 + q] * lam[1] + pk[6 + q] * lam[2];
              const float wq = a.w[3 * i + q];
              vn[q] = owner ? vs[q] + wq * F : vs[q] - wq * F;
            }
            if (owner) {
              s_br[il] = (unsigned char)b_;
#pragma unroll
              for (int q = 0; q < 3; ++q) a.lambda[3 * (int64_t)m + q] = lam[q];
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              if (cheb) {
                const float pv = (l == 1) ? vo[q] : a.vprev[3 * i + q];
                a.vprev[3 * i + q] = vo[q];
                vn[q] = nu * (uu * (vn[q] - vo[q]) + vo[q] - pv) + pv;
              }
              vnx[3 * il + q] = vn[q];
              const double dd = (double)(vn[q] - vo[q]);
              th2 += dd * dd;
            }
          }
        }
      }
      th2 = wave_sum(th2);
      if (lane == 0) s_red[l & 1][wave] = th2;
      __syncthreads();
      double tot = 0.0;
#pragma unroll
      for (int k = 0; k < NW; ++k) tot += s_red[l & 1][k];
      const double theta = sqrt(tot);
      const bool conv = !a.fixed && theta < a.tol;
      const bool stop = conv || l >= a.max_iters;
      cur ^= 1;
      if (stop) {
        if (threadIdx.x == 0) {
          vfpi_stats* st = a.stats + r.e;
          st->iters = l;
          st->status = conv ? VFPI_S_CONVERGED : VFPI_S_MAXITER;
          st->theta = theta;
        }
        break;
      }
      ch.observe(theta);
    }
    // outputs: the final iterate, and the branch counts of the last sweep
    int cb[3] = {0, 0, 0};
    for (int il = threadIdx.x; il < nn; il += blockDim.x) {
      const int64_t i = n_lo + il;
#pragma unroll
      for (int q = 0; q < 3; ++q) a.v_user[3 * i + q] = s_v[cur][3 * il + q];
      const int m = a.cmap[i];
      if (m >= 0 && (!a.has_d || a.cpair[2 * (int64_t)m] == i)) cb[s_br[il]] += 1;
    }
    block_sum4_int(cb[0], cb[1], cb[2], s_ired);
    if (threadIdx.x == 0) {
      vfpi_stats* st = a.stats + r.e;
      st->n_open = cb[0];
      st->n_stick = cb[1];
      st->n_slip = cb[2];
      st->reserved = 0;
    }
    __syncthreads();
  }
}

}  // namespace vfpi

using namespace vfpi;

namespace {

template <int TPN, int NW, int MW = 1>
hipError_t launch_batched(const BatchArgs& ba, int grid_req, int num_cu, hipStream_t st) {
  auto kern = k_vfpi_batched<TPN, NW, MW>;
  const int threads = 64 * TPN * NW;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0);
  if (e != hipSuccess) return e;
  int64_t g = (int64_t)per_cu * num_cu;
  if (grid_req > 0 && grid_req < g) g = grid_req;
  if (g > ba.n_env) g = ba.n_env;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(1), 0, st, ba.queue);
  hipLaunchKernelGGL(kern, dim3((unsigned)g), dim3(threads), 0, st, ba);
  return hipGetLastError();
}

template <int NW, int RP, int KC, int MAXN, int U>
hipError_t launch_batched_lds(const BatchArgs& ba, int grid_req, int num_cu, hipStream_t st) {
  auto kern = k_vfpi_batched_lds<NW, RP, KC, MAXN, U>;
  const int threads = 64 * NW;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  int64_t g = (int64_t)per_cu * num_cu;
  if (grid_req > 0 && grid_req < g) g = grid_req;
  if (g > ba.n_env) g = ba.n_env;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(1), 0, st, ba.queue);
  hipLaunchKernelGGL(kern, dim3((unsigned)g), dim3(threads), 0, st, ba);
  return hipGetLastError();
}

}  // namespace

extern "C" int vfpi_step_batched(vfpi_ctx* ctx, int32_t n_env, const int32_t* env_node_off,
                                 const int32_t* env_con_off, const int32_t* env_order, const vfpi_bsr* A,
                                 const float* b, const vfpi_contacts* Jc, float* v, float* lambda,
                                 const vfpi_opts* opts, vfpi_stats* per_env_stats, hipStream_t stream) {
  if (!ctx || !A || !b || !Jc || !v || !opts || !per_env_stats || !env_node_off || !env_con_off) return VFPI_E_NULL;
  const int32_t N = A->n_nodes, nc = Jc->n_contacts;
  if (n_env < 0 || N < 0 || nc < 0 || A->nnzb < 0 || Jc->nnzb < 0 || nc > N) return VFPI_E_SHAPE;
  if (N > 0 && (!A->row_ptr || !A->col_idx || !A->val)) return VFPI_E_NULL;
  if (nc > 0 && (!Jc->row_ptr || !Jc->col_idx || !Jc->val || !Jc->phi || !Jc->mu || !lambda)) return VFPI_E_NULL;
  if (N > ctx->max_nodes || A->nnzb > ctx->max_nnzb || nc > ctx->max_contacts || n_env > ctx->max_envs)
    return VFPI_E_CAPACITY;
  int rc = vfpi_check_opts(opts, true);
  if (rc) return rc;
  if (Jc->nnzb > 2 * (int64_t)nc) return VFPI_E_SHAPE;
  if (Jc->mu2 && opts->projection != VFPI_PROJ_STRICT) return VFPI_E_UNSUPPORTED;
  if (opts->reuse_w && ctx->stats_nodes != N) return VFPI_E_OPTS;
  const int kind = opts->variant & 0xff;
  if (kind > 4) return VFPI_E_OPTS;
  if (n_env == 0) return VFPI_OK;
  VFPI_CHECK_HIP(hipSetDevice(ctx->device));

  BatchArgs ba;
  ba.n_env = n_env;
  ba.n_nodes = N;
  ba.n_contacts = nc;
  ba.env_node_off = env_node_off;
  ba.env_con_off = env_con_off;
  ba.env_order = env_order;
  ba.row_ptr = A->row_ptr;
  ba.col_idx = A->col_idx;
  ba.val = static_cast<const float*>(A->val);
  ba.nnzb = A->nnzb;
  ba.b = b;
  ba.crp = Jc->row_ptr;
  ba.ccol = Jc->col_idx;
  ba.cval = static_cast<const float*>(Jc->val);
  ba.phi = static_cast<const float*>(Jc->phi);
  ba.mu = static_cast<const float*>(Jc->mu);
  ba.mu2 = static_cast<const float*>(Jc->mu2);
  ba.nnzb_c = Jc->nnzb;
  ba.scol = ctx->scol;
  ba.sval = static_cast<float*>(ctx->sval);
  ba.diag = ctx->diag;
  ba.rn2 = ctx->rn2;
  ba.w = static_cast<float*>(ctx->w);
  ba.cmap = ctx->cmap;
  ba.cpack = static_cast<float*>(ctx->cpack);
  ba.cpair = ctx->cpair;
  ba.has_d = Jc->nnzb > nc;
  ba.v_user = v;
  ba.v_alt = static_cast<float*>(ctx->vbuf);
  ba.lambda = lambda;
  ba.max_iters = opts->max_iters;
  ba.fixed = opts->fixed_iters;
  ba.tol = opts->tol;
  ba.proj = opts->projection;
  ba.ra.nnzb = A->nnzb;
  ba.ra.w_mode = opts->w_mode;
  ba.ra.reuse = opts->reuse_w != 0;
  ba.ra.alpha = opts->alpha_user;
  ba.ra.omega = opts->omega;
  ba.stats = per_env_stats;
  ba.queue = ctx->sync + SY_QUEUE;
  ba.vprev = static_cast<float*>(ctx->vprev);
  ba.cheby_ls = opts->cheby_ls;
  ba.cheby_u = opts->cheby_u == 0.0 ? 1.0 : opts->cheby_u;
  ctx->stats_nodes = N;

  const int nw = (opts->variant >> 8) & 0xff;
  const int grid = (opts->variant >> 16) & 0xff;
  vfpi_mark(ctx, 0, stream);
  vfpi_mark(ctx, 1, stream);  // setup is fused into the batched kernel
  hipError_t e;
  if (kind == 2) {
    e = (nw >= 2) ? launch_batched<3, 2>(ba, grid, ctx->num_cu, stream)
                  : launch_batched<3, 1>(ba, grid, ctx->num_cu, stream);
  } else if (kind == 3) {  // lane per node, two workgroups per CU
    e = (nw >= 8) ? launch_batched<1, 8, 4>(ba, grid, ctx->num_cu, stream)
                  : launch_batched<1, 4, 4>(ba, grid, ctx->num_cu, stream);
  } else if (kind == 4 || kind == 0) {  // iterate in LDS (the library default)
    const int ug = (opts->variant >> 26) & 0x3;
    e = (nw >= 16) ? launch_batched_lds<16, 0, 1, 3072, 2>(ba, grid, ctx->num_cu, stream)
                   : (ug == 1 ? launch_batched_lds<8, 1, 9, 3072, 4>(ba, grid, ctx->num_cu, stream)
                              : launch_batched_lds<8, 1, 9, 3072, 2>(ba, grid, ctx->num_cu, stream));
  } else if (kind == 1) {
    e = (nw >= 8)   ? launch_batched<1, 8>(ba, grid, ctx->num_cu, stream)
        : (nw >= 4) ? launch_batched<1, 4>(ba, grid, ctx->num_cu, stream)
        : (nw >= 2 || nw == 0) ? launch_batched<1, 2>(ba, grid, ctx->num_cu, stream)
                               : launch_batched<1, 1>(ba, grid, ctx->num_cu, stream);
  } else {
    return VFPI_E_OPTS;
  }
  vfpi_mark(ctx, 2, stream);
  return e == hipSuccess ? VFPI_OK : VFPI_E_HIP;
}
