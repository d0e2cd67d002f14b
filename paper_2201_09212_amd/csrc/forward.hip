// (compiled as part of vfpi_lib.hip)
// Plain FP64 V-FPI step: setup kernels + one persistent kernel that runs the
// whole iteration (Alg. 1 inner loop) on the device, with a deterministic
// grid-wide residual reduction and early exit.
#include <math.h>

#include "internal.h"
#include "setup.h"
#include "sweep.h"
#include "gridsync.h"

namespace vfpi {

// Per-call reset: node->contact map, error flags, work-queue word, barrier
// slots and the stats record (its branch counters are accumulated later).
__global__ void k_prep(int32_t n_nodes, int32_t* cmap, int32_t* flags, uint32_t* sync, uint64_t* slots,
                       vfpi_stats* stats) {
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < n_nodes; i += stride) cmap[i] = -1;
  for (int64_t i = i0; i < kSlotRings * kMaxGridSlots; i += stride) {  // region 0: both words of a slot
    slots[i * kSlotPad] = 0ull;
    slots[i * kSlotPad + 1] = 0ull;
  }
  for (int64_t i = i0; i < 12 * kMaxGridSlots; i += stride) slots[kBBSlotOffset + i] = 0ull;
  for (int64_t i = i0; i < 2 * kMaxGridSlots; i += stride) slots[kDSlotOffset + i * kSlotPad] = 0ull;
  if (i0 == 0) {
    flags[0] = 0;
    for (int k = 0; k < kSyncWords; ++k) sync[k] = 0u;
    stats->iters = 0;
    stats->status = 0;
    stats->theta = 0.0;
    stats->n_open = stats->n_stick = stats->n_slip = stats->reserved = 0;
  }
}

__global__ void k_stats_empty(vfpi_stats* st) {
  st->iters = 0;
  st->status = VFPI_S_MAXITER;
  st->theta = 0.0;
  st->n_open = st->n_stick = st->n_slip = st->reserved = 0;
}

template <class T>
__global__ void k_contacts(int32_t nc, int32_t nnzb_c, const int32_t* crp, const int32_t* ccol, const T* cval,
                           const T* phi, const T* mu, const T* mu2, int32_t n_nodes, int32_t* cmap, T* cpack,
                           int32_t* cpair, int32_t* flags, double orth_tol) {
  int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (m < nc)
    contact_setup<T>(m, nnzb_c, crp, ccol, cval, phi, mu, mu2, 0, n_nodes, cmap, cpack, cpair, flags, orth_tol);
}

// Shared W and gamma of every D-contact pair (after the row pass).
template <class T>
__global__ void k_pairs(int32_t nc, const int32_t* cpair, const double* diag, const double* rn2, RowsArgs ra, T* w,
                        double* tape_w, T* cpack, int32_t* flags) {
  int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (m < nc) pair_setup<T>(m, cpair, diag, rn2, ra, w, tape_w, cpack, flags);
}

template <class T>
__global__ void __launch_bounds__(256) k_rows(int32_t n_nodes, const int32_t* row_ptr, const int32_t* col_idx,
                                              const T* val, int32_t* scol, T* sval, double* diag, double* rn2,
                                              RowsArgs ra, const T* w_user, const int32_t* cmap, T* cpack, T* w,
                                              double* tape_w, const T* bvec, const T* vvec, int32_t* flags) {
  const int64_t chunk = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t n0 = chunk * 64;
  if (n0 >= n_nodes) return;  // whole wave leaves together
  const int cnt = (int)min<int64_t>(64, n_nodes - n0);
  rows_chunk<T>(n0, cnt, threadIdx.x & 63, row_ptr, col_idx, val, scol, sval, 0, n_nodes, diag, rn2, ra, w_user,
                cmap, cpack, w, tape_w, bvec, vvec, flags);
}

struct GridArgs {
  SweepData<double> d;
  int32_t n_nodes, n_contacts;
  double* v_user;
  double* v_alt;
  double* tape_v;
  int32_t max_iters, fixed;
  double tol;
  const int32_t* flags;
  vfpi_stats* stats;
  uint64_t* slots;
  double* vprev;       // Chebyshev v^{l-1} buffer (streaming kernels)
  int32_t cheby_ls;    // 0: off
  double cheby_u;
  // Barzilai-Borwein step sizes (k_vfpi_bb only)
  int32_t bb2;                        // 0: BB1 s's/s'z, 1: BB2 s'z/z'z
  double omega;                       // gamma_m = alpha + omega (S-contacts)
  double* avbuf;                      // [n] A v^l of the previous sweep (own DOFs)
  const unsigned long long* amax;     // max_d sum_j |a_dj| from the setup
  double* tape_w;                     // nullable: receives the final alpha
  // lagged residual (k_vfpi_regs with LAG): contact results of the last two
  // sweeps, [2][n_contacts][8] (lambda, lambda*, branch), then (D-contacts)
  // v* of the two sweep parities, [2][3 n_nodes]
  double* lring;
};

// Persistent V-FPI kernel: the whole sweep loop of one step.  TPN = threads
// per node (1: a lane owns a node's three rows; 3: three waves own rows 0/1/2
// of the same 64 nodes), NW = chunk slots per workgroup.  With more than one
// workgroup it needs a cooperative launch of at most one workgroup per CU;
// the workgroups meet once per sweep in the residual reduction.  A workgroup
// keeps the same nodes in every sweep, and the iterate moves between
// workgroups through coherent loads / stores only (see gridsync.h).
template <int TPN, int NW, int U = (TPN == 3 ? (64 * TPN * NW >= 960 ? 4 : 8) : (64 * TPN * NW >= 960 ? 2 : 4))>
__global__ void __launch_bounds__(64 * TPN * NW) k_vfpi_grid(GridArgs a) {
  constexpr bool COH = true;
  __shared__ double s_vs[2][TPN == 3 ? NW : 1][3][64];
  __shared__ double s_red[TPN * NW];
  __shared__ double s_poll[3 * TPN * NW];  // see grid_sum
  __shared__ int s_ired[3 * TPN * NW];

  const int G = gridDim.x;
  const int lb = xcd_logical_block(blockIdx.x, G);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = wave / TPN, r = (TPN == 3) ? wave % 3 : 0;
  const int64_t nch = (a.n_nodes + 63) / 64;
  const int64_t c0 = lb * nch / G, c1 = (lb + 1) * nch / G;
  const int passes = (int)((c1 - c0 + NW - 1) / NW);

  const int flags = *a.flags;
  if (flags != 0 || a.max_iters <= 0) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < 3 * (int64_t)a.n_contacts;
         k += (int64_t)G * blockDim.x)
      a.d.lambda[k] = 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.stats->iters = 0;
      a.stats->status = flags ? flags : VFPI_S_MAXITER;
      a.stats->theta = INFINITY;
    }
    return;
  }

  double* vcur = a.v_user;
  double* vnext = a.v_alt;
  int cb[3] = {0, 0, 0};
  SweepData<double> d = a.d;
  Cheby ch;
  ch.ls = a.cheby_ls;
  ch.u = a.cheby_u;
  d.vprev = ch.ls ? a.vprev : nullptr;
  d.u = ch.u;
  for (int l = 1;; ++l) {
    double th2 = 0.0;
    cb[0] = cb[1] = cb[2] = 0;
    d.nu = ch.next_nu(l);
    d.first = (l == 1);
    for (int p = 0; p < passes; ++p) {
      const int64_t c = c0 + (int64_t)p * NW + slot;
      const int64_t n0 = c * 64;
      const int cnt = (c < c1) ? (int)min<int64_t>(64, a.n_nodes - n0) : 0;
      if (TPN == 3)
        sweep_chunk_row<double, COH, U>(d, vcur, vnext, n0, cnt, lane, r,
                                                                      s_vs[p & 1][TPN == 3 ? slot : 0], th2, cb);
      else
        sweep_chunk_node<double, COH, U>(d, vcur, vnext, n0, cnt, lane, th2, cb);
    }
    th2 = block_sum(th2, s_red);
    double theta;
    const bool stop =
        grid_residual_step(a.slots, G, lb, l, th2, l, a.max_iters, a.fixed, a.tol, a.stats, s_poll, &theta);
    double* t = vcur;
    vcur = vnext;
    vnext = t;
    if (stop) break;
    ch.observe(theta);
  }
  block_sum4_int(cb[0], cb[1], cb[2], s_ired);
  add_counts(a.stats, cb[0], cb[1], cb[2]);
  // The final iterate is in vcur.  Each thread copies only entries it wrote
  // itself in the last sweep, so no further synchronization is needed.
  if (vcur != a.v_user || a.tape_v) {
    for (int p = 0; p < passes; ++p) {
      const int64_t c = c0 + (int64_t)p * NW + slot;
      const int64_t n0 = c * 64;
      const int cnt = (c < c1) ? (int)min<int64_t>(64, a.n_nodes - n0) : 0;
      if (lane < cnt) {
        const int64_t i = n0 + lane;
        for (int rr = (TPN == 3 ? r : 0); rr < (TPN == 3 ? r + 1 : 3); ++rr) {
          const double x = ldv<COH>(vcur + 3 * i + rr);
          if (vcur != a.v_user) a.v_user[3 * i + rr] = x;
          if (a.tape_v) a.tape_v[3 * i + rr] = x;
        }
      }
    }
  }
}


// Persistent V-FPI kernel with Barzilai-Borwein step sizes W = alpha^l I
// (Sec. IV-C.2): alpha^1 = 1 / max_d sum_j |a_dj| (Gershgorin), and for l >= 2
// alpha^l = s's / s'z (BB1) or s'z / z'z (BB2) with s = v^l - v^{l-1},
// z = A v^l - A v^{l-1}; the previous alpha is kept when the quotient is not
// defined and positive.  A sweep has two phases: A v^l for the workgroup's own
// rows (kept in avbuf for the next z) with the three dot products, one grid
// reduction, then the rest of the sweep with gamma_m = alpha + omega and the
// residual reduction of Alg. 1.  Thread = node, NW chunk slots per workgroup.
template <int NW>
__global__ void __launch_bounds__(64 * NW) k_vfpi_bb(GridArgs a) {
  constexpr bool COH = true;
  constexpr int U = (64 * NW >= 960) ? 2 : 4;
  __shared__ double s_red[NW];
  __shared__ double s_poll[3 * NW];  // see grid_sum
  __shared__ int s_ired[3 * NW];
  const int G = gridDim.x;
  const int lb = xcd_logical_block(blockIdx.x, G);
  const int slot = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nch = (a.n_nodes + 63) / 64;
  const int64_t c0 = lb * nch / G, c1 = (lb + 1) * nch / G;
  const int passes = (int)((c1 - c0 + NW - 1) / NW);

  const int flags = *a.flags;
  if (flags != 0 || a.max_iters <= 0) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < 3 * (int64_t)a.n_contacts;
         k += (int64_t)G * blockDim.x)
      a.d.lambda[k] = 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.stats->iters = 0;
      a.stats->status = flags ? flags : VFPI_S_MAXITER;
      a.stats->theta = INFINITY;
    }
    return;
  }
  const SweepData<double>& d = a.d;
  double* vcur = a.v_user;
  double* vnext = a.v_alt;
  double alpha = 1.0 / __builtin_bit_cast(double, (uint64_t)*a.amax);
  int cb[3] = {0, 0, 0};
  for (int l = 1;; ++l) {
    // phase 1: A v^l of the own rows, s = v^l - v^{l-1}, z = A v^l - A v^{l-1}
    double dots[3] = {0.0, 0.0, 0.0};  // s's, s'z, z'z
    for (int p = 0; p < passes; ++p) {
      const int64_t c = c0 + (int64_t)p * NW + slot;
      const int64_t n0 = c * 64;
      const int cnt = (c < c1) ? (int)min<int64_t>(64, a.n_nodes - n0) : 0;
      const int64_t i = n0 + lane;
      const bool act = lane < cnt;
      const int nk = act ? d.row_ptr[i + 1] - d.row_ptr[i] : 0;
      const int64_t base = cnt > 0 ? d.row_ptr[n0] : 0;
      double Av[3];
      spmv_rows3<double, COH, U>(d.scol, d.sval, vcur, base, nk, lane, Av);
      if (act) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const int64_t k = 3 * i + r;
          if (l >= 2) {
            const double s = ldv<COH>(vcur + k) - ldv<COH>(vnext + k);
            const double z = Av[r] - a.avbuf[k];
            dots[0] += s * s;
            dots[1] += s * z;
            dots[2] += z * z;
          }
          a.avbuf[k] = Av[r];
        }
      }
    }
    if (l >= 2) {
      grid_sum3(a.slots + kBBSlotOffset, G, lb, l - 1, dots, s_red, s_poll);
      if (!a.bb2 && dots[0] > 0.0 && dots[1] > 0.0) alpha = dots[0] / dots[1];
      else if (a.bb2 && dots[1] > 0.0 && dots[2] > 0.0) alpha = dots[1] / dots[2];
    }
    // phase 2: v* = v^l - alpha (A v^l - b), contact step, v^{l+1}
    const double g = alpha + a.omega;
    double th2 = 0.0;
    cb[0] = cb[1] = cb[2] = 0;
    for (int p = 0; p < passes; ++p) {
      const int64_t c = c0 + (int64_t)p * NW + slot;
      const int64_t n0 = c * 64;
      const int cnt = (c < c1) ? (int)min<int64_t>(64, a.n_nodes - n0) : 0;
      const int64_t i = n0 + lane;
      if (lane >= cnt) continue;
      double v[3], vs[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        v[r] = ldv<COH>(vcur + 3 * i + r);
        vs[r] = v[r] - alpha * (a.avbuf[3 * i + r] - d.b[3 * i + r]);
      }
      double vn[3] = {vs[0], vs[1], vs[2]};
      const int m = d.cmap[i];
      if (m >= 0 && is_dcontact(d, m)) {  // gamma = w_i + w_j = 2 alpha (+ omega)
        double lam[3], ls[3];
        int br;
        if (dcontact_node<double, COH>(d, vcur, nullptr, alpha, 2.0 * alpha + a.omega, i, m, vs, vn, lam, ls, br)) {
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            d.lambda[3 * (int64_t)m + r] = lam[r];
            if (d.tape_lamstar) d.tape_lamstar[3 * (int64_t)m + r] = ls[r];
          }
          if (d.tape_branch) d.tape_branch[m] = br;
          cb[br] += 1;
        }
      } else if (m >= 0) {
        ContactRec<double> cr = load_contact<double>(d.cpack + kPack * (int64_t)m);
        cr.g = g;
        double lam[3], ls[3];
        const int br = contact_solve<double>(cr, vs[0], vs[1], vs[2], d.proj, lam, ls);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const double F = cr.R[r] * lam[0] + cr.R[3 + r] * lam[1] + cr.R[6 + r] * lam[2];
          vn[r] = vs[r] + alpha * F;
          d.lambda[3 * (int64_t)m + r] = lam[r];
          if (d.tape_lamstar) d.tape_lamstar[3 * (int64_t)m + r] = ls[r];
        }
        if (d.tape_branch) d.tape_branch[m] = br;
        cb[br] += 1;
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        stv<COH>(vnext + 3 * i + r, vn[r]);
        const double dd = vn[r] - v[r];
        th2 += dd * dd;
      }
    }
    th2 = block_sum(th2, s_red);
    const bool stop = grid_residual_step(a.slots, G, lb, l, th2, l, a.max_iters, a.fixed, a.tol, a.stats, s_poll);
    double* t = vcur;
    vcur = vnext;
    vnext = t;
    if (stop) break;
  }
  block_sum4_int(cb[0], cb[1], cb[2], s_ired);
  add_counts(a.stats, cb[0], cb[1], cb[2]);
  for (int p = 0; p < passes; ++p) {
    const int64_t c = c0 + (int64_t)p * NW + slot;
    const int64_t n0 = c * 64;
    const int cnt = (c < c1) ? (int)min<int64_t>(64, a.n_nodes - n0) : 0;
    if (lane >= cnt) continue;
    const int64_t i = n0 + lane;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double x = ldv<COH>(vcur + 3 * i + r);
      if (vcur != a.v_user) a.v_user[3 * i + r] = x;
      if (a.tape_v) a.tape_v[3 * i + r] = x;
      if (a.tape_w) a.tape_w[3 * i + r] = alpha;
    }
  }
}

// Register-resident variant of the persistent kernel (variant kind 5): each
// workgroup owns at most NW chunks (one pass), so a lane keeps, for the whole
// step, its node's first KC block levels of A (values and columns), b, W, the
// contact record, and its own iterate v^l (which it wrote itself).  The next
// KL levels are kept in LDS, so rows longer than KC blocks (solid meshes) do
// not stream them either.  A sweep gathers the neighbours' v (coherent loads
// when COH, i.e. more than one workgroup), streams the levels beyond KC + KL
// in groups of U, runs the epilogue, and writes v^{l+1} through LDS so every
// wave stores whole cache lines; lambda and the tape are written once, after
// the last sweep.  Same arithmetic and order as the streaming kernel, except
// for node-node contacts: their nodes publish v* and read the pair's v* back
// after a barrier (two phases per sweep: the whole grid, or with LD the
// workgroups that share D pairs) instead of recomputing both rows.  BB:
// Barzilai-Borwein step sizes (W = alpha^l I, see k_vfpi_bb), with the node's
// own v^{l-1} and A v^{l-1} kept in registers and one more grid reduction
// (the three dot products) per sweep.  LAG: the lagged stop test (below);
// LD (with LAG): D-contacts, met with their partner workgroups only (without
// it the lagged form is compiled for S-contacts alone).
template <int NW, int KC, int KL, int U, bool COH, bool CH, bool BB = false, bool LAG = false, bool LD = false>
__global__ void __launch_bounds__(64 * NW) k_vfpi_regs(GridArgs a) {
  // Registers hold what every sweep streams through the FMA chains: A's first
  // KC levels, the gathered neighbour values and the node's own iterate.  The
  // per-node constants (b, W, the contact record) and the last sweep's contact
  // results live in LDS, which keeps the kernel within the 256 architectural
  // VGPRs (beyond them the compiler parks A in AGPRs and copies it back every
  // sweep).  CH: Chebyshev acceleration (keeps v^{l-1} in registers).
  __shared__ double s_red[NW];
  __shared__ double s_poll[3 * NW];  // see grid_sum
  __shared__ int s_ired[3 * NW];
  __shared__ double s_out[NW][192];
  __shared__ double s_bw[NW][6][64];      // b (3), W (3)
  __shared__ double s_cr[NW][kPack][64];  // contact record of the lane's node
  // lambda, lambda* of the last sweep (LAG: the contact ring holds them)
  __shared__ double s_lam[LAG ? 1 : NW][6][64];
  __shared__ double s_al[KL > 0 ? NW : 1][KL > 0 ? KL : 1][9][64];
  __shared__ int s_cl[KL > 0 ? NW : 1][KL > 0 ? KL : 1][64];
  // LAG (no Chebyshev, no BB, more than one workgroup): the stop test of
  // sweep l is taken after sweep l + 1, and between sweeps a workgroup waits
  // only for its neighbours (lag_sync in gridsync.h)
  __shared__ uint32_t s_nbm[LAG ? kMaxGridSlots / 32 : 1];
  __shared__ int s_lflag;
  // LAG with D-contacts: the workgroups owning the other nodes of this
  // workgroup's D-contacts (pair_sync in gridsync.h), and whether it has any
  __shared__ uint32_t s_pbm[LD ? kMaxGridSlots / 32 : 1];
  __shared__ int s_pflag, s_anyd;
  const int G = gridDim.x;
  const int lb = xcd_logical_block(blockIdx.x, G);
  const int slot = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nch = (a.n_nodes + 63) / 64;
  const int64_t c0 = lb * nch / G, c1 = (lb + 1) * nch / G;
  const int64_t c = c0 + slot;
  const int64_t n0 = c * 64;
  const int cnt = (c < c1) ? (int)min<int64_t>(64, a.n_nodes - n0) : 0;
  const int64_t i = n0 + lane;
  const bool act = lane < cnt;

  const int flags = *a.flags;
  if (flags != 0 || a.max_iters <= 0) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < 3 * (int64_t)a.n_contacts;
         k += (int64_t)G * blockDim.x)
      a.d.lambda[k] = 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.stats->iters = 0;
      a.stats->status = flags ? flags : VFPI_S_MAXITER;
      a.stats->theta = INFINITY;
    }
    return;
  }
  const SweepData<double>& d = a.d;
  const int nk = act ? d.row_ptr[i + 1] - d.row_ptr[i] : 0;
  const int64_t base = cnt > 0 ? d.row_ptr[n0] : 0;
  int col[KC];
  double av[KC][9];
  int64_t off = 0;
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const uint64_t m = ballot(k < nk);
    const int ck = __popcll(m);
    // a level the row lacks: a zero block on column 0, so the sweep's
    // register levels run without branches (adding the exact zero)
    col[k] = 0;
#pragma unroll
    for (int e = 0; e < 9; ++e) av[k][e] = 0.0;
    if (k < nk) {
      const int pos = lanes_below(m, lane);
      const int64_t q = base + off;
      col[k] = d.scol[q + pos];
      load_sblock(d.sval, q, ck, pos, av[k]);
    }
    off += ck;
  }
#pragma unroll
  for (int k = 0; k < KL; ++k) {
    const uint64_t m = ballot(KC + k < nk);
    const int ck = __popcll(m);
    if (KC + k < nk) {
      const int pos = lanes_below(m, lane);
      const int64_t q = base + off;
      s_cl[slot][k][lane] = d.scol[q + pos];
#pragma unroll
      for (int e = 0; e < 9; ++e) s_al[slot][k][e][lane] = d.sval[sval_at<double>(q, ck, pos, e)];
    } else {
      // a zero block on a valid column: the sweep's LDS levels then run
      // without branches (adding the exact zero leaves A v unchanged)
      s_cl[slot][k][lane] = act ? (int)i : 0;
#pragma unroll
      for (int e = 0; e < 9; ++e) s_al[slot][k][e][lane] = 0.0;
    }
    off += ck;
  }
  const int64_t off_tail = off;
  double vo[3] = {0.0, 0.0, 0.0};
  int m = -1;
  if (act) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      s_bw[slot][r][lane] = d.b[3 * i + r];
      s_bw[slot][3 + r][lane] = d.w[3 * i + r];
      vo[r] = a.v_user[3 * i + r];
    }
    m = d.cmap[i];
    if (m >= 0)
      for (int e = 0; e < kPack; ++e) s_cr[slot][e][lane] = d.cpack[kPack * (int64_t)m + e];
  }
  if constexpr (!LAG) {
#pragma unroll
    for (int e = 0; e < 6; ++e) s_lam[slot][e][lane] = 0.0;
  }
  const bool isd = m >= 0 && is_dcontact(d, m);
  const int64_t pi = isd ? d.cpair[2 * (int64_t)m] : -1, pj = isd ? d.cpair[2 * (int64_t)m + 1] : -1;
  const bool owner = !isd || pi == i;  // reports lambda
  // the same in every workgroup (the lagged form without LD: S-contacts only)
  const bool has_d = (!LAG || LD) && d.cpair != nullptr;
  double vp[3] = {vo[0], vo[1], vo[2]};  // v^{l-1} (Chebyshev only; v^0 = v^1)
  int br = BR_OPEN;
  double* vcur = a.v_user;
  double* vnext = a.v_alt;
  Cheby ch;
  ch.ls = CH ? a.cheby_ls : 0;
  ch.u = a.cheby_u;
  // BB: alpha^1 from the Gershgorin bound; v^{l-1} and A v^{l-1} of the own node
  double alpha = BB ? 1.0 / __builtin_bit_cast(double, (uint64_t)*a.amax) : 0.0;
  double vq[3] = {0.0, 0.0, 0.0}, aq[3] = {0.0, 0.0, 0.0};
  if constexpr (LAG) {
    // neighbour workgroups: the owners of the columns of this workgroup's
    // rows (chunk q belongs to the workgroup lg with lg nch / G <= q, i.e.
    // lg = ((q + 1) G - 1) / nch)
    for (int k = threadIdx.x; k < kMaxGridSlots / 32; k += blockDim.x) {
      s_nbm[k] = 0u;
      if constexpr (LD) s_pbm[k] = 0u;
    }
    if (threadIdx.x == 0) s_anyd = 0;
    __syncthreads();
    if (act) {
      const int64_t r1 = d.row_ptr[i + 1];
      for (int64_t k = d.row_ptr[i]; k < r1; ++k) {
        const int64_t q = (int64_t)d.col_idx[k] / 64;
        const int lg = (int)(((q + 1) * G - 1) / nch);
        if (lg != lb) atomicOr(&s_nbm[lg >> 5], 1u << (lg & 31));
      }
      if (LD && isd) {
        const int64_t q = (owner ? pj : pi) / 64;
        const int lg = (int)(((q + 1) * G - 1) / nch);
        if (lg != lb) atomicOr(&s_pbm[lg >> 5], 1u << (lg & 31));
        atomicOr(&s_anyd, 1);
      }
    }
    __syncthreads();
  }
  for (int l = 1;; ++l) {
    const double nu = CH ? ch.next_nu(l) : 1.0;
    double xs[KC][3];
#pragma unroll
    for (int k = 0; k < KC; ++k) ldv3<COH>(vcur, col[k], xs[k]);
    // up to four LDS levels: their gathers go out with the register levels'
    // (one round trip for both); more would cost the registers of A's levels
    constexpr bool EL = KL > 0 && KL <= 4;
    double xe[EL ? KL : 1][3];
    if constexpr (EL) {
      int ce[KL];
#pragma unroll
      for (int k = 0; k < KL; ++k) ce[k] = s_cl[slot][k][lane];
#pragma unroll
      for (int k = 0; k < KL; ++k) ldv3<COH>(vcur, ce[k], xe[k]);
    }
    double Av[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      Av[0] += dot3(av[k][0], av[k][1], av[k][2], xs[k][0], xs[k][1], xs[k][2]);
      Av[1] += dot3(av[k][3], av[k][4], av[k][5], xs[k][0], xs[k][1], xs[k][2]);
      Av[2] += dot3(av[k][6], av[k][7], av[k][8], xs[k][0], xs[k][1], xs[k][2]);
    }
    // LDS levels: gathered above with the register levels (up to four), or
    // here all at once (one round trip; gathering two at a time took four);
    // levels a row lacks hold zero blocks, so there is no branch here
    constexpr int LG = EL ? 2 : (KL > 0 ? KL : 1);
#pragma unroll
    for (int k0 = 0; k0 < KL; k0 += LG) {
      double xl[LG][3];
#pragma unroll
      for (int u = 0; u < LG; ++u) {
        const int k = k0 + u;
        if (k < KL) {
          if constexpr (EL) {
#pragma unroll
            for (int r = 0; r < 3; ++r) xl[u][r] = xe[k][r];
          } else {
            ldv3<COH>(vcur, s_cl[slot][k][lane], xl[u]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < LG; ++u) {
        const int k = k0 + u;
        if (k < KL) {
          // all five LDS reads of the block issue before its products
          double al[9];
#pragma unroll
          for (int e = 0; e < 9; ++e) al[e] = s_al[slot][k][e][lane];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int r = 0; r < 3; ++r)
            Av[r] += dot3(al[3 * r], al[3 * r + 1], al[3 * r + 2], xl[u][0], xl[u][1], xl[u][2]);
        }
      }
    }
    spmv_rows3_from<double, COH, U>(d.scol, d.sval, vcur, base, nk, lane, KC + KL, off_tail, Av);
    if (BB) {
      // s = v^l - v^{l-1}, z = A v^l - A v^{l-1}: s's, s'z, z'z over the grid
      if (l >= 2) {
        double dots[3] = {0.0, 0.0, 0.0};
        if (act) {
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            const double s = vo[r] - vq[r], z = Av[r] - aq[r];
            dots[0] += s * s;
            dots[1] += s * z;
            dots[2] += z * z;
          }
        }
        grid_sum3(a.slots + kBBSlotOffset, G, lb, l - 1, dots, s_red, s_poll);
        if (!a.bb2 && dots[0] > 0.0 && dots[1] > 0.0) alpha = dots[0] / dots[1];
        else if (a.bb2 && dots[1] > 0.0 && dots[2] > 0.0) alpha = dots[1] / dots[2];
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        vq[r] = vo[r];
        aq[r] = Av[r];
      }
    }
    double th2 = 0.0;
    double vn[3] = {0.0, 0.0, 0.0};
    double vs[3] = {0.0, 0.0, 0.0};
    if (act) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        vs[r] = vo[r] - (BB ? alpha : s_bw[slot][3 + r][lane]) * (Av[r] - s_bw[slot][r][lane]);
        vn[r] = vs[r];
      }
    }
    bool pair_ok = true;
    if (has_d) {
      // node-node contacts in two phases: the nodes of D pairs publish v*,
      // and after a barrier (the whole grid; LAG: the partner workgroups,
      // v* double-buffered by sweep parity behind the lagged contact ring)
      // both nodes of a pair read the same two values, so they form the same
      // lambda
      double* vsb = LAG ? a.lring + 16 * (int64_t)a.n_contacts + (int64_t)(l & 1) * 3 * a.n_nodes : a.avbuf;
      if (act && isd) {
#pragma unroll
        for (int r = 0; r < 3; ++r) stv<COH>(vsb + 3 * i + r, vs[r]);
      }
      if constexpr (LD) {
        if (s_anyd) pair_ok = pair_sync(a.slots, G, lb, l, s_pbm, &s_pflag);
      } else if constexpr (!LAG) {
        grid_barrier(a.slots, G, lb, 2 * l - 1, s_poll);
      }
      if (act && isd) {
        ContactRec<double> cr;
#pragma unroll
        for (int e = 0; e < 9; ++e) cr.R[e] = s_cr[slot][e][lane];
        cr.phi = s_cr[slot][9][lane];
        cr.mu = s_cr[slot][10][lane];
        cr.g = BB ? 2.0 * alpha + a.omega : s_cr[slot][11][lane];  // gamma = w_i + w_j (+ omega)
        cr.mu2 = s_cr[slot][12][lane];
        double eta[3], lam[3], ls[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) eta[r] = ldv<COH>(vsb + 3 * pi + r) - ldv<COH>(vsb + 3 * pj + r);
        br = contact_solve<double>(cr, eta[0], eta[1], eta[2], d.proj, lam, ls);
        const double sg = owner ? 1.0 : -1.0;  // +W R^T lambda on node i, -W R^T lambda on node j
        double* rg = (LAG && owner) ? a.lring + ((int64_t)(l & 1) * a.n_contacts + m) * 8 : nullptr;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const double F = cr.R[r] * lam[0] + cr.R[3 + r] * lam[1] + cr.R[6 + r] * lam[2];
          vn[r] = vs[r] + sg * (BB ? alpha : s_bw[slot][3 + r][lane]) * F;
          if constexpr (LAG) {
            if (owner) {
              rg[r] = lam[r];
              rg[3 + r] = ls[r];
            }
          } else {
            s_lam[slot][r][lane] = lam[r];
            s_lam[slot][3 + r][lane] = ls[r];
          }
        }
        if (LAG && owner) rg[6] = (double)br;
      }
    }
    if (act) {
      if (m >= 0 && !isd) {
        ContactRec<double> cr;
#pragma unroll
        for (int e = 0; e < 9; ++e) cr.R[e] = s_cr[slot][e][lane];
        cr.phi = s_cr[slot][9][lane];
        cr.mu = s_cr[slot][10][lane];
        cr.g = BB ? alpha + a.omega : s_cr[slot][11][lane];
        cr.mu2 = s_cr[slot][12][lane];
        double lam[3], ls[3];
        br = contact_solve<double>(cr, vs[0], vs[1], vs[2], d.proj, lam, ls);
        double* rg = LAG ? a.lring + ((int64_t)(l & 1) * a.n_contacts + m) * 8 : nullptr;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const double F = cr.R[r] * lam[0] + cr.R[3 + r] * lam[1] + cr.R[6 + r] * lam[2];
          vn[r] = vs[r] + (BB ? alpha : s_bw[slot][3 + r][lane]) * F;
          if constexpr (LAG) {
            rg[r] = lam[r];
            rg[3 + r] = ls[r];
          } else {
            s_lam[slot][r][lane] = lam[r];
            s_lam[slot][3 + r][lane] = ls[r];
          }
        }
        if (LAG) rg[6] = (double)br;
      }
      if (CH && ch.ls) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const double p = vp[r];
          vp[r] = vo[r];
          vn[r] = nu * (ch.u * (vn[r] - vo[r]) + vo[r] - p) + p;
        }
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double dd = vn[r] - vo[r];
        th2 += dd * dd;
        s_out[slot][3 * lane + r] = vn[r];
      }
    }
    __syncthreads();
    // the wave's 3*cnt values are contiguous in v: store them as whole lines
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int e = lane + 64 * j;
      if (e < 3 * cnt) stv<COH>(vnext + 3 * n0 + e, s_out[slot][e]);
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) vo[r] = vn[r];
    th2 = block_sum(th2, s_red);
    if constexpr (LAG) {
      LagResult lr = lag_sync(a.slots, G, lb, l, th2, a.max_iters, a.fixed, a.tol, s_nbm, s_poll, &s_lflag);
      if (!pair_ok) lr = {l, VFPI_S_SYNC_TIMEOUT, (double)INFINITY};
      if (lr.stop == 0) {
        double* t = vcur;
        vcur = vnext;
        vnext = t;
        continue;
      }
      // Alg. 1 stopped at sweep s = l (results of this sweep) or l - 1 (v^l
      // is in vcur, the contact results in the ring's other half)
      const int s = lr.stop;
      if (lr.status == VFPI_S_SYNC_TIMEOUT) {
        if (threadIdx.x == 0) atomicOr(&a.stats->status, VFPI_S_SYNC_TIMEOUT);
      } else if (lb == 0 && threadIdx.x == 0) {
        a.stats->iters = s;
        a.stats->status = lr.status;
        a.stats->theta = lr.theta;
      }
      int cb[3] = {0, 0, 0};
      if (act) {
        if (s != l) {
#pragma unroll
          for (int r = 0; r < 3; ++r) vo[r] = ldv<COH>(vcur + 3 * i + r);
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          a.v_user[3 * i + r] = vo[r];
          if (a.tape_v) a.tape_v[3 * i + r] = vo[r];
        }
        if (m >= 0 && owner) {
          const double* rg = a.lring + ((int64_t)(s & 1) * a.n_contacts + m) * 8;
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            d.lambda[3 * (int64_t)m + r] = rg[r];
            if (d.tape_lamstar) d.tape_lamstar[3 * (int64_t)m + r] = rg[3 + r];
          }
          const int bs = (int)rg[6];
          if (d.tape_branch) d.tape_branch[m] = bs;
          cb[bs] = 1;
        }
      }
      block_sum4_int(cb[0], cb[1], cb[2], s_ired);
      add_counts(a.stats, cb[0], cb[1], cb[2]);
      return;
    } else {
      double theta;
      const bool stop = grid_residual_step(a.slots, G, lb, has_d ? 2 * l : l, th2, l, a.max_iters, a.fixed,
                                           a.tol, a.stats, s_poll, &theta);
      double* t = vcur;
      vcur = vnext;
      vnext = t;
      if (stop) break;
      if (CH) ch.observe(theta);
    }
  }
  if constexpr (LAG) return;  // (the lagged form returns inside the loop)
  int cb[3] = {0, 0, 0};
  if (act && m >= 0 && owner) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      d.lambda[3 * (int64_t)m + r] = s_lam[slot][r][lane];
      if (d.tape_lamstar) d.tape_lamstar[3 * (int64_t)m + r] = s_lam[slot][3 + r][lane];
    }
    if (d.tape_branch) d.tape_branch[m] = br;
    cb[br] = 1;
  }
  block_sum4_int(cb[0], cb[1], cb[2], s_ired);
  add_counts(a.stats, cb[0], cb[1], cb[2]);
  if (act && (vcur != a.v_user || a.tape_v)) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      if (vcur != a.v_user) a.v_user[3 * i + r] = vo[r];
      if (a.tape_v) a.tape_v[3 * i + r] = vo[r];
    }
  }
  if (BB && act && a.tape_w) {
#pragma unroll
    for (int r = 0; r < 3; ++r) a.tape_w[3 * i + r] = alpha;
  }
}

}  // namespace vfpi

using namespace vfpi;

namespace {

struct Variant {
  int kind;   // 1: grid TPN=1, 2: grid TPN=3, 3: single workgroup TPN=1, 4: single workgroup TPN=3
  int nw;     // chunk slots per workgroup
  int grid;   // workgroup cap (0 = one per CU)
  int lds;    // kind 5: LDS levels 0 = when rows average more than 9 blocks, 1 = off, 2 = on
  int u;      // kind 1 with 8 chunk slots: levels per load group, 1 = two, else four
  int sync;   // kind 5: 1 = the residual reduction and barrier of every sweep (no lag)
};

// Library default (variant 0): the register-resident kernel with the fewest
// chunk slots per workgroup that still fits one workgroup per CU; the
// streaming kernel (kind 1) when the problem is larger, with eight chunk
// slots (waves) per workgroup and levels loaded two at a time: the most
// loads in flight per CU that the registers allow.
Variant decode_variant(int32_t v, int32_t n_nodes, int num_cu) {
  Variant x;
  x.kind = v & 0xff;
  x.nw = (v >> 8) & 0xff;
  x.grid = (v >> 16) & 0xff;
  x.lds = (v >> 24) & 0x3;
  x.u = (v >> 26) & 0x3;
  x.sync = (v >> 28) & 0x1;
  if (x.kind == 0) {
    const int64_t nch = ((int64_t)n_nodes + 63) / 64;
    const int64_t cap = num_cu < kMaxGridSlots ? num_cu : kMaxGridSlots;
    x.kind = 1;
    for (int nw : {2, 4, 5, 6, 8}) {
      int64_t g = (nch + nw - 1) / nw;
      if (g > 8 && g % 8 != 0) g += 8 - g % 8;
      if (g > nch) g = nch;
      if (g <= cap) {
        x.kind = 5;
        if (x.nw == 0) x.nw = nw;
        break;
      }
    }
    if (x.kind == 1 && x.nw == 0 && x.u == 0) {
      x.nw = 8;
      x.u = 1;
    }
  }
  if (x.nw == 0) x.nw = (x.kind == 3) ? 16 : (x.kind == 4 ? 5 : (x.kind == 1 ? 2 : (x.kind == 5 ? 2 : 1)));
  return x;
}

// Cooperative launch of at most one workgroup per CU (capped by the number of
// chunk groups and the caller's cap); the grid is a multiple of 8 above 8 so
// the XCD-aware numbering is exact.
hipError_t launch_persistent(void (*kern)(GridArgs), int threads, int nw, const GridArgs& ga, int grid_req,
                             int num_cu, int n_nodes, bool single, hipStream_t st) {
  if (single) {
    hipLaunchKernelGGL(kern, dim3(1), dim3(threads), 0, st, ga);
    return hipGetLastError();
  }
  const int64_t nch = (n_nodes + 63) / 64;
  int64_t g = (nch + nw - 1) / nw;
  int64_t cap = num_cu < kMaxGridSlots ? num_cu : kMaxGridSlots;
  if (g > cap) g = cap;
  if (grid_req > 0 && grid_req < g) g = grid_req;
  if (g > 8) g -= g % 8;
  if (g < 1) g = 1;
  GridArgs arg = ga;
  void* params[] = {&arg};
  return hipLaunchCooperativeKernel((const void*)kern, dim3((unsigned)g), dim3(threads), params, 0, st);
}

template <int TPN, int NW, int... U>
hipError_t launch_grid(const GridArgs& ga, int grid_req, int num_cu, int n_nodes, bool single, hipStream_t st) {
  return launch_persistent(k_vfpi_grid<TPN, NW, U...>, 64 * TPN * NW, NW, ga, grid_req, num_cu, n_nodes, single,
                           st);
}

template <int NW>
hipError_t launch_bb(const GridArgs& ga, int grid_req, int num_cu, int n_nodes, bool single, hipStream_t st) {
  return launch_persistent(k_vfpi_bb<NW>, 64 * NW, NW, ga, grid_req, num_cu, n_nodes, single, st);
}

// Chunk slots of the register-resident instance a requested slot count maps to.
int regs_slots(int nw) { return nw <= 1 ? 1 : nw <= 2 ? 2 : nw <= 4 ? 4 : nw <= 5 ? 5 : nw <= 6 ? 6 : 8; }

// Grid of the register-resident kernel: one pass per workgroup, so the grid
// must cover every chunk with at most NW chunks per workgroup; -1 when that
// needs more than one workgroup per CU.
int64_t regs_grid(int NW, int grid_req, int num_cu, int n_nodes) {
  const int64_t nch = (n_nodes + 63) / 64;
  int64_t g = (nch + NW - 1) / NW;
  const int64_t cap = num_cu < kMaxGridSlots ? num_cu : kMaxGridSlots;
  if (grid_req > 0 && grid_req > g) g = grid_req < nch ? grid_req : nch;
  if (g > 8 && g % 8 != 0) g += 8 - g % 8;  // round up: every workgroup still gets <= NW chunks
  if (g > nch) g = nch;
  return g > cap ? -1 : g;
}

// Register-resident launch (refused with invalid value when the grid does not
// fit).  KC register levels and KL LDS levels per lane (KLL in the lagged
// form, which keeps no per-lane lambda buffer); the rest streamed in groups
// of U levels (UD in the lagged form with D-contacts).  The lagged
// S-contact form, the leanest in registers, takes KCL register levels and
// groups of UL.
template <int NW, int KC, int KL, int U, bool BB, int KLL = KL, int UD = U, int KCL = KC, int UL = U>
hipError_t launch_regs(const GridArgs& ga, int grid_req, int num_cu, int n_nodes, bool sync, hipStream_t st) {
  const int64_t g = regs_grid(NW, grid_req, num_cu, n_nodes);
  if (g < 0) return hipErrorInvalidValue;
  GridArgs arg = ga;
  void* params[] = {&arg};
  const void* kern;
  if constexpr (BB) {  // no Chebyshev with BB step sizes
    if (g == 1) {      // one workgroup: plain loads, no cooperative launch needed
      hipLaunchKernelGGL((k_vfpi_regs<NW, KC, KL, U, false, false, true>), dim3(1), dim3(64 * NW), 0, st, ga);
      return hipGetLastError();
    }
    kern = (const void*)k_vfpi_regs<NW, KC, KL, U, true, false, true>;
  } else {
    const bool ch = ga.cheby_ls > 0;
    if (g == 1) {
      if (ch)
        hipLaunchKernelGGL((k_vfpi_regs<NW, KC, KL, U, false, true>), dim3(1), dim3(64 * NW), 0, st, ga);
      else
        hipLaunchKernelGGL((k_vfpi_regs<NW, KC, KL, U, false, false>), dim3(1), dim3(64 * NW), 0, st, ga);
      return hipGetLastError();
    }
    // the lagged residual needs no Chebyshev (nu of sweep l + 1 depends on
    // theta_l); D-contacts take its instance with the partner barrier
    const bool lag = !ch && !sync;
    kern = ch    ? (const void*)k_vfpi_regs<NW, KC, KL, U, true, true>
           : !lag ? (const void*)k_vfpi_regs<NW, KC, KL, U, true, false>
           : ga.d.cpair ? (const void*)k_vfpi_regs<NW, KC, KLL, UD, true, false, false, true, true>
                        : (const void*)k_vfpi_regs<NW, KCL, KLL, UL, true, false, false, true>;
  }
  return hipLaunchCooperativeKernel(kern, dim3((unsigned)g), dim3(64 * NW), params, 0, st);
}

// Kind 5: (chunk slots, register levels, LDS levels, tail unroll); the LDS
// levels use what the per-node constants leave of the 160 KB.  Their code
// costs register space even when no row reaches them, so rows of at most 9
// blocks on average (cloth) take the instances without them.
template <bool BB>
hipError_t launch_kind5(const Variant& vr, const GridArgs& ga, int num_cu, int N, bool long_rows,
                        hipStream_t stream) {
  const bool kl = vr.lds == 2 || (vr.lds == 0 && long_rows);
  if (kl)
    return (vr.nw <= 1)   ? launch_regs<1, 9, 8, 1, BB>(ga, vr.grid, num_cu, N, vr.sync != 0, stream)
           : (vr.nw <= 2) ? launch_regs<2, 9, 8, 2, BB>(ga, vr.grid, num_cu, N, vr.sync != 0, stream)
           : (vr.nw <= 4) ? launch_regs<4, 9, 4, 2, BB>(ga, vr.grid, num_cu, N, vr.sync != 0, stream)
           : (vr.nw <= 5) ? launch_regs<5, 6, 3, BB ? 2 : 3, BB, 4, 2, 7, 2>(ga, vr.grid, num_cu, N, vr.sync != 0, stream)
           : (vr.nw <= 6) ? launch_regs<6, 4, 2, BB ? 2 : 3, BB, 3, 2, 6, 2>(ga, vr.grid, num_cu, N, vr.sync != 0, stream)
                          : launch_regs<8, 4, 0, 2, BB, 0, 2, 6, 2>(ga, vr.grid, num_cu, N, vr.sync != 0, stream);
  return (vr.nw <= 1)   ? launch_regs<1, 9, 0, 1, BB>(ga, vr.grid, num_cu, N, vr.sync != 0, stream)
         : (vr.nw <= 2) ? launch_regs<2, 9, 0, 1, BB>(ga, vr.grid, num_cu, N, vr.sync != 0, stream)
         : (vr.nw <= 4) ? launch_regs<4, 9, 0, 1, BB>(ga, vr.grid, num_cu, N, vr.sync != 0, stream)
         : (vr.nw <= 5) ? launch_regs<5, 6, 0, 2, BB, 0, 2, 7, 2>(ga, vr.grid, num_cu, N, vr.sync != 0, stream)
         : (vr.nw <= 6) ? launch_regs<6, 6, 0, 2, BB, 0, 2, 7, 2>(ga, vr.grid, num_cu, N, vr.sync != 0, stream)
                        : launch_regs<8, 6, 0, 2, BB, 0, 2, 7, 2>(ga, vr.grid, num_cu, N, vr.sync != 0, stream);
}

// Barzilai-Borwein step sizes: the register-resident kernel (kind 5) or the
// two-phase streaming kernel, grid (kind 1) or one workgroup (kind 3); the
// other kinds do not implement it.
hipError_t launch_variant_bb(const Variant& vr, const GridArgs& ga, int num_cu, int N, bool long_rows,
                             hipStream_t stream) {
  switch (vr.kind) {
    case 5:
      return launch_kind5<true>(vr, ga, num_cu, N, long_rows, stream);
    case 1:
      return (vr.nw <= 1)   ? launch_bb<1>(ga, vr.grid, num_cu, N, false, stream)
             : (vr.nw <= 2) ? launch_bb<2>(ga, vr.grid, num_cu, N, false, stream)
                            : launch_bb<4>(ga, vr.grid, num_cu, N, false, stream);
    case 3:
      return (vr.nw <= 4) ? launch_bb<4>(ga, 1, num_cu, N, true, stream)
                          : launch_bb<16>(ga, 1, num_cu, N, true, stream);
    default:
      return hipErrorNotSupported;
  }
}

hipError_t launch_variant(const Variant& vr, const GridArgs& ga, int num_cu, int N, bool long_rows,
                          hipStream_t stream) {
  switch (vr.kind) {
    case 5:
      return launch_kind5<false>(vr, ga, num_cu, N, long_rows, stream);
    case 1:
      return (vr.nw <= 1)   ? launch_grid<1, 1>(ga, vr.grid, num_cu, N, false, stream)
             : (vr.nw <= 2) ? launch_grid<1, 2>(ga, vr.grid, num_cu, N, false, stream)
             : (vr.nw <= 4) ? launch_grid<1, 4>(ga, vr.grid, num_cu, N, false, stream)
             : (vr.nw <= 8) ? (vr.u == 1 ? launch_grid<1, 8, 2>(ga, vr.grid, num_cu, N, false, stream)
                                         : launch_grid<1, 8>(ga, vr.grid, num_cu, N, false, stream))
                            : launch_grid<1, 16>(ga, vr.grid, num_cu, N, false, stream);
    case 2:
      return (vr.nw <= 1)   ? launch_grid<3, 1>(ga, vr.grid, num_cu, N, false, stream)
             : (vr.nw <= 2) ? launch_grid<3, 2>(ga, vr.grid, num_cu, N, false, stream)
                            : launch_grid<3, 4>(ga, vr.grid, num_cu, N, false, stream);
    case 3:
      return (vr.nw <= 4) ? launch_grid<1, 4>(ga, 1, num_cu, N, true, stream)
                          : launch_grid<1, 16>(ga, 1, num_cu, N, true, stream);
    case 4:
      return launch_grid<3, 5>(ga, 1, num_cu, N, true, stream);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

extern "C" int vfpi_step(vfpi_ctx* ctx, const vfpi_bsr* A, const double* b, const vfpi_contacts* Jc, double* v,
                         double* lambda, const vfpi_opts* opts, vfpi_stats* stats, void* tape, hipStream_t stream) {
  if (!ctx || !A || !b || !Jc || !v || !opts || !stats) return VFPI_E_NULL;
  const int32_t N = A->n_nodes, nc = Jc->n_contacts;
  if (N < 0 || nc < 0 || A->nnzb < 0 || Jc->nnzb < 0 || nc > N) return VFPI_E_SHAPE;
  if (N > 0 && (!A->row_ptr || !A->col_idx || !A->val)) return VFPI_E_NULL;
  if (nc > 0 && (!Jc->row_ptr || !Jc->col_idx || !Jc->val || !Jc->phi || !Jc->mu || !lambda)) return VFPI_E_NULL;
  if (N > ctx->max_nodes || A->nnzb > ctx->max_nnzb || nc > ctx->max_contacts) return VFPI_E_CAPACITY;
  int rc = vfpi_check_opts(opts, false);
  if (rc) return rc;
  const bool bb = opts->w_mode == VFPI_W_BB1 || opts->w_mode == VFPI_W_BB2;
  if (bb && opts->cheby_ls > 0) return VFPI_E_UNSUPPORTED;
  if (Jc->mu2 && opts->projection != VFPI_PROJ_STRICT) return VFPI_E_UNSUPPORTED;
  if (Jc->nnzb > 2 * (int64_t)nc) return VFPI_E_SHAPE;  // at most two blocks per contact row
  if (opts->reuse_w && ctx->stats_nodes != N) return VFPI_E_OPTS;
  if (N == 0) {
    hipLaunchKernelGGL(k_stats_empty, dim3(1), dim3(1), 0, stream, stats);
    VFPI_CHECK_HIP(hipGetLastError());
    return VFPI_OK;
  }
  // the launch variant is checked before anything is enqueued
  const Variant vr = decode_variant(opts->variant, N, ctx->num_cu);
  if (vr.kind < 1 || vr.kind > 5) return VFPI_E_OPTS;
  if (bb && vr.kind != 1 && vr.kind != 3 && vr.kind != 5) return VFPI_E_UNSUPPORTED;
  if (vr.kind == 5 && regs_grid(regs_slots(vr.nw), vr.grid, ctx->num_cu, N) < 0) return VFPI_E_OPTS;
  VFPI_CHECK_HIP(hipSetDevice(ctx->device));

  TapeView tv = {nullptr, nullptr, nullptr, nullptr};
  if (tape) tv = tape_view(tape, N, nc);
  double* cpack = static_cast<double*>(ctx->cpack);
  double* w = static_cast<double*>(ctx->w);

  vfpi_mark(ctx, 0, stream);
  // setup kernels in one-wave workgroups: spread over every CU (faster than
  // four waves on a quarter of them)
  hipLaunchKernelGGL(k_prep, dim3((N + 63) / 64), dim3(64), 0, stream, N, ctx->cmap, ctx->flags, ctx->sync,
                     ctx->slots, stats);
  if (nc > 0)
    hipLaunchKernelGGL(k_contacts<double>, dim3((nc + 63) / 64), dim3(64), 0, stream, nc, Jc->nnzb, Jc->row_ptr,
                       Jc->col_idx, static_cast<const double*>(Jc->val), static_cast<const double*>(Jc->phi),
                       static_cast<const double*>(Jc->mu), static_cast<const double*>(Jc->mu2), N, ctx->cmap,
                       cpack, ctx->cpair, ctx->flags, 1e-10);
  RowsArgs ra;
  ra.nnzb = A->nnzb;
  ra.w_mode = opts->w_mode;
  ra.reuse = opts->reuse_w != 0;
  ra.alpha = bb ? 1.0 : opts->alpha_user;  // BB: alpha is set on the device
  ra.omega = opts->omega;
  ra.amax = bb ? reinterpret_cast<unsigned long long*>(ctx->sync + SY_AMAX) : nullptr;
  const int64_t nch = (N + 63) / 64;
  hipLaunchKernelGGL(k_rows<double>, dim3((unsigned)nch), dim3(64), 0, stream, N, A->row_ptr, A->col_idx,
                     static_cast<const double*>(A->val), ctx->scol, static_cast<double*>(ctx->sval), ctx->diag,
                     ctx->rn2, ra, static_cast<const double*>(opts->w_user), ctx->cmap, cpack, w, tv.w, b, v,
                     ctx->flags);
  if (nc > 0 && Jc->nnzb > nc)
    hipLaunchKernelGGL(k_pairs<double>, dim3((nc + 255) / 256), dim3(256), 0, stream, nc, ctx->cpair, ctx->diag,
                       ctx->rn2, ra, w, tv.w, cpack, ctx->flags);
  VFPI_CHECK_HIP(hipGetLastError());
  ctx->stats_nodes = N;

  GridArgs ga;
  ga.d.row_ptr = A->row_ptr;
  ga.d.scol = ctx->scol;
  ga.d.sval = static_cast<const double*>(ctx->sval);
  ga.d.b = b;
  ga.d.w = w;
  ga.d.cmap = ctx->cmap;
  ga.d.cpack = cpack;
  ga.d.lambda = lambda;
  ga.d.tape_lamstar = tv.lamstar;
  ga.d.tape_branch = tv.branch;
  ga.d.proj = opts->projection;
  ga.d.col_idx = A->col_idx;
  ga.d.val = static_cast<const double*>(A->val);
  ga.d.cpair = (Jc->nnzb > nc) ? ctx->cpair : nullptr;
  ga.n_nodes = N;
  ga.n_contacts = nc;
  ga.v_user = v;
  ga.v_alt = static_cast<double*>(ctx->vbuf);
  ga.tape_v = tv.v;
  ga.max_iters = opts->max_iters;
  ga.fixed = opts->fixed_iters;
  ga.tol = opts->tol;
  ga.flags = ctx->flags;
  ga.stats = stats;
  ga.slots = ctx->slots;
  ga.vprev = static_cast<double*>(ctx->vprev);
  ga.cheby_ls = opts->cheby_ls;
  ga.cheby_u = opts->cheby_u == 0.0 ? 1.0 : opts->cheby_u;
  ga.bb2 = opts->w_mode == VFPI_W_BB2;
  ga.omega = opts->omega;
  ga.avbuf = ctx->adj;
  ga.amax = reinterpret_cast<const unsigned long long*>(ctx->sync + SY_AMAX);
  ga.tape_w = tv.w;
  ga.lring = ctx->adj;

  vfpi_mark(ctx, 1, stream);
  const bool long_rows = A->nnzb > 9 * (int64_t)N;
  hipError_t e = bb ? launch_variant_bb(vr, ga, ctx->num_cu, N, long_rows, stream)
                    : launch_variant(vr, ga, ctx->num_cu, N, long_rows, stream);
  if (e == hipErrorInvalidValue) return VFPI_E_OPTS;
  if (e == hipErrorNotSupported) return VFPI_E_UNSUPPORTED;
  vfpi_mark(ctx, 2, stream);
  return e == hipSuccess ? VFPI_OK : VFPI_E_HIP;
}
