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
  constexpr int NWAVES = TPN * NW;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = wave / TPN, r = (TPN == 3) ? wave % 3 : 0;

  for (;;) {
    if (threadIdx.x == 0) {
      s_env = (int)atomicAdd(a.queue, 1u);
      s_flag = 0;
    }
    __syncthreads();
    int e = s_env;
    if (e >= a.n_env) break;
    if (a.env_order) e = a.env_order[e];
    if (e < 0 || e >= a.n_env) {  // not a permutation entry: nothing safe to touch
      __syncthreads();
      continue;
    }
    const int64_t n_lo = a.env_node_off[e], n_hi = a.env_node_off[e + 1];
    const int64_t m_lo = a.env_con_off[e], m_hi = a.env_con_off[e + 1];
    const bool bad_off = n_lo < 0 || n_hi < n_lo || n_hi > a.n_nodes || m_lo < 0 || m_hi < m_lo ||
                         m_hi > a.n_contacts || m_hi - m_lo > n_hi - n_lo;
    if (bad_off) {
      if (threadIdx.x == 0) {
        vfpi_stats* st = a.stats + e;
        st->iters = 0;
        st->status = VFPI_S_BAD_PATTERN;
        st->theta = INFINITY;
        st->n_open = st->n_stick = st->n_slip = st->reserved = 0;
      }
      __syncthreads();
      continue;
    }
    // ---- setup (a0): contact map, records, chunk-interleaved A, W, gamma
    for (int64_t i = n_lo + threadIdx.x; i < n_hi; i += blockDim.x) a.cmap[i] = -1;
    __syncthreads();
    for (int64_t m = m_lo + threadIdx.x; m < m_hi; m += blockDim.x)
      contact_setup<float>(m, a.nnzb_c, a.crp, a.ccol, a.cval, a.phi, a.mu, a.mu2, n_lo, n_hi, a.cmap, a.cpack,
                           a.cpair, &s_flag, 1e-5);
    __syncthreads();
    const int64_t nn = n_hi - n_lo;
    const int64_t nch = (nn + 63) / 64;
    for (int64_t c = wave; c < nch; c += NWAVES) {
      const int64_t n0 = n_lo + 64 * c;
      rows_chunk<float>(n0, (int)min<int64_t>(64, n_hi - n0), lane, a.row_ptr, a.col_idx, a.val, a.scol, a.sval,
                        n_lo, n_hi, a.diag, a.rn2, a.ra, nullptr, a.cmap, a.cpack, a.w, nullptr, a.b, a.v_user,
                        &s_flag);
    }
    __syncthreads();
    if (a.has_d) {
      for (int64_t m = m_lo + threadIdx.x; m < m_hi; m += blockDim.x)
        pair_setup<float>(m, a.cpair, a.diag, a.rn2, a.ra, a.w, nullptr, a.cpack, &s_flag);
      __syncthreads();
    }
    const int flag = s_flag;
    if (flag != 0 || a.max_iters <= 0) {
      for (int64_t k = 3 * m_lo + threadIdx.x; k < 3 * m_hi; k += blockDim.x) a.lambda[k] = 0.0f;
      if (threadIdx.x == 0) {
        vfpi_stats* st = a.stats + e;
        st->iters = 0;
        st->status = flag ? flag : VFPI_S_MAXITER;
        st->theta = INFINITY;
        st->n_open = st->n_stick = st->n_slip = st->reserved = 0;
      }
      __syncthreads();
      continue;
    }
    // ---- V-FPI loop (a1-a5), workgroup-local
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
          sweep_chunk_row<float>(d, vcur, vnext, n0, cnt, lane, r, s_vs[p & 1][TPN == 3 ? slot : 0], th2, cb);
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
          vfpi_stats* st = a.stats + e;
          st->iters = l;
          st->status = conv ? VFPI_S_CONVERGED : VFPI_S_MAXITER;
          st->theta = theta;
          st->n_open = o;
          st->n_stick = s;
          st->n_slip = sl;
          st->reserved = 0;
        }
        s_stop = stop;
      }
      __syncthreads();
      const bool stop = s_stop != 0;
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
  if (kind > 3) return VFPI_E_OPTS;
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
  } else if (kind == 0 || kind == 1) {
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
