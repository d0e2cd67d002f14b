// (compiled as part of vfpi_lib.hip)
// Adjoint of a converged V-FPI step (FP64).
//
// The step's fixed-point map (Sec. IV, Lemma 1 framing) is
//   f(v) = v* + W J^T P(-Gamma^-1 (J v* + phi e1)),  v* = v - W (A v - b),
// with P the strict or the proximal projection (eq. operator), or the strict
// one on the elliptic cone (anisotropic friction).  Holding W constant (the fixed
// point does not depend on it, consistency remark of Sec. III-B) and writing
// D_P for P's Jacobian on the branch taken in the last sweep, G = I - W J^T D_P
// Gamma^-1 J, the adjoint u of a loss with gradients (g_v, g_lam) solves
//     u = g~ + (I - A W) G^T u,   g~ = g_v - (I - A W) J^T Gamma^-1 D_P^T g_lam.
// It is iterated in the variables t = G^T u, s = W t:
//     u^{l+1} = g~ + t^l - A s^l,  t^{l+1} = G^T u^{l+1},  s^{l+1} = W t^{l+1}
// so every sweep is one product with A plus node-local work, like the forward
// sweep.  Then, with r = J W u + g_lam and q = u - J^T Gamma^-1 D_P^T r:
//     dL/db = W q,  dL/dA_ij = -(dL/db)_i v_j,  dL/dphi_m = -(D_P^T r)_n / gamma_m,
//     dL/dmu_m = (dP/dmu)^T r_m  (and dL/dmu2_m = (dP/dmu2)^T r_m).
#include <math.h>

#include "gridsync.h"
#include "internal.h"
#include "setup.h"
#include "sweep.h"

namespace vfpi {

struct AdjArgs {
  int32_t n_nodes, n_contacts, nnzb;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* val;       // A in the caller's layout (rows of D-contact partners)
  const int32_t* cpair;    // contact nodes i, j (j = -1: S); nullptr: S only
  const int32_t* scol;
  const double* sval;
  const double* w;
  const int32_t* cmap;
  const double* cpack;
  const double* lamstar;
  const int32_t* branch;
  const double* vsol;
  const double* gv;
  const double* gl;
  double* gt;
  double* U[2];
  double* T[2];
  double* S[2];
  double* E;
  double* grad_b;
  double* grad_A;
  double* grad_phi;
  double* grad_mu;
  double* grad_mu2;  // anisotropic friction only (else nullptr)
  int32_t max_iters, fixed;
  double tol;
  const int32_t* flags;
  vfpi_stats* stats;
  uint64_t* slots;
  int32_t proj;  // the forward's projection (VFPI_PROJ_*)
};

// Slip branch of the strict operator on the elliptic cone (mu1 != mu2):
// lambda_n = n and x_i = A_i t_i / D_i, D_i = A_i + s, A_i = (mu_i n)^2, with s
// the root of F(s) = sum_i A_i t_i^2 / D_i^2 - 1 (recomputed from lambda* by
// the forward's own iteration).  Implicit differentiation, F_s = -2 sum_i
// A_i t_i^2 / D_i^3: ds = -(sum_i 2 A_i t_i / D_i^2 dt_i + sum_i t_i^2 (s - A_i)
// / D_i^3 dA_i) / F_s, dx_i = (t_i s / D_i^2) dA_i + (A_i / D_i) dt_i - (x_i /
// D_i) ds, dA_i = 2 mu_i^2 n dn + 2 mu_i n^2 dmu_i.  With a zero coefficient
// the ellipse is a segment and each tangent component is clamped on its own;
// the zero coefficient's derivative is the one-sided one of the opening
// ellipse (0 past the segment's tip; beside it dx_i = sign(t_i) n r dmu_i and
// dx_j = -n t_j |t_i| / (b^2 r) dmu_i, r = sqrt(1 - t_j^2 / b^2), b = mu_j n).
VFPI_DEV void dp_transpose_ellipse(const double* ls, double mu1, double mu2, const double x[3], double y[3],
                                   double* dmu1, double* dmu2) {
  const double n = ls[0], t[2] = {ls[1], ls[2]}, mu[2] = {mu1, mu2};
  double dm[2] = {0.0, 0.0};
  y[0] = x[0];
  if (mu1 * n == 0.0 || mu2 * n == 0.0) {  // the forward's test for a segment
    for (int i = 0; i < 2; ++i) {
      if (fabs(t[i]) > mu[i] * n) {
        const double sg = t[i] > 0.0 ? 1.0 : -1.0;
        y[0] += sg * mu[i] * x[1 + i];
        y[1 + i] = 0.0;
        dm[i] = sg * n * x[1 + i];
      } else {
        y[1 + i] = x[1 + i];
      }
    }
    const int i = mu1 * n == 0.0 ? 0 : 1, j = 1 - i;
    dm[i] = 0.0;
    const double b = mu[j] * n;
    if (b > 0.0 && fabs(t[j]) < b) {
      const double q = t[j] / b, r = sqrt(1.0 - q * q);
      dm[i] = (t[i] > 0.0 ? 1.0 : -1.0) * n * r * x[1 + i] - n * t[j] * fabs(t[i]) / (b * b * r) * x[1 + j];
    }
    *dmu1 = dm[0];
    *dmu2 = dm[1];
    return;
  }
  const double s = ellipse_multiplier(mu1 * n, mu2 * n, t[0], t[1]);
  double A[2], D[2], P = 0.0, Fs = 0.0, gA_An = 0.0;
  for (int i = 0; i < 2; ++i) {
    A[i] = (mu[i] * n) * (mu[i] * n);
    D[i] = A[i] + s;
    const double iD = 1.0 / D[i];
    P += A[i] * t[i] * iD * iD * x[1 + i];  // sum_i (x_i / D_i) z_i
    Fs -= 2.0 * A[i] * t[i] * t[i] * iD * iD * iD;
    gA_An += t[i] * t[i] * (s - A[i]) * iD * iD * iD * (2.0 * mu[i] * mu[i] * n);
  }
  const double ds_dn = -gA_An / Fs;
  for (int i = 0; i < 2; ++i) {
    const double iD = 1.0 / D[i];
    const double An = 2.0 * mu[i] * mu[i] * n, Amu = 2.0 * mu[i] * n * n;
    const double ds_dt = -2.0 * A[i] * t[i] * iD * iD / Fs;
    const double ds_dmu = -t[i] * t[i] * (s - A[i]) * iD * iD * iD * Amu / Fs;
    y[0] += t[i] * s * iD * iD * An * x[1 + i];
    y[1 + i] = A[i] * iD * x[1 + i] - ds_dt * P;
    dm[i] = t[i] * s * iD * iD * Amu * x[1 + i] - ds_dmu * P;
  }
  y[0] -= ds_dn * P;
  *dmu1 = dm[0];
  *dmu2 = dm[1];
}

// y = D_P^T x for the contact's branch; *dmu = (dP/dmu)^T x and *dmu2 =
// (dP/dmu2)^T x (zero with isotropic friction).  R is the contact's packed
// record (mu = R[10], mu2 = R[12]; mu2 != mu selects the elliptic cone, as in
// the forward).  Slip, strict operator: dl_n/dn = 1, dl_t/dn = mu h,
// dl_t/dt = (mu n / s)(I - h h^T), dl_t/dmu = n h with (n, t) = lambda*,
// s = |t|, h = t / s.  Slip, proximal operator (projection onto the cone,
// P = a (1, mu h), a = (n + mu s) c, c = 1 / (1 + mu^2)): the symmetric
// D_P = [c, mu c h^T; mu c h, mu^2 c h h^T + (mu a / s)(I - h h^T)],
// dP_n/dmu = c (s - 2 mu a), dP_t/dmu = (a + mu dP_n/dmu) h.
VFPI_DEV void dp_transpose(const double* ls, int br, const double* R, int proj, const double x[3], double y[3],
                           double* dmu, double* dmu2) {
  *dmu2 = 0.0;
  if (br == BR_STICK) {
    y[0] = x[0];
    y[1] = x[1];
    y[2] = x[2];
    *dmu = 0.0;
    return;
  }
  if (br != BR_SLIP) {
    y[0] = y[1] = y[2] = 0.0;
    *dmu = 0.0;
    return;
  }
  const double mu = R[10];
  if (proj != VFPI_PROJ_PROXIMAL && R[12] != mu) {
    dp_transpose_ellipse(ls, mu, R[12], x, y, dmu, dmu2);
    return;
  }
  const double n = ls[0], t1 = ls[1], t2 = ls[2];
  const double s = sqrt(t1 * t1 + t2 * t2);
  const double h1 = t1 / s, h2 = t2 / s;
  const double ht = h1 * x[1] + h2 * x[2];
  if (proj == VFPI_PROJ_PROXIMAL) {
    const double c = 1.0 / (1.0 + mu * mu);
    const double al = (n + mu * s) * c;
    const double z = c * (x[0] + mu * ht);
    const double kp = mu * al / s;
    y[0] = z;
    y[1] = mu * h1 * z + kp * (x[1] - h1 * ht);
    y[2] = mu * h2 * z + kp * (x[2] - h2 * ht);
    const double da = c * (s - 2.0 * mu * al);
    *dmu = da * x[0] + (al + mu * da) * ht;
    return;
  }
  const double k = mu * n / s;
  y[0] = x[0] + mu * ht;
  y[1] = k * (x[1] - h1 * ht);
  y[2] = k * (x[2] - h2 * ht);
  *dmu = n * ht;
}

// (G^T u)_i for a node: u - R^T D_P^T R (w_i u) / g on a contact node, with g
// = gamma_m (+ omega), u elsewhere.
VFPI_DEV void gt_node(const AdjArgs& a, int64_t i, int m, const double u[3], double out[3]) {
  out[0] = u[0];
  out[1] = u[1];
  out[2] = u[2];
  if (m < 0) return;
  const double* R = a.cpack + kPack * (int64_t)m;
  const double f = a.w[3 * i] / R[11];
  double x[3], y[3], dmu, dmu2;
  for (int k = 0; k < 3; ++k) x[k] = (R[3 * k] * u[0] + R[3 * k + 1] * u[1] + R[3 * k + 2] * u[2]) * f;
  dp_transpose(a.lamstar + 3 * (int64_t)m, a.branch[m], R, a.proj, x, y, &dmu, &dmu2);
  for (int r = 0; r < 3; ++r) out[r] -= R[r] * y[0] + R[3 + r] * y[1] + R[6 + r] * y[2];
}

// D-contact m (J_m = [R, -R] on nodes i, j) seen from one of its nodes:
// (G^T u) there = u_x -+ R^T D_P^T R (w_i u_i - w_j u_j) / g.
VFPI_DEV void gt_pair(const AdjArgs& a, int m, bool first, const double ui[3], const double uj[3], double out[3]) {
  const double* R = a.cpack + kPack * (int64_t)m;
  const int64_t i = a.cpair[2 * (int64_t)m], j = a.cpair[2 * (int64_t)m + 1];
  const double fi = a.w[3 * i] / R[11], fj = a.w[3 * j] / R[11];
  double x[3], y[3], dmu, dmu2;
  for (int k = 0; k < 3; ++k)
    x[k] = (R[3 * k] * ui[0] + R[3 * k + 1] * ui[1] + R[3 * k + 2] * ui[2]) * fi -
           (R[3 * k] * uj[0] + R[3 * k + 1] * uj[1] + R[3 * k + 2] * uj[2]) * fj;
  dp_transpose(a.lamstar + 3 * (int64_t)m, a.branch[m], R, a.proj, x, y, &dmu, &dmu2);
  const double* u = first ? ui : uj;
  for (int r = 0; r < 3; ++r) {
    const double f = R[r] * y[0] + R[3 + r] * y[1] + R[6 + r] * y[2];
    out[r] = first ? u[r] - f : u[r] + f;
  }
}

VFPI_DEV bool adj_isd(const AdjArgs& a, int m) { return m >= 0 && a.cpair && a.cpair[2 * (int64_t)m + 1] >= 0; }

// (A y)_x from A's block row x in the caller's layout; y read coherently.
VFPI_DEV void arow_bsr(const AdjArgs& a, const double* y, int64_t x, double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
  const int64_t r1 = a.row_ptr[x + 1];
  for (int64_t k = a.row_ptr[x]; k < r1; ++k) {
    const int64_t c = a.col_idx[k];
    const double* B = a.val + 9 * k;
    const double y0 = ldv<true>(y + 3 * c), y1 = ldv<true>(y + 3 * c + 1), y2 = ldv<true>(y + 3 * c + 2);
    for (int r = 0; r < 3; ++r) out[r] += dot3(B[3 * r], B[3 * r + 1], B[3 * r + 2], y0, y1, y2);
  }
}

template <int NW>
__global__ void __launch_bounds__(64 * NW) k_adjoint(AdjArgs a) {
  __shared__ double s_red[NW];
  __shared__ double s_poll[3 * NW];  // see grid_sum
  int seq = 0;
  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int lb = xcd_logical_block(b, G);
  const int slot = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nch = (a.n_nodes + 63) / 64;
  const int64_t c0 = lb * nch / G, c1 = (lb + 1) * nch / G;
  const int passes = (int)((c1 - c0 + NW - 1) / NW);
  const int flags = *a.flags;
  if (flags != 0) {
    for (int64_t k = b * (int64_t)blockDim.x + threadIdx.x; k < 3 * (int64_t)a.n_nodes; k += (int64_t)G * blockDim.x)
      a.grad_b[k] = 0.0;
    for (int64_t k = b * (int64_t)blockDim.x + threadIdx.x; k < a.n_contacts; k += (int64_t)G * blockDim.x) {
      a.grad_phi[k] = a.grad_mu[k] = 0.0;
      if (a.grad_mu2) a.grad_mu2[k] = 0.0;
    }
    if (a.grad_A)
      for (int64_t k = b * (int64_t)blockDim.x + threadIdx.x; k < 9 * (int64_t)a.nnzb;
           k += (int64_t)G * blockDim.x)
        a.grad_A[k] = 0.0;
    if (b == 0 && threadIdx.x == 0) {
      a.stats->iters = 0;
      a.stats->status = flags;
      a.stats->theta = INFINITY;
      a.stats->n_open = a.stats->n_stick = a.stats->n_slip = a.stats->reserved = 0;
    }
    return;
  }
  auto for_my_nodes = [&](auto&& fn) {
    for (int p = 0; p < passes; ++p) {
      const int64_t c = c0 + (int64_t)p * NW + slot;
      const int64_t n0 = c * 64;
      const int cnt = (c < c1) ? (int)min<int64_t>(64, a.n_nodes - n0) : 0;
      fn(n0, cnt);
    }
  };
  // phase A: e = J^T Gamma^-1 D_P^T g_lam (node-local), p = W e into S[1]
  if (a.gl) {
    for_my_nodes([&](int64_t n0, int cnt) {
      if (lane >= cnt) return;
      const int64_t i = n0 + lane;
      const int m = a.cmap[i];
      double e[3] = {0.0, 0.0, 0.0};
      if (m >= 0) {
        const double* R = a.cpack + kPack * (int64_t)m;
        double x[3] = {a.gl[3 * (int64_t)m], a.gl[3 * (int64_t)m + 1], a.gl[3 * (int64_t)m + 2]}, y[3], dmu, dmu2;
        dp_transpose(a.lamstar + 3 * (int64_t)m, a.branch[m], R, a.proj, x, y, &dmu, &dmu2);
        const double gi = (adj_isd(a, m) && a.cpair[2 * (int64_t)m] != i) ? -1.0 / R[11] : 1.0 / R[11];
        for (int r = 0; r < 3; ++r) e[r] = (R[r] * y[0] + R[3 + r] * y[1] + R[6 + r] * y[2]) * gi;
      }
      for (int r = 0; r < 3; ++r) {
        stv<true>(a.E + 3 * i + r, e[r]);
        stv<true>(a.S[1] + 3 * i + r, a.w[3 * i + r] * e[r]);
      }
    });
    grid_barrier(a.slots, G, lb, ++seq, s_poll);
  }
  // phase B: g~ = g_v - e + A p; u0 = g~, t0 = G^T u0, s0 = W t0
  for_my_nodes([&](int64_t n0, int cnt) {
    const int64_t i = n0 + lane;
    const bool act = lane < cnt;
    double Ap[3] = {0.0, 0.0, 0.0};
    if (a.gl) {
      const int nk = act ? a.row_ptr[i + 1] - a.row_ptr[i] : 0;
      spmv_rows3<double, true>(a.scol, a.sval, a.S[1], cnt > 0 ? a.row_ptr[n0] : 0, nk, lane, Ap);
    }
    if (!act) return;
    double u[3], t[3];
    const int m = a.cmap[i];
    if (adj_isd(a, m)) {  // u0 of both nodes of the pair, from A's rows
      double uu[2][3];
      for (int s = 0; s < 2; ++s) {
        const int64_t z = a.cpair[2 * (int64_t)m + s];
        double Az[3] = {0.0, 0.0, 0.0};
        if (a.gl) arow_bsr(a, a.S[1], z, Az);
        for (int r = 0; r < 3; ++r)
          uu[s][r] = a.gl ? a.gv[3 * z + r] - ldv<true>(a.E + 3 * z + r) + Az[r] : a.gv[3 * z + r];
      }
      const bool first = a.cpair[2 * (int64_t)m] == i;
      gt_pair(a, m, first, uu[0], uu[1], t);
      for (int r = 0; r < 3; ++r) u[r] = first ? uu[0][r] : uu[1][r];
    } else {
      for (int r = 0; r < 3; ++r) u[r] = a.gl ? a.gv[3 * i + r] - ldv<true>(a.E + 3 * i + r) + Ap[r] : a.gv[3 * i + r];
      gt_node(a, i, m, u, t);
    }
    for (int r = 0; r < 3; ++r) {
      stv<true>(a.gt + 3 * i + r, u[r]);
      stv<true>(a.U[0] + 3 * i + r, u[r]);
      stv<true>(a.T[0] + 3 * i + r, t[r]);
      stv<true>(a.S[0] + 3 * i + r, a.w[3 * i + r] * t[r]);
    }
  });
  grid_barrier(a.slots, G, lb, ++seq, s_poll);
  int cur = 0;
  if (a.max_iters > 0) {
    int l = 0;
    for (;;) {
      ++l;
      const int nxt = cur ^ 1;
      double th2 = 0.0;
      for_my_nodes([&](int64_t n0, int cnt) {
        const int64_t i = n0 + lane;
        const bool act = lane < cnt;
        const int nk = act ? a.row_ptr[i + 1] - a.row_ptr[i] : 0;
        double As[3];
        spmv_rows3<double, true>(a.scol, a.sval, a.S[cur], cnt > 0 ? a.row_ptr[n0] : 0, nk, lane, As);
        if (!act) return;
        double un[3], tn[3];
        const int m = a.cmap[i];
        if (adj_isd(a, m)) {  // u of both nodes of the pair, from A's rows
          double uu[2][3];
          for (int s = 0; s < 2; ++s) {
            const int64_t z = a.cpair[2 * (int64_t)m + s];
            double Az[3];
            arow_bsr(a, a.S[cur], z, Az);
            for (int r = 0; r < 3; ++r) uu[s][r] = ldv<true>(a.gt + 3 * z + r) + ldv<true>(a.T[cur] + 3 * z + r) - Az[r];
          }
          const bool first = a.cpair[2 * (int64_t)m] == i;
          gt_pair(a, m, first, uu[0], uu[1], tn);
          for (int r = 0; r < 3; ++r) un[r] = first ? uu[0][r] : uu[1][r];
        } else {
          for (int r = 0; r < 3; ++r) un[r] = ldv<true>(a.gt + 3 * i + r) + ldv<true>(a.T[cur] + 3 * i + r) - As[r];
          gt_node(a, i, m, un, tn);
        }
        for (int r = 0; r < 3; ++r) {
          const double d = un[r] - ldv<true>(a.U[cur] + 3 * i + r);
          th2 += d * d;
          stv<true>(a.U[nxt] + 3 * i + r, un[r]);
          stv<true>(a.T[nxt] + 3 * i + r, tn[r]);
          stv<true>(a.S[nxt] + 3 * i + r, a.w[3 * i + r] * tn[r]);
        }
      });
      th2 = block_sum(th2, s_red);
      const bool stop = grid_residual_step(a.slots, G, lb, ++seq, th2, l, a.max_iters, a.fixed, a.tol, a.stats, s_poll);
      cur = nxt;
      if (stop) break;
    }
  } else if (b == 0 && threadIdx.x == 0) {
    a.stats->iters = 0;
    a.stats->status = VFPI_S_MAXITER;
    a.stats->theta = INFINITY;
    a.stats->n_open = a.stats->n_stick = a.stats->n_slip = a.stats->reserved = 0;
  }
  // final gradients (node-local in u; A_bar reads the solution v of neighbours)
  const double* u_fin = a.U[cur];
  for_my_nodes([&](int64_t n0, int cnt) {
    if (lane >= cnt) return;
    const int64_t i = n0 + lane;
    const int m = a.cmap[i];
    double u[3] = {ldv<true>(u_fin + 3 * i), ldv<true>(u_fin + 3 * i + 1), ldv<true>(u_fin + 3 * i + 2)};
    double q[3] = {u[0], u[1], u[2]};
    if (m >= 0) {
      const double* R = a.cpack + kPack * (int64_t)m;
      const bool isd = adj_isd(a, m);
      const bool first = !isd || a.cpair[2 * (int64_t)m] == i;
      // r = J_m W u + g_lam (both nodes of a D-contact)
      const int64_t ni = isd ? a.cpair[2 * (int64_t)m] : i;
      double ui[3], rr[3], y[3], dmu, dmu2;
      for (int r = 0; r < 3; ++r) ui[r] = ldv<true>(u_fin + 3 * ni + r);
      const double wi = a.w[3 * ni];
      for (int k = 0; k < 3; ++k) {
        rr[k] = R[3 * k] * (wi * ui[0]) + R[3 * k + 1] * (wi * ui[1]) + R[3 * k + 2] * (wi * ui[2]);
        if (a.gl) rr[k] += a.gl[3 * (int64_t)m + k];
      }
      if (isd) {
        const int64_t nj = a.cpair[2 * (int64_t)m + 1];
        double uj[3];
        for (int r = 0; r < 3; ++r) uj[r] = ldv<true>(u_fin + 3 * nj + r);
        const double wj = a.w[3 * nj];
        for (int k = 0; k < 3; ++k)
          rr[k] -= R[3 * k] * (wj * uj[0]) + R[3 * k + 1] * (wj * uj[1]) + R[3 * k + 2] * (wj * uj[2]);
      }
      dp_transpose(a.lamstar + 3 * (int64_t)m, a.branch[m], R, a.proj, rr, y, &dmu, &dmu2);
      const double gi = 1.0 / R[11];
      const double sg = first ? gi : -gi;
      for (int r = 0; r < 3; ++r) q[r] -= (R[r] * y[0] + R[3 + r] * y[1] + R[6 + r] * y[2]) * sg;
      if (first) {
        a.grad_phi[m] = -y[0] * gi;
        a.grad_mu[m] = dmu;
        if (a.grad_mu2) a.grad_mu2[m] = dmu2;
      }
    }
    double bb[3];
    for (int r = 0; r < 3; ++r) {
      bb[r] = a.w[3 * i + r] * q[r];
      a.grad_b[3 * i + r] = bb[r];
    }
    if (a.grad_A) {
      const int64_t rp = a.row_ptr[i], re = a.row_ptr[i + 1];
      for (int64_t k = rp; k < re; ++k) {
        const int64_t c = a.col_idx[k];
        const double v0 = a.vsol[3 * c], v1 = a.vsol[3 * c + 1], v2 = a.vsol[3 * c + 2];
        double* g = a.grad_A + 9 * k;
        for (int r = 0; r < 3; ++r) {
          g[3 * r] = -bb[r] * v0;
          g[3 * r + 1] = -bb[r] * v1;
          g[3 * r + 2] = -bb[r] * v2;
        }
      }
    }
  });
}

// Register-resident adjoint (one pass: every workgroup owns at most NW
// chunks).  A lane keeps its node's first KC block levels of A and its own t
// and u in registers for the whole solve; only s = W t goes through memory,
// written as whole lines through LDS and gathered coherently by the
// neighbours' products.  The contact term of G^T is formed once, before the
// iteration: a contact node keeps P = R^T D_P^T R (D_P of the taped branch,
// for the elliptic cone with its closest-point multiplier solved once) and
// two factors in LDS, so a sweep applies t = u - P (a u - c u_p) with no
// further reads of the contact record or the tape: a = w_i / gamma, c = 0
// for an S-contact; for a D-contact (J_m = [R, -R]) u_p is the partner
// node's u of the same sweep, a = w_x / gamma and c = w_p / gamma for node x
// and its partner p, and the two nodes exchange u through memory in a second
// grid barrier per sweep.  Same sweeps as k_adjoint (the contact term in
// another rounding order).
template <int NW, int KC>
__global__ void __launch_bounds__(64 * NW) k_adjoint_regs(AdjArgs a) {
  __shared__ double s_red[NW];
  __shared__ double s_poll[3 * NW];  // see grid_sum
  __shared__ double s_out[NW][192];
  __shared__ double s_M[NW][9][64];   // P = R^T D_P^T R of the lane's contact (0 off contacts)
  __shared__ double s_ac[NW][2][64];  // factors a, c of t = u - P (a u - c u_p)
  __shared__ int s_pn[NW][64];        // the partner node of a D-contact (else the node itself)
  __shared__ double s_gw[NW][6][64];  // g~ (3) and W (3) of the lane's node
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
  if (flags != 0) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < 3 * (int64_t)a.n_nodes; k += (int64_t)G * blockDim.x)
      a.grad_b[k] = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < a.n_contacts; k += (int64_t)G * blockDim.x) {
      a.grad_phi[k] = a.grad_mu[k] = 0.0;
      if (a.grad_mu2) a.grad_mu2[k] = 0.0;
    }
    if (a.grad_A)
      for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < 9 * (int64_t)a.nnzb;
           k += (int64_t)G * blockDim.x)
        a.grad_A[k] = 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.stats->iters = 0;
      a.stats->status = flags;
      a.stats->theta = INFINITY;
      a.stats->n_open = a.stats->n_stick = a.stats->n_slip = a.stats->reserved = 0;
    }
    return;
  }
  const int nk = act ? a.row_ptr[i + 1] - a.row_ptr[i] : 0;
  const int64_t base = cnt > 0 ? a.row_ptr[n0] : 0;
  int col[KC];
  double av[KC][9];
  int64_t off = 0;
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const uint64_t mk = ballot(k < nk);
    const int ck = __popcll(mk);
    // a level the row lacks: a zero block on column 0 (no branch in spmv)
    col[k] = 0;
#pragma unroll
    for (int e = 0; e < 9; ++e) av[k][e] = 0.0;
    if (k < nk) {
      const int pos = lanes_below(mk, lane);
      const int64_t q = base + off;
      col[k] = a.scol[q + pos];
      load_sblock(a.sval, q, ck, pos, av[k]);
    }
    off += ck;
  }
  const int64_t off_tail = off;
  const int m = act ? a.cmap[i] : -1;
  {
    double w3[3] = {0.0, 0.0, 0.0};
    if (act)
      for (int r = 0; r < 3; ++r) w3[r] = a.w[3 * i + r];
#pragma unroll
    for (int r = 0; r < 3; ++r) s_gw[slot][3 + r][lane] = w3[r];
    // P = R^T D_P^T R and the factors (zero off contacts: t = u exactly)
    double M[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double fa = 0.0, fc = 0.0;
    int pn = act ? (int)i : 0;
    if (m >= 0) {
      const double* R = a.cpack + kPack * (int64_t)m;
      if (adj_isd(a, m)) {
        const int64_t pi = a.cpair[2 * (int64_t)m], pj = a.cpair[2 * (int64_t)m + 1];
        const bool first = pi == i;
        pn = (int)(first ? pj : pi);
        fa = w3[0] / R[11];
        fc = a.w[3 * (int64_t)pn] / R[11];
      } else {
        fa = w3[0] / R[11];
      }
      double Dt[3][3];  // Dt[.][k] = D_P^T e_k
      for (int k = 0; k < 3; ++k) {
        double x[3] = {0.0, 0.0, 0.0}, y[3], dmu, dmu2;
        x[k] = 1.0;
        dp_transpose(a.lamstar + 3 * (int64_t)m, a.branch[m], R, a.proj, x, y, &dmu, &dmu2);
        for (int r = 0; r < 3; ++r) Dt[r][k] = y[r];
      }
      for (int r = 0; r < 3; ++r)
        for (int c2 = 0; c2 < 3; ++c2) {
          double acc = 0.0;
          for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) acc += R[3 * p + r] * Dt[p][q] * R[3 * q + c2];
          M[3 * r + c2] = acc;
        }
    }
    // without D-contacts the factor goes into M: t = u - M u, M = (w / gamma) P
    const bool sonly = a.cpair == nullptr;
#pragma unroll
    for (int e = 0; e < 9; ++e) s_M[slot][e][lane] = sonly ? fa * M[e] : M[e];
    s_ac[slot][0][lane] = fa;
    s_ac[slot][1][lane] = fc;
    s_pn[slot][lane] = pn;
  }
  const bool has_d = a.cpair != nullptr;  // the same in every workgroup
  auto W = [&](int r) { return s_gw[slot][3 + r][lane]; };
  // t = G^T u for this lane's node: u - P (a u - c u_p); without D-contacts
  // u - M u (the factor a is in M)
  auto gtm = [&](const double u[3], const double up[3], double out[3]) {
    double Mr[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) Mr[e] = s_M[slot][e][lane];
    double z[3] = {u[0], u[1], u[2]};
    if (has_d) {
      const double fa_ = s_ac[slot][0][lane], fc_ = s_ac[slot][1][lane];
#pragma unroll
      for (int r = 0; r < 3; ++r) z[r] = fa_ * u[r] - fc_ * up[r];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) out[r] = u[r] - (Mr[3 * r] * z[0] + Mr[3 * r + 1] * z[1] + Mr[3 * r + 2] * z[2]);
  };
  // y = A x for this lane's row (every thread calls)
  auto spmv = [&](const double* x, double out[3]) {
    double xs[KC][3];
#pragma unroll
    for (int k = 0; k < KC; ++k) ldv3<true>(x, col[k], xs[k]);
    out[0] = out[1] = out[2] = 0.0;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      out[0] += dot3(av[k][0], av[k][1], av[k][2], xs[k][0], xs[k][1], xs[k][2]);
      out[1] += dot3(av[k][3], av[k][4], av[k][5], xs[k][0], xs[k][1], xs[k][2]);
      out[2] += dot3(av[k][6], av[k][7], av[k][8], xs[k][0], xs[k][1], xs[k][2]);
    }
    spmv_rows3_from<double, true, 2>(a.scol, a.sval, x, base, nk, lane, KC, off_tail, out);
  };
  // store this wave's node values as whole lines (every thread calls)
  auto publish = [&](double* dst, const double x[3]) {
    if (act)
      for (int r = 0; r < 3; ++r) s_out[slot][3 * lane + r] = x[r];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int e = lane + 64 * j;
      if (e < 3 * cnt) stv<true>(dst + 3 * n0 + e, s_out[slot][e]);
    }
  };
  int seq = 0;
  // u of the D-contact partner (every thread calls): published in E, a grid
  // barrier, then read back; for any other node its own u
  auto partner_u = [&](const double u[3], double up[3]) {
    const int pn = s_pn[slot][lane];
    const bool dl = act && pn != (int)i;
    if (dl)
      for (int r = 0; r < 3; ++r) stv<true>(a.E + 3 * i + r, u[r]);
    grid_barrier(a.slots, G, lb, ++seq, s_poll);
    for (int r = 0; r < 3; ++r) up[r] = dl ? ldv<true>(a.E + 3 * (int64_t)pn + r) : u[r];
  };
  // phase A: e = J^T Gamma^-1 D_P^T g_lam, p = W e
  double e3[3] = {0.0, 0.0, 0.0};
  if (a.gl) {
    if (m >= 0) {
      const double* R = a.cpack + kPack * (int64_t)m;
      double x[3] = {a.gl[3 * (int64_t)m], a.gl[3 * (int64_t)m + 1], a.gl[3 * (int64_t)m + 2]}, y[3], dmu, dmu2;
      dp_transpose(a.lamstar + 3 * (int64_t)m, a.branch[m], R, a.proj, x, y, &dmu, &dmu2);
      const double gi = (adj_isd(a, m) && a.cpair[2 * (int64_t)m] != i) ? -1.0 / R[11] : 1.0 / R[11];
      for (int r = 0; r < 3; ++r) e3[r] = (R[r] * y[0] + R[3 + r] * y[1] + R[6 + r] * y[2]) * gi;
    }
    const double p3[3] = {W(0) * e3[0], W(1) * e3[1], W(2) * e3[2]};
    publish(a.S[1], p3);
    grid_barrier(a.slots, G, lb, ++seq, s_poll);
  }
  // phase B: g~ = g_v - e + A p; u0 = g~, t0 = G^T u0, s0 = W t0
  double uu[3] = {0.0, 0.0, 0.0}, tt[3] = {0.0, 0.0, 0.0};
  {
    double Ap[3] = {0.0, 0.0, 0.0};
    if (a.gl) spmv(a.S[1], Ap);
    double gt[3] = {0.0, 0.0, 0.0};
    if (act)
      for (int r = 0; r < 3; ++r) gt[r] = a.gl ? a.gv[3 * i + r] - e3[r] + Ap[r] : a.gv[3 * i + r];
    double gp[3] = {gt[0], gt[1], gt[2]};
    if (has_d) partner_u(gt, gp);
    if (act) {
      gtm(gt, gp, tt);
      for (int r = 0; r < 3; ++r) uu[r] = gt[r];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) s_gw[slot][r][lane] = gt[r];
    const double s3[3] = {W(0) * tt[0], W(1) * tt[1], W(2) * tt[2]};
    publish(a.S[0], s3);
    grid_barrier(a.slots, G, lb, ++seq, s_poll);
  }
  int cur = 0;
  if (a.max_iters > 0) {
    for (int l = 1;; ++l) {
      const int nxt = cur ^ 1;
      double As[3];
      spmv(a.S[cur], As);
      double th2 = 0.0;
      double un[3] = {0.0, 0.0, 0.0};
      if (act)
        for (int r = 0; r < 3; ++r) un[r] = s_gw[slot][r][lane] + tt[r] - As[r];
      double up[3] = {un[0], un[1], un[2]};
      if (has_d) partner_u(un, up);
      if (act) {
        double tn[3];
        gtm(un, up, tn);
        for (int r = 0; r < 3; ++r) {
          const double d = un[r] - uu[r];
          th2 += d * d;
          uu[r] = un[r];
          tt[r] = tn[r];
        }
      }
      const double s3[3] = {W(0) * tt[0], W(1) * tt[1], W(2) * tt[2]};
      publish(a.S[nxt], s3);
      th2 = block_sum(th2, s_red);
      const bool stop = grid_residual_step(a.slots, G, lb, ++seq, th2, l, a.max_iters, a.fixed, a.tol, a.stats, s_poll);
      cur = nxt;
      if (stop) break;
    }
  } else if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.stats->iters = 0;
    a.stats->status = VFPI_S_MAXITER;
    a.stats->theta = INFINITY;
    a.stats->n_open = a.stats->n_stick = a.stats->n_slip = a.stats->reserved = 0;
  }
  // final gradients (A_bar reads the solution v of the neighbours from the tape)
  double uf[3] = {uu[0], uu[1], uu[2]};
  if (has_d) partner_u(uu, uf);  // u of the partner (every thread calls)
  if (!act) return;
  double q[3] = {uu[0], uu[1], uu[2]};
  if (m >= 0) {
    const double* R = a.cpack + kPack * (int64_t)m;
    const bool isd = adj_isd(a, m);
    const bool first = !isd || a.cpair[2 * (int64_t)m] == i;
    // r = J_m W u + g_lam with J_m = [R] or [R, -R] on nodes (i, j)
    const double* ui = first ? uu : uf;
    const double wi = first ? W(0) : a.w[3 * (int64_t)s_pn[slot][lane]];
    double rr[3], y[3], dmu, dmu2;
    for (int k = 0; k < 3; ++k) {
      rr[k] = R[3 * k] * (wi * ui[0]) + R[3 * k + 1] * (wi * ui[1]) + R[3 * k + 2] * (wi * ui[2]);
      if (a.gl) rr[k] += a.gl[3 * (int64_t)m + k];
    }
    if (isd) {
      const double* uj = first ? uf : uu;
      const double wj = first ? a.w[3 * (int64_t)s_pn[slot][lane]] : W(0);
      for (int k = 0; k < 3; ++k)
        rr[k] -= R[3 * k] * (wj * uj[0]) + R[3 * k + 1] * (wj * uj[1]) + R[3 * k + 2] * (wj * uj[2]);
    }
    dp_transpose(a.lamstar + 3 * (int64_t)m, a.branch[m], R, a.proj, rr, y, &dmu, &dmu2);
    const double gi = 1.0 / R[11];
    const double sg = first ? gi : -gi;
    for (int r = 0; r < 3; ++r) q[r] -= (R[r] * y[0] + R[3 + r] * y[1] + R[6 + r] * y[2]) * sg;
    if (first) {
      a.grad_phi[m] = -y[0] * gi;
      a.grad_mu[m] = dmu;
      if (a.grad_mu2) a.grad_mu2[m] = dmu2;
    }
  }
  double bb[3];
  for (int r = 0; r < 3; ++r) {
    bb[r] = W(r) * q[r];
    a.grad_b[3 * i + r] = bb[r];
  }
  if (a.grad_A) {
    const int64_t rp = a.row_ptr[i], re = a.row_ptr[i + 1];
    for (int64_t k = rp; k < re; ++k) {
      const int64_t cc = a.col_idx[k];
      const double v0 = a.vsol[3 * cc], v1 = a.vsol[3 * cc + 1], v2 = a.vsol[3 * cc + 2];
      double* g = a.grad_A + 9 * k;
      for (int r = 0; r < 3; ++r) {
        g[3 * r] = -bb[r] * v0;
        g[3 * r + 1] = -bb[r] * v1;
        g[3 * r + 2] = -bb[r] * v2;
      }
    }
  }
}

}  // namespace vfpi

using namespace vfpi;

extern "C" int vfpi_step_backward(vfpi_ctx* ctx, const vfpi_bsr* A, const vfpi_contacts* Jc, const void* tape,
                                  const double* grad_v, const double* grad_lambda, double* grad_b, double* grad_A_val,
                                  double* grad_phi, double* grad_mu, double* grad_mu2, const vfpi_opts* opts,
                                  vfpi_stats* stats, hipStream_t stream) {
  if (!ctx || !A || !Jc || !grad_v || !grad_b || !opts || !stats) return VFPI_E_NULL;
  if (!tape) return VFPI_E_NO_TAPE;
  const int32_t N = A->n_nodes, nc = Jc->n_contacts;
  if (N < 0 || nc < 0 || A->nnzb < 0 || Jc->nnzb < 0 || nc > N) return VFPI_E_SHAPE;
  if (N > 0 && (!A->row_ptr || !A->col_idx || !A->val)) return VFPI_E_NULL;
  if (nc > 0 && (!Jc->row_ptr || !Jc->col_idx || !Jc->val || !Jc->phi || !Jc->mu || !grad_phi || !grad_mu))
    return VFPI_E_NULL;
  if (N > ctx->max_nodes || A->nnzb > ctx->max_nnzb || nc > ctx->max_contacts) return VFPI_E_CAPACITY;
  if (opts->max_iters < 0 || !(opts->tol >= 0.0)) return VFPI_E_OPTS;
  if (nc > 0 && Jc->mu2 && !grad_mu2) return VFPI_E_NULL;
  if (opts->projection != VFPI_PROJ_STRICT && opts->projection != VFPI_PROJ_PROXIMAL) return VFPI_E_OPTS;
  if (Jc->mu2 && opts->projection != VFPI_PROJ_STRICT) return VFPI_E_UNSUPPORTED;
  if (Jc->nnzb > 2 * (int64_t)nc) return VFPI_E_SHAPE;
  if (N == 0) {
    hipLaunchKernelGGL(k_stats_empty, dim3(1), dim3(1), 0, stream, stats);
    VFPI_CHECK_HIP(hipGetLastError());
    return VFPI_OK;
  }
  VFPI_CHECK_HIP(hipSetDevice(ctx->device));
  TapeView tv = tape_view(const_cast<void*>(tape), N, nc);
  double* cpack = static_cast<double*>(ctx->cpack);
  double* w = static_cast<double*>(ctx->w);

  vfpi_mark(ctx, 0, stream);
  hipLaunchKernelGGL(k_prep, dim3((N + 63) / 64), dim3(64), 0, stream, N, ctx->cmap, ctx->flags, ctx->sync,
                     ctx->slots, stats);
  if (nc > 0)
    hipLaunchKernelGGL(k_contacts<double>, dim3((nc + 63) / 64), dim3(64), 0, stream, nc, Jc->nnzb, Jc->row_ptr,
                       Jc->col_idx, static_cast<const double*>(Jc->val), static_cast<const double*>(Jc->phi),
                       static_cast<const double*>(Jc->mu), static_cast<const double*>(Jc->mu2), N, ctx->cmap,
                       cpack, ctx->cpair, ctx->flags,
                       1e-10);
  // W comes from the forward tape; the row pass rebuilds the interleaved copy of A.
  RowsArgs ra;
  ra.nnzb = A->nnzb;
  ra.w_mode = VFPI_W_USER_DIAG;
  ra.reuse = false;
  ra.alpha = 0.0;
  ra.omega = opts->omega;
  const int64_t nch = (N + 63) / 64;
  hipLaunchKernelGGL(k_rows<double>, dim3((unsigned)nch), dim3(64), 0, stream, N, A->row_ptr, A->col_idx,
                     static_cast<const double*>(A->val), ctx->scol, static_cast<double*>(ctx->sval), nullptr, nullptr,
                     ra, tv.w, ctx->cmap, cpack, w, nullptr, grad_v, tv.v,
                     ctx->flags);
  if (nc > 0 && Jc->nnzb > nc)
    hipLaunchKernelGGL(k_pairs<double>, dim3((nc + 255) / 256), dim3(256), 0, stream, nc, ctx->cpair, nullptr,
                       nullptr, ra, w, nullptr, cpack, ctx->flags);
  VFPI_CHECK_HIP(hipGetLastError());

  const int64_t n = 3 * (int64_t)N;
  AdjArgs aa;
  aa.n_nodes = N;
  aa.n_contacts = nc;
  aa.nnzb = A->nnzb;
  aa.row_ptr = A->row_ptr;
  aa.col_idx = A->col_idx;
  aa.val = static_cast<const double*>(A->val);
  aa.cpair = (Jc->nnzb > nc) ? ctx->cpair : nullptr;
  aa.scol = ctx->scol;
  aa.sval = static_cast<const double*>(ctx->sval);
  aa.w = w;
  aa.cmap = ctx->cmap;
  aa.cpack = cpack;
  aa.lamstar = tv.lamstar;
  aa.branch = tv.branch;
  aa.vsol = tv.v;
  aa.gv = grad_v;
  aa.gl = grad_lambda;
  aa.gt = ctx->adj;
  aa.U[0] = ctx->adj + n;
  aa.U[1] = ctx->adj + 2 * n;
  aa.T[0] = ctx->adj + 3 * n;
  aa.T[1] = ctx->adj + 4 * n;
  aa.S[0] = ctx->adj + 5 * n;
  aa.S[1] = ctx->adj + 6 * n;
  aa.E = ctx->adj + 7 * n;
  aa.grad_b = grad_b;
  aa.grad_A = grad_A_val;
  aa.grad_phi = grad_phi;
  aa.grad_mu = grad_mu;
  aa.grad_mu2 = Jc->mu2 ? grad_mu2 : nullptr;
  aa.max_iters = opts->max_iters;
  aa.fixed = opts->fixed_iters;
  aa.tol = opts->tol;
  aa.flags = ctx->flags;
  aa.stats = stats;
  aa.slots = ctx->slots;
  aa.proj = opts->projection;

  const int kind = opts->variant & 0xff;
  const int grid_req = (opts->variant >> 16) & 0xff;
  // register-resident adjoint: variant 0 or kind 5, one workgroup per CU at
  // most with the fewest chunk slots that fit
  if (kind == 0 || kind == 5) {
    const int64_t cap = ctx->num_cu < kMaxGridSlots ? ctx->num_cu : kMaxGridSlots;
    int want_nw = (opts->variant >> 8) & 0xff;
    for (int nw : {2, 4, 5, 8}) {
      if (want_nw && nw < want_nw) continue;
      int64_t g = (nch + nw - 1) / nw;
      if (g > 8 && g % 8 != 0) g += 8 - g % 8;
      if (g > nch) g = nch;
      if (g > cap) continue;
      void* params[] = {&aa};
      const void* kern = nw == 2   ? (const void*)k_adjoint_regs<2, 9>
                         : nw == 4 ? (const void*)k_adjoint_regs<4, 9>
                         : nw == 5 ? (const void*)k_adjoint_regs<5, 7>
                                   : (const void*)k_adjoint_regs<8, 4>;
      vfpi_mark(ctx, 1, stream);
      VFPI_CHECK_HIP(hipLaunchCooperativeKernel(kern, dim3((unsigned)g), dim3(64 * nw), params, 0, stream));
      vfpi_mark(ctx, 2, stream);
      return VFPI_OK;
    }
  }
  constexpr int NW = 4;
  auto kern = k_adjoint<NW>;
  const int threads = 64 * NW;
  const int64_t want = (nch + NW - 1) / NW;
  int64_t g = 1;
  if (kind != 3) {  // at most one workgroup per CU (see gridsync.h)
    const int64_t cap = ctx->num_cu < kMaxGridSlots ? ctx->num_cu : kMaxGridSlots;
    g = want < cap ? want : cap;
    if (grid_req > 0 && grid_req < g) g = grid_req;
    if (g > 8) g -= g % 8;
    if (g < 1) g = 1;
  }
  void* params[] = {&aa};
  vfpi_mark(ctx, 1, stream);
  VFPI_CHECK_HIP(hipLaunchCooperativeKernel((const void*)kern, dim3((unsigned)g), dim3(threads), params, 0, stream));
  vfpi_mark(ctx, 2, stream);
  return VFPI_OK;
}
