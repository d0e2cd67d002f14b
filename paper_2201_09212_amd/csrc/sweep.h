// One V-FPI sweep over one chunk of <= 64 nodes (Alg. 1 inner loop body):
//   v*      = v^l - W (A v^l - b)                       (eq. pgd1)
//   lambda* = -(R_m v*_i + phi_m e1) / gamma_m           (Alg. 2, eq. subp)
//   lambda  = ProjectFC(lambda*)                         (eq. operator)
//   v^{l+1} = v* + W R_m^T lambda                        (eq. vup, nodal J_c)
// and the squared residual contribution |v^{l+1} - v^l|^2 (Alg. 1).
// For S-contacts everything after the sparse product is local to the node,
// so the gather (eta = J_c v*), the one-shot contact solve and the scatter
// (W J_c^T lambda) are fused into the product's epilogue.
#pragma once

#include "common.h"

namespace vfpi {

template <class T>
struct SweepData {
  const int32_t* row_ptr;
  const int32_t* scol;
  const T* sval;
  const T* b;
  const T* w;
  const int32_t* cmap;
  const T* cpack;
  T* lambda;
  double* tape_lamstar;   // nullable (FP64 path only)
  int32_t* tape_branch;   // nullable
  int proj;
  // Chebyshev acceleration (Alg. 3): v^{l+1} = nu (u (v** - v^l) + v^l - v^{l-1}) + v^{l-1}
  T* vprev;               // v^{l-1} per DOF, node-local (nullptr: off)
  double nu, u;
  int first;              // sweep 1: v^0 = v^1
  // D-contacts: A's block rows in the caller's layout and the contact's nodes
  const int32_t* col_idx;
  const T* val;
  const int32_t* cpair;   // [2 n_c]: i, j (j = -1: S-contact); nullptr: S only
};

// Chebyshev update of one DOF (identity when d.vprev is null); keeps v^l as the
// next sweep's v^{l-1}.
template <class T>
VFPI_DEV T cheby_update(const SweepData<T>& a, int64_t k, T vss, T v) {
  if (!a.vprev) return vss;
  const T vp = a.first ? v : a.vprev[k];
  a.vprev[k] = v;
  return (T)a.nu * ((T)a.u * (vss - v) + v - vp) + vp;
}

// One contact's packed record: R (row 0 = normal), phi, mu, gamma, mu2
// (friction along tangent 2; equal to mu unless friction is anisotropic).
template <class T>
struct ContactRec {
  T R[9];
  T phi, mu, g, mu2;
};

template <class T>
VFPI_DEV ContactRec<T> load_contact(const T* __restrict__ pk) {
  ContactRec<T> c;
#pragma unroll
  for (int e = 0; e < 9; ++e) c.R[e] = pk[e];
  c.phi = pk[9];
  c.mu = pk[10];
  c.g = pk[11];
  c.mu2 = pk[12];
  return c;
}

// Contact step for one S-contact given v* of its node; returns the branch and
// writes lambda (and lambda* for the tape).
template <class T>
VFPI_DEV int contact_solve(const ContactRec<T>& cr, T vs0, T vs1, T vs2, int proj, T lam[3], T ls[3]) {
  const T* R = cr.R;
  const T phi = cr.phi, mu = cr.mu, g = cr.g, mu2 = cr.mu2;
  const T e0 = R[0] * vs0 + R[1] * vs1 + R[2] * vs2;
  const T e1 = R[3] * vs0 + R[4] * vs1 + R[5] * vs2;
  const T e2 = R[6] * vs0 + R[7] * vs1 + R[8] * vs2;
  ls[0] = -(e0 + phi) / g;
  ls[1] = -e1 / g;
  ls[2] = -e2 / g;
  lam[0] = ls[0];
  lam[1] = ls[1];
  lam[2] = ls[2];
  return project(proj, lam[0], lam[1], lam[2], mu, mu2);
}

template <class T>
VFPI_DEV int contact_step(const T* __restrict__ pk, T vs0, T vs1, T vs2, int proj, T lam[3], T ls[3]) {
  return contact_solve<T>(load_contact<T>(pk), vs0, vs1, vs2, proj, lam, ls);
}

// v*_x = v_x - W_x (A_x v - b_x) from node x's block row in A's own layout
// (blocks in row order).  A D-contact needs v* of both of its nodes; each of
// the two nodes' threads forms both with this one routine, so the two sides
// compute the same lambda.  w == nullptr: W = alpha I.
template <class T, bool COH>
VFPI_DEV void vstar_bsr(const SweepData<T>& a, const T* __restrict__ vcur, const T* w, T alpha, int64_t x,
                        T vs[3]) {
  T acc[3] = {T(0), T(0), T(0)};
  const int64_t r1 = a.row_ptr[x + 1];
  for (int64_t k = a.row_ptr[x]; k < r1; ++k) {
    const int64_t c = a.col_idx[k];
    const T* B = a.val + 9 * k;
    const T y0 = ldv<COH>(vcur + 3 * c), y1 = ldv<COH>(vcur + 3 * c + 1), y2 = ldv<COH>(vcur + 3 * c + 2);
#pragma unroll
    for (int r = 0; r < 3; ++r) acc[r] += dot3(B[3 * r], B[3 * r + 1], B[3 * r + 2], y0, y1, y2);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const T wr = w ? w[3 * x + r] : alpha;
    vs[r] = ldv<COH>(vcur + 3 * x + r) - wr * (acc[r] - a.b[3 * x + r]);
  }
}

// D-contact m (nodes i, j; J_m = [R, -R], eq. jcnode) seen from its node x:
// lambda* = -(R (v*_i - v*_j) + phi e1) / gamma, projected (Alg. 2), and x's
// own v* and update v*_x +- W_x R^T lambda.  g > 0 overrides gamma_m, w ==
// nullptr means W = alpha I.  Returns true when x is node i (which reports
// lambda, the tape entries and the branch count).
template <class T, bool COH>
VFPI_DEV bool dcontact_node(const SweepData<T>& a, const T* __restrict__ vcur, const T* w, T alpha, T g, int64_t x,
                            int m, T vs_own[3], T vn_own[3], T lam[3], T ls[3], int& br) {
  const int64_t i = a.cpair[2 * (int64_t)m], j = a.cpair[2 * (int64_t)m + 1];
  T vi[3], vj[3];
  vstar_bsr<T, COH>(a, vcur, w, alpha, i, vi);
  vstar_bsr<T, COH>(a, vcur, w, alpha, j, vj);
  ContactRec<T> cr = load_contact<T>(a.cpack + kPack * (int64_t)m);
  if (g > T(0)) cr.g = g;
  br = contact_solve<T>(cr, vi[0] - vj[0], vi[1] - vj[1], vi[2] - vj[2], a.proj, lam, ls);
  const bool first = (x == i);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const T F = cr.R[r] * lam[0] + cr.R[3 + r] * lam[1] + cr.R[6 + r] * lam[2];
    const T wr = w ? w[3 * x + r] : alpha;
    vs_own[r] = first ? vi[r] : vj[r];
    vn_own[r] = first ? vs_own[r] + wr * F : vs_own[r] - wr * F;
  }
  return first;
}

template <class T>
VFPI_DEV bool is_dcontact(const SweepData<T>& a, int m) {
  return a.cpair && a.cpair[2 * (int64_t)m + 1] >= 0;
}

// Thread = node (all three rows).  Every lane of the wave calls; cnt may be 0.
template <class T, bool COH = false, int U = 4>
VFPI_DEV void sweep_chunk_node(const SweepData<T>& a, const T* __restrict__ vcur, T* __restrict__ vnext,
                               int64_t n0, int cnt, int lane, double& th2, int cb[3]) {
  const int64_t i = n0 + lane;
  const bool act = lane < cnt;
  const int nk = act ? a.row_ptr[i + 1] - a.row_ptr[i] : 0;
  const int64_t base = cnt > 0 ? a.row_ptr[n0] : 0;  // idle slots may lie past the end
  T Av[3];
  spmv_rows3<T, COH, U>(a.scol, a.sval, vcur, base, nk, lane, Av);
  if (!act) return;
  T v[3], vs[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    v[r] = ldv<COH>(vcur + 3 * i + r);
    vs[r] = v[r] - a.w[3 * i + r] * (Av[r] - a.b[3 * i + r]);
  }
  T vn[3] = {vs[0], vs[1], vs[2]};
  const int m = a.cmap[i];
  if (m >= 0 && is_dcontact(a, m)) {
    T lam[3], ls[3];
    int br;
    if (dcontact_node<T, COH>(a, vcur, a.w, T(0), T(0), i, m, vs, vn, lam, ls, br)) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        a.lambda[3 * (int64_t)m + r] = lam[r];
        if (a.tape_lamstar) a.tape_lamstar[3 * (int64_t)m + r] = (double)ls[r];
      }
      if (a.tape_branch) a.tape_branch[m] = br;
      cb[br] += 1;
    }
  } else if (m >= 0) {
    const T* pk = a.cpack + kPack * (int64_t)m;
    T lam[3], ls[3];
    int br = contact_step<T>(pk, vs[0], vs[1], vs[2], a.proj, lam, ls);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      T F = pk[r] * lam[0] + pk[3 + r] * lam[1] + pk[6 + r] * lam[2];
      vn[r] = vs[r] + a.w[3 * i + r] * F;
      a.lambda[3 * (int64_t)m + r] = lam[r];
      if (a.tape_lamstar) a.tape_lamstar[3 * (int64_t)m + r] = (double)ls[r];
    }
    if (a.tape_branch) a.tape_branch[m] = br;
    cb[br] += 1;
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    vn[r] = cheby_update<T>(a, 3 * i + r, vn[r], v[r]);
    stv<COH>(vnext + 3 * i + r, vn[r]);
    double d = (double)(vn[r] - v[r]);
    th2 += d * d;
  }
}

// Thread = one row r of a node; the three rows of a chunk are three waves of
// the same workgroup that swap v* through LDS (double-buffered by pass parity
// so one barrier per pass suffices).  Every thread of the workgroup calls.
template <class T, bool COH = false, int U = 8>
VFPI_DEV void sweep_chunk_row(const SweepData<T>& a, const T* __restrict__ vcur, T* __restrict__ vnext,
                              int64_t n0, int cnt, int lane, int r, T (*s_vs)[64], double& th2, int cb[3]) {
  const int64_t i = n0 + lane;
  const bool act = lane < cnt;
  const int nk = act ? a.row_ptr[i + 1] - a.row_ptr[i] : 0;
  const int64_t base = cnt > 0 ? a.row_ptr[n0] : 0;  // idle slots may lie past the end
  const T Av = spmv_row1<T, COH, U>(a.scol, a.sval, vcur, base, nk, lane, r);
  T v = T(0), vs = T(0);
  if (act) {
    v = ldv<COH>(vcur + 3 * i + r);
    vs = v - a.w[3 * i + r] * (Av - a.b[3 * i + r]);
    s_vs[r][lane] = vs;
  }
  __syncthreads();
  if (!act) return;
  T vn = vs;
  const int m = a.cmap[i];
  if (m >= 0 && is_dcontact(a, m)) {
    T lam[3], ls[3], vs3[3], vn3[3];
    int br;
    const bool first = dcontact_node<T, COH>(a, vcur, a.w, T(0), T(0), i, m, vs3, vn3, lam, ls, br);
    vn = vn3[r];
    if (first) {
      a.lambda[3 * (int64_t)m + r] = lam[r];
      if (a.tape_lamstar) a.tape_lamstar[3 * (int64_t)m + r] = (double)ls[r];
      if (r == 0) {
        if (a.tape_branch) a.tape_branch[m] = br;
        cb[br] += 1;
      }
    }
  } else if (m >= 0) {
    const T* pk = a.cpack + kPack * (int64_t)m;
    T lam[3], ls[3];
    int br = contact_step<T>(pk, s_vs[0][lane], s_vs[1][lane], s_vs[2][lane], a.proj, lam, ls);
    T F = pk[r] * lam[0] + pk[3 + r] * lam[1] + pk[6 + r] * lam[2];
    vn = vs + a.w[3 * i + r] * F;
    a.lambda[3 * (int64_t)m + r] = lam[r];
    if (a.tape_lamstar) a.tape_lamstar[3 * (int64_t)m + r] = (double)ls[r];
    if (r == 0) {
      if (a.tape_branch) a.tape_branch[m] = br;
      cb[br] += 1;
    }
  }
  vn = cheby_update<T>(a, 3 * i + r, vn, v);
  stv<COH>(vnext + 3 * i + r, vn);
  double d = (double)(vn - v);
  th2 += d * d;
}

}  // namespace vfpi
