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

// One contact's packed record: R (row 0 = normal), phi, mu, gamma.
template <class T>
struct ContactRec {
  T R[9];
  T phi, mu, g;
};

template <class T>
VFPI_DEV ContactRec<T> load_contact(const T* __restrict__ pk) {
  ContactRec<T> c;
#pragma unroll
  for (int e = 0; e < 9; ++e) c.R[e] = pk[e];
  c.phi = pk[9];
  c.mu = pk[10];
  c.g = pk[11];
  return c;
}

// Contact step for one S-contact given v* of its node; returns the branch and
// writes lambda (and lambda* for the tape).
template <class T>
VFPI_DEV int contact_solve(const ContactRec<T>& cr, T vs0, T vs1, T vs2, int proj, T lam[3], T ls[3]) {
  const T* R = cr.R;
  const T phi = cr.phi, mu = cr.mu, g = cr.g;
  const T e0 = R[0] * vs0 + R[1] * vs1 + R[2] * vs2;
  const T e1 = R[3] * vs0 + R[4] * vs1 + R[5] * vs2;
  const T e2 = R[6] * vs0 + R[7] * vs1 + R[8] * vs2;
  ls[0] = -(e0 + phi) / g;
  ls[1] = -e1 / g;
  ls[2] = -e2 / g;
  lam[0] = ls[0];
  lam[1] = ls[1];
  lam[2] = ls[2];
  return project(proj, lam[0], lam[1], lam[2], mu);
}

template <class T>
VFPI_DEV int contact_step(const T* __restrict__ pk, T vs0, T vs1, T vs2, int proj, T lam[3], T ls[3]) {
  return contact_solve<T>(load_contact<T>(pk), vs0, vs1, vs2, proj, lam, ls);
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
  if (m >= 0) {
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
  if (m >= 0) {
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
