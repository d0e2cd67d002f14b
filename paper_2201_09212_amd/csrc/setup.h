// Per-step setup shared by the plain, batched and adjoint kernels:
//  * contact records: validate each J_c block row (one SO(3) block at a
//    node, eq. jcnode), build the node -> contact map, pack R, phi, mu;
//  * block rows of A: copy into the chunk-interleaved layout (see common.h),
//    accumulate a_dd and ||A_d*||^2, and form the step sizes W (Sec. IV-C.1)
//    and gamma_m = w_i of Prop. 3 (plus omega for the invertible contact of
//    eq. invt, whose Omega_c = omega I is simply added to Gamma_c).
#pragma once

#include "common.h"

namespace vfpi {

// Contact m: one block row of J_c with either one block R at node i
// (S-contact) or, when `cpair` is given, two blocks R at node i and -R at node
// j != i (D-contact, eq. jcnode); anything else is NOT_NODAL.  Both nodes enter
// the node -> contact map; cpair[2m], cpair[2m+1] = i, j (-1 for S).
template <class T>
VFPI_DEV void contact_setup(int64_t m, int32_t nnzb_c, const int32_t* __restrict__ crp,
                            const int32_t* __restrict__ ccol, const T* __restrict__ cval,
                            const T* __restrict__ phi, const T* __restrict__ mu, const T* __restrict__ mu2,
                            int64_t node_lo,
                            int64_t node_hi, int32_t* cmap, T* cpack, int32_t* cpair, int32_t* flag,
                            double orth_tol) {
  if (cpair) {  // a rejected row must not leave a stale pair behind
    cpair[2 * m] = -1;
    cpair[2 * m + 1] = -1;
  }
  const int64_t r0 = crp[m], r1 = crp[m + 1];
  const int64_t nb = r1 - r0;
  if ((nb != 1 && !(nb == 2 && cpair)) || r0 < 0 || r1 > nnzb_c) {
    set_flag(flag, VFPI_S_NOT_NODAL);
    return;
  }
  const int64_t i = ccol[r0];
  const int64_t j = nb == 2 ? ccol[r0 + 1] : -1;
  if (i < node_lo || i >= node_hi || (nb == 2 && (j < node_lo || j >= node_hi))) {
    set_flag(flag, VFPI_S_BAD_PATTERN);
    return;
  }
  if (j == i) {
    set_flag(flag, VFPI_S_NOT_NODAL);
    return;
  }
  T R[9];
  bool fin = true, neg = true;
  for (int e = 0; e < 9; ++e) {
    R[e] = cval[9 * r0 + e];
    fin &= finite(R[e]);
    if (nb == 2) {
      const T x = cval[9 * (r0 + 1) + e];
      fin &= finite(x);
      neg &= (x == -R[e]);
    }
  }
  T ph = phi[m], mm = mu[m], m2 = mu2 ? mu2[m] : mu[m];
  fin &= finite(ph) && finite(mm) && finite(m2);
  if (!fin) {
    set_flag(flag, VFPI_S_NONFINITE);
    return;
  }
  if (!neg) {
    set_flag(flag, VFPI_S_NOT_NODAL);
    return;
  }
  if (!(mm >= T(0)) || !(m2 >= T(0))) set_flag(flag, VFPI_S_BAD_MU);
  double err = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double d = (double)R[3 * a] * R[3 * b] + (double)R[3 * a + 1] * R[3 * b + 1] +
                 (double)R[3 * a + 2] * R[3 * b + 2] - (a == b ? 1.0 : 0.0);
      err = fmax(err, fabs(d));
    }
  if (!(err <= orth_tol)) set_flag(flag, VFPI_S_NOT_ORTHONORMAL);
  if (atomicCAS(cmap + i, -1, (int)m) != -1) set_flag(flag, VFPI_S_SHARED_NODE);
  if (j >= 0 && atomicCAS(cmap + j, -1, (int)m) != -1) set_flag(flag, VFPI_S_SHARED_NODE);
  if (cpair) {
    cpair[2 * m] = (int32_t)i;
    cpair[2 * m + 1] = (int32_t)j;
  }
  T* pk = cpack + kPack * m;
  for (int e = 0; e < 9; ++e) pk[e] = R[e];
  pk[9] = ph;
  pk[10] = mm;
  pk[12] = m2;
}

// One 3x3 block (9 consecutive values) of the caller's A into registers with
// 16-byte loads (the blocks are only 8- or 4-byte aligned; unaligned vector
// loads are legal on global memory), 5 load instructions instead of 9 for
// FP64 and 3 for FP32: the row pass reads each lane's own row, so every load
// touches another cache line per lane, and fewer, wider loads cost fewer
// address cycles.
VFPI_DEV void load_block9(const double* __restrict__ src, double x[9]) {
  typedef double d2 __attribute__((ext_vector_type(2), aligned(8)));
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const d2 t = *reinterpret_cast<const d2*>(src + 2 * q);
    x[2 * q] = t.x;
    x[2 * q + 1] = t.y;
  }
  x[8] = src[8];
}
VFPI_DEV void load_block9(const float* __restrict__ src, float x[9]) {
  typedef float f4 __attribute__((ext_vector_type(4), aligned(4)));
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const f4 t = *reinterpret_cast<const f4*>(src + 4 * q);
    x[4 * q] = t.x;
    x[4 * q + 1] = t.y;
    x[4 * q + 2] = t.z;
    x[4 * q + 3] = t.w;
  }
  x[8] = src[8];
}

struct RowsArgs {
  int32_t nnzb;
  int w_mode;
  bool reuse;
  double alpha;
  double omega;  // invertible contact: the contact step divides by gamma + omega
  unsigned long long* amax = nullptr;  // nullable: max_d sum_j |a_dj| (bits of a non-negative double)
};

// One wave converts one chunk of <= 64 consecutive nodes [n0, n0 + cnt).
// Every lane of the wave must call.  Nodes of the chunk must lie in
// [node_lo, node_hi), and so must every column index (else BAD_PATTERN).
// bvec / vvec (nullable) are checked for NaN/Inf along with the row.
template <class T>
VFPI_DEV void rows_chunk(int64_t n0, int cnt, int lane, const int32_t* __restrict__ row_ptr,
                         const int32_t* __restrict__ col_idx, const T* __restrict__ val,
                         int32_t* __restrict__ scol, T* __restrict__ sval, int64_t node_lo,
                         int64_t node_hi, double* __restrict__ diag, double* __restrict__ rn2,
                         const RowsArgs ra, const T* __restrict__ w_user, const int32_t* __restrict__ cmap,
                         T* __restrict__ cpack, T* __restrict__ w, double* __restrict__ tape_w,
                         const T* __restrict__ bvec, const T* __restrict__ vvec, int32_t* flag) {
  const int64_t i = n0 + lane;
  const bool act = lane < cnt;
  int64_t rp = 0;
  int nk = 0;
  bool bad = false;
  if (act) {
    int64_t r1;
    rp = row_ptr[i];
    r1 = row_ptr[i + 1];
    nk = (int)(r1 - rp);
    bad = rp < 0 || r1 < rp || r1 > ra.nnzb || (i == 0 && rp != 0);
  }
  if (ballot(bad) != 0) {  // row offsets unusable: skip the whole chunk
    if (lane == 0) set_flag(flag, VFPI_S_BAD_PATTERN);
    return;
  }
  const int64_t base = row_ptr[n0];
  double d[3] = {0.0, 0.0, 0.0}, s[3] = {0.0, 0.0, 0.0}, ab[3] = {0.0, 0.0, 0.0};
  bool has_diag = false, fin = true, badcol = false;
  int64_t off = 0;
  // levels in groups of four: the group's loads are all issued before its
  // blocks are converted (in level order, so the row sums keep their order)
  constexpr int UG = 4;
  for (int k0 = 0;; k0 += UG) {
    uint64_t mask[UG];
#pragma unroll
    for (int u = 0; u < UG; ++u) mask[u] = ballot(k0 + u < nk);
    if (mask[0] == 0) break;
    int64_t cg[UG];
    T x[UG][9];
#pragma unroll
    for (int u = 0; u < UG; ++u) {
      if (k0 + u < nk) {
        cg[u] = col_idx[rp + k0 + u];
        load_block9(val + 9 * (rp + k0 + u), x[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < UG; ++u) {
      const int c_ = __popcll(mask[u]);
      if (k0 + u < nk) {
        const int pos = lanes_below(mask[u], lane);
        const int64_t q = base + off;
        int64_t c = cg[u];
        if (c < node_lo || c >= node_hi) {
          badcol = true;
          c = i;
        }
        scol[q + pos] = (int32_t)c;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
          sval[sval_at<T>(q, c_, pos, e)] = x[u][e];
          fin &= finite(x[u][e]);
        }
        // FP64: the column also goes into the block's record, beside entry 8
        if constexpr (sizeof(T) == 8)
          sval[sval_at<T>(q, c_, pos, 8) + 1] = __builtin_bit_cast(double, (uint64_t)(uint32_t)c);
#pragma unroll
        for (int r = 0; r < 3; ++r)
          for (int cc = 0; cc < 3; ++cc) {
            s[r] += (double)x[u][3 * r + cc] * (double)x[u][3 * r + cc];
            ab[r] += fabs((double)x[u][3 * r + cc]);
          }
        if (c == i) {
          has_diag = true;
          d[0] = x[u][0];
          d[1] = x[u][4];
          d[2] = x[u][8];
        }
      }
      off += c_;
    }
  }
  if (!act) return;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    if (bvec) fin &= finite(bvec[3 * i + r]);
    if (vvec) fin &= finite(vvec[3 * i + r]);
  }
  if (badcol) set_flag(flag, VFPI_S_BAD_PATTERN);
  if (ra.amax) {  // Gershgorin bound for the first Barzilai-Borwein step (order-free max)
    const double mx = fmax(ab[0], fmax(ab[1], ab[2]));
    if (mx >= 0.0) atomicMax(ra.amax, (unsigned long long)__builtin_bit_cast(uint64_t, mx));
  }
  if (!fin) set_flag(flag, VFPI_S_NONFINITE);
  if (ra.reuse) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      d[r] = diag[3 * i + r];
      s[r] = rn2[3 * i + r];
    }
  } else if (diag) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      diag[3 * i + r] = d[r];
      rn2[3 * i + r] = s[r];
    }
  }
  if (!has_diag || !(d[0] > 0.0) || !(d[1] > 0.0) || !(d[2] > 0.0)) set_flag(flag, VFPI_S_NONPOS_DIAG);
  const int m = cmap[i];
  double wr[3];
  if (ra.w_mode == VFPI_W_FROBENIUS) {
    if (m >= 0) {
      double wb = (d[0] + d[1] + d[2]) / (s[0] + s[1] + s[2]);
      wr[0] = wr[1] = wr[2] = wb;
    } else {
      for (int r = 0; r < 3; ++r) wr[r] = d[r] / s[r];
    }
  } else if (ra.w_mode == VFPI_W_USER_DIAG) {
    for (int r = 0; r < 3; ++r) wr[r] = (double)w_user[3 * i + r];
    if (!(wr[0] > 0.0 && wr[1] > 0.0 && wr[2] > 0.0) || !finite(wr[0] + wr[1] + wr[2]) ||
        (m >= 0 && (wr[0] != wr[1] || wr[1] != wr[2])))
      set_flag(flag, VFPI_S_BAD_W);
  } else {
    wr[0] = wr[1] = wr[2] = ra.alpha;
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    w[3 * i + r] = (T)wr[r];
    if (tape_w) tape_w[3 * i + r] = wr[r];
  }
  if (m >= 0) cpack[kPack * (int64_t)m + 11] = (T)(wr[0] + ra.omega);
}

// D-contact m after the row pass (which grouped each node's 3 DOFs alone):
// the pair's 6 DOFs share one w-bar (Frobenius: sum a_dd / sum ||A_d*||^2
// over the six, Sec. IV-C.1), and gamma_m = w_i + w_j (Prop. 3), plus omega.
// A user W must already be equal on the six DOFs (else BAD_W).
template <class T>
VFPI_DEV void pair_setup(int64_t m, const int32_t* __restrict__ cpair, const double* __restrict__ diag,
                         const double* __restrict__ rn2, const RowsArgs ra, T* __restrict__ w,
                         double* __restrict__ tape_w, T* __restrict__ cpack, int32_t* flag) {
  const int64_t i = cpair[2 * m], j = cpair[2 * m + 1];
  if (i < 0 || j < 0) return;
  double wi, wj;
  if (ra.w_mode == VFPI_W_FROBENIUS) {
    double dn = 0.0, sn = 0.0;
    for (int r = 0; r < 3; ++r) {
      dn += diag[3 * i + r];
      sn += rn2[3 * i + r];
    }
    for (int r = 0; r < 3; ++r) {
      dn += diag[3 * j + r];
      sn += rn2[3 * j + r];
    }
    wi = wj = dn / sn;
    for (int r = 0; r < 3; ++r) {
      w[3 * i + r] = (T)wi;
      w[3 * j + r] = (T)wj;
      if (tape_w) {
        tape_w[3 * i + r] = wi;
        tape_w[3 * j + r] = wj;
      }
    }
  } else {
    wi = (double)w[3 * i];
    wj = (double)w[3 * j];
    if (ra.w_mode == VFPI_W_USER_DIAG && wi != wj) set_flag(flag, VFPI_S_BAD_W);
  }
  cpack[kPack * m + 11] = (T)(wi + wj + ra.omega);
}

}  // namespace vfpi
