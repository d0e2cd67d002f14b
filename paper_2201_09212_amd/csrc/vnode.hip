// (compiled as part of vfpi_lib.hip)
// Virtual nodes (Sec. III-A): the system of eq. vnode,
//
//   [ A_o + k_v J_v^T J_v   -k_v J_v^T ] [v_o]   [b_o]
//   [ -k_v J_v               k_v I     ] [v_v] = [ 0 ] + J_c^T lambda,
//
// built in two calls: the block pattern on the host (it depends on the index
// arrays only), then the values on the device.  Virtual node q is node n_o + q
// of the result; J_v's block row q holds the 3x3 blocks J_qa mapping the
// velocity of original node a to the velocity of the point the virtual node
// sits on (eq. vforce).
#include <algorithm>
#include <vector>

#include "internal.h"

namespace vfpi {

// One thread per block row of the result.  Row a < n_o: blocks of A_o row a
// plus k_v sum_{q in Q(a)} J_qa^T J_qc for original columns c, and -k_v J_qa^T
// for the virtual columns n_o + q; Q(a) (the virtual nodes whose row touches a)
// is read off the virtual columns of the row itself.  Row n_o + q: -k_v J_qa,
// and k_v I on the diagonal.  Also b = [b_o; 0] and v = [v_o; J_v v_o].
__global__ void k_vnode_values(int32_t n_o, const int32_t* __restrict__ a_ptr, const int32_t* __restrict__ a_col,
                               const double* __restrict__ a_val, const double* __restrict__ b_o,
                               const double* __restrict__ v_o, int32_t n_v, const int32_t* __restrict__ jv_ptr,
                               const int32_t* __restrict__ jv_col, const double* __restrict__ jv_val, double k_v,
                               const int32_t* __restrict__ g_ptr, const int32_t* __restrict__ g_col,
                               double* __restrict__ g_val, double* __restrict__ b, double* __restrict__ v) {
  const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (row >= (int64_t)n_o + n_v) return;
  const int64_t g0 = g_ptr[row], g1 = g_ptr[row + 1];
  if (row >= n_o) {  // virtual node q
    const int64_t q = row - n_o;
    double vv[3] = {0.0, 0.0, 0.0};
    for (int64_t k = g0; k < g1; ++k) {
      const int64_t c = g_col[k];
      double* out = g_val + 9 * k;
      if (c == row) {
        for (int e = 0; e < 9; ++e) out[e] = (e % 4 == 0) ? k_v : 0.0;
        continue;
      }
      for (int e = 0; e < 9; ++e) out[e] = 0.0;
      for (int64_t t = jv_ptr[q]; t < jv_ptr[q + 1]; ++t)
        if (jv_col[t] == c)
          for (int e = 0; e < 9; ++e) out[e] = -k_v * jv_val[9 * t + e];
    }
    for (int64_t t = jv_ptr[q]; t < jv_ptr[q + 1]; ++t) {
      const double* J = jv_val + 9 * t;
      const int64_t a = jv_col[t];
      for (int r = 0; r < 3; ++r) vv[r] += J[3 * r] * v_o[3 * a] + J[3 * r + 1] * v_o[3 * a + 1] + J[3 * r + 2] * v_o[3 * a + 2];
    }
    for (int r = 0; r < 3; ++r) {
      b[3 * row + r] = 0.0;
      v[3 * row + r] = vv[r];
    }
    return;
  }
  // original node a = row: the virtual columns are the last ones of the row
  const int64_t a = row;
  int64_t gv = g1;
  while (gv > g0 && g_col[gv - 1] >= n_o) --gv;
  int64_t ak = a_ptr[a];
  const int64_t a1 = a_ptr[a + 1];
  for (int64_t k = g0; k < g1; ++k) {
    const int64_t c = g_col[k];
    double* out = g_val + 9 * k;
    double acc[9];
    for (int e = 0; e < 9; ++e) acc[e] = 0.0;
    if (c < n_o) {
      while (ak < a1 && a_col[ak] < c) ++ak;  // both rows sorted by column
      if (ak < a1 && a_col[ak] == c)
        for (int e = 0; e < 9; ++e) acc[e] = a_val[9 * ak + e];
      for (int64_t s = gv; s < g1; ++s) {  // k_v sum_q J_qa^T J_qc
        const int64_t q = g_col[s] - n_o;
        const double* Ja = nullptr;
        const double* Jc = nullptr;
        for (int64_t t = jv_ptr[q]; t < jv_ptr[q + 1]; ++t) {
          if (jv_col[t] == a) Ja = jv_val + 9 * t;
          if (jv_col[t] == c) Jc = jv_val + 9 * t;
        }
        if (!Ja || !Jc) continue;
        for (int r = 0; r < 3; ++r)
          for (int cc = 0; cc < 3; ++cc)
            acc[3 * r + cc] += k_v * (Ja[r] * Jc[cc] + Ja[3 + r] * Jc[3 + cc] + Ja[6 + r] * Jc[6 + cc]);
      }
    } else {  // -k_v J_qa^T
      const int64_t q = c - n_o;
      for (int64_t t = jv_ptr[q]; t < jv_ptr[q + 1]; ++t)
        if (jv_col[t] == a)
          for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc) acc[3 * r + cc] = -k_v * jv_val[9 * t + 3 * cc + r];
    }
    for (int e = 0; e < 9; ++e) out[e] = acc[e];
  }
  for (int r = 0; r < 3; ++r) {
    b[3 * a + r] = b_o[3 * a + r];
    v[3 * a + r] = v_o[3 * a + r];
  }
}

}  // namespace vfpi

using namespace vfpi;

extern "C" int vfpi_vnode_pattern(int32_t n_o, const int32_t* row_ptr, const int32_t* col_idx, int32_t n_v,
                                  const int32_t* jv_ptr, const int32_t* jv_col, int32_t* aug_row_ptr,
                                  int32_t* aug_col_idx, int64_t cap, int64_t* aug_nnzb) {
  if (!row_ptr || !jv_ptr || !aug_row_ptr || !aug_nnzb) return VFPI_E_NULL;
  if (n_o < 0 || n_v < 0 || (int64_t)n_o + n_v > INT32_MAX) return VFPI_E_SHAPE;
  if ((row_ptr[n_o] > 0 && !col_idx) || (jv_ptr[n_v] > 0 && !jv_col)) return VFPI_E_NULL;
  if (row_ptr[0] != 0 || jv_ptr[0] != 0) return VFPI_E_SHAPE;
  // Q(a): virtual nodes whose J_v row touches original node a
  std::vector<std::vector<int32_t>> Q(n_o);
  std::vector<std::vector<int32_t>> supp(n_v);
  for (int32_t q = 0; q < n_v; ++q) {
    if (jv_ptr[q + 1] < jv_ptr[q]) return VFPI_E_SHAPE;
    for (int32_t t = jv_ptr[q]; t < jv_ptr[q + 1]; ++t) {
      const int32_t a = jv_col[t];
      if (a < 0 || a >= n_o) return VFPI_E_SHAPE;
      supp[q].push_back(a);
      Q[a].push_back(q);
    }
    std::sort(supp[q].begin(), supp[q].end());
    if (std::adjacent_find(supp[q].begin(), supp[q].end()) != supp[q].end()) return VFPI_E_SHAPE;
  }
  int64_t nnz = 0;
  std::vector<int32_t> cols;
  aug_row_ptr[0] = 0;
  for (int32_t a = 0; a < n_o; ++a) {
    if (row_ptr[a + 1] < row_ptr[a]) return VFPI_E_SHAPE;
    cols.assign(col_idx + row_ptr[a], col_idx + row_ptr[a + 1]);
    for (size_t k = 0; k < cols.size(); ++k)  // in range, strictly increasing (the value pass merges rows)
      if (cols[k] < 0 || cols[k] >= n_o || (k > 0 && cols[k] <= cols[k - 1])) return VFPI_E_SHAPE;
    for (int32_t q : Q[a]) cols.insert(cols.end(), supp[q].begin(), supp[q].end());
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    for (int32_t q : Q[a]) cols.push_back(n_o + q);  // Q[a] is increasing
    if (aug_col_idx) {
      if (nnz + (int64_t)cols.size() > cap) return VFPI_E_CAPACITY;
      std::copy(cols.begin(), cols.end(), aug_col_idx + nnz);
    }
    nnz += (int64_t)cols.size();
    if (nnz > INT32_MAX) return VFPI_E_SHAPE;
    aug_row_ptr[a + 1] = (int32_t)nnz;
  }
  for (int32_t q = 0; q < n_v; ++q) {
    cols = supp[q];
    cols.push_back(n_o + q);
    if (aug_col_idx) {
      if (nnz + (int64_t)cols.size() > cap) return VFPI_E_CAPACITY;
      std::copy(cols.begin(), cols.end(), aug_col_idx + nnz);
    }
    nnz += (int64_t)cols.size();
    if (nnz > INT32_MAX) return VFPI_E_SHAPE;
    aug_row_ptr[n_o + q + 1] = (int32_t)nnz;
  }
  *aug_nnzb = nnz;
  return VFPI_OK;
}

extern "C" int vfpi_vnode_values(const vfpi_bsr* A_o, const double* b_o, const double* v_o, int32_t n_v,
                                 const int32_t* jv_ptr, const int32_t* jv_col, const double* jv_val, double k_v,
                                 const int32_t* aug_row_ptr, const int32_t* aug_col_idx, double* aug_val,
                                 double* b, double* v, hipStream_t stream) {
  if (!A_o || !b_o || !v_o || !jv_ptr || !aug_row_ptr || !b || !v) return VFPI_E_NULL;
  const int32_t n_o = A_o->n_nodes;
  if (n_o < 0 || n_v < 0) return VFPI_E_SHAPE;
  if (!(k_v > 0.0) || !__builtin_isfinite(k_v)) return VFPI_E_OPTS;
  const int64_t rows = (int64_t)n_o + n_v;
  if (rows == 0) return VFPI_OK;
  if (!aug_col_idx || !aug_val || (n_o > 0 && (!A_o->row_ptr || !A_o->col_idx || !A_o->val))) return VFPI_E_NULL;
  if (n_v > 0 && (!jv_col || !jv_val)) return VFPI_E_NULL;
  hipLaunchKernelGGL(k_vnode_values, dim3((unsigned)((rows + 127) / 128)), dim3(128), 0, stream, n_o, A_o->row_ptr,
                     A_o->col_idx, static_cast<const double*>(A_o->val), b_o, v_o, n_v, jv_ptr, jv_col, jv_val, k_v,
                     aug_row_ptr, aug_col_idx, aug_val, b, v);
  VFPI_CHECK_HIP(hipGetLastError());
  return VFPI_OK;
}
