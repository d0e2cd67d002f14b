// Library-internal declarations: the context, launch helpers, tape layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vfpi.h"

#define VFPI_CHECK_HIP(expr)                  \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return VFPI_E_HIP;  \
  } while (0)

namespace vfpi {

constexpr int kSyncWords = 64;

// Words of ctx->sync
enum { SY_QUEUE = 2, SY_AMAX = 4 /* 64-bit, words 4-5 */ };

}  // namespace vfpi

struct vfpi_ctx {
  int device = 0;
  int num_cu = 0;
  int32_t max_nodes = 0, max_nnzb = 0, max_contacts = 0, max_envs = 0;
  int32_t* scol = nullptr;     // [max_nnzb]   chunk-interleaved column indices
  void* sval = nullptr;        // [10 max_nnzb] doubles: chunk-interleaved values (FP64: 80 bytes a block, with the column; FP32: 36)
  double* diag = nullptr;      // [3 max_nodes] a_dd
  double* rn2 = nullptr;       // [3 max_nodes] ||A_d*||^2
  void* w = nullptr;           // [3 max_nodes] step sizes
  void* vbuf = nullptr;        // [3 max_nodes] second buffer of the V-FPI iterate
  void* vprev = nullptr;       // [3 max_nodes] v^{l-1} for Chebyshev acceleration (node-local)
  int32_t* cmap = nullptr;     // [max_nodes] node -> contact (-1: none)
  void* cpack = nullptr;       // [12 max_contacts] R, phi, mu, gamma per contact
  int32_t* cpair = nullptr;    // [2 max_contacts] nodes i, j of each contact (j = -1: S)
  double* adj = nullptr;       // [8 * 3 max_nodes] adjoint vectors (forward BB: A v^l)
  uint64_t* slots = nullptr;   // [kSlotWords] tagged per-workgroup partial sums
  uint32_t* sync = nullptr;    // [kSyncWords] work-queue counter of the batched kernel
  int32_t* flags = nullptr;    // [1 + max_envs] device-detected data errors
  int32_t stats_nodes = -1;    // N for which diag/rn2 hold valid row sums (W reuse)
  int32_t timing = 0;          // record events around setup / solve
  int32_t timed_calls = 0;     // calls recorded since enabling
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
};

// Event marks for the timing aid (no-ops unless enabled).
inline void vfpi_mark(vfpi_ctx* c, int k, hipStream_t s) {
  if (c->timing) {
    (void)hipEventRecord(c->ev[k], s);
    if (k == 2) c->timed_calls++;
  }
}

// Tape layout (bytes from the start): w[n] f64, v[n] f64, lambda*[3nc] f64, branch[nc] i32
struct TapeView {
  double* w;
  double* v;
  double* lamstar;
  int32_t* branch;
};

inline TapeView tape_view(void* base, int32_t n_nodes, int32_t n_contacts) {
  char* p = static_cast<char*>(base);
  int64_t n = 3 * (int64_t)n_nodes;
  TapeView t;
  t.w = reinterpret_cast<double*>(p);
  t.v = reinterpret_cast<double*>(p + 8 * n);
  t.lamstar = reinterpret_cast<double*>(p + 16 * n);
  t.branch = reinterpret_cast<int32_t*>(p + 16 * n + 24 * (int64_t)n_contacts);
  return t;
}

int vfpi_check_opts(const vfpi_opts* o, bool batched);
