// (compiled as part of vfpi_lib.hip)
// Context management, option checks, tape size and error strings.
#include <string.h>

#include "common.h"
#include "internal.h"

namespace {

template <class T>
hipError_t alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

void release(vfpi_ctx* c) {
  void* ptrs[] = {c->scol, c->sval, c->diag, c->rn2, c->w, c->vbuf, c->vprev, c->cmap, c->cpack,
                  c->cpair, c->adj, c->slots, c->sync, c->flags};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int k = 0; k < 3; ++k)
    if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
}

}  // namespace

int vfpi_check_opts(const vfpi_opts* o, bool batched) {
  if (o->max_iters < 0) return VFPI_E_OPTS;
  if (!(o->tol >= 0.0)) return VFPI_E_OPTS;
  if (o->w_mode < VFPI_W_FROBENIUS || o->w_mode > VFPI_W_BB2) return VFPI_E_OPTS;
  if (o->projection != VFPI_PROJ_STRICT && o->projection != VFPI_PROJ_PROXIMAL) return VFPI_E_OPTS;
  if (o->w_mode == VFPI_W_USER_DIAG && !o->w_user) return VFPI_E_NULL;
  if (o->w_mode == VFPI_W_USER_SCALAR && !(o->alpha_user > 0.0)) return VFPI_E_OPTS;
  if (batched && o->w_mode != VFPI_W_FROBENIUS && o->w_mode != VFPI_W_USER_SCALAR) return VFPI_E_UNSUPPORTED;
  if (o->cheby_ls < 0 || !(o->cheby_u >= 0.0 && o->cheby_u <= 1.0)) return VFPI_E_OPTS;
  if (!(o->omega >= 0.0) || !__builtin_isfinite(o->omega)) return VFPI_E_OPTS;
  return VFPI_OK;
}

extern "C" int vfpi_create(vfpi_ctx** out, int32_t max_nodes, int32_t max_nnzb, int32_t max_contacts,
                           int32_t max_envs) {
  if (!out) return VFPI_E_NULL;
  *out = nullptr;
  if (max_nodes < 0 || max_nnzb < 0 || max_contacts < 0 || max_envs < 0) return VFPI_E_SHAPE;
  vfpi_ctx* c = new vfpi_ctx();
  c->max_nodes = max_nodes;
  c->max_nnzb = max_nnzb;
  c->max_contacts = max_contacts;
  c->max_envs = max_envs;
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device);
  const size_t n = 3 * (size_t)max_nodes;
  if (e == hipSuccess) e = alloc(&c->scol, (size_t)max_nnzb);
  if (e == hipSuccess) e = alloc(reinterpret_cast<double**>(&c->sval), vfpi::kSvalWords64 * (size_t)max_nnzb);
  if (e == hipSuccess) e = alloc(&c->diag, n);
  if (e == hipSuccess) e = alloc(&c->rn2, n);
  if (e == hipSuccess) e = alloc(reinterpret_cast<double**>(&c->w), n);
  if (e == hipSuccess) e = alloc(reinterpret_cast<double**>(&c->vbuf), n);
  if (e == hipSuccess) e = alloc(reinterpret_cast<double**>(&c->vprev), n);
  if (e == hipSuccess) e = alloc(&c->cmap, (size_t)max_nodes);
  if (e == hipSuccess) e = alloc(reinterpret_cast<double**>(&c->cpack), vfpi::kPack * (size_t)max_contacts);
  if (e == hipSuccess) e = alloc(&c->cpair, 2 * (size_t)max_contacts);
  if (e == hipSuccess) e = alloc(&c->adj, 8 * n);
  if (e == hipSuccess) e = alloc(&c->slots, (size_t)vfpi::kSlotWords);
  if (e == hipSuccess) e = alloc(&c->sync, (size_t)vfpi::kSyncWords);
  if (e == hipSuccess) e = alloc(&c->flags, 1 + (size_t)max_envs);
  for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipEventCreate(&c->ev[k]);
  if (e == hipSuccess) e = hipMemset(c->sync, 0, vfpi::kSyncWords * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(c->flags, 0, (1 + (size_t)max_envs) * sizeof(int32_t));
  if (e != hipSuccess) {
    release(c);
    delete c;
    return VFPI_E_HIP;
  }
  *out = c;
  return VFPI_OK;
}

extern "C" int vfpi_destroy(vfpi_ctx* c) {
  if (!c) return VFPI_OK;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  release(c);
  delete c;
  return VFPI_OK;
}

extern "C" int64_t vfpi_tape_bytes(int32_t n_nodes, int32_t n_contacts) {
  if (n_nodes < 0 || n_contacts < 0) return VFPI_E_SHAPE;
  const int64_t raw = 48 * (int64_t)n_nodes + 28 * (int64_t)n_contacts;
  return (raw + 255) / 256 * 256;
}

extern "C" int vfpi_timing_enable(vfpi_ctx* c, int32_t on) {
  if (!c) return VFPI_E_NULL;
  c->timing = on ? 1 : 0;
  c->timed_calls = 0;
  return VFPI_OK;
}

extern "C" int vfpi_timing_read(vfpi_ctx* c, float* setup_ms, float* solve_ms) {
  if (!c || !setup_ms || !solve_ms) return VFPI_E_NULL;
  if (!c->timing || c->timed_calls == 0) return VFPI_E_OPTS;
  VFPI_CHECK_HIP(hipEventSynchronize(c->ev[2]));
  VFPI_CHECK_HIP(hipEventElapsedTime(setup_ms, c->ev[0], c->ev[1]));
  VFPI_CHECK_HIP(hipEventElapsedTime(solve_ms, c->ev[1], c->ev[2]));
  return VFPI_OK;
}

extern "C" const char* vfpi_error_string(int code) {
  switch (code) {
    case VFPI_OK: return "ok";
    case VFPI_E_NULL: return "a required pointer is NULL";
    case VFPI_E_SHAPE: return "inconsistent sizes";
    case VFPI_E_OPTS: return "invalid option";
    case VFPI_E_CAPACITY: return "problem larger than the context capacity";
    case VFPI_E_UNSUPPORTED: return "input form not supported by the library";
    case VFPI_E_HIP: return "HIP runtime error";
    case VFPI_E_NO_TAPE: return "backward called without a forward tape";
    default: return "unknown error code";
  }
}
