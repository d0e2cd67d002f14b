// (compiled as part of vfpi_lib.hip)
// vfpi_step_noalloc: the plain FP64 solve of vfpi_step with its workspace in a
// fixed device array instead of a context's hipMalloc'd buffers, for callers
// that cannot allocate (graph capture, serving loops).  The kernels are
// vfpi_step's own; only where their scratch lives differs.
#include <mutex>

#include "common.h"
#include "internal.h"

namespace {

// The workspace, one copy per GPU the library runs on, held until the
// process ends.  Host code must never use this name as a device address: it
// is a host-side stand-in.  The device address comes from
// hipGetSymbolAddress, once per device (scratch_on_device).
static __device__ __align__(256) unsigned char scratch[VFPI_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};
int g_scratch_cu[kMaxDevices] = {};

constexpr int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

// Carve the workspace of one call out of `base` in the order of vfpi_ctx's
// buffers.  With base == nullptr only the byte count is computed.
int64_t carve(unsigned char* base, int32_t N, int32_t nnzb, int32_t nc, vfpi_ctx* c) {
  const int64_t n = 3 * (int64_t)N;
  int64_t off = 0;
  auto take = [&](int64_t bytes) -> unsigned char* {
    unsigned char* p = base ? base + off : nullptr;
    off += align256(bytes > 0 ? bytes : 1);
    return p;
  };
  unsigned char* p;
  p = take(4 * (int64_t)nnzb);                         if (c) c->scol = reinterpret_cast<int32_t*>(p);
  p = take(80 * (int64_t)nnzb);                        if (c) c->sval = p;
  p = take(8 * n);                                     if (c) c->diag = reinterpret_cast<double*>(p);
  p = take(8 * n);                                     if (c) c->rn2 = reinterpret_cast<double*>(p);
  p = take(8 * n);                                     if (c) c->w = p;
  p = take(8 * n);                                     if (c) c->vbuf = p;
  p = take(8 * n);                                     if (c) c->vprev = p;
  p = take(4 * (int64_t)N);                            if (c) c->cmap = reinterpret_cast<int32_t*>(p);
  p = take(8 * (int64_t)vfpi::kPack * nc);             if (c) c->cpack = p;
  p = take(4 * 2 * (int64_t)nc);                       if (c) c->cpair = reinterpret_cast<int32_t*>(p);
  p = take(8 * 8 * n);                                 if (c) c->adj = reinterpret_cast<double*>(p);
  p = take(8 * (int64_t)vfpi::kSlotWords);             if (c) c->slots = reinterpret_cast<uint64_t*>(p);
  p = take(4 * (int64_t)vfpi::kSyncWords);             if (c) c->sync = reinterpret_cast<uint32_t*>(p);
  p = take(4);                                         if (c) c->flags = reinterpret_cast<int32_t*>(p);
  return off;
}

// Device address of this device's copy of `scratch` and its CU count, looked
// up once per device with that device current.
hipError_t scratch_on_device(int dev, unsigned char** ptr, int* num_cu) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    int cu = 0;
    e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    g_scratch_cu[dev] = cu;
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *ptr = g_scratch_ptr[dev];
  *num_cu = g_scratch_cu[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int vfpi_step_noalloc(const vfpi_bsr* A, const double* b, const vfpi_contacts* Jc, double* v,
                                 double* lambda, const vfpi_opts* opts, vfpi_stats* stats, void* tape,
                                 hipStream_t stream) {
  if (!A || !b || !Jc || !v || !opts || !stats) return VFPI_E_NULL;
  const int32_t N = A->n_nodes, nnzb = A->nnzb, nc = Jc->n_contacts;
  if (N < 0 || nnzb < 0 || nc < 0) return VFPI_E_SHAPE;
  if (opts->reuse_w) return VFPI_E_OPTS;  // other calls on this GPU may have overwritten the row sums
  if (carve(nullptr, N, nnzb, nc, nullptr) > (int64_t)VFPI_NOALLOC_SCRATCH_BYTES) return VFPI_E_CAPACITY;
  int dev = 0;
  VFPI_CHECK_HIP(hipGetDevice(&dev));
  unsigned char* base = nullptr;
  int num_cu = 0;
  VFPI_CHECK_HIP(scratch_on_device(dev, &base, &num_cu));
  // A context on the stack whose buffers lie in this device's scratch array.
  // vfpi_step clears what must start at zero (flags, sync words, reduction
  // slots, stats) in its first kernel, so nothing left by an earlier call
  // matters; timing stays off and no events are touched.
  vfpi_ctx c;
  c.device = dev;
  c.num_cu = num_cu;
  c.max_nodes = N;
  c.max_nnzb = nnzb;
  c.max_contacts = nc;
  c.max_envs = 0;
  (void)carve(base, N, nnzb, nc, &c);
  return vfpi_step(&c, A, b, Jc, v, lambda, opts, stats, tape, stream);
}
