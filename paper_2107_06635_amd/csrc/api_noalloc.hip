// ntu_metric_fix_noalloc (declared in include/ntu.h): the metric repair for
// callers that cannot allocate device memory.  Its scratch space (the
// Hermitisation's partial norms, then the eigen-solve's two matrices per
// item) is a file-scope device array instead of a context's workspace, so the
// call allocates nothing and needs no context.
#include <mutex>
#include <string>
#include "ntu.h"
#include "kernels.h"

// One copy per device, held by every device the library runs on until the
// process ends.  Host code never passes this name to a kernel: on the host it
// is a stand-in, not a device address; the address comes from
// hipGetSymbolAddress (scratch_ptr below).
static __device__ __align__(256) unsigned char scratch[NTU_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = NTU_NOALLOC_SCRATCH_BYTES;  // per device
constexpr int NOALLOC_MAX_DEVICES = 64;

void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
std::mutex g_scratch_mu;

// the message is read with ntu_last_error(NULL)
ntu_status nfail(ntu_status s, const std::string& m) {
  ntu::set_global_error(m.c_str());
  return s;
}

// The device address of this device's `scratch`, looked up once per device
// with that device current (the caller's current device).
hipError_t scratch_ptr(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

ntu_status check_dense(const ntu_tensor* t, const char* name, int ndim, int dev) {
  const std::string nm(name);
  if (!t->data) return nfail(NTU_ERR_ARG, nm + ": NULL data pointer");
  if (t->ndim != ndim) return nfail(NTU_ERR_SHAPE, nm + ": wrong number of dimensions");
  long long st = 1;
  for (int i = ndim - 1; i >= 0; --i) {
    if (t->shape[i] < 0) return nfail(NTU_ERR_SHAPE, nm + ": negative extent");
    if (t->shape[i] != 1 && t->stride[i] != st) return nfail(NTU_ERR_SHAPE, nm + ": not a dense row-major array");
    st *= t->shape[i];
  }
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, t->data) != hipSuccess) {
    (void)hipGetLastError();
    return nfail(NTU_ERR_ARG, nm + ": not device memory");
  }
  if ((attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) || attr.device != dev)
    return nfail(NTU_ERR_ARG, nm + ": not memory of the current device");
  return NTU_OK;
}

}  // namespace

extern "C" {

ntu_status ntu_metric_fix_noalloc(void* stream, int batch, ntu_tensor* g, int mode, ntu_tensor* stats) {
  ntu::set_global_error("");
  if (batch < 0) return nfail(NTU_ERR_ARG, "batch must be >= 0");
  if (mode != NTU_FIX_HERM && mode != NTU_FIX_HERM_CLIP) return nfail(NTU_ERR_ARG, "unknown mode");
  if (batch == 0) return NTU_OK;
  if (!g) return nfail(NTU_ERR_ARG, "g: NULL descriptor");
  if (g->dtype != NTU_F64 && g->dtype != NTU_C128) return nfail(NTU_ERR_DTYPE, "g: element type must be F64 or C128");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return nfail(NTU_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nfail(NTU_ERR_UNSUPPORTED, "device ordinal beyond the table");
  ntu_status s = check_dense(g, "g", 3, dev);
  if (s) return s;
  const long long n = g->shape[1];
  if (g->shape[0] != batch || g->shape[2] != n || n < 1)
    return nfail(NTU_ERR_SHAPE, "g: expected shape (batch, n, n)");
  if (n > 1024) return nfail(NTU_ERR_SHAPE, "g: n above 1024");
  if (stats) {
    if (stats->dtype != NTU_F64) return nfail(NTU_ERR_DTYPE, "stats: element type must be F64");
    if ((s = check_dense(stats, "stats", 2, dev))) return s;
    if (stats->shape[0] != batch || stats->shape[1] != 8) return nfail(NTU_ERR_SHAPE, "stats: expected (batch, 8)");
  }
  const bool cplx = g->dtype == NTU_C128;
  const size_t need = ntu::fix_workspace_bytes(cplx, batch, (int)n);
  if (need > NOALLOC_SCRATCH_BYTES)
    return nfail(NTU_ERR_WORKSPACE, "batch x n exceeds the " + std::to_string(NOALLOC_SCRATCH_BYTES >> 20) +
                                        " MiB scratch of ntu_metric_fix_noalloc (needs " + std::to_string(need) +
                                        " bytes)");
  void* ws = nullptr;
  if ((e = scratch_ptr(dev, &ws)) != hipSuccess)
    return nfail(NTU_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
  const ntu::ProfHook none{nullptr, nullptr};
  e = ntu::launch_metric_fix(cplx, batch, (int)n, g->data, mode, stats ? (double*)stats->data : nullptr, 8, ws,
                             (hipStream_t)stream, none);
  return e == hipSuccess ? NTU_OK : nfail(NTU_ERR_HIP, std::string("metric_fix: ") + hipGetErrorString(e));
}

}  // extern "C"
