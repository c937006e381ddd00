// tnn_query without a caller-supplied scratch buffer: for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).  The scratch lives in a file-scope device
// array, one copy per GPU, resolved once per device to its device address.
#include <mutex>

#include "tnn_internal.h"

namespace tnn {
namespace {

// One copy per device, held until the process ends.  In host code this name
// is only a stand-in for the symbol: its device address comes from
// hipGetSymbolAddress and is the only form ever handed to a kernel or copy.
static __device__ __align__(256) unsigned char scratch[TNN_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

// Device address of this device's `scratch`, resolved on the first call with
// that device current; null when the runtime cannot resolve it.
void *scratch_ptr(int dev) {
  static void *ptr[kMaxDevices] = {};
  static bool tried[kMaxDevices] = {};
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (!tried[dev]) {
    tried[dev] = true;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) ptr[dev] = p;
  }
  return ptr[dev];
}

}  // namespace
}  // namespace tnn

extern "C" tnn_status tnn_query_noalloc(const tnn_index *index, tnn_points queries,
                                        const tnn_query_params *params, int32_t *d_out_idx,
                                        double *d_out_dist, void *stream) {
  size_t need = 0;
  const tnn_status c = tnn_query_workspace(index, queries.n, params, &need);
  if (c != TNN_OK) return c;
  if (need > TNN_NOALLOC_SCRATCH_BYTES) return TNN_E_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TNN_E_HIP;
  if (dev < 0 || dev >= tnn::kMaxDevices) return TNN_E_UNSUPPORTED;
  void *p = tnn::scratch_ptr(dev);
  if (!p) return TNN_E_HIP;
  // tnn_query writes every byte of the scratch it reads (the search's work
  // counters are cleared by its preparation kernel), so the previous call's
  // contents do no harm
  return tnn_query(index, queries, params, d_out_idx, d_out_dist, p, TNN_NOALLOC_SCRATCH_BYTES,
                   stream);
}
