// Gaussian kernel averaging of measured values over each query's k-NN
// context (Sec. 3.2, Eq. gka), run after the search on its outputs.
#include <cmath>

#include "gka.h"
#include "tnn_internal.h"

namespace tnn {
namespace {

constexpr int kGkaWaves = 4;  // queries per workgroup, one per wave

// One wave per query, lane r = context slot r.
__global__ __launch_bounds__(64 * kGkaWaves) void gka_kernel(const int32_t *idx, const double *dist,
                                                             int64_t nq, int k,
                                                             const float *values, int n_comp,
                                                             int64_t n_points, double *out) {
  const int64_t q = (int64_t)blockIdx.x * kGkaWaves + (threadIdx.x >> 6);
  if (q >= nq) return;
  const int lane = lane_id();
  int id = -1;
  double d = __builtin_huge_val();
  if (lane < k) {
    id = idx[q * k + lane];
    d = dist[q * k + lane];
  }
  const bool used = id >= 0 && (int64_t)id < n_points && d < __builtin_huge_val();
  gka_context_average(used, id, d, values, n_comp, out + q * n_comp);
}

}  // namespace

hipError_t launch_gka(const int32_t *idx, const double *dist, int64_t nq, int k,
                      const float *values, int n_comp, int64_t n_points, double *out,
                      hipStream_t st) {
  if (nq == 0) return hipSuccess;
  const int64_t grid = (nq + kGkaWaves - 1) / kGkaWaves;
  hipLaunchKernelGGL(gka_kernel, dim3((unsigned)grid), dim3(64 * kGkaWaves), 0, st, idx, dist, nq,
                     k, values, n_comp, n_points, out);
  return hipGetLastError();
}

}  // namespace tnn

using namespace tnn;

extern "C" tnn_status tnn_gka_average(const int32_t *d_idx, const double *d_dist,
                                      int64_t n_queries, int32_t k, const float *d_values,
                                      int32_t n_comp, int64_t n_points, double *d_out,
                                      void *stream) {
  if (n_queries < 0 || n_points < 0 || k < 1 || k > kMaxK || n_comp < 1 || n_comp > kGkaMaxComp)
    return TNN_E_ARG;
  if (n_queries == 0) return TNN_OK;
  if (!d_idx || !d_dist || !d_out || (n_points > 0 && !d_values)) return TNN_E_ARG;
  return launch_gka(d_idx, d_dist, n_queries, k, d_values, n_comp, n_points, d_out,
                    static_cast<hipStream_t>(stream)) == hipSuccess
             ? TNN_OK
             : TNN_E_HIP;
}
