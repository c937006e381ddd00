// Gaussian kernel averaging of measured values over each query's k-NN
// context (Sec. 3.2, Eq. gka), run after the search on its outputs.
#include <cmath>

#include "tnn_internal.h"
#include "wave.h"

namespace tnn {
namespace {

constexpr int kGkaMaxComp = 8;
constexpr int kGkaWaves = 4;  // queries per workgroup, one per wave

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

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
  const uint64_t um = ballot(used);
  if (!um) {
    if (lane < n_comp) out[q * n_comp + lane] = __builtin_nan("");
    return;
  }
  // the nearest used slot (the slots are sorted by distance)
  const double d0 = readlane_d(d, __ffsll((long long)um) - 1);
  const double w = used ? exp(-(d - d0)) : 0.0;
  const double den = wave_sum_d(w);
  for (int c = 0; c < n_comp; ++c) {
    const double v = used ? (double)values[(int64_t)id * n_comp + c] : 0.0;
    const double num = wave_sum_d(w * v);
    if (lane == 0) out[q * n_comp + c] = num / den;
  }
}

}  // namespace
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
  const int64_t grid = (n_queries + kGkaWaves - 1) / kGkaWaves;
  hipLaunchKernelGGL(gka_kernel, dim3((unsigned)grid), dim3(64 * kGkaWaves), 0,
                     static_cast<hipStream_t>(stream), d_idx, d_dist, n_queries, k, d_values,
                     n_comp, n_points, d_out);
  return hipGetLastError() == hipSuccess ? TNN_OK : TNN_E_HIP;
}
