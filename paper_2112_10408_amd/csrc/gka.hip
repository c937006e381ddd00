// Gaussian kernel averaging of measured values over each query's k-NN
// context (Sec. 3.2, Eq. gka), run after the search on its outputs.
#include <cmath>

#include "gka.h"
#include "tnn_internal.h"

namespace tnn {
namespace {

constexpr int kGkaWaves = 4;  // waves per workgroup

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

// Two queries per wave when k <= 32: lanes 0-31 hold the first query's
// slots, lanes 32-63 the second's.  The sums are those of
// gka_context_average bit for bit: a query's slots fill two rows of 16 lanes
// there too (the other two rows adding +0), and each row is reduced by the
// same DPP steps.
__device__ __forceinline__ double row_pair_sum(double v, int half) {
  v += dpp_d<kDppQuadXor1>(v);
  v += dpp_d<kDppQuadXor2>(v);
  v += dpp_d<kDppRowRor4>(v);
  v += dpp_d<kDppRowRor8>(v);
  const double a = (readlane_d(v, 0) + readlane_d(v, 16)) + 0.0;
  const double b = (readlane_d(v, 32) + readlane_d(v, 48)) + 0.0;
  return half ? b : a;
}

__global__ __launch_bounds__(64 * kGkaWaves) void gka_pair_kernel(
    const int32_t *idx, const double *dist, int64_t nq, int k, const float *values, int n_comp,
    int64_t n_points, double *out) {
  const int64_t q0 = ((int64_t)blockIdx.x * kGkaWaves + (threadIdx.x >> 6)) * 2;
  if (q0 >= nq) return;
  const int lane = lane_id();
  const int half = lane >> 5, r = lane & 31;
  const int64_t q = q0 + half;
  const bool real = q < nq;
  int id = -1;
  double d = __builtin_huge_val();
  if (real && r < k) {
    id = idx[q * k + r];
    d = dist[q * k + r];
  }
  const bool used = id >= 0 && (int64_t)id < n_points && d < __builtin_huge_val();
  const uint64_t um = ballot(used);
  const uint32_t ua = (uint32_t)um, ub = (uint32_t)(um >> 32);
  const bool any = half ? ub != 0 : ua != 0;
  double *row = out + q * n_comp;
  if (real && !any && r < n_comp) row[r] = __builtin_nan("");
  if (um == 0) return;
  float v[kGkaMaxComp];
#pragma unroll
  for (int c = 0; c < kGkaMaxComp; ++c)
    v[c] = (used && c < n_comp) ? values[(int64_t)id * n_comp + c] : 0.0f;
  // the nearest used slot of each query
  const double da = ua ? readlane_d(d, __ffs(ua) - 1) : 0.0;
  const double db = ub ? readlane_d(d, 32 + __ffs(ub) - 1) : 0.0;
  const double d0 = half ? db : da;
  const double w = used ? exp(-(d - d0)) : 0.0;
  const double den = row_pair_sum(w, half);
#pragma unroll
  for (int c = 0; c < kGkaMaxComp; ++c) {
    if (c >= n_comp) break;
    const double num = row_pair_sum(w * (double)v[c], half);
    if (r == 0 && real && any) row[c] = num / den;
  }
}

}  // namespace

hipError_t launch_gka(const int32_t *idx, const double *dist, int64_t nq, int k,
                      const float *values, int n_comp, int64_t n_points, double *out,
                      hipStream_t st) {
  if (nq == 0) return hipSuccess;
  if (k <= 32) {
    const int64_t grid = ((nq + 1) / 2 + kGkaWaves - 1) / kGkaWaves;
    hipLaunchKernelGGL(gka_pair_kernel, dim3((unsigned)grid), dim3(64 * kGkaWaves), 0, st, idx,
                       dist, nq, k, values, n_comp, n_points, out);
    return hipGetLastError();
  }
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
