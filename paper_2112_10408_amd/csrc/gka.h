// Gaussian kernel averaging over one query's k-NN context (Sec. 3.2, Eq.
// gka), held one slot per lane of a wavefront: the one-query averaging
// kernel and the batched search's epilogue run this same code.
#pragma once
#include "wave.h"

namespace tnn {

constexpr int kGkaMaxComp = 8;

// Sum of a double over the 64 lanes of a wave, in every lane, in a fixed
// order: DPP steps add lane pairs 1 and 2 apart within quads, then 4 and 8
// apart within rows of 16, and the four row sums are combined as
// (row 0 + row 1) + (row 2 + row 3).  DPP moves each 32-bit half; no LDS.
template <int Ctrl>
__device__ __forceinline__ double dpp_d(double v) {
  return mk_double(dpp_i<Ctrl>(lo32(v)), dpp_i<Ctrl>(hi32(v)));
}

__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_d<kDppQuadXor1>(v);
  v += dpp_d<kDppQuadXor2>(v);
  v += dpp_d<kDppRowRor4>(v);
  v += dpp_d<kDppRowRor8>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Lane r holds context slot r: `used` (slot r is a neighbour), its caller
// index `id` and scaled squared distance `d`, slots ascending by distance.
// Writes out_row[c] = sum_r w_r v[id_r][c] / sum_r w_r, w_r = exp(-(d_r - d_0))
// with d_0 the nearest used slot (the same ratio as exp(-d), without 0/0 for
// far contexts); NaN when no slot is used.  Every lane of the wave calls it.
// The value gathers of every component are issued before the weights are
// computed, so their latency overlaps the exponentials.
__device__ __forceinline__ void gka_context_average(bool used, int id, double d,
                                                    const float *values, int n_comp,
                                                    double *out_row) {
  const int lane = lane_id();
  const uint64_t um = ballot(used);
  if (!um) {
    if (lane < n_comp) out_row[lane] = __builtin_nan("");
    return;
  }
  float v[kGkaMaxComp];
#pragma unroll
  for (int c = 0; c < kGkaMaxComp; ++c)
    v[c] = (used && c < n_comp) ? values[(int64_t)id * n_comp + c] : 0.0f;
  const double d0 = readlane_d(d, __ffsll((long long)um) - 1);
  const double w = used ? exp(-(d - d0)) : 0.0;
  const double den = wave_sum_d(w);
#pragma unroll
  for (int c = 0; c < kGkaMaxComp; ++c) {
    if (c >= n_comp) break;
    const double num = wave_sum_d(w * (double)v[c]);
    if (lane == 0) out_row[c] = num / den;
  }
}

}  // namespace tnn
