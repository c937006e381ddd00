// Host launchers of the query kernels.
#pragma once
#include "tnn_internal.h"

namespace tnn {

// One airspace of a batch, as the persistent kernel reads it.
struct BatchItemDev {
  IndexDesc ix;
  Prep pr;
  QueryArgs a;
  const float *qx, *qy, *qz, *qt;
  int64_t nq;
  int32_t *out_idx;
  double *out_dist;
};

// Everything tnn_query_batched launches with (lives in tnn_batch_plan).
struct BatchLaunch {
  uint32_t magic;
  int32_t n;
  int32_t chunk;
  int32_t waves_per_block;
  int32_t stats;  // some item collects statistics
  int32_t gka;    // some item averages values over its neighbours
  int64_t grid;
  int64_t total_q;
  int64_t total_seg;
  const BatchItemDev *items;
  const int64_t *qprefix;
  const int32_t *order;
  const int64_t *seg_prefix;
  unsigned long long *counter;
  unsigned *done;
  unsigned long long *ticks;
};
static_assert(sizeof(BatchLaunch) <= sizeof(tnn_batch_plan), "batch plan too large");
constexpr uint32_t kBatchMagic = 0x544e4e42u;  // "TNNB"

hipError_t launch_batch(const BatchLaunch &bl, hipStream_t st);

// per_query_scales: records carry the deviation bounds instead of the
// per-call cylinder constants (each query forms its own).
hipError_t launch_prep(const IndexDesc &ix, const QueryArgs &a, const Prep &pr, hipStream_t st,
                       bool per_query_scales = false);
// The preparation and, in the same launch, the radius prediction of every
// query into pr.radius2 with a.model and a.alpha.
hipError_t launch_prep_infer(const IndexDesc &ix, const QueryArgs &a, const Prep &pr,
                             const tnn_points &qs, hipStream_t st, bool per_query_scales);
// query_scale: per-query scales [n][4] (device) or null for the shared ones.
hipError_t launch_query(const IndexDesc &ix, const Prep &pr, const QueryArgs &a,
                        const tnn_points &qs, int waves_per_block, int32_t *out_idx,
                        double *out_dist, hipStream_t st, const double *query_scale = nullptr);
hipError_t launch_brute(const IndexDesc &ix, const QueryArgs &a, const tnn_points &qs,
                        int waves_per_block, int32_t *out_idx, double *out_dist, hipStream_t st,
                        const double *query_scale = nullptr);
hipError_t launch_gka(const int32_t *idx, const double *dist, int64_t nq, int k,
                      const float *values, int n_comp, int64_t n_points, double *out,
                      hipStream_t st);
size_t mixed_scratch_bytes(int64_t n_points, int64_t n_queries, int k);
hipError_t launch_mixed_brute(const IndexDesc &ix, const QueryArgs &a, const tnn_points &qs,
                              int32_t *out_idx, double *out_dist, void *scratch, hipStream_t st);
hipError_t launch_debug_lb(const IndexDesc &ix, const Prep &pr, const QueryArgs &a,
                           const tnn_points &qs, double *seg_lb_out, float *block_lb_out,
                           hipStream_t st, const double *query_scale = nullptr);

// Index construction (build.hip).
hipError_t launch_seg_stats(const tnn_points &pts, const int32_t *start, const int32_t *cnt_flags,
                            int64_t n_seg, const float *order_sqrt_scale, float *ax, float *ay,
                            float *az, float *bx, float *by, float *bz, float *tmin, float *tmax,
                            float *ex, float *ey, float *ez, float *keys, uint32_t *status,
                            hipStream_t st);
hipError_t launch_seg_scatter(const tnn_points &pts, int64_t n_seg, const int32_t *perm,
                              const int32_t *src_start, const int32_t *src_cnt_flags,
                              const int32_t *dst_pstart, const float *const src_f[11],
                              float *const dst_f[11], int32_t *dst_pstart_out, int32_t *dst_pcount,
                              int32_t *dst_sorig, int32_t *dst_first, float4 *pt4, int32_t *pid,
                              hipStream_t st);
hipError_t launch_block_box(const IndexDesc &ix, float *box, hipStream_t st);
hipError_t launch_export(const IndexDesc &ix, float *seg_f32, int32_t *seg_i32, int32_t *point_id,
                         float *block_box, hipStream_t st);

}  // namespace tnn
