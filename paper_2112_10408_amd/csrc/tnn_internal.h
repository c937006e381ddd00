// Internal layout shared by the host entry points and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tnn.h"

namespace tnn {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlockSegs = 64;     // segments per culling block (one per lane)
constexpr int kSuperBlocks = 64;   // blocks per superblock (one per lane)
constexpr int kMaxK = 64;          // top-k held one rank per lane
constexpr int kMaxSegLen = 64;

// Everything a kernel needs to read a built index.  Lives inside tnn_index.
struct IndexDesc {
  uint32_t magic;
  int32_t seg_len;     // K
  int32_t kpad;        // K rounded up to a power of two (points per lane group)
  int32_t n_blocks;
  int64_t n_points;
  int64_t n_seg;
  // sorted points (segment order): (x, y, z, t) of slot p in pt4[p]
  const float4 *pt4;
  const int32_t *pid;  // caller index of each slot
  // segments (block order), SoA
  const float *ax, *ay, *az, *bx, *by, *bz, *tmin, *tmax, *ex, *ey, *ez;
  const int32_t *pstart, *pcount, *sorig;
  const int32_t *sfirst;  // 1 for the first segment of its trajectory
  // block boxes: box[8 b + f] for f = 0..7 (lo x y z t, hi x y z t)
  const float *box;
  // superblock boxes (64 consecutive blocks each), same layout
  const float *sbox;
  int32_t n_super;
  int32_t pad_;
  float lo[4], hi[4];  // bounding box of all points
};
static_assert(sizeof(IndexDesc) <= sizeof(tnn_index), "index descriptor too large");
constexpr uint32_t kIndexMagic = 0x544e4e31u;  // "TNN1"

// Per-call segment records (the radius and projection constants depend on
// the scales), in four planes of n_seg entries each (plane f of segment s at
// rec[f * n_seg + s], so that the 64 lanes of a wave reading the records of
// 64 consecutive segments read 1 KiB of contiguous memory per plane):
//   [0] A.x, A.y, A.z, t_min
//   [1] (B - A).x, .y, .z (float32 differences), t_max
//   [2] 1 / |AB|_s^2 (0 for a degenerate segment), radius R = sqrt(sum s_f
//       e_f^2) rounded up, absolute slack 2^-17 |AB|_s rounded up, 0
//   [3] first point slot, member count (an int2 array over the plane)
constexpr int kSegRec = 4;
struct Prep {
  float4 *rec;
  unsigned long long *ticket;  // work-queue counters of the resident search kernel
  float *radius2;              // predicted radii (in-call prediction) or null
  int64_t n_seg;               // entries per record plane
};

struct QueryArgs {
  double inf;          // +infinity, from the host (see TopK::init)
  double s[4];
  float sf[4];         // scales rounded toward zero to float32 (block bounds)
  double t_window;
  int32_t k;
  uint32_t flags;
  int32_t seed_segments;
  const float *radius2;
  unsigned long long *stats;
  double floor_tau;    // smallest search radius a growing round starts from (radius_floor)
  // radius predicted by the preparation launch (model null: none)
  const tnn_radius_model *model;
  float alpha;
  // Gaussian kernel averaging asked with the search (gka_values null: none)
  const float *gka_values;
  int32_t gka_comp;
  double *gka_out;
};

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Float32 bounds and BF16 tiles take scaled squared norms up to this: the
// scaled squared half-diagonal of the index box, sum_f s_f ((hi_f - lo_f) / 2)^2,
// must stay below it (queries may lie far outside the box, up to about 1e8
// box widths, before float32 products could overflow).
constexpr double kMaxScaledNorm = 1e30;

__host__ __device__ inline bool scaled_box_ok(const float lo[4], const float hi[4],
                                              const double s[4]) {
  double n2 = 0.0;
  for (int f = 0; f < 4; ++f) {
    const double h = 0.5 * ((double)hi[f] - (double)lo[f]);
    n2 += s[f] * h * h;
  }
  return n2 < kMaxScaledNorm;
}

// Scale of the data for a metric: 2^-24 of the scaled squared diagonal of the
// index box (at least 1e-300), the radius a round grows from when a query has
// found nothing yet.
__host__ __device__ inline double radius_floor(const float lo[4], const float hi[4],
                                               const double s[4]) {
  double diag2 = 0.0;
  for (int f = 0; f < 4; ++f) {
    const double e = (double)hi[f] - (double)lo[f];
    diag2 += s[f] * e * e;
  }
  const double v = diag2 * 0x1p-24;
  return v > 1e-300 ? v : 1e-300;
}

}  // namespace tnn

#define TNN_HIP_CHECK(expr)                   \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return TNN_E_HIP;   \
  } while (0)
