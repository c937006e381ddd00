// Lower bounds and exact distances shared by the query kernels.
//
// Every bound here is conservative: it never exceeds the binary64 distance
// (the value the result reports) of any member point that passes the time
// mask.  Rounding slack is derived in the design notes; in short:
//  * block bound (float32): each term carries at most 7 float32 roundings of
//    a non-negative quantity, so multiplying by (1 - 2^-18) stays below the
//    real bound, which is below the real distance, which is within a
//    2^-50 relative error of the reported one;
//  * cylinder bound (float32): see seg_lb.
#pragma once
#include "tnn_internal.h"
#include "wave.h"

namespace tnn {

// Scaled squared distance, each operation rounded once in this order (no
// contraction): the value the result reports.
__device__ __forceinline__ double exact_dist(const double s[4], float qx, float qy, float qz,
                                             float qt, float px, float py, float pz, float pt) {
#pragma clang fp contract(off)
  const double dx = (double)qx - (double)px;
  const double dy = (double)qy - (double)py;
  const double dz = (double)qz - (double)pz;
  const double dt = (double)qt - (double)pt;
  const double a = s[0] * (dx * dx);
  const double b = s[1] * (dy * dy);
  const double c = s[2] * (dz * dz);
  const double e = s[3] * (dt * dt);
  return ((a + b) + c) + e;
}

// Per-query constants of the time mask.
struct QueryPoint {
  float x, y, z, t;
  double thr;   // (double)t - t_w: a point is a candidate iff (double)t_p < thr
  float thrf;   // thr rounded up to float32: for a float32 t_p, t_p < thr iff
                // t_p < thrf, and t_min >= thr iff t_min >= thrf (no float lies
                // strictly between thr and thrf), so the masks compare floats
  double gw;    // lower bound on t - t_p for any candidate (0 when t_w = 0)
  float gwf;    // the same, rounded down to float32
};

__device__ __forceinline__ QueryPoint make_query(float x, float y, float z, float t, double t_window) {
  QueryPoint q;
  q.x = x;
  q.y = y;
  q.z = z;
  q.t = t;
  q.thr = (double)t - t_window;
  q.thrf = __double2float_ru(q.thr);
  double gw = 0.0;
  if (t_window > 0.0) gw = fmax(t_window - 0x1p-50 * (fabs((double)t) + t_window), 0.0);
  q.gw = gw;
  q.gwf = __double2float_rd(gw);
  return q;
}

// Lower bound from a query to every point of block b: scaled squared
// distance to the block's (x, y, z, t) bounding box.  +inf when no point of
// the block is early enough.
// `box` is the index's box array (box[8 b + f]) in global memory or a copy of
// it in LDS.
__device__ __forceinline__ float block_lb(const float *box, int b, const QueryPoint &q,
                                          const float sf[4]) {
  const float4 lo = reinterpret_cast<const float4 *>(box)[2 * b];
  const float4 hi = reinterpret_cast<const float4 *>(box)[2 * b + 1];
  if (lo.w >= q.thrf) return __builtin_huge_valf();
  const float gx = fmaxf(fmaxf(lo.x - q.x, q.x - hi.x), 0.0f);
  const float gy = fmaxf(fmaxf(lo.y - q.y, q.y - hi.y), 0.0f);
  const float gz = fmaxf(fmaxf(lo.z - q.z, q.z - hi.z), 0.0f);
  const float gt = fmaxf(fmaxf(q.t - hi.w, q.gwf), 0.0f);
  const float v = sf[0] * (gx * gx) + sf[1] * (gy * gy) + sf[2] * (gz * gz) + sf[3] * (gt * gt);
  // saturate: a float32 overflow (huge scales or coordinates) must not read
  // as +inf, which means "masked"; the largest float is still a lower bound
  return fminf(v * (1.0f - 0x1p-18f), 0x1.fffffep+127f);
}

// A segment's record as the search reads it.
struct SegView {
  float4 r0, r1, r2;
  int ps, pc;  // first point slot, member count
};

__device__ __forceinline__ SegView load_seg(const Prep &pr, int64_t s) {
  const int64_t S = pr.n_seg;
  SegView v;
  v.r0 = pr.rec[s];
  v.r1 = pr.rec[S + s];
  v.r2 = pr.rec[2 * S + s];
  const int2 r3 = reinterpret_cast<const int2 *>(pr.rec + 3 * S)[s];
  v.ps = r3.x;
  v.pc = r3.y;
  return v;
}

// Cylinder lower bound (Sec. 3.4 masked distance minus approximation error,
// Algorithm 1, corrected): +inf if t_min >= t_q - t_w; otherwise
// max(0, D - R)^2 + s_t max(0, t_q - t_max, t_w)^2 with D the distance from
// the query to segment AB in the scaled metric (projection in that metric).
// Float32 with a proven margin: the computed distance to the segment exceeds
// the true one by at most 8u D + 14u |AB|_s (u = 2^-24; rounding of the
// differences, the projection parameter's second-order effect, and the
// hardware square root v_sqrt_f32, within 1 ulp = 2u relative), which the
// (1 - 2^-18) = (1 - 64u) factor and the 2^-17 |AB|_s slack remove; the
// scales are rounded toward zero, R is rounded up, and the final (1 - 2^-20)
// factor covers the remaining float32 roundings.  (The square root flushes a
// denormal argument to 0: a smaller distance, still a lower bound.)
__device__ __forceinline__ float seg_lb(const SegView &v, const QueryPoint &q, const float sf[4]) {
  if (v.r0.w >= q.thrf) return __builtin_huge_valf();
  const float abx = v.r1.x, aby = v.r1.y, abz = v.r1.z;
  const float apx = q.x - v.r0.x, apy = q.y - v.r0.y, apz = q.z - v.r0.z;
  const float dot = sf[0] * (apx * abx) + sf[1] * (apy * aby) + sf[2] * (apz * abz);
  const float del = fminf(fmaxf(dot * v.r2.x, 0.0f), 1.0f);
  const float rx = apx - del * abx, ry = apy - del * aby, rz = apz - del * abz;
  const float d2 = sf[0] * (rx * rx) + sf[1] * (ry * ry) + sf[2] * (rz * rz);
  const float dlo = __builtin_amdgcn_sqrtf(d2) * (1.0f - 0x1p-18f) - v.r2.z;
  const float g = fmaxf(dlo - v.r2.y, 0.0f);
  const float gt = fmaxf(fmaxf(q.t - v.r1.w, q.gwf), 0.0f);
  // saturated like block_lb (an overflow gives a NaN or +inf on the way,
  // which fmaxf / fminf turn into 0 or the largest float: both lower bounds)
  return fminf((g * g + sf[3] * (gt * gt)) * (1.0f - 0x1p-20f), 0x1.fffffep+127f);
}

// The same bound when every query has its own scales s (per-query metric):
// the record's third float4 then holds the segment's per-axis deviation
// bounds (e_x, e_y, e_z) instead of the per-call constants, and this computes
// those constants for s as the per-call preparation would.  1/|AB|^2_s and
// R are formed the same way; the slack uses 2^-17 |f|_s (1 + 2^-20), which
// is at least the per-call slack 2^-17 (|AB|_s + |f|_s) / 2 (1 + 2^-30):
// f = fl(B - A) is within a relative 2^-24 of B - A in every component.
__device__ __forceinline__ float seg_lb_q(SegView v, const QueryPoint &q, const double s[4],
                                          const float sf[4]) {
  const double fx = (double)v.r1.x, fy = (double)v.r1.y, fz = (double)v.r1.z;
  const double n2 = s[0] * fx * fx + s[1] * fy * fy + s[2] * fz * fz;
  const double ex = (double)v.r2.x, ey = (double)v.r2.y, ez = (double)v.r2.z;
  v.r2.x = n2 > 0.0 ? (float)(1.0 / n2) : 0.0f;
  v.r2.y = __double2float_ru(sqrt(s[0] * ex * ex + s[1] * ey * ey + s[2] * ez * ez) * (1.0 + 0x1p-40));
  v.r2.z = __double2float_ru(0x1p-17 * sqrt(n2) * (1.0 + 0x1p-20));
  return seg_lb(v, q, sf);
}

}  // namespace tnn
