// Index construction kernels (Sec. 3.4: partition into runs of K points,
// segment from first to last point, approximation error) and the test export.
#include "kdorder.h"
#include "query.h"
#include "wave.h"

namespace tnn {

constexpr uint32_t kBadUnsorted = 1u;
constexpr uint32_t kBadNonFinite = 2u;

// One thread per segment, trajectory order.  cnt_flags[s] = member count in
// bits 0..15, bit 16 set when s is the first segment of its trajectory.
__global__ void seg_stats_kernel(tnn_points pts, const int32_t *start, const int32_t *cnt_flags,
                                 int64_t n_seg, const float *osc, float *ax, float *ay, float *az,
                                 float *bx, float *by, float *bz, float *tmin, float *tmax,
                                 float *ex, float *ey, float *ez, float *keys, uint32_t *status) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_seg) return;
  const int p0 = start[s];
  const int c = cnt_flags[s] & 0xffff;
  const bool first = (cnt_flags[s] >> 16) & 1;
  const int p1 = p0 + c - 1;
  uint32_t bad = 0;
  if (!first && pts.t[p0 - 1] > pts.t[p0]) bad |= kBadUnsorted;
  const double A[3] = {pts.x[p0], pts.y[p0], pts.z[p0]};
  const double B[3] = {pts.x[p1], pts.y[p1], pts.z[p1]};
  const double AB[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
  const double n2 = AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2];
  double e[3] = {0.0, 0.0, 0.0};
  float tlo = pts.t[p0], thi = pts.t[p0];
  float tprev = pts.t[p0];
  for (int i = 0; i < c; ++i) {
    const float fx = pts.x[p0 + i], fy = pts.y[p0 + i], fz = pts.z[p0 + i], ft = pts.t[p0 + i];
    if (!isfinite(fx) || !isfinite(fy) || !isfinite(fz) || !isfinite(ft)) bad |= kBadNonFinite;
    if (ft < tprev) bad |= kBadUnsorted;
    tprev = ft;
    tlo = fminf(tlo, ft);
    thi = fmaxf(thi, ft);
    const double P[3] = {fx, fy, fz};
    double u = 0.0;
    if (n2 > 0.0) {
      u = ((P[0] - A[0]) * AB[0] + (P[1] - A[1]) * AB[1] + (P[2] - A[2]) * AB[2]) / n2;
      u = fmin(fmax(u, 0.0), 1.0);
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      // |P - Q| for Q = A + u AB, plus room for the rounding of Q
      const double q = A[f] + u * AB[f];
      const double dev = fabs(P[f] - q) + 0x1p-40 * (fabs(A[f]) + fabs(B[f]) + fabs(P[f]));
      e[f] = fmax(e[f], dev);
    }
  }
  ax[s] = (float)A[0];
  ay[s] = (float)A[1];
  az[s] = (float)A[2];
  bx[s] = (float)B[0];
  by[s] = (float)B[1];
  bz[s] = (float)B[2];
  tmin[s] = tlo;
  tmax[s] = thi;
  ex[s] = __double2float_ru(e[0]);
  ey[s] = __double2float_ru(e[1]);
  ez[s] = __double2float_ru(e[2]);
  if (osc) {
    keys[4 * s + 0] = (float)(0.5 * (A[0] + B[0])) * osc[0];
    keys[4 * s + 1] = (float)(0.5 * (A[1] + B[1])) * osc[1];
    keys[4 * s + 2] = (float)(0.5 * (A[2] + B[2])) * osc[2];
    keys[4 * s + 3] = (float)(0.5 * ((double)tlo + (double)thi)) * osc[3];
  }
  if (bad) atomicOr(status, bad);
}

struct F11 {
  const float *p[11];
};
struct F11w {
  float *p[11];
};

// One workgroup of 64 lanes per segment in index order: copies the segment's
// fields and its member points into index order.
__global__ void seg_scatter_kernel(tnn_points pts, int64_t n_seg, const int32_t *perm,
                                   const int32_t *src_start, const int32_t *src_cf,
                                   const int32_t *dst_pstart, F11 src, F11w dst,
                                   int32_t *out_pstart, int32_t *out_pcount, int32_t *out_sorig,
                                   int32_t *out_first, float4 *pt4, int32_t *pid) {
  const int64_t j = blockIdx.x;
  if (j >= n_seg) return;
  const int o = perm[j];
  const int c = src_cf[o] & 0xffff;
  const int p0 = src_start[o];
  const int d0 = dst_pstart[j];
  const int t = threadIdx.x;
  if (t < c) {
    pt4[d0 + t] = make_float4(pts.x[p0 + t], pts.y[p0 + t], pts.z[p0 + t], pts.t[p0 + t]);
    pid[d0 + t] = p0 + t;
  }
  if (t < 11) dst.p[t][j] = src.p[t][o];
  if (t == 0) {
    out_pstart[j] = d0;
    out_pcount[j] = c;
    out_sorig[j] = o;
    out_first[j] = (src_cf[o] >> 16) & 1;
  }
}

// One wavefront per block of 64 segments: bounding box of its points.
__global__ void block_box_kernel(IndexDesc ix, float *box) {
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t s = (int64_t)b * kBlockSegs + lane;
  float lo[4], hi[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    lo[f] = __builtin_huge_valf();
    hi[f] = -__builtin_huge_valf();
  }
  if (s < ix.n_seg) {
    const int ps = ix.pstart[s], pc = ix.pcount[s];
    for (int i = 0; i < pc; ++i) {
      const float4 p = ix.pt4[ps + i];
      const float v[4] = {p.x, p.y, p.z, p.w};
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        lo[f] = fminf(lo[f], v[f]);
        hi[f] = fmaxf(hi[f], v[f]);
      }
    }
  }
#pragma unroll
  for (int f = 0; f < 4; ++f) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
      lo[f] = fminf(lo[f], __shfl_xor(lo[f], m, 64));
      hi[f] = fmaxf(hi[f], __shfl_xor(hi[f], m, 64));
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      box[8 * b + f] = lo[f];
      box[8 * b + 4 + f] = hi[f];
    }
  }
}

__global__ void export_kernel(IndexDesc ix, float *seg_f32, int32_t *seg_i32, int32_t *point_id,
                              float *block_box) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ix.n_seg) {
    if (seg_f32) {
      float *o = seg_f32 + 12 * i;
      o[0] = ix.ax[i];
      o[1] = ix.ay[i];
      o[2] = ix.az[i];
      o[3] = ix.bx[i];
      o[4] = ix.by[i];
      o[5] = ix.bz[i];
      o[6] = ix.tmin[i];
      o[7] = ix.tmax[i];
      o[8] = ix.ex[i];
      o[9] = ix.ey[i];
      o[10] = ix.ez[i];
      o[11] = 0.0f;
    }
    if (seg_i32) {
      int32_t *o = seg_i32 + 4 * i;
      o[0] = ix.sorig[i];
      o[1] = ix.pstart[i];
      o[2] = ix.pcount[i];
      o[3] = (int32_t)(i / kBlockSegs);
    }
  }
  if (point_id && i < ix.n_points) point_id[i] = ix.pid[i];
  if (block_box && i < ix.n_blocks) {
    for (int f = 0; f < 8; ++f) block_box[8 * i + f] = ix.box[8 * i + f];
  }
}

// ---------------------------------------------------------------------------
// kd order on the device, one level per launch and one workgroup per split.
// ---------------------------------------------------------------------------
constexpr int kKdThreads = 1024;
constexpr int kKdWaves = kKdThreads / kWave;

__global__ void iota_kernel(int32_t *perm, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) perm[i] = (int32_t)i;
}

// Unsigned image of a float32 key with the same order (-0 taken as +0, so
// that equal keys compare equal).
__device__ __forceinline__ uint32_t kd_ordered(float v) {
  const uint32_t u = __float_as_uint(v == 0.0f ? 0.0f : v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// A split range [start, start + n) of perm: the widest key axis over the
// range (extent hi - lo, the first of equal extents), the entry of rank m by
// (key on that axis, segment index) found by radix selection over the 64-bit
// (ordered key, index) with 8-bit digits, then a stable partition of the
// range into the entries below it and the rest, staged in tmp and copied
// back.
__global__ __launch_bounds__(kKdThreads) void kd_split_kernel(const float4 *__restrict__ keys,
                                                              int32_t *perm, int32_t *tmp,
                                                              const host::KdSplit *splits) {
  const host::KdSplit sp = splits[blockIdx.x];
  int32_t *r = perm + sp.start;
  int32_t *o = tmp + sp.start;
  const int n = sp.n, m = sp.m;
  const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
  __shared__ float s_ext[kKdWaves][8];
  __shared__ uint32_t s_hist[256];
  __shared__ uint64_t s_pref, s_piv;
  __shared__ int s_rank, s_cnt, s_axis;
  __shared__ int s_wl[kKdWaves], s_wv[kKdWaves];

  // widest axis
  float lo[4], hi[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    lo[f] = __builtin_huge_valf();
    hi[f] = -__builtin_huge_valf();
  }
  for (int i = t; i < n; i += kKdThreads) {
    const float4 k = keys[r[i]];
    const float v[4] = {k.x, k.y, k.z, k.w};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      lo[f] = fminf(lo[f], v[f]);
      hi[f] = fmaxf(hi[f], v[f]);
    }
  }
#pragma unroll
  for (int f = 0; f < 4; ++f)
    for (int off = kWave / 2; off > 0; off >>= 1) {
      lo[f] = fminf(lo[f], __shfl_xor(lo[f], off));
      hi[f] = fmaxf(hi[f], __shfl_xor(hi[f], off));
    }
  if (lane == 0)
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      s_ext[w][f] = lo[f];
      s_ext[w][4 + f] = hi[f];
    }
  __syncthreads();
  if (t == 0) {
    float l[4], h[4];
    for (int f = 0; f < 4; ++f) {
      l[f] = s_ext[0][f];
      h[f] = s_ext[0][4 + f];
      for (int x = 1; x < kKdWaves; ++x) {
        l[f] = fminf(l[f], s_ext[x][f]);
        h[f] = fmaxf(h[f], s_ext[x][4 + f]);
      }
    }
    int axis = 0;
    for (int f = 1; f < 4; ++f)
      if (h[f] - l[f] > h[axis] - l[axis]) axis = f;
    s_axis = axis;
    s_pref = 0;
    s_rank = m;
  }
  __syncthreads();
  const int axis = s_axis;
  auto composite = [&](int i, int32_t *id_out) -> uint64_t {
    const int32_t id = r[i];
    const float4 k = keys[id];
    const float v = axis == 0 ? k.x : axis == 1 ? k.y : axis == 2 ? k.z : k.w;
    *id_out = id;
    return ((uint64_t)kd_ordered(v) << 32) | (uint32_t)id;
  };

  // the entry of rank m: digits from the top until one candidate is left
  // (the composites are distinct, so at the latest after the last digit)
  uint64_t mask = 0;
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    for (int b = t; b < 256; b += kKdThreads) s_hist[b] = 0;
    __syncthreads();
    const uint64_t pref = s_pref;
    for (int i = t; i < n; i += kKdThreads) {
      int32_t id;
      const uint64_t c = composite(i, &id);
      if ((c & mask) == pref) atomicAdd(&s_hist[(c >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (t == 0) {
      const uint32_t rank = (uint32_t)s_rank;
      uint32_t cum = 0;
      int d = 0;
      while (d < 255 && rank >= cum + s_hist[d]) cum += s_hist[d++];
      s_rank = (int)(rank - cum);
      s_pref = pref | ((uint64_t)d << shift);
      s_cnt = (int)s_hist[d];
    }
    __syncthreads();
    mask |= (uint64_t)255 << shift;
    if (s_cnt <= 1) break;
  }
  {
    const uint64_t pref = s_pref;
    if (t == 0) s_piv = pref;  // all digits fixed, or overwritten below
    __syncthreads();
    for (int i = t; i < n; i += kKdThreads) {
      int32_t id;
      const uint64_t c = composite(i, &id);
      if ((c & mask) == pref) s_piv = c;
    }
    __syncthreads();
  }
  const uint64_t pivot = s_piv;

  // stable partition: entries below the pivot to o[0, m), the rest to
  // o[m, n), each in range order, chunk by chunk
  int nl = 0, nr = 0;
  for (int base = 0; base < n; base += kKdThreads) {
    const int i = base + t;
    const bool valid = i < n;
    int32_t id = 0;
    bool left = false;
    if (valid) left = composite(i, &id) < pivot;
    const uint64_t bl = ballot(left), bv = ballot(valid);
    if (lane == 0) {
      s_wl[w] = __popcll(bl);
      s_wv[w] = __popcll(bv);
    }
    __syncthreads();
    int offl = 0, offv = 0, totl = 0, totv = 0;
    for (int x = 0; x < kKdWaves; ++x) {
      if (x < w) {
        offl += s_wl[x];
        offv += s_wv[x];
      }
      totl += s_wl[x];
      totv += s_wv[x];
    }
    if (valid) {
      if (left) {
        const uint64_t below = bl & ((1ull << lane) - 1ull);
        o[nl + offl + __popcll(below)] = id;
      } else {
        const uint64_t below = (bv & ~bl) & ((1ull << lane) - 1ull);
        o[m + nr + (offv - offl) + __popcll(below)] = id;
      }
    }
    nl += totl;
    nr += totv - totl;
    __syncthreads();
  }
  for (int i = t; i < n; i += kKdThreads) r[i] = o[i];
}

// Inside every block of the kd order (kBlockSegs entries, the last one
// shorter) the splits go on down to single entries: a range of n >= 2
// entries splits along its widest axis into its n/2 smallest (by key, ties
// by segment index) and the rest, each part keeping its order.  One wave per
// block, lane = position; per level each lane finds its range, the range's
// extents and its own rank in it by reading every lane, and moves to its new
// position through LDS.
__global__ __launch_bounds__(kWave) void kd_leaf_kernel(const float4 *__restrict__ keys,
                                                        int32_t *perm, int64_t n_seg) {
  __shared__ int32_t s_id[kWave];
  const int64_t b0 = (int64_t)blockIdx.x * kBlockSegs;
  const int lane = lane_id();
  const int n = (int)(n_seg - b0 < kBlockSegs ? n_seg - b0 : kBlockSegs);
  const bool ok = lane < n;
  int32_t id = ok ? perm[b0 + lane] : 0;
  for (int level = 0; (1 << level) < n; ++level) {
    // this lane's range at this level: descend from [0, n)
    int rs = 0, rn = n;
    for (int d = 0; d < level; ++d) {
      const int m = rn / 2;
      if (lane < rs + m) {
        rn = m;
      } else {
        rs += m;
        rn -= m;
      }
    }
    const float4 k = ok ? keys[id] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const bool in_split = ok && rn >= 2;
    // extents of the lane's range
    float lo[4], hi[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      lo[f] = __builtin_huge_valf();
      hi[f] = -__builtin_huge_valf();
    }
    for (int j = 0; j < n; ++j) {
      const float kx = __shfl(k.x, j), ky = __shfl(k.y, j), kz = __shfl(k.z, j),
                  kw = __shfl(k.w, j);
      if (j >= rs && j < rs + rn) {
        lo[0] = fminf(lo[0], kx);
        hi[0] = fmaxf(hi[0], kx);
        lo[1] = fminf(lo[1], ky);
        hi[1] = fmaxf(hi[1], ky);
        lo[2] = fminf(lo[2], kz);
        hi[2] = fmaxf(hi[2], kz);
        lo[3] = fminf(lo[3], kw);
        hi[3] = fmaxf(hi[3], kw);
      }
    }
    int axis = 0;
#pragma unroll
    for (int f = 1; f < 4; ++f)
      if (hi[f] - lo[f] > hi[axis] - lo[axis]) axis = f;
    const float key = axis == 0 ? k.x : axis == 1 ? k.y : axis == 2 ? k.z : k.w;
    const uint64_t c = ((uint64_t)kd_ordered(key) << 32) | (uint32_t)id;
    // rank in the range (axes may differ between ranges: each lane compares
    // within its own range, where every lane took the same axis)
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const uint32_t hj = (uint32_t)__shfl((int)(uint32_t)(c >> 32), j);
      const uint32_t lj = (uint32_t)__shfl((int)(uint32_t)c, j);
      if (j >= rs && j < rs + rn && (((uint64_t)hj << 32) | lj) < c) ++rank;
    }
    const int m = rn / 2;
    const bool left = in_split && rank < m;
    const uint64_t bl = ballot(left);
    // position: the range's lefts first, then the rest, each in lane order
    const uint64_t below = ((1ull << lane) - 1ull) & ~((1ull << rs) - 1ull);
    const int lefts_before = __popcll(bl & below);
    const int pos = !in_split ? lane
                    : left    ? rs + lefts_before
                              : rs + m + (lane - rs - lefts_before);
    if (ok) s_id[pos] = id;
    wave_sync();
    id = ok ? s_id[lane] : 0;
    wave_sync();
  }
  if (ok) perm[b0 + lane] = id;
}

// One workgroup: each thread sums a contiguous run of the counts, the run
// sums are scanned in LDS, then each thread writes its run's offsets.
__global__ __launch_bounds__(1024) void point_offsets_kernel(const int32_t *perm,
                                                             const int32_t *cnt_flags,
                                                             int64_t n_seg, int32_t *dpstart) {
  __shared__ int64_t s[1024];
  const int t = threadIdx.x;
  const int64_t per = (n_seg + 1023) / 1024;
  const int64_t b0 = t * per < n_seg ? t * per : n_seg;
  const int64_t b1 = b0 + per < n_seg ? b0 + per : n_seg;
  int64_t sum = 0;
  for (int64_t i = b0; i < b1; ++i) sum += cnt_flags[perm[i]] & 0xffff;
  s[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  int64_t acc = s[t] - sum;
  for (int64_t i = b0; i < b1; ++i) {
    dpstart[i] = (int32_t)acc;
    acc += cnt_flags[perm[i]] & 0xffff;
  }
}

hipError_t launch_iota(int32_t *perm, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(iota_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, perm, n);
  return hipGetLastError();
}

hipError_t launch_kd_level(const float *keys, int32_t *perm, int32_t *tmp,
                           const host::KdSplit *splits, int64_t n_splits, hipStream_t st) {
  if (n_splits == 0) return hipSuccess;
  hipLaunchKernelGGL(kd_split_kernel, dim3((unsigned)n_splits), dim3(kKdThreads), 0, st,
                     reinterpret_cast<const float4 *>(keys), perm, tmp, splits);
  return hipGetLastError();
}

hipError_t launch_kd_leaves(const float *keys, int32_t *perm, int64_t n_seg, hipStream_t st) {
  if (n_seg == 0) return hipSuccess;
  hipLaunchKernelGGL(kd_leaf_kernel, dim3((unsigned)((n_seg + kBlockSegs - 1) / kBlockSegs)),
                     dim3(kWave), 0, st, reinterpret_cast<const float4 *>(keys), perm, n_seg);
  return hipGetLastError();
}

hipError_t launch_point_offsets(const int32_t *perm, const int32_t *cnt_flags, int64_t n_seg,
                                int32_t *dpstart, hipStream_t st) {
  if (n_seg == 0) return hipSuccess;
  hipLaunchKernelGGL(point_offsets_kernel, dim3(1), dim3(1024), 0, st, perm, cnt_flags, n_seg,
                     dpstart);
  return hipGetLastError();
}

hipError_t launch_seg_stats(const tnn_points &pts, const int32_t *start, const int32_t *cnt_flags,
                            int64_t n_seg, const float *osc, float *ax, float *ay, float *az,
                            float *bx, float *by, float *bz, float *tmin, float *tmax, float *ex,
                            float *ey, float *ez, float *keys, uint32_t *status, hipStream_t st) {
  if (n_seg == 0) return hipSuccess;
  const int tpb = 256;
  hipLaunchKernelGGL(seg_stats_kernel, dim3((unsigned)((n_seg + tpb - 1) / tpb)), dim3(tpb), 0, st,
                     pts, start, cnt_flags, n_seg, osc, ax, ay, az, bx, by, bz, tmin, tmax, ex, ey,
                     ez, keys, status);
  return hipGetLastError();
}

hipError_t launch_seg_scatter(const tnn_points &pts, int64_t n_seg, const int32_t *perm,
                              const int32_t *src_start, const int32_t *src_cnt_flags,
                              const int32_t *dst_pstart, const float *const src_f[11],
                              float *const dst_f[11], int32_t *dst_pstart_out, int32_t *dst_pcount,
                              int32_t *dst_sorig, int32_t *dst_first, float4 *pt4, int32_t *pid,
                              hipStream_t st) {
  if (n_seg == 0) return hipSuccess;
  F11 src;
  F11w dst;
  for (int i = 0; i < 11; ++i) {
    src.p[i] = src_f[i];
    dst.p[i] = dst_f[i];
  }
  hipLaunchKernelGGL(seg_scatter_kernel, dim3((unsigned)n_seg), dim3(kWave), 0, st, pts, n_seg, perm,
                     src_start, src_cnt_flags, dst_pstart, src, dst, dst_pstart_out, dst_pcount,
                     dst_sorig, dst_first, pt4, pid);
  return hipGetLastError();
}

hipError_t launch_block_box(const IndexDesc &ix, float *box, hipStream_t st) {
  if (ix.n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(block_box_kernel, dim3((unsigned)ix.n_blocks), dim3(kWave), 0, st, ix, box);
  return hipGetLastError();
}

hipError_t launch_export(const IndexDesc &ix, float *seg_f32, int32_t *seg_i32, int32_t *point_id,
                         float *block_box, hipStream_t st) {
  int64_t n = ix.n_seg;
  if (ix.n_points > n) n = ix.n_points;
  if (ix.n_blocks > n) n = ix.n_blocks;
  if (n == 0) return hipSuccess;
  const int tpb = 256;
  hipLaunchKernelGGL(export_kernel, dim3((unsigned)((n + tpb - 1) / tpb)), dim3(tpb), 0, st, ix,
                     seg_f32, seg_i32, point_id, block_box);
  return hipGetLastError();
}

}  // namespace tnn
