// Linear search with BF16 matrix-core distance tiles (TNN_BRUTE |
// TNN_MIXED_BF16).  Not in the paper: the all-pairs distance of Sec. 3.6's
// linear search runs on MFMA as a proven lower-bound filter, and every pair
// that passes it is rescored with the binary64 formula before the top-k, so
// the result is identical to the exact linear search.
//
// Distance as a matrix product.  With v_f = sqrt(s_f) (p_f - c_f) and
// u_f = sqrt(s_f) (q_f - c_f) (c = centre of the data box),
//     d(q, p) = |u|^2 + |v|^2 - 2 u.v .
// Each coordinate is split into three bfloat16 terms (h + m + l carries 24
// bits) and the six products that matter (hh, hm, mh, hl, mm, lh) fill 24 of
// the 32 K-slots of v_mfma_f32_16x16x32_bf16; the norms, pre-scaled by
// (1 - gamma) and split the same way, fill six more.  The tile value is then
//     c' = (1 - gamma)(|u|^2 + |v|^2) - 2 u.v  <=  d(q, p)
// because the split, the float32 accumulation of 32 terms and the float32
// inputs err by at most 1.6 * 2^-18 (|u|^2 + |v|^2), below gamma = 2^-16.
#include "bounds.h"
#include "query.h"

namespace tnn {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr float kGamma = 0x1p-16f;
constexpr int kMQ = 16;      // queries per wave (MFMA rows)
constexpr int kStep = 64;    // points per step (four 16-column MFMA tiles)

__device__ __forceinline__ __bf16 to_bf16(float x) {
  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  const unsigned short h = (unsigned short)(u >> 16);
  return __builtin_bit_cast(__bf16, h);
}

__device__ __forceinline__ float from_bf16(__bf16 b) {
  const unsigned short h = __builtin_bit_cast(unsigned short, b);
  return __uint_as_float((uint32_t)h << 16);
}

__device__ __forceinline__ void split3(float x, __bf16 &h, __bf16 &m, __bf16 &l) {
  h = to_bf16(x);
  const float r1 = x - from_bf16(h);
  m = to_bf16(r1);
  const float r2 = r1 - from_bf16(m);
  l = to_bf16(r2);
}

struct MixedCtx {
  float c[4];   // centre
  float sq[4];  // sqrt of the scales
};

// Scaled, centred coordinates and their squared norm.
__device__ __forceinline__ float scaled(const MixedCtx &mc, float x, float y, float z, float t,
                                        float u[4]) {
  const float v[4] = {x, y, z, t};
  float n = 0.0f;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    u[f] = mc.sq[f] * (v[f] - mc.c[f]);
    n += u[f] * u[f];
  }
  return n;
}

// B operand (point side) for K-group g (lanes 16g..16g+15 supply slots
// 8g..8g+7): see the slot table in the file comment.
__device__ __forceinline__ bf16x8 point_group(const float v[4], float nvs, int g) {
  __bf16 h[4], m[4], l[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) split3(v[f], h[f], m[f], l[f]);
  bf16x8 o;
  const __bf16 one = to_bf16(1.0f), zero = to_bf16(0.0f);
  if (g == 0) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      o[f] = to_bf16(-2.0f * from_bf16(h[f]));
      o[4 + f] = to_bf16(-2.0f * from_bf16(m[f]));
    }
  } else if (g == 1) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      o[f] = to_bf16(-2.0f * from_bf16(h[f]));
      o[4 + f] = to_bf16(-2.0f * from_bf16(l[f]));
    }
  } else if (g == 2) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      o[f] = to_bf16(-2.0f * from_bf16(m[f]));
      o[4 + f] = to_bf16(-2.0f * from_bf16(h[f]));
    }
  } else {
    __bf16 nh, nm, nl;
    split3(nvs, nh, nm, nl);
    o[0] = one;
    o[1] = one;
    o[2] = one;
    o[3] = nh;
    o[4] = nm;
    o[5] = nl;
    o[6] = zero;
    o[7] = zero;
  }
  return o;
}

// A operand (query side), paired slot by slot with point_group.
__device__ __forceinline__ bf16x8 query_group(const float u[4], float nus, int g) {
  __bf16 h[4], m[4], l[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) split3(u[f], h[f], m[f], l[f]);
  bf16x8 o;
  const __bf16 one = to_bf16(1.0f), zero = to_bf16(0.0f);
  if (g == 0) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      o[f] = h[f];
      o[4 + f] = h[f];
    }
  } else if (g == 1) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      o[f] = m[f];
      o[4 + f] = h[f];
    }
  } else if (g == 2) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      o[f] = m[f];
      o[4 + f] = l[f];
    }
  } else {
    __bf16 nh, nm, nl;
    split3(nus, nh, nm, nl);
    o[0] = nh;
    o[1] = nm;
    o[2] = nl;
    o[3] = one;
    o[4] = one;
    o[5] = one;
    o[6] = zero;
    o[7] = zero;
  }
  return o;
}

// Per call: the point operands in index order (4 groups of 8 bf16 per
// point, 64 bytes), |v|^2 and a copy of the times (read densely by the
// distance tiles).
__global__ void mixed_prep_kernel(IndexDesc ix, MixedCtx mc, bf16x8 *ops, float *nv, float *tv) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ix.n_points) return;
  float v[4];
  const float4 pv = ix.pt4[p];
  tv[p] = pv.w;
  const float n = scaled(mc, pv.x, pv.y, pv.z, pv.w, v);
  const float ns = (1.0f - kGamma) * n;
#pragma unroll
  for (int g = 0; g < 4; ++g) ops[4 * p + g] = point_group(v, ns, g);
  nv[p] = n;
}

__device__ __forceinline__ float round_up_f(double x) {
  return x < kInf ? __double2float_ru(x) : __builtin_huge_valf();
}

// One wavefront = one workgroup answers 16 queries (the MFMA rows).  Point
// operands stream straight from global memory (64 points per step, four
// 16-column MFMA tiles); no workgroup barrier is needed.  Per-query state in
// LDS: the top-k (k entries) and a candidate queue of one step's points.
__global__ __launch_bounds__(64) void mixed_brute_kernel(
    IndexDesc ix, QueryArgs a, MixedCtx mc, const bf16x8 *ops, const float *nv, const float *tv,
    const float *qxp,
    const float *qyp, const float *qzp, const float *qtp, int64_t nq, int32_t *out_idx,
    double *out_dist, int64_t tile_stride) {
  extern __shared__ double s_dyn[];
  const int k = a.k;
  double *s_tkd = s_dyn;                                            // [kMQ][k]
  int *s_tkid = reinterpret_cast<int *>(s_tkd + kMQ * k);           // [kMQ][k]
  int *s_qp = s_tkid + kMQ * k;                                     // [kMQ][kStep]
  float *s_qc = reinterpret_cast<float *>(s_qp + kMQ * kStep);      // [kMQ][kStep]
  int *s_qn = reinterpret_cast<int *>(s_qc + kMQ * kStep);          // [kMQ]
  float *s_tau = reinterpret_cast<float *>(s_qn + kMQ);             // [kMQ]
  float *s_thr = s_tau + kMQ;                                       // [kMQ]
  float *s_nu = s_thr + kMQ;                                        // [kMQ]

  const int lane = lane_id();
  const int64_t qbase = (int64_t)blockIdx.x * kMQ;
  const int g = lane >> 4;    // K-group this lane supplies
  const int row = lane & 15;  // A row (query) / C column (point)
  const int64_t qa = qbase + row;
  float u[4] = {0, 0, 0, 0};
  float nu = 0.0f;
  if (qa < nq) nu = scaled(mc, qxp[qa], qyp[qa], qzp[qa], qtp[qa], u);
  const bf16x8 aop = query_group(u, (1.0f - kGamma) * nu, g);
  if (lane < kMQ) {
    const int64_t q = qbase + lane;
    s_qn[lane] = 0;
    s_nu[lane] = nu;
    if (q < nq) {
      s_tau[lane] = __builtin_huge_valf();
      s_thr[lane] = round_up_f((double)qtp[q] - a.t_window);
    } else {
      s_tau[lane] = -__builtin_huge_valf();  // inactive row: nothing passes
      s_thr[lane] = -__builtin_huge_valf();
    }
  }
  for (int i = lane; i < kMQ * k; i += 64) {
    s_tkd[i] = a.inf;
    s_tkid[i] = kNoId;
  }
  __syncthreads();
  uint32_t rescored = 0;
  double max_err = 0.0;
  const int64_t n = ix.n_points;
  const int64_t n_steps = (n + kStep - 1) / kStep;
  float tau[4], thr[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    tau[e] = s_tau[g * 4 + e];
    thr[e] = s_thr[g * 4 + e];
  }
  for (int64_t si = 0; si < n_steps; ++si) {
    // Steps in a scattered order: index order is spatially sorted, and a
    // scan that approaches the query gradually would improve the k-th
    // distance at almost every point, sending nearly all of them to the
    // binary64 rescoring.  tile_stride is coprime with n_steps.
    const int64_t p0 = (int64_t)(((unsigned long long)si * (unsigned long long)tile_stride) %
                                 (unsigned long long)n_steps) * kStep;
    bf16x8 bop[kStep / 16];
    float pts[kStep / 16];
#pragma unroll
    for (int cb = 0; cb < kStep / 16; ++cb) {
      const int64_t p = p0 + cb * 16 + row;
      bf16x8 v = {};
      float t = __builtin_huge_valf();
      if (p < n) {
        v = ops[4 * p + g];
        t = tv[p];
      }
      bop[cb] = v;
      pts[cb] = t;
    }
    bool any = false;
#pragma unroll
    for (int cb = 0; cb < kStep / 16; ++cb) {
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop[cb], acc, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // row (query) g*4+e, column (point) cb*16 + row; the point's time is
        // held by the lane that loaded column `row`, i.e. this lane
        if ((acc[e] <= tau[e]) & (pts[cb] < thr[e])) {
          const int m = g * 4 + e;
          const int slot = atomicAdd(&s_qn[m], 1);
          s_qp[m * kStep + slot] = (int)(p0 + cb * 16 + row);
          s_qc[m * kStep + slot] = acc[e];
          any = true;
        }
      }
    }
    if (!ballot(any)) continue;
    // ---- rescore survivors in binary64 and merge them into each top-k
    for (int m = 0; m < kMQ; ++m) {
      const int cnt = s_qn[m];
      const int64_t q = qbase + m;
      if (cnt == 0 || q >= nq) continue;
      const QueryPoint qp = make_query(qxp[q], qyp[q], qzp[q], qtp[q], a.t_window);
      const bool has = lane < cnt;
      const int p = has ? s_qp[m * kStep + lane] : 0;
      double d = a.inf;
      int pid = kNoId;
      bool valid = false;
      if (has) {
        const float4 pv = ix.pt4[p];
        const float pt = pv.w;
        d = exact_dist(a.s, qp.x, qp.y, qp.z, qp.t, pv.x, pv.y, pv.z, pt);
        pid = ix.pid[p];
        valid = (double)pt < qp.thr;
        const double approx = (double)s_qc[m * kStep + lane] +
                              (double)kGamma * ((double)s_nu[m] + (double)nv[p]);
        max_err = fmax(max_err, fabs(approx - d));
      }
      rescored += (uint32_t)cnt;
      TopK tk;
      tk.init(k, a.inf);
      if (lane < k) {
        tk.d = s_tkd[m * k + lane];
        tk.id = s_tkid[m * k + lane];
      }
      tk.refresh();
      const bool gate = valid && tk.admits(d, pid);
      const uint64_t gm = ballot(gate);
      if (gm) {
        tk.offer(gm, gate, d, pid);
        if (lane < k) {
          s_tkd[m * k + lane] = tk.d;
          s_tkid[m * k + lane] = tk.id;
        }
        if (lane == 0) s_tau[m] = round_up_f(tk.kd);
      }
      if (lane == 0) s_qn[m] = 0;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) tau[e] = s_tau[g * 4 + e];
  }
  for (int m = 0; m < kMQ; ++m) {
    const int64_t q = qbase + m;
    if (q < nq && lane < k) {
      const int id = s_tkid[m * k + lane];
      out_idx[q * k + lane] = id == kNoId ? -1 : id;
      out_dist[q * k + lane] = s_tkd[m * k + lane];
    }
  }
  if (a.stats) {
    for (int o = 32; o > 0; o >>= 1) max_err = fmax(max_err, __shfl_xor(max_err, o, 64));
    if (lane == 0) {
      int64_t nvalid = nq - qbase;
      nvalid = nvalid < 0 ? 0 : (nvalid > kMQ ? kMQ : nvalid);
      atomicAdd(a.stats + TNN_STAT_QUERIES, (unsigned long long)nvalid);
      atomicAdd(a.stats + TNN_STAT_POINTS, (unsigned long long)(nvalid * n));
      atomicAdd(a.stats + TNN_STAT_RESCORED, (unsigned long long)rescored);
      atomicMax(a.stats + TNN_STAT_MAX_ERR, (unsigned long long)__double_as_longlong(max_err));
    }
  }
}

}  // namespace

size_t mixed_scratch_bytes(int64_t n_points) {
  return align_up((size_t)n_points * 64) + 2 * align_up((size_t)n_points * 4);
}

MixedCtx make_ctx(const IndexDesc &ix, const QueryArgs &a) {
  MixedCtx mc;
  for (int f = 0; f < 4; ++f) {
    mc.c[f] = 0.5f * (ix.lo[f] + ix.hi[f]);
    mc.sq[f] = (float)sqrt(a.s[f]);
  }
  return mc;
}

hipError_t launch_mixed_brute(const IndexDesc &ix, const QueryArgs &a, const tnn_points &qs,
                              int32_t *out_idx, double *out_dist, void *scratch, hipStream_t st) {
  if (qs.n == 0) return hipSuccess;
  const MixedCtx mc = make_ctx(ix, a);
  bf16x8 *ops = static_cast<bf16x8 *>(scratch);
  float *nv = reinterpret_cast<float *>(static_cast<char *>(scratch) +
                                        align_up((size_t)ix.n_points * 64));
  float *tv = reinterpret_cast<float *>(reinterpret_cast<char *>(nv) +
                                        align_up((size_t)ix.n_points * 4));
  if (ix.n_points > 0) {
    hipLaunchKernelGGL(mixed_prep_kernel, dim3((unsigned)((ix.n_points + 255) / 256)), dim3(256), 0,
                       st, ix, mc, ops, nv, tv);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t n_steps = (ix.n_points + kStep - 1) / kStep;
  int64_t stride = 1;
  if (n_steps > 2) {
    auto gcd = [](int64_t x, int64_t y) {
      while (y) {
        const int64_t r = x % y;
        x = y;
        y = r;
      }
      return x;
    };
    stride = (int64_t)(0.6180339887 * (double)n_steps) | 1;
    while (gcd(stride, n_steps) != 1) stride += 2;
  }
  const size_t lds = (size_t)kMQ * a.k * 12 + (size_t)kMQ * kStep * 8 + (size_t)kMQ * 16;
  hipLaunchKernelGGL(mixed_brute_kernel, dim3((unsigned)((qs.n + kMQ - 1) / kMQ)), dim3(64), lds,
                     st, ix, a, mc, ops, nv, tv, qs.x, qs.y, qs.z, qs.t, qs.n, out_idx, out_dist,
                     stride);
  return hipGetLastError();
}

}  // namespace tnn
