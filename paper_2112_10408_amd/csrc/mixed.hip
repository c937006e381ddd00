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
#include <mutex>

#include "bounds.h"
#include "query.h"

namespace tnn {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr float kGamma = 0x1p-16f;
// Largest scaled squared norm |u|^2 of a point or query the float32 tiles
// take: tile values then stay below 4e30, far from float32 overflow.
constexpr float kMaxNorm = (float)kMaxScaledNorm;
constexpr int kWaves = 4;                 // waves per workgroup
constexpr int kMQ = 16;                   // queries per wave (the MFMA rows)
constexpr int kTileQ = kWaves * kMQ;      // queries per work item
constexpr int kStage = 128;               // points per LDS stage
constexpr int kStageTiles = kStage / 16;  // 16-column MFMA tiles per stage
constexpr int kQCap = 64;                 // queued survivors per wave (one row of a tile)
constexpr int kBatch = 4;                 // tiles whose reads and MFMAs are issued together
constexpr int kMaxChunks = 8;             // point chunks per query tile
// Workgroups resident on a full chip, nominally (256 CUs x 3): only sets
// how finely the points are chunked, so the workspace size does not depend
// on the device.
constexpr int64_t kNominalSlots = 768;

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

// Per call: the point operands and |v|^2.  Operands are stored tile-major:
// the 16-byte group g of point p sits at unit (p / 16 * 4 + g) * 16 + p % 16,
// so a 16-point MFMA tile is 1 KB laid out lane by lane and a stage is one
// contiguous block.  Operands are padded to whole stages with zeros.
__global__ void mixed_prep_kernel(IndexDesc ix, MixedCtx mc, bf16x8 *ops, float *nv,
                                  int64_t n_pad) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pad) return;
  const int64_t unit0 = (p >> 4) * 64 + (p & 15);
  if (p >= ix.n_points) {
#pragma unroll
    for (int g = 0; g < 4; ++g) ops[unit0 + 16 * g] = bf16x8{};
    return;
  }
  float v[4];
  const float4 pv = ix.pt4[p];
  const float n = scaled(mc, pv.x, pv.y, pv.z, pv.w, v);
  const float ns = (1.0f - kGamma) * n;
#pragma unroll
  for (int g = 0; g < 4; ++g) ops[unit0 + 16 * g] = point_group(v, ns, g);
  nv[p] = n;
}

// Per call: no chunk has a k-th distance yet; the work counter starts at 0.
__global__ void mixed_reset_kernel(float *part_kd, int64_t n, unsigned long long *counter) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) part_kd[i] = __builtin_huge_valf();
  if (i == 0) *counter = 0;
}

__device__ __forceinline__ float round_up_f(double x) {
  return x < kInf ? __double2float_ru(x) : __builtin_huge_valf();
}

// What only the rescoring needs, parked in LDS so that the scan loop keeps
// few scalar registers live.
struct SlowArgs {
  double s[4];
  double t_window;
  double inf;
  const float *nv;
  unsigned long long *stats;
  int k;
};

// LDS stage buffer: the operands of kStage points (tile-major), their
// coordinates and their caller indices.
struct Stage {
  bf16x8 op[kStage * 4];
  float4 pt[kStage];
  int pid[kStage];
};

// Work item = (query tile of kTileQ queries, chunk of the point stages).
// A persistent grid of 4-wave workgroups takes items from a counter, chunk
// by chunk.  The workgroup streams the chunk's stages through two LDS
// buffers (loaded by all 256 lanes, one stage ahead), and each wave answers
// its 16 queries against every stage: a tile whose values all exceed their
// queries' bounds costs one LDS read, one MFMA and four compares per lane.
// For the others the survivors (bound and time mask passed) go to the wave's
// queue (slots from ballots), which is rescored in binary64 from the staged
// coordinates (one lane per survivor) and merged into each query's top-k.
// That top-k is kept in place in the chunk's list in global memory (L2
// resident while the item runs): LDS holds only the stages, so four
// workgroups fit on a CU.  A query's bound starts at the least k-th distance
// among the chunks of its tile already finished (each is an upper bound on
// the final k-th distance), and mixed_merge_kernel combines the chunk lists.
__global__ __launch_bounds__(kWaves * 64) void mixed_brute_kernel(
    IndexDesc ix, QueryArgs a, MixedCtx mc, const bf16x8 *ops, const float *nv, const float *qxp,
    const float *qyp, const float *qzp, const float *qtp, int64_t nq, double *part_d,
    int32_t *part_i, float *part_kd, unsigned long long *counter, int64_t n_tiles, int n_chunks,
    int64_t n_steps, int64_t tile_stride) {
  // 16-byte aligned: the stage buffers are read with 16-byte LDS loads
  extern __shared__ float4 s_dyn4[];
  __shared__ SlowArgs s_a;
  __shared__ long long s_item;
  __shared__ float4 s_q[kWaves][kMQ];   // query coordinates (x, y, z, t)
  __shared__ float s_tau[kWaves][kMQ];  // bound on the top-k's k-th distance, rounded up
  __shared__ float s_nu[kWaves][kMQ];   // |u|^2 of each query
  __shared__ int s_qp[kWaves][kQCap];   // queued survivor: index in the stage
  __shared__ float s_qc[kWaves][kQCap];  //                 its tile value
  __shared__ unsigned char s_qm[kWaves][kQCap];  //         its query row
  const int k = a.k;
  const int lane = lane_id();
  const int wave = (int)(threadIdx.x >> 6);
  const int tid = (int)threadIdx.x;
  const int g = lane >> 4;    // K-group this lane supplies
  const int row = lane & 15;  // A row (query) / C column (point)
  // dynamic LDS: the two stages
  Stage *s_stage = reinterpret_cast<Stage *>(s_dyn4);
  if (tid == 0) {
    for (int f = 0; f < 4; ++f) s_a.s[f] = a.s[f];
    s_a.t_window = a.t_window;
    s_a.inf = a.inf;
    s_a.nv = nv;
    s_a.stats = a.stats;
    s_a.k = k;
  }
  const int64_t n_real = ix.n_points;
  uint32_t rescored = 0;
  double max_err = 0.0;
  int64_t queries_done = 0;
  // The current item's top-k of query row m lives in place in its chunk list
  // (in the L2 while the item runs): tkd_base[m * tk_stride + rank].
  double *tkd_base = part_d;
  int *tkid_base = part_i;
  int64_t tk_stride = k;

  // Rescore the wave's queued survivors (stage `st`, first point p0) in
  // binary64, one lane each, and merge them query by query.
  auto flush = [&](int queued, const Stage *st, int64_t p0) {
    const int kk = __builtin_amdgcn_readfirstlane(s_a.k);
    double sc[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) sc[f] = s_a.s[f];
    const double tw = s_a.t_window, inf = s_a.inf;
    const bool want_err = s_a.stats != nullptr;
    const bool has = lane < queued;
    int mi = -1;
    double d = inf;
    int pid = kNoId;
    bool valid = false;
    if (has) {
      mi = s_qm[wave][lane];
      const int j = s_qp[wave][lane];
      const float4 qv = s_q[wave][mi];
      const QueryPoint qp = make_query(qv.x, qv.y, qv.z, qv.w, tw);
      const float4 pv = st->pt[j];
      d = exact_dist(sc, qp.x, qp.y, qp.z, qp.t, pv.x, pv.y, pv.z, pv.w);
      pid = st->pid[j];
      valid = (double)pv.w < qp.thr;
      if (want_err) {
        const double approx = (double)s_qc[wave][lane] +
                              (double)kGamma * ((double)s_nu[wave][mi] + (double)s_a.nv[p0 + j]);
        max_err = fmax(max_err, fabs(approx - d));
      }
    }
    uint64_t pending = ballot(has);
    while (pending) {
      const int m = __builtin_amdgcn_readlane(mi, __ffsll((long long)pending) - 1);
      const bool mine = has && mi == m;
      pending &= ~ballot(mine);
      TopK tk;
      tk.init(kk, inf);
      if (lane < kk) {
        tk.d = tkd_base[m * tk_stride + lane];
        tk.id = tkid_base[m * tk_stride + lane];
      }
      tk.refresh();
      const bool gate = mine && valid && tk.admits(d, pid);
      const uint64_t gm = ballot(gate);
      if (gm) {
        tk.offer(gm, d, pid);
        if (lane < kk) {
          tkd_base[m * tk_stride + lane] = tk.d;
          tkid_base[m * tk_stride + lane] = tk.id;
        }
        if (lane == 0) s_tau[wave][m] = round_up_f(tk.kd);
      }
    }
    rescored += (uint32_t)queued;
  };

  const int64_t n_items = n_tiles * n_chunks;
  for (;;) {
    if (tid == 0) s_item = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const long long item = s_item;
    if (item >= n_items) break;
    const int chunk = (int)(item / n_tiles);
    const int64_t qbase = (item % n_tiles) * kTileQ + wave * kMQ;

    // ---- this wave's queries: A operands, bounds, time thresholds
    float tau[4], thr[4];
    bf16x8 aop;
    {
      const int64_t qa = qbase + row;
      float u[4] = {0, 0, 0, 0};
      float nu = 0.0f;
      if (qa < nq) nu = scaled(mc, qxp[qa], qyp[qa], qzp[qa], qtp[qa], u);
      aop = query_group(u, (1.0f - kGamma) * nu, g);
      if (g == 0) s_nu[wave][row] = nu;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t q = qbase + g * 4 + e;
      float t = -__builtin_huge_valf();  // an inactive row lets nothing pass
      float h = -__builtin_huge_valf();
      // a query too far out for the float32 tiles takes no part (its rows
      // are reported as (-1, NaN) by the merge)
      if (q < nq && s_nu[wave][g * 4 + e] < kMaxNorm) {
        t = __builtin_huge_valf();
        for (int c = 0; c < n_chunks; ++c)
          if (c != chunk) t = fminf(t, part_kd[q * n_chunks + c]);
        h = round_up_f((double)qtp[q] - a.t_window);
      }
      tau[e] = t;
      thr[e] = h;
    }
    if (lane < kMQ) {
      const int64_t q = qbase + lane;
      s_q[wave][lane] = q < nq ? make_float4(qxp[q], qyp[q], qzp[q], qtp[q]) : make_float4(0, 0, 0, 0);
      // NaN marks a query outside the tiles' range in its chunk bound
      s_tau[wave][lane] = s_nu[wave][lane] < kMaxNorm ? __builtin_huge_valf() : __builtin_nanf("");
    }
    tk_stride = (int64_t)n_chunks * k;
    tkd_base = part_d + ((size_t)qbase * n_chunks + chunk) * k;
    tkid_base = part_i + ((size_t)qbase * n_chunks + chunk) * k;
    for (int m = 0; m < kMQ && qbase + m < nq; ++m)
      if (lane < k) {
        tkd_base[m * tk_stride + lane] = a.inf;
        tkid_base[m * tk_stride + lane] = kNoId;
      }

    // ---- stream the chunk's stages
    const int64_t s_lo = n_steps * chunk / n_chunks, s_hi = n_steps * (chunk + 1) / n_chunks;
    // stage of step si: (si * tile_stride) mod n_steps
    int64_t sb = (int64_t)(((unsigned long long)s_lo * (unsigned long long)tile_stride) %
                           (unsigned long long)n_steps);
    bf16x8 r_op[2];  // this lane's share of the next stage
    float4 r_pt = make_float4(0, 0, 0, 0);
    int r_pid = kNoId;
    auto load_stage = [&](int64_t stage) {
      const bf16x8 *src = ops + stage * (kStage * 4);
      r_op[0] = src[tid];
      r_op[1] = src[tid + kWaves * 64];
      // lanes 0..127 fetch the coordinates, 128..255 the indices
      const int64_t p = stage * kStage + (tid & (kStage - 1));
      if (tid < kStage) {
        r_pt = p < n_real ? ix.pt4[p] : make_float4(0, 0, 0, __builtin_huge_valf());
      } else {
        r_pid = p < n_real ? ix.pid[p] : kNoId;
      }
    };
    auto store_stage = [&](int buf) {
      Stage *dst = s_stage + buf;
      dst->op[tid] = r_op[0];
      dst->op[tid + kWaves * 64] = r_op[1];
      if (tid < kStage)
        dst->pt[tid] = r_pt;
      else
        dst->pid[tid - kStage] = r_pid;
    };
    auto next_stage = [&](int64_t x) {
      x += tile_stride;
      return x >= n_steps ? x - n_steps : x;
    };
    load_stage(sb);
    store_stage(0);
    int64_t sb_next = next_stage(sb);
    if (s_lo + 1 < s_hi) load_stage(sb_next);
    __syncthreads();
    for (int64_t si = s_lo; si < s_hi; ++si) {
      const int buf = (int)((si - s_lo) & 1);
      const Stage *st = s_stage + buf;
      const int64_t p0 = sb * kStage;
      // all operand reads, then all MFMAs, then the tests: no dependency
      // between tiles, so the latencies overlap
      uint32_t near_tiles = 0;  // tiles with a value within its query's bound
#pragma unroll
      for (int c0 = 0; c0 < kStageTiles; c0 += kBatch) {
        bf16x8 b[kBatch];
#pragma unroll
        for (int c = 0; c < kBatch; ++c) b[c] = st->op[(c0 + c) * 64 + lane];
        f32x4 acc[kBatch];
#pragma unroll
        for (int c = 0; c < kBatch; ++c) {
          const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
          acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, b[c], z, 0, 0, 0);
        }
#pragma unroll
        for (int c = 0; c < kBatch; ++c) {
          bool near = false;
#pragma unroll
          for (int e = 0; e < 4; ++e) near |= acc[c][e] <= tau[e];
          near_tiles |= (ballot(near) != 0 ? 1u : 0u) << (c0 + c);
        }
      }
      while (near_tiles) {
        const int cb = __ffs(near_tiles) - 1;
        near_tiles &= near_tiles - 1;
        const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
        const f32x4 acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, st->op[cb * 64 + lane], z, 0, 0, 0);
        const int j = cb * 16 + row;  // this lane's point in the stage
        const float pt = st->pt[j].w;
        int queued = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          // row (query) g*4+e, column (point) j; padding has time +inf
          const float v = acc1[e];
          const bool pass = (v <= tau[e]) & (pt < thr[e]);
          const uint64_t pm = ballot(pass);
          if (pm == 0) continue;
          const int np = __popcll(pm);
          if (queued + np > kQCap) {
            flush(queued, st, p0);
            queued = 0;
          }
          if (pass) {
            const int slot = queued + (int)__builtin_amdgcn_mbcnt_hi(
                                          (uint32_t)(pm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)pm, 0u));
            s_qp[wave][slot] = j;
            s_qc[wave][slot] = v;
            s_qm[wave][slot] = (unsigned char)(g * 4 + e);
          }
          queued += np;
        }
        if (queued == 0) continue;
        flush(queued, st, p0);
#pragma unroll
        for (int e = 0; e < 4; ++e) tau[e] = fminf(tau[e], s_tau[wave][g * 4 + e]);
      }
      // the other buffer was last read before the previous barrier
      if (si + 1 < s_hi) store_stage(buf ^ 1);
      __syncthreads();
      sb = sb_next;
      sb_next = next_stage(sb);
      if (si + 2 < s_hi) load_stage(sb_next);
    }

    // ---- this chunk's top-k of each query, and its k-th distance
    for (int m = 0; m < kMQ; ++m) {
      const int64_t q = qbase + m;
      if (q >= nq) break;
      // the rounded-up k-th distance (+inf with fewer than k)
      if (lane == 0) part_kd[q * n_chunks + chunk] = s_tau[wave][m];
    }
    if (chunk == 0) {
      const int64_t left = nq - qbase;
      queries_done += left < 0 ? 0 : (left > kMQ ? kMQ : left);
    }
    __syncthreads();
  }
  if (a.stats) {
    for (int o = 32; o > 0; o >>= 1) max_err = fmax(max_err, __shfl_xor(max_err, o, 64));
    if (lane == 0) {
      atomicAdd(a.stats + TNN_STAT_QUERIES, (unsigned long long)queries_done);
      atomicAdd(a.stats + TNN_STAT_POINTS, (unsigned long long)(queries_done * ix.n_points));
      atomicAdd(a.stats + TNN_STAT_RESCORED, (unsigned long long)rescored);
      atomicMax(a.stats + TNN_STAT_MAX_ERR, (unsigned long long)__double_as_longlong(max_err));
    }
  }
}

// One wave per query: the exact top-k of the union of its chunks' partial
// lists (each sorted by (distance, index), padded with (+inf, none)).
__global__ __launch_bounds__(256) void mixed_merge_kernel(const double *part_d,
                                                          const int32_t *part_i,
                                                          const float *part_kd, int n_chunks,
                                                          int64_t nq, int k, double inf,
                                                          int32_t *out_idx, double *out_dist) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= nq) return;
  const int lane = lane_id();
  bool out_of_range = false;
  for (int c = 0; c < n_chunks; ++c) out_of_range = out_of_range || __builtin_isnan(part_kd[q * n_chunks + c]);
  if (out_of_range) {  // the query's scaled norm exceeds the tiles' range
    if (lane < k) {
      out_idx[q * k + lane] = -1;
      out_dist[q * k + lane] = inf - inf;  // NaN (no 64-bit literal)
    }
    return;
  }
  TopK tk;
  tk.init(k, inf);
  for (int c = 0; c < n_chunks; ++c) {
    const size_t o = ((size_t)q * n_chunks + c) * k;
    double d = inf;
    int id = kNoId;
    if (lane < k) {
      d = part_d[o + lane];
      id = part_i[o + lane];
    }
    if (c == 0) {
      tk.d = d;
      tk.id = id;
      tk.refresh();
      continue;
    }
    const bool gate = id != kNoId && tk.admits(d, id);
    const uint64_t gm = ballot(gate);
    if (gm) tk.offer(gm, d, id);
  }
  if (lane < k) {
    out_idx[q * k + lane] = tk.id == kNoId ? -1 : tk.id;
    out_dist[q * k + lane] = tk.d;
  }
}

}  // namespace

// Points padded to whole stages.
static int64_t padded_points(int64_t n_points) {
  return (n_points + kStage - 1) / kStage * kStage;
}

// Point chunks per query tile: enough work items to keep a full chip busy
// to the end, at most one chunk per stage.
static int mixed_chunks(int64_t n_points, int64_t nq) {
  const int64_t tiles = (nq + kTileQ - 1) / kTileQ;
  const int64_t stages = padded_points(n_points) / kStage;
  int64_t c = tiles > 0 ? (8 * kNominalSlots + tiles - 1) / tiles : 1;
  if (c > kMaxChunks) c = kMaxChunks;
  if (c > stages) c = stages;
  return c < 1 ? 1 : (int)c;
}

namespace {
struct MixedLayout {
  int64_t np, chunks;
  size_t ops, nv, part_d, part_i, part_kd, counter, total;
};

MixedLayout mixed_layout(int64_t n_points, int64_t nq, int k) {
  MixedLayout l;
  l.np = padded_points(n_points);
  l.chunks = mixed_chunks(n_points, nq);
  const size_t entries = (size_t)nq * l.chunks * k;
  size_t o = 0;
  l.ops = o;
  o += align_up((size_t)l.np * 64);
  l.nv = o;
  o += align_up((size_t)n_points * 4);
  l.part_d = o;
  o += align_up(entries * 8);
  l.part_i = o;
  o += align_up(entries * 4);
  l.part_kd = o;
  o += align_up((size_t)nq * l.chunks * 4);
  l.counter = o;
  o += 256;
  l.total = o;
  return l;
}

// Workgroups of mixed_brute_kernel resident on one CU, per (device, LDS).
int mixed_per_cu(size_t lds) {
  struct Entry {
    int dev;
    size_t lds;
    int per_cu;
  };
  static Entry cache[16];
  static int used = 0;
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  std::lock_guard<std::mutex> lock(mu);
  for (int i = 0; i < used; ++i)
    if (cache[i].dev == dev && cache[i].lds == lds) return cache[i].per_cu;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mixed_brute_kernel, kWaves * 64, lds) !=
          hipSuccess ||
      n <= 0)
    n = 1;
  if (used < 16) cache[used++] = Entry{dev, lds, n};
  return n;
}

int cu_count_mixed() {
  int dev = 0, c = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
    return 256;
  return c;
}
}  // namespace

size_t mixed_scratch_bytes(int64_t n_points, int64_t n_queries, int k) {
  return mixed_layout(n_points, n_queries, k).total;
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
  const MixedLayout l = mixed_layout(ix.n_points, qs.n, a.k);
  char *base = static_cast<char *>(scratch);
  bf16x8 *ops = reinterpret_cast<bf16x8 *>(base + l.ops);
  float *nv = reinterpret_cast<float *>(base + l.nv);
  double *part_d = reinterpret_cast<double *>(base + l.part_d);
  int32_t *part_i = reinterpret_cast<int32_t *>(base + l.part_i);
  float *part_kd = reinterpret_cast<float *>(base + l.part_kd);
  unsigned long long *counter = reinterpret_cast<unsigned long long *>(base + l.counter);
  const int64_t n_steps = l.np / kStage;
  const int64_t n_tiles = (qs.n + kTileQ - 1) / kTileQ;
  const int64_t n_kd = qs.n * l.chunks;
  if (n_steps == 0) {
    // no points: merging no lists leaves every slot a pad
    hipLaunchKernelGGL(mixed_merge_kernel, dim3((unsigned)((qs.n + 3) / 4)), dim3(256), 0, st,
                       part_d, part_i, part_kd, 0, qs.n, a.k, a.inf, out_idx, out_dist);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(mixed_prep_kernel, dim3((unsigned)((l.np + 255) / 256)), dim3(256), 0, st, ix,
                     mc, ops, nv, l.np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mixed_reset_kernel, dim3((unsigned)((n_kd + 255) / 256)), dim3(256), 0, st,
                     part_kd, n_kd, counter);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
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
  const size_t lds = 2 * sizeof(Stage);
  const int64_t items = n_tiles * l.chunks;
  const int64_t resident = (int64_t)cu_count_mixed() * mixed_per_cu(lds);
  const int64_t grid = items < resident ? items : resident;
  hipLaunchKernelGGL(mixed_brute_kernel, dim3((unsigned)grid), dim3(kWaves * 64), lds, st, ix, a,
                     mc, ops, nv, qs.x, qs.y, qs.z, qs.t, qs.n, part_d, part_i, part_kd, counter,
                     n_tiles, (int)l.chunks, n_steps, stride);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mixed_merge_kernel, dim3((unsigned)((qs.n + 3) / 4)), dim3(256), 0, st, part_d,
                     part_i, part_kd, (int)l.chunks, qs.n, a.k, a.inf, out_idx, out_dist);
  return hipGetLastError();
}

}  // namespace tnn
