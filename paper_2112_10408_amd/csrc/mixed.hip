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
// (1 - gamma) and split the same way, fill six more, and the last two carry
// minus the query's current bound T (two bfloat16 terms on the query side,
// ones on the point side).  The tile value is
//     c = (1 - gamma)(|u|^2 + |v|^2) - 2 u.v - T .
// Without the T terms it errs by at most 1.6 * 2^-18 (|u|^2 + |v|^2) (the
// split, the float32 accumulation of 32 terms and the float32 inputs),
// below gamma = 2^-16; the T terms add at most 31 * 2^-23 T < 2^-18 T to the
// accumulation error.  So c < d - (1 - 2^-18) T, and with T >= tau (1 + 2^-16)
// and T >= 2^-100 every pair whose distance is at most the query's k-th
// distance bound tau gets a negative tile value: the sign bit is the filter,
// and one OR over a batch of tile values tells whether any pair passes.
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
constexpr int kWaves = 4;                   // waves per workgroup
constexpr int kMQ = 16;                     // queries per MFMA row block
constexpr int kRowBlocks = 4;               // row blocks per wave (four named A operands)
constexpr int kWaveQ = kMQ * kRowBlocks;    // queries per wave
constexpr int kTileQ = kWaves * kWaveQ;     // queries per work item
constexpr int kStage = 128;                 // points per LDS stage
constexpr int kStageTiles = kStage / 16;    // 16-column MFMA tiles per stage
constexpr int kQCap = 64;                   // queued survivors per wave (one per lane)
constexpr int kBatch = 2;                   // tiles whose tile values are tested together
constexpr int kMaxChunks = 16;              // point chunks per query tile
constexpr int kPilotStages = 32;            // stages of a tile's home range (pilot pass)
constexpr int kShareSteps = 16;             // steps between two poolings of a tile's bounds
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

// Rounded toward +infinity (finite inputs).
__device__ __forceinline__ __bf16 to_bf16_up(float x) {
  const uint32_t u = __float_as_uint(x);
  uint32_t t = u & 0xffff0000u;
  if ((u & 0xffffu) != 0 && !(u >> 31)) t += 0x10000u;
  return __builtin_bit_cast(__bf16, (unsigned short)(t >> 16));
}

__device__ __forceinline__ __bf16 neg_bf16(__bf16 b) {
  return __builtin_bit_cast(__bf16, (unsigned short)(__builtin_bit_cast(unsigned short, b) ^ 0x8000u));
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

// The bound slots of a query row: bfloat16 terms h, m with h + m >= T,
// T = max(tau (1 + 2^-15) rounded to float, 2^-100) >= tau (1 + 2^-16), and
// their sum as a float (for the statistics).  tau = +inf (no bound yet), or
// T overflowing, gives h = +inf: every tile value of the row is -inf.
// tau = -inf (a row that takes no part) gives h = -inf: tile values +inf.
__device__ __forceinline__ void bound_terms(float tau, __bf16 &h, __bf16 &m, float &sum) {
  const __bf16 zero = __builtin_bit_cast(__bf16, (unsigned short)0);
  if (tau == -__builtin_huge_valf()) {
    h = __builtin_bit_cast(__bf16, (unsigned short)0xff80u);
    m = zero;
    sum = -__builtin_huge_valf();
    return;
  }
  const float t = fmaxf(tau * (1.0f + 0x1p-15f), 0x1p-100f);
  const __bf16 th = to_bf16(t);
  if (!(t < __builtin_huge_valf()) || !(from_bf16(th) < __builtin_huge_valf())) {
    h = __builtin_bit_cast(__bf16, (unsigned short)0x7f80u);
    m = zero;
    sum = __builtin_huge_valf();
    return;
  }
  h = th;
  m = to_bf16_up(t - from_bf16(th));  // the difference is exact
  sum = from_bf16(h) + from_bf16(m);
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
  const __bf16 one = to_bf16(1.0f);
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
    o[6] = one;  // times the query's -T terms
    o[7] = one;
  }
  return o;
}

// A operand (query side), paired slot by slot with point_group; th, tm are
// the query's bound terms (bound_terms), entered negated.
__device__ __forceinline__ bf16x8 query_group(const float u[4], float nus, int g, __bf16 th,
                                              __bf16 tm) {
  __bf16 h[4], m[4], l[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) split3(u[f], h[f], m[f], l[f]);
  bf16x8 o;
  const __bf16 one = to_bf16(1.0f);
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
    o[6] = neg_bf16(th);
    o[7] = neg_bf16(tm);
  }
  return o;
}

// Per call: the point operands and |v|^2.  Operands are stored tile-major:
// the 16-byte group g of point p sits at unit (p / 16 * 4 + g) * 16 + p % 16,
// so a 16-point MFMA tile is 1 KB laid out lane by lane and a stage is one
// contiguous block.  Operands are padded to whole stages with zeros (a
// padding column's tile values are 0 or NaN: the time mask drops it).
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

// Per call: no query has a bound yet; the block counts and the work counter
// start at 0.
__global__ void mixed_reset_kernel(float *bound, int64_t n, int32_t *bcount, int64_t nb,
                                   unsigned long long *counter) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) bound[i] = __builtin_huge_valf();
  if (i < nb) bcount[i] = 0;
  if (i == 0) *counter = 0;
}

// Scan order (not in the paper; any order gives the same result).  Every
// query gets a home block: the index block nearest to it by the block box
// lower bound, searched in the nearest superblock.  Queries are then
// ordered by home block (a counting sort), so that a tile of kTileQ
// consecutive queries is spatially compact, and a pilot pass scans each
// tile's home range of stages first: its k-th distances, near the final
// ones, bound the main pass from its first stage on.
__global__ void mixed_home_kernel(IndexDesc ix, QueryArgs a, const float *qxp, const float *qyp,
                                  const float *qzp, const float *qtp, int64_t nq, int32_t *home,
                                  int32_t *bcount) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const QueryPoint qp = make_query(qxp[q], qyp[q], qzp[q], qtp[q], a.t_window);
  int best_s = 0;
  float lb_s = __builtin_huge_valf();
  for (int sb = 0; sb < ix.n_super; ++sb) {
    const float lb = block_lb(ix.sbox, sb, qp, a.sf);
    if (lb < lb_s) {
      lb_s = lb;
      best_s = sb;
    }
  }
  const int b_lo = best_s * kSuperBlocks;
  const int b_hi = min(b_lo + kSuperBlocks, ix.n_blocks);
  int best = b_lo;
  float lb_b = __builtin_huge_valf();
  for (int b = b_lo; b < b_hi; ++b) {
    const float lb = block_lb(ix.box, b, qp, a.sf);
    if (lb < lb_b) {
      lb_b = lb;
      best = b;
    }
  }
  home[q] = best;
  atomicAdd(bcount + best, 1);
}

// Exclusive prefix sums of the block counts, in place (one workgroup of
// 1024 threads).
__global__ __launch_bounds__(1024) void mixed_offsets_kernel(int32_t *bcount, int64_t nb) {
  __shared__ int s_v[1024];
  __shared__ int s_carry;
  const int tid = (int)threadIdx.x;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t i = base + tid;
    const int v = i < nb ? bcount[i] : 0;
    s_v[tid] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int add = tid >= o ? s_v[tid - o] : 0;
      __syncthreads();
      s_v[tid] += add;
      __syncthreads();
    }
    const int carry = s_carry;
    if (i < nb) bcount[i] = carry + s_v[tid] - v;
    __syncthreads();
    if (tid == 1023) s_carry = carry + s_v[1023];
    __syncthreads();
  }
}

// perm[position] = caller index, grouped by home block (the order within a
// block is whatever the atomics give: only the scan order depends on it).
__global__ void mixed_scatter_kernel(const int32_t *home, int64_t nq, int32_t *bcount,
                                     int32_t *perm) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  perm[atomicAdd(bcount + home[q], 1)] = (int32_t)q;
}

// First stage of each tile's home range: starting a little before the
// first stage of its middle query's home block.
__global__ void mixed_tile_start_kernel(IndexDesc ix, const int32_t *home, const int32_t *perm,
                                        int64_t nq, int64_t n_tiles, int64_t n_steps,
                                        int64_t *tstart) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  int64_t mid = t * kTileQ + kTileQ / 2;
  if (mid >= nq) mid = nq - 1;
  const int b = home[perm[mid]];
  const int64_t first = ix.pstart[(int64_t)b * kBlockSegs] / kStage;
  int64_t s0 = (first - kPilotStages / 4) % n_steps;  // in [0, n_steps)
  if (s0 < 0) s0 += n_steps;
  tstart[t] = s0;
}

__device__ __forceinline__ float round_up_f(double x) {
  return x < kInf ? __double2float_ru(x) : __builtin_huge_valf();
}

// The pooled bound of a query: the least upper bound on its k-th distance
// any of its lists has found (non-negative floats order as their bit
// patterns, so a signed integer minimum is a float minimum; -0 is made +0
// first).  Read and lowered at device scope, so that the items of a tile
// on other dies see it.
__device__ __forceinline__ void lower_bound_to(float *b, float v) {
  __hip_atomic_fetch_min(reinterpret_cast<int *>(b), __float_as_int(v + 0.0f), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float read_bound(const float *b) {
  return __hip_atomic_load(b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The call's arguments the MFMA search needs beyond its arrays, parked in
// LDS so that the scan loop keeps few scalar registers live.
struct SlowArgs {
  double s[4];
  double t_window;
  double inf;
  const float *nv;
  unsigned long long *stats;
  int k;
};

// Earliest time of each stage's points (+inf for a stage of padding only):
// a stage not earlier than every query's time threshold in a tile holds no
// candidate of the tile (every pair is masked, Sec. 3.4), and the tile
// skips it.  One wave per stage.
__global__ void mixed_stage_time_kernel(const float4 *pt4, int64_t n_real, int64_t n_steps,
                                        float *stage_tmin) {
  const int64_t stg = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (stg >= n_steps) return;
  const int lane = lane_id();
  float t = __builtin_huge_valf();
  for (int h = 0; h < kStage / kWave; ++h) {
    const int64_t p = stg * kStage + h * kWave + lane;
    if (p < n_real) t = fminf(t, pt4[p].w);
  }
  for (int o = 32; o > 0; o >>= 1) t = fminf(t, __shfl_xor(t, o, 64));
  if (lane == 0) stage_tmin[stg] = t;
}

// Pilot pass: the exact top-k of each query over its tile's home range
// (stages t0 .. t0 + n_home - 1, mod n_steps) in binary64, one wave per
// kPilotQ consecutive queries of the scan order (all in one tile), each
// 64-point pass of the range loaded once for them.  The list goes to slot
// n_slots - 1, its rounded-up k-th distance to the query's bound.
constexpr int kPilotQ = 4;
static_assert(kTileQ % kPilotQ == 0, "a pilot wave stays within one tile");
__global__ __launch_bounds__(256) void mixed_pilot_kernel(
    IndexDesc ix, QueryArgs a, const float *qxp, const float *qyp, const float *qzp,
    const float *qtp, const int32_t *perm, int64_t nq, const int64_t *tstart,
    const float *stage_tmin, int n_home, int64_t n_steps, int n_slots, double *part_d,
    int32_t *part_i, float *bound) {
  const int64_t q0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + uniform_i((int)(threadIdx.x >> 6))) *
                     kPilotQ;
  if (q0 >= nq) return;
  const int lane = lane_id();
  const double s[4] = {a.s[0], a.s[1], a.s[2], a.s[3]};
  // positions past the end repeat the last one and are not written
  QueryPoint q[kPilotQ];
  TopK tk[kPilotQ];
#pragma unroll
  for (int j = 0; j < kPilotQ; ++j) {
    const int64_t qc = perm[q0 + j < nq ? q0 + j : nq - 1];
    q[j] = make_query(qxp[qc], qyp[qc], qzp[qc], qtp[qc], a.t_window);
    tk[j].init(a.k, a.inf);
  }
  const int64_t t0 = tstart[q0 / kTileQ];
  const int64_t n = ix.n_points;
  int scanned = 0;
  // a stage not earlier than every one of these queries' time thresholds
  // holds none of their candidates
  float thr_max = -__builtin_huge_valf();
#pragma unroll
  for (int j = 0; j < kPilotQ; ++j) thr_max = fmaxf(thr_max, q[j].thrf);
  // The home range's stages that can hold a candidate of these queries (one
  // stage per lane, read at once), then the points of each such stage, both
  // halves requested together.
  static_assert(kPilotStages <= kWave, "one home stage per lane");
  uint64_t live = 0;
  {
    float tm = __builtin_huge_valf();
    if (lane < n_home) {
      int64_t stage = t0 + lane;
      if (stage >= n_steps) stage -= n_steps;
      tm = stage_tmin[stage];
    }
    live = ballot(tm < thr_max);
  }
  constexpr int kHalves = kStage / kWave;
  while (live) {
    const int h = __ffsll((long long)live) - 1;
    live &= live - 1;
    int64_t stage = t0 + h;
    if (stage >= n_steps) stage -= n_steps;
    ++scanned;
    float4 pv[kHalves];
    int pid[kHalves];
    bool ok[kHalves];
    // (unconditional loads, a padding lane reading point 0, which the gate
    // drops: a branch around each load, or a use scheduled among them, would
    // make the compiler wait for the first half's before requesting the
    // second's; the launch has points)
#pragma unroll
    for (int half = 0; half < kHalves; ++half) {
      const int64_t p = stage * kStage + half * kWave + lane;
      ok[half] = p < n;
      const int64_t pl = ok[half] ? p : 0;
      pv[half] = ix.pt4[pl];
      pid[half] = ix.pid[pl];
    }
    __builtin_amdgcn_sched_barrier(0);  // every load issued before the first use
#pragma unroll
    for (int half = 0; half < kHalves; ++half) {
#pragma unroll
      for (int j = 0; j < kPilotQ; ++j) {
        const double d = exact_dist(s, q[j].x, q[j].y, q[j].z, q[j].t, pv[half].x, pv[half].y,
                                    pv[half].z, pv[half].w);
        const bool gate = ok[half] & (pv[half].w < q[j].thrf) & tk[j].admits(d, pid[half]);
        const uint64_t gm = ballot(gate);
        if (gm) tk[j].offer(gm, d, pid[half]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kPilotQ; ++j) {
    const int64_t qi = q0 + j;
    if (qi < nq) {
      const size_t o = ((size_t)qi * n_slots + (n_slots - 1)) * a.k;
      if (lane < a.k) {
        part_d[o + lane] = tk[j].d;
        part_i[o + lane] = tk[j].id;
      }
      if (lane == 0) bound[qi] = round_up_f(tk[j].kd);
    }
  }
  if (a.stats && lane == 0) {
    const int nmine = (int)(nq - q0 < kPilotQ ? nq - q0 : kPilotQ);
    atomicAdd(a.stats + TNN_STAT_RESCORED, (unsigned long long)scanned * kStage * nmine);
    atomicAdd(a.stats + TNN_STAT_POINTS, (unsigned long long)scanned * kStage * nmine);
  }
}

// LDS stage buffer: the operands of kStage points (tile-major), their
// times and their caller indices (the rescoring reads a survivor's
// coordinates from global memory).
struct Stage {
  bf16x8 op[kStage * 4];
  float t[kStage];
  int pid[kStage];
};

constexpr int kStageBufs = 3;  // LDS stage buffers: loads run two stages ahead
constexpr int kStageLoads = 3;  // load instructions per wave and stage

// M0 is written only here: the compiler uses it for nothing else in this
// file (no other LDS-direct load, no indexed register move), so the clobber
// it warns about is taken on purpose.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
// Loads straight into LDS (no registers): each lane's 16 or 4 bytes land at
// the wave-uniform LDS byte address `lds` plus lane * size (M0 holds it).
// Written out because the compiler, not seeing which buffer a later LDS
// read hits, would wait for every such load right away; the waits are
// explicit (stage_wait_barrier).
__device__ __forceinline__ void lds_load16(const void *src, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
               :
               : "v"(src), "s"(__builtin_amdgcn_readfirstlane(lds))
               : "memory", "m0");
}
__device__ __forceinline__ void lds_load4(const void *src, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dword %0, off"
               :
               : "v"(src), "s"(__builtin_amdgcn_readfirstlane(lds))
               : "memory", "m0");
}

#pragma clang diagnostic pop

// Wait until this wave's stage loads have landed, except the newest
// stage's kStageLoads when `keep_newest` (vector memory operations complete
// in issue order), and until its LDS reads are done; then the workgroup
// barrier, after which every wave's loads of the older stages are visible.
__device__ __forceinline__ void stage_wait_barrier(bool keep_newest) {
  static_assert(kStageLoads == 3, "the wait below keeps kStageLoads operations in flight");
  if (keep_newest)
    asm volatile("s_waitcnt vmcnt(3) lgkmcnt(0)\n\ts_barrier" ::: "memory");
  else
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ uint32_t lds_addr(const void *p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}

// Work item = (query tile of kTileQ queries in scan order, chunk of the
// point stages).  A persistent grid of 4-wave workgroups takes items from a
// counter, chunk by chunk.  The workgroup streams the chunk's stages
// through three LDS buffers, loaded straight into LDS by all 256 lanes two
// stages ahead, and each wave answers its 64 queries (four MFMA row blocks)
// against every stage: each 16-point tile read from LDS feeds four MFMAs,
// and a batch of 2 tiles (2,048 pairs) costs one OR over its 32 tile values
// and one ballot when nothing passes.  Otherwise the survivors (negative
// tile value, time mask passed) go to the wave's queue (slots from
// ballots), which is rescored in binary64 (one lane per survivor) and
// merged into each query's top-k; then the bound terms of the A operands
// are refreshed.  That top-k is kept in place in the item's list in global
// memory (L2 resident while the item runs).  A query's bound starts at the
// least k-th distance among its lists already finished, the pilot pass's
// first (each is an upper bound on the final k-th distance), and
// mixed_merge_kernel combines the lists.
__global__ __launch_bounds__(kWaves * 64, 4) void mixed_brute_kernel(
    const float4 *pt4, const int32_t *pidv, int64_t n_real, SlowArgs sa, MixedCtx mc,
    const bf16x8 *ops, const float *qxp,
    const float *qyp, const float *qzp, const float *qtp, const int32_t *perm, int64_t nq,
    double *part_d, int32_t *part_i, float *bound, unsigned long long *counter,
    const int64_t *tstart, const float *stage_tmin, int64_t n_tiles, int n_chunks, int n_home,
    int n_steps, int tile_stride) {
  // 16-byte aligned: the stage buffers are read with 16-byte LDS loads
  extern __shared__ float4 s_dyn4[];
  __shared__ SlowArgs s_a;
  __shared__ long long s_item;
  __shared__ float s_wthr[kWaves];  // each wave's largest time threshold
  __shared__ float4 s_q[kWaves][kWaveQ];    // query coordinates (x, y, z, t)
  __shared__ float4 s_thr4[kWaves][kWaveQ / 4];  // time thresholds (float, rounded up)
  __shared__ float s_tau[kWaves][kWaveQ];   // bound on the k-th distance, rounded up
  __shared__ float s_trep[kWaves][kWaveQ];  // the bound terms' sum folded in the A operand
  __shared__ float s_nu[kWaves][kWaveQ];    // |u|^2 of each query
  __shared__ int s_qp[kWaves][kQCap];       // queued survivor: point slot
  __shared__ int s_qi[kWaves][kQCap];       //                 its caller index
  __shared__ float s_qc[kWaves][kQCap];     //                 tile value + bound terms
  __shared__ unsigned char s_qm[kWaves][kQCap];  //            its query row
  const int k = sa.k;
  const int lane = lane_id();
  const int wave = uniform_i((int)(threadIdx.x >> 6));
  const int tid = (int)threadIdx.x;
  const int g = lane >> 4;    // K-group this lane supplies
  const int row = lane & 15;  // A row (query) / C column (point)
  float *s_thr = reinterpret_cast<float *>(s_thr4[wave]);
  // dynamic LDS: the stage buffers (and their LDS byte address, for the
  // loads that write them)
  Stage *s_stage = reinterpret_cast<Stage *>(s_dyn4);
  const uint32_t lds_stage0 = uniform_i((int)lds_addr(s_dyn4));
  if (tid == 0) s_a = sa;
  uint32_t rescored = 0;
  double max_err = 0.0;
  int64_t queries_done = 0;
  unsigned long long pairs_scanned = 0;  // (query, point) pairs of the stages scanned
  // The current item's top-k of query row m lives in place in its chunk list
  // (in the L2 while the item runs): tkd_base[m * tk_stride + rank].
  double *tkd_base = part_d;
  int *tkid_base = part_i;
  int64_t tk_stride = k;

  // Rescore the wave's queued survivors in binary64, one lane each (their
  // coordinates read from global memory), and merge them query by query.
  auto flush = [&](int queued) {
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
      const int64_t p = s_qp[wave][lane];
      const float4 qv = s_q[wave][mi];
      const QueryPoint qp = make_query(qv.x, qv.y, qv.z, qv.w, tw);
      const float4 pv = pt4[p];
      d = exact_dist(sc, qp.x, qp.y, qp.z, qp.t, pv.x, pv.y, pv.z, pv.w);
      pid = s_qi[wave][lane];
      // a candidate beyond the row's bound cannot be among the query's k
      // nearest (the bound is the rounded-up k-th distance of some list of k
      // of its candidates), so it skips the merge; a row whose survivors all
      // fail this reads no list
      valid = (double)pv.w < qp.thr && d <= (double)s_tau[wave][mi];
      const float c = s_qc[wave][lane];
      if (want_err && c > -__builtin_huge_valf() && c < __builtin_huge_valf()) {
        const double approx = (double)c + (double)kGamma * ((double)s_nu[wave][mi] + (double)s_a.nv[p]);
        max_err = fmax(max_err, fabs(approx - d));
      }
    }
    uint64_t pending = ballot(has && valid);
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
        if (lane == 0) s_tau[wave][m] = fminf(s_tau[wave][m], round_up_f(tk.kd));
      }
    }
    rescored += (uint32_t)queued;
  };

  const int n_slots = n_chunks + 1;
  const int64_t n_items = n_tiles * n_chunks;
  for (;;) {
    if (tid == 0) s_item = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const long long item = s_item;
    if (item >= n_items) break;
    const int chunk = (int)(item / n_tiles);
    const int64_t tile = item % n_tiles;
    const int slot = chunk;
    const int64_t qbase = tile * kTileQ + wave * kWaveQ;  // positions in scan order

    // ---- this wave's queries: norms, bounds, time thresholds, A operands
    float u[kRowBlocks][4];
#pragma unroll
    for (int bb = 0; bb < kRowBlocks; ++bb) {
      const int64_t qa = qbase + bb * kMQ + row;
      float nu = 0.0f;
#pragma unroll
      for (int f = 0; f < 4; ++f) u[bb][f] = 0.0f;
      if (qa < nq) {
        const int64_t qc = perm[qa];
        nu = scaled(mc, qxp[qc], qyp[qc], qzp[qc], qtp[qc], u[bb]);
      }
      if (g == 0) s_nu[wave][bb * kMQ + row] = nu;
    }
    if (lane < kWaveQ) {
      const int64_t q = qbase + lane;
      float t = -__builtin_huge_valf();  // a row that takes no part lets nothing pass
      float h = -__builtin_huge_valf();
      float4 qv = make_float4(0, 0, 0, 0);
      if (q < nq) {
        const int64_t qc = perm[q];
        qv = make_float4(qxp[qc], qyp[qc], qzp[qc], qtp[qc]);
        if (s_nu[wave][lane] < kMaxNorm) {
          t = read_bound(bound + q);
          h = round_up_f((double)qv.w - sa.t_window);
        } else {
          // too far out for the float32 tiles: NaN marks it in its bound
          // (which no list lowers then), and the merge reports its rows as
          // (-1, NaN)
          t = __builtin_nanf("");
          bound[q] = t;
        }
      }
      s_q[wave][lane] = qv;
      s_thr[lane] = h;
      s_tau[wave][lane] = t;
    }
    // the tile's largest time threshold: a stage not earlier is skipped
    {
      float h = s_thr[lane];
      for (int o = 32; o > 0; o >>= 1) h = fmaxf(h, __shfl_xor(h, o, 64));
      if (lane == 0) s_wthr[wave] = h;
    }
    __syncthreads();
    const float thr_max = fmaxf(fmaxf(s_wthr[0], s_wthr[1]), fmaxf(s_wthr[2], s_wthr[3]));
    static_assert(kWaves == 4, "four waves' thresholds");
    // the A operands of the row blocks (named, not an array: a
    // dynamically indexed array would live in scratch memory)
    static_assert(kRowBlocks == 4, "four named A operands");
    bf16x8 aop0, aop1, aop2, aop3;
#pragma unroll
    for (int bb = 0; bb < kRowBlocks; ++bb) {
      const int r = bb * kMQ + row;
      const float t = s_tau[wave][r];
      __bf16 th, tm;
      float sum;
      bound_terms(t != t ? -__builtin_huge_valf() : t, th, tm, sum);
      const bf16x8 o = query_group(u[bb], (1.0f - kGamma) * s_nu[wave][r], g, th, tm);
      if (bb == 0) aop0 = o;
      if (bb == 1) aop1 = o;
      if (bb == 2) aop2 = o;
      if (bb == 3) aop3 = o;
      if (g == 3) s_trep[wave][r] = sum;
    }
    // block bb's tile against operand tile b (a branch per block: selecting
    // among the named operands by value would put them in scratch memory)
    auto mfma_block = [&](int bb, const bf16x8 &b) {
      const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
      if (bb == 0) return __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop0, b, z, 0, 0, 0);
      if (bb == 1) return __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop1, b, z, 0, 0, 0);
      if (bb == 2) return __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop2, b, z, 0, 0, 0);
      return __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop3, b, z, 0, 0, 0);
    };
    tk_stride = (int64_t)n_slots * k;
    tkd_base = part_d + ((size_t)qbase * n_slots + slot) * k;
    tkid_base = part_i + ((size_t)qbase * n_slots + slot) * k;
    for (int m = 0; m < kWaveQ && qbase + m < nq; ++m)
      if (lane < k) {
        tkd_base[m * tk_stride + lane] = sa.inf;
        tkid_base[m * tk_stride + lane] = kNoId;
      }

    // ---- the item's stages: the chunk's share of the steps; step si scans
    // stage (si * tile_stride) mod n_steps, so that the chunk is spread over
    // the index, skipping the tile's home range (the pilot pass scanned it)
    // (in scalar registers: a vector register loaded from memory would make
    // the compiler wait for every load in flight, the stage loads included,
    // where the loop first reads it)
    // (stage numbers fit 32 bits: the host checks n_steps)
    const int t0 = uniform_i((int)tstart[tile]);
    int li = (int)((int64_t)n_steps * chunk / n_chunks);  // next step to load
    const int l_end = (int)((int64_t)n_steps * (chunk + 1) / n_chunks);
    int lx = (int)((int64_t)li * tile_stride % n_steps);
    auto in_home = [&](int x) {
      int d = x - t0;
      if (d < 0) d += n_steps;
      return d < n_home;
    };
    // the stage of the next step to load, or -1 when the item has no more
    // Earliest times of the next 64 steps' stages, one per lane (steps
    // win .. win + 63), read 64 at a time.
    int win = li - 64;
    float win_tmin = __builtin_huge_valf();
    auto next_stage = [&]() -> int {
      while (li < l_end) {
        if (li >= win + 64) {
          win = li;
          const int step = li + lane;
          win_tmin = step < l_end ? stage_tmin[(int64_t)step * tile_stride % n_steps]
                                  : __builtin_huge_valf();
        }
        const float tmin = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(win_tmin), li - win));
        const int x = lx;
        ++li;
        lx += tile_stride;
        if (lx >= n_steps) lx -= n_steps;
        if (!in_home(x) && tmin < thr_max) return x;
      }
      return -1;
    };
    // Stage `stage` into buffer `buf`: all 256 lanes load two operand
    // units; waves 0-1 load the times, waves 2-3 the caller indices (a
    // padding point loads point 0's, which the scan never uses).
    auto load_stage = [&](int stage, int buf) {
      const uint32_t dst = lds_stage0 + (uint32_t)buf * (uint32_t)sizeof(Stage);
      const bf16x8 *src = ops + (int64_t)stage * (kStage * 4);
      lds_load16(src + tid, dst + (uint32_t)offsetof(Stage, op) + wave * 1024u);
      lds_load16(src + kWaves * 64 + tid, dst + (uint32_t)offsetof(Stage, op) + (kWaves + wave) * 1024u);
      const int64_t p = (int64_t)stage * kStage + (tid & (kStage - 1));
      const int64_t pl = p < n_real ? p : 0;
      if (tid < kStage)
        lds_load4(&pt4[pl].w, dst + (uint32_t)offsetof(Stage, t) + wave * 256u);
      else
        lds_load4(pidv + pl, dst + (uint32_t)offsetof(Stage, pid) + (wave - 2) * 256u);
    };
    static_assert(kStage == 2 * 64 && kWaves == 4, "stage loads assume 4 waves and 128 points");

    // The bound terms of the A operands from the rows' current bounds.
    auto refresh_bounds = [&]() {
      if (g != 3) return;
#pragma unroll
      for (int bb = 0; bb < kRowBlocks; ++bb) {
        const int r = bb * kMQ + row;
        const float t = s_tau[wave][r];
        __bf16 th, tm;
        float sum;
        bound_terms(t != t ? -__builtin_huge_valf() : t, th, tm, sum);
        if (bb == 0) {
          aop0[6] = neg_bf16(th);
          aop0[7] = neg_bf16(tm);
        }
        if (bb == 1) {
          aop1[6] = neg_bf16(th);
          aop1[7] = neg_bf16(tm);
        }
        if (bb == 2) {
          aop2[6] = neg_bf16(th);
          aop2[7] = neg_bf16(tm);
        }
        if (bb == 3) {
          aop3[6] = neg_bf16(th);
          aop3[7] = neg_bf16(tm);
        }
        s_trep[wave][r] = sum;
      }
    };

    // Queue one survivor set: `pm` (a ballot) holds the lanes whose column j
    // passes for row r; v is the tile value.  Slots from the ballot.
    int queued = 0;  // survivors waiting in the wave's queue
    auto enqueue = [&](uint64_t pm, bool pass, int j, int r, float v, int64_t p0, const Stage *st) {
      if (pass) {
        const int slot = queued + (int)__builtin_amdgcn_mbcnt_hi(
                                      (uint32_t)(pm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)pm, 0u));
        s_qp[wave][slot] = (int)(p0 + j);
        s_qi[wave][slot] = st->pid[j];
        s_qc[wave][slot] = v + s_trep[wave][r];
        s_qm[wave][slot] = (unsigned char)r;
      }
      queued += __popcll(pm);
    };

    // One stage: every batch of tiles through the filter; the survivors go
    // to the queue (a full queue is flushed on the way).  Returns whether
    // a flush happened.
    auto scan_stage = [&](const Stage *st, int64_t p0) {
      bool flushed = false;
      // The stage's tiles through the filter, batch by batch (straight-line
      // code: the loop is unrolled), noting the tiles that hold a negative
      // value: bit (c * kRowBlocks + bb) for point tile c and row block bb.
      static_assert(kStageTiles * kRowBlocks == 32, "one bit per tile of the stage");
      uint32_t near = 0;
#pragma unroll
      for (int c0 = 0; c0 < kStageTiles; c0 += kBatch) {
        f32x4 acc[kRowBlocks][kBatch];
        {
          const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int c = 0; c < kBatch; ++c) {
            const bf16x8 b = st->op[(c0 + c) * 64 + lane];
            acc[0][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop0, b, z, 0, 0, 0);
            acc[1][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop1, b, z, 0, 0, 0);
            acc[2][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop2, b, z, 0, 0, 0);
            acc[3][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop3, b, z, 0, 0, 0);
          }
        }
        // sign bits of the batch's tile values, ORed as a tree
        uint32_t o[kRowBlocks * kBatch];
#pragma unroll
        for (int c = 0; c < kBatch; ++c)
#pragma unroll
          for (int bb = 0; bb < kRowBlocks; ++bb)
            o[c * kRowBlocks + bb] =
                (__float_as_uint(acc[bb][c][0]) | __float_as_uint(acc[bb][c][1])) |
                (__float_as_uint(acc[bb][c][2]) | __float_as_uint(acc[bb][c][3]));
        static_assert(kRowBlocks * kBatch == 8, "the OR tree below takes 8 tiles");
        const uint32_t any = ((o[0] | o[1]) | (o[2] | o[3])) | ((o[4] | o[5]) | (o[6] | o[7]));
        if (ballot((int)any < 0) == 0) continue;
#pragma unroll
        for (int t = 0; t < kRowBlocks * kBatch; ++t)
          near |= (ballot((int)o[t] < 0) != 0 ? 1u : 0u) << (c0 * kRowBlocks + t);
      }
      // Each such tile's values again (the same MFMA, so that few registers
      // stay live), and its survivors (negative tile value, the time mask, a
      // real point; row g*4+e of block bb, column j) to the queue.
      while (near) {
        const int t = __ffs(near) - 1;
        near &= near - 1;
        const int c = t / kRowBlocks, bb = t % kRowBlocks;
        const int j = c * 16 + row;
        const f32x4 v4 = mfma_block(bb, st->op[c * 64 + lane]);
        const float pt = (p0 + j < n_real) ? st->t[j] : __builtin_huge_valf();
        const float4 th4 = s_thr4[wave][bb * 4 + g];
        const int r0 = bb * kMQ + g * 4;
        bool ps[4];
        uint64_t pm[4];
        int np = 0;
        ps[0] = (__float_as_int(v4[0]) < 0) & (pt < th4.x);
        ps[1] = (__float_as_int(v4[1]) < 0) & (pt < th4.y);
        ps[2] = (__float_as_int(v4[2]) < 0) & (pt < th4.z);
        ps[3] = (__float_as_int(v4[3]) < 0) & (pt < th4.w);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          pm[e] = ballot(ps[e]);
          np += __popcll(pm[e]);
        }
        if (np == 0) continue;
        if (queued + np <= kQCap) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (pm[e] != 0) enqueue(pm[e], ps[e], j, r0 + e, v4[e], p0, st);
          continue;
        }
        // a full queue: set by set, flushing whenever the next would not fit
#pragma unroll 1
        for (int e = 0; e < 4; ++e) {
          const uint64_t m = e == 0 ? pm[0] : e == 1 ? pm[1] : e == 2 ? pm[2] : pm[3];
          if (m == 0) continue;
          if (queued + __popcll(m) > kQCap) {
            flush(queued);
            flushed = true;
            queued = 0;
          }
          const bool pe = e == 0 ? ps[0] : e == 1 ? ps[1] : e == 2 ? ps[2] : ps[3];
          const float ve = e == 0 ? v4[0] : e == 1 ? v4[1] : e == 2 ? v4[2] : v4[3];
          enqueue(m, pe, j, r0 + e, ve, p0, st);
        }
      }
      return flushed;
    };

    // Each step scans one buffer while the loads of the stage two steps
    // ahead (issued as the step starts, into the buffer the previous step
    // used) are in flight; a step ends once the next stage's loads have
    // landed.  st0, st1, st2: the stages in the current buffer and the next
    // two (-1: none).
    int st0 = next_stage(), st1 = -1, st2 = -1;
    if (st0 >= 0) load_stage(st0, 0);
    if (st0 >= 0) st1 = next_stage();
    if (st1 >= 0) load_stage(st1, 1);
    // the loads of the previous item's last steps and this item's top-k
    // initialisation are older: waited for as well
    stage_wait_barrier(st1 >= 0);
    int buf = 0;
    int step_no = 0;
    int scanned = 0;
    while (st0 >= 0) {
      // Every kShareSteps steps the items of the tile that run at the same
      // time pool their bounds: lower the query's pooled bound to this
      // list's, and read it back (applied after the scan, so that the load
      // has time to arrive).  Lane = row.
      const bool share = ++step_no == kShareSteps;
      if (share) step_no = 0;
      float pooled = __builtin_huge_valf();
      if (share && qbase + lane < nq) {
        const float t = s_tau[wave][lane];
        if (t >= 0.0f && t < __builtin_huge_valf()) lower_bound_to(bound + qbase + lane, t);
        pooled = read_bound(bound + qbase + lane);
      }
      const int buf_load = buf == 0 ? 2 : buf - 1;  // (buf + 2) % 3
      st2 = st1 >= 0 ? next_stage() : -1;
      if (st2 >= 0) load_stage(st2, buf_load);
      const bool flushed = scan_stage(s_stage + buf, (int64_t)st0 * kStage);
      if (share) {
        // the queued survivors, then the pooled bound (not for a row
        // outside the tiles' range (NaN) or without a query)
        if (queued > 0) flush(queued);
        queued = 0;
        const float t = s_tau[wave][lane];
        if (t == t && pooled < t) s_tau[wave][lane] = pooled;
        refresh_bounds();
      } else if (flushed) {
        refresh_bounds();
      }
      stage_wait_barrier(st2 >= 0);
      st0 = st1;
      st1 = st2;
      buf = buf == 2 ? 0 : buf + 1;
      ++scanned;
    }
    {
      const int64_t left = nq - qbase;
      pairs_scanned += (unsigned long long)scanned * kStage * (left > kWaveQ ? kWaveQ : left);
    }

    if (queued > 0) flush(queued);
    queued = 0;
    // ---- this list's k-th distance bound to each query's pooled bound
    if (lane < kWaveQ && qbase + lane < nq) {
      const float t = s_tau[wave][lane];
      if (t >= 0.0f && t < __builtin_huge_valf()) lower_bound_to(bound + qbase + lane, t);
    }
    if (chunk == 0) {
      const int64_t left = nq - qbase;
      queries_done += left < 0 ? 0 : (left > kWaveQ ? kWaveQ : left);
    }
    __syncthreads();
  }
  if (sa.stats) {
    for (int o = 32; o > 0; o >>= 1) max_err = fmax(max_err, __shfl_xor(max_err, o, 64));
    if (lane == 0) {
      atomicAdd(sa.stats + TNN_STAT_QUERIES, (unsigned long long)queries_done);
      atomicAdd(sa.stats + TNN_STAT_POINTS, pairs_scanned);
      atomicAdd(sa.stats + TNN_STAT_RESCORED, (unsigned long long)rescored);
      atomicMax(sa.stats + TNN_STAT_MAX_ERR, (unsigned long long)__double_as_longlong(max_err));
    }
  }
}

// One wave per query: the exact top-k of the union of its partial lists
// (each sorted by (distance, index), padded with (+inf, none)); position q
// of the scan order is caller query perm[q].
__global__ __launch_bounds__(256) void mixed_merge_kernel(const double *part_d,
                                                          const int32_t *part_i,
                                                          const float *bound, int n_slots,
                                                          const int32_t *perm, int64_t nq, int k,
                                                          double inf, int32_t *out_idx,
                                                          double *out_dist) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= nq) return;
  const int lane = lane_id();
  const int64_t qc = perm ? perm[q] : q;
  if (bound && __builtin_isnan(bound[q])) {  // the query's scaled norm exceeds the tiles' range
    if (lane < k) {
      out_idx[qc * k + lane] = -1;
      out_dist[qc * k + lane] = inf - inf;  // NaN (no 64-bit literal)
    }
    return;
  }
  TopK tk;
  tk.init(k, inf);
  for (int c = 0; c < n_slots; ++c) {
    const size_t o = ((size_t)q * n_slots + c) * k;
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
    out_idx[qc * k + lane] = tk.id == kNoId ? -1 : tk.id;
    out_dist[qc * k + lane] = tk.d;
  }
}

}  // namespace

// Points padded to whole stages.
static int64_t padded_points(int64_t n_points) {
  return (n_points + kStage - 1) / kStage * kStage;
}

// Point chunks per query tile: enough work items to keep a full chip busy
// to the end, each chunk at least kMinChunkStages stages (an item's set-up
// writes its lists: short chunks would spend more on that than on the scan).
constexpr int64_t kMinChunkStages = 64;
static int mixed_chunks(int64_t n_points, int64_t nq) {
  const int64_t tiles = (nq + kTileQ - 1) / kTileQ;
  const int64_t stages = padded_points(n_points) / kStage;
  int64_t c = tiles > 0 ? (8 * kNominalSlots + tiles - 1) / tiles : 1;
  if (c > kMaxChunks) c = kMaxChunks;
  if (c > (stages + kMinChunkStages - 1) / kMinChunkStages)
    c = (stages + kMinChunkStages - 1) / kMinChunkStages;
  return c < 1 ? 1 : (int)c;
}

namespace {
struct MixedLayout {
  int64_t np, chunks, slots, tiles, max_blocks;
  size_t ops, nv, part_d, part_i, bound, home, perm, bcount, tstart, stage_tmin, counter, total;
};

MixedLayout mixed_layout(int64_t n_points, int64_t nq, int k) {
  MixedLayout l;
  l.np = padded_points(n_points);
  l.chunks = mixed_chunks(n_points, nq);
  l.slots = l.chunks + 1;  // the chunks' lists and the pilot's
  l.tiles = (nq + kTileQ - 1) / kTileQ;
  // blocks of 64 segments, a segment holding at least one point
  l.max_blocks = (n_points + kBlockSegs - 1) / kBlockSegs + 1;
  const size_t entries = (size_t)nq * l.slots * k;
  size_t o = 0;
  l.ops = o;
  o += align_up((size_t)l.np * 64);
  l.nv = o;
  o += align_up((size_t)n_points * 4);
  l.part_d = o;
  o += align_up(entries * 8);
  l.part_i = o;
  o += align_up(entries * 4);
  l.bound = o;
  o += align_up((size_t)nq * 4);
  l.home = o;
  o += align_up((size_t)nq * 4);
  l.perm = o;
  o += align_up((size_t)nq * 4);
  l.bcount = o;
  o += align_up((size_t)l.max_blocks * 4);
  l.tstart = o;
  o += align_up((size_t)l.tiles * 8);
  l.stage_tmin = o;
  o += align_up((size_t)(l.np / kStage) * 4);
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
  // stage numbers, point slots and query positions are 32-bit in the search
  if (ix.n_blocks > l.max_blocks || l.np > INT32_MAX || qs.n > INT32_MAX)
    return hipErrorInvalidValue;
  char *base = static_cast<char *>(scratch);
  bf16x8 *ops = reinterpret_cast<bf16x8 *>(base + l.ops);
  float *nv = reinterpret_cast<float *>(base + l.nv);
  double *part_d = reinterpret_cast<double *>(base + l.part_d);
  int32_t *part_i = reinterpret_cast<int32_t *>(base + l.part_i);
  float *bound = reinterpret_cast<float *>(base + l.bound);
  int32_t *home = reinterpret_cast<int32_t *>(base + l.home);
  int32_t *perm = reinterpret_cast<int32_t *>(base + l.perm);
  int32_t *bcount = reinterpret_cast<int32_t *>(base + l.bcount);
  int64_t *tstart = reinterpret_cast<int64_t *>(base + l.tstart);
  float *stage_tmin = reinterpret_cast<float *>(base + l.stage_tmin);
  unsigned long long *counter = reinterpret_cast<unsigned long long *>(base + l.counter);
  const int64_t n_steps = l.np / kStage;
  const int64_t n_kd = qs.n;
  const int n_slots = (int)l.slots;
  if (n_steps == 0) {
    // no points: merging no lists leaves every slot a pad
    hipLaunchKernelGGL(mixed_merge_kernel, dim3((unsigned)((qs.n + 3) / 4)), dim3(256), 0, st,
                       part_d, part_i, (const float *)nullptr, 0, (const int32_t *)nullptr, qs.n,
                       a.k, a.inf,
                       out_idx, out_dist);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(mixed_prep_kernel, dim3((unsigned)((l.np + 255) / 256)), dim3(256), 0, st, ix,
                     mc, ops, nv, l.np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mixed_stage_time_kernel, dim3((unsigned)((n_steps + 3) / 4)), dim3(256), 0, st,
                     ix.pt4, ix.n_points, n_steps, stage_tmin);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n_reset = n_kd > ix.n_blocks ? n_kd : ix.n_blocks;
  hipLaunchKernelGGL(mixed_reset_kernel, dim3((unsigned)((n_reset + 255) / 256)), dim3(256), 0, st,
                     bound, n_kd, bcount, (int64_t)ix.n_blocks, counter);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // scan order: home blocks, counting sort, home ranges of the tiles
  const unsigned qgrid = (unsigned)((qs.n + 255) / 256);
  hipLaunchKernelGGL(mixed_home_kernel, dim3(qgrid), dim3(256), 0, st, ix, a, qs.x, qs.y, qs.z,
                     qs.t, qs.n, home, bcount);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mixed_offsets_kernel, dim3(1), dim3(1024), 0, st, bcount,
                     (int64_t)ix.n_blocks);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mixed_scatter_kernel, dim3(qgrid), dim3(256), 0, st, home, qs.n, bcount, perm);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mixed_tile_start_kernel, dim3((unsigned)((l.tiles + 255) / 256)), dim3(256), 0,
                     st, ix, home, perm, qs.n, l.tiles, n_steps, tstart);
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
  const int n_home = (int)(n_steps < kPilotStages ? n_steps : kPilotStages);
  const size_t lds = kStageBufs * sizeof(Stage);
  const int64_t resident = (int64_t)cu_count_mixed() * mixed_per_cu(lds);
  const int64_t pilot_waves = (qs.n + kPilotQ - 1) / kPilotQ;
  hipLaunchKernelGGL(mixed_pilot_kernel, dim3((unsigned)((pilot_waves + 3) / 4)), dim3(256), 0, st,
                     ix, a, qs.x, qs.y, qs.z, qs.t, perm, qs.n, tstart, stage_tmin, n_home, n_steps,
                     n_slots, part_d, part_i, bound);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t items = l.tiles * l.chunks;
  const int64_t grid = items < resident ? items : resident;
  SlowArgs sa;
  for (int f = 0; f < 4; ++f) sa.s[f] = a.s[f];
  sa.t_window = a.t_window;
  sa.inf = a.inf;
  sa.nv = nv;
  sa.stats = a.stats;
  sa.k = a.k;
  hipLaunchKernelGGL(mixed_brute_kernel, dim3((unsigned)grid), dim3(kWaves * 64), lds, st, ix.pt4,
                     ix.pid, ix.n_points, sa, mc, ops, qs.x, qs.y, qs.z, qs.t, perm, qs.n, part_d,
                     part_i, bound,
                     counter, tstart, stage_tmin, l.tiles, n_slots - 1, n_home, (int)n_steps,
                     (int)stride);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mixed_merge_kernel, dim3((unsigned)((qs.n + 3) / 4)), dim3(256), 0, st, part_d,
                     part_i, bound, n_slots, perm, qs.n, a.k, a.inf, out_idx, out_dist);
  return hipGetLastError();
}

}  // namespace tnn
