// Wavefront-level primitives for gfx950 (64 lanes): broadcasts, reductions
// and a register-resident top-k of (distance, index) keys, one rank per lane.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tnn {

constexpr double kInf = __builtin_huge_val();
constexpr int kNoId = 0x7fffffff;
// Newcomers up to this count are inserted one by one; more are sorted and
// merged with a bitonic network.
constexpr int kInsertMax = 12;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p); }

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32));
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(v & 0xffffffffull));
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Lexicographic (distance, caller index) order of the result.
// Branch-free on purpose: short-circuit forms turn every compare-exchange of
// the sorting network into divergent branches.
__device__ __forceinline__ bool key_lt(double a, int ia, double b, int ib) {
  return (a < b) | ((a == b) & (ia < ib));
}

// Wave-wide argmin; every lane returns the same (value, index); ties take the
// smaller index.
__device__ __forceinline__ void wave_argmin_f(float &v, int &i) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const float ov = __shfl_xor(v, m, 64);
    const int oi = __shfl_xor(i, m, 64);
    if (ov < v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
}

__device__ __forceinline__ void wave_argmin_d(double &v, int &i) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const double ov = __shfl_xor(v, m, 64);
    const int oi = __shfl_xor(i, m, 64);
    if (ov < v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
  return v;
}

// Value of lane ^ j (j a power of two known after unrolling): DPP quad
// permutes for 1 and 2, LDS swizzle for 4..16, a permute for 32.
__device__ __forceinline__ int xor_lane(int v, int j) {
  if (j == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  if (j == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  if (j == 4) return __builtin_amdgcn_ds_swizzle(v, 0x1F | (4 << 10));
  if (j == 8) return __builtin_amdgcn_ds_swizzle(v, 0x1F | (8 << 10));
  if (j == 16) return __builtin_amdgcn_ds_swizzle(v, 0x1F | (16 << 10));
  return __shfl_xor(v, j, 64);
}

__device__ __forceinline__ double xor_lane_d(double v, int j) {
  const long long b = __double_as_longlong(v);
  const int lo = xor_lane((int)(b & 0xffffffffll), j);
  const int hi = xor_lane((int)(b >> 32), j);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Compare-exchange with lane ^ j: keep the smaller key if `keep_min`.
__device__ __forceinline__ void cmpx(double &d, int &id, int j, bool keep_min) {
  const double od = xor_lane_d(d, j);
  const int oid = xor_lane(id, j);
  const bool other_lt = key_lt(od, oid, d, id);
  const bool other_gt = key_lt(d, id, od, oid);
  if (keep_min ? other_lt : other_gt) {
    d = od;
    id = oid;
  }
}

// Bitonic sort of 64 keys, ascending by lane.
__device__ __forceinline__ void sort64(double &d, int &id) {
  const int l = lane_id();
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
    for (int j = size >> 1; j > 0; j >>= 1) {
      const bool asc = (l & size) == 0;
      const bool lower = (l & j) == 0;
      cmpx(d, id, j, lower == asc);
    }
  }
}

// Sort a bitonic sequence of 64 keys ascending.
__device__ __forceinline__ void merge64(double &d, int &id) {
  const int l = lane_id();
#pragma unroll
  for (int j = 32; j > 0; j >>= 1) cmpx(d, id, j, (l & j) == 0);
}

// Top-k over (distance, index): lane r holds the r-th smallest key seen so
// far (r < 64; ranks >= k are kept but never reported).  kd/kid mirror rank
// k-1 in every lane and are the admission threshold.
struct TopK {
  double d;
  int id;
  double kd;
  int kid;
  int k;
  double inf_;

  // `inf` must be +infinity passed in from the host (a kernel argument):
  // a compile-time +inf held in a scalar register pair is materialised with
  // a 64-bit literal move that the gfx950 assembler truncates to 0.
  __device__ __forceinline__ void init(int k_, double inf) {
    d = inf;
    id = kNoId;
    kd = inf;
    kid = kNoId;
    k = k_;
    inf_ = inf;
  }

  __device__ __forceinline__ bool admits(double nd, int nid) const {
    return (nd < kInf) & key_lt(nd, nid, kd, kid);
  }

  __device__ __forceinline__ void refresh() {
    kd = readlane_d(d, k - 1);
    kid = readlane_i(id, k - 1);
  }

  // Insert one key (wave-uniform) keeping lanes sorted.
  __device__ __forceinline__ void insert_one(double c, int cid) {
    const int l = lane_id();
    const bool before = key_lt(c, cid, d, id);  // candidate ranks ahead of my key
    const int src = l > 0 ? l - 1 : 0;
    const double up = __shfl(d, src, 64);
    const int upid = __shfl(id, src, 64);
    const bool prev_before = __shfl((int)before, src, 64) != 0 && l > 0;
    if (before) {
      if (prev_before) {
        d = up;
        id = upid;
      } else {
        d = c;
        id = cid;
      }
    }
  }

  // Offer one key per lane; lanes with gate=false offer nothing.  `gm` is the
  // ballot of gate.  Returns nothing; updates the threshold.
  __device__ __forceinline__ void offer(uint64_t gm, bool gate, double nd, int nid) {
    const int n = __popcll(gm);
    if (n <= kInsertMax) {
      while (gm) {
        const int l = __ffsll((long long)gm) - 1;
        gm &= gm - 1;
        insert_one(readlane_d(nd, l), readlane_i(nid, l));
      }
    } else {
      double cd = gate ? nd : inf_;
      int cid = gate ? nid : kNoId;
      sort64(cd, cid);
      if (!(readlane_d(d, 0) < inf_)) {  // empty top-k: the sorted batch is the result
        d = cd;
        id = cid;
        refresh();
        return;
      }
      const int rl = 63 - lane_id();
      const double rd = __shfl(cd, rl, 64);
      const int rid = __shfl(cid, rl, 64);
      if (key_lt(rd, rid, d, id)) {
        d = rd;
        id = rid;
      }
      merge64(d, id);
    }
    refresh();
  }
};

}  // namespace tnn
