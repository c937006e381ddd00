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

// Orders a wave's own LDS writes before its later reads of other lanes'
// entries (the lanes of a wave run in lockstep; this only stops the compiler
// from moving memory operations across the point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lexicographic (distance, caller index) order of the result.
// Branch-free on purpose: short-circuit forms turn every compare-exchange of
// the sorting network into divergent branches.
__device__ __forceinline__ bool key_lt(double a, int ia, double b, int ib) {
  return (a < b) | ((a == b) & (ia < ib));
}

// DPP controls (gfx9 encoding) used below.
constexpr int kDppQuadXor1 = 0xB1;  // quad_perm [1,0,3,2]: lane ^ 1
constexpr int kDppQuadXor2 = 0x4E;  // quad_perm [2,3,0,1]: lane ^ 2
constexpr int kDppRowRor4 = 0x124;  // lane (l - 4) mod 16 within its row of 16
constexpr int kDppRowRor8 = 0x128;  // lane (l + 8) mod 16 = lane ^ 8
constexpr int kDppWaveShr1 = 0x138; // lane l - 1

template <int Ctrl>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, Ctrl, 0xF, 0xF, false);
}
template <int Ctrl>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), Ctrl, 0xF, 0xF, false));
}

// Both values of each lane pair (l, l ^ J), J = 16 or 32, in every lane:
// `lo` from the lane whose bit J is clear, `hi` from the lane whose bit J is
// set (gfx950 permlane swaps: no LDS round trip).
template <int J>
__device__ __forceinline__ void lane_pair(int v, int &lo, int &hi) {
  static_assert(J == 16 || J == 32, "pair exchange spans 16 or 32 lanes");
  if constexpr (J == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    lo = (int)r[0];
    hi = (int)r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    lo = (int)r[0];
    hi = (int)r[1];
  }
}

// Wave-wide minimum / maximum of non-negative floats (or +inf), the result in
// every lane: quad and row steps by DPP, row pairs and wave halves by
// permlane swaps.  Non-negative floats order like their bit patterns as
// int32, so integer min / max does the comparisons.
template <bool Max>
__device__ __forceinline__ int wave_ext_bits(int v) {
  auto f = [](int a, int b) { return Max ? max(a, b) : min(a, b); };
  v = f(v, dpp_i<kDppQuadXor1>(v));
  v = f(v, dpp_i<kDppQuadXor2>(v));
  v = f(v, dpp_i<kDppRowRor4>(v));
  v = f(v, dpp_i<kDppRowRor8>(v));
  int a, b;
  lane_pair<16>(v, a, b);
  v = f(a, b);
  lane_pair<32>(v, a, b);
  return f(a, b);
}

__device__ __forceinline__ float wave_min_nonneg(float v) {
  return __int_as_float(wave_ext_bits<false>(__float_as_int(v)));
}

__device__ __forceinline__ float wave_max_nonneg(float v) {
  return __int_as_float(wave_ext_bits<true>(__float_as_int(v)));
}

// Wave-wide argmin of a non-negative float (or +inf): the minimum and the
// lowest lane that holds it, in every lane.
__device__ __forceinline__ int wave_argmin_lane(float v, float &vmin) {
  vmin = wave_min_nonneg(v);
  return __ffsll((long long)ballot(v == vmin)) - 1;
}

// Value of lane ^ J for J = 1, 2, 4, 8 (DPP quad permutes and row rotation;
// an LDS swizzle for 4).
template <int J>
__device__ __forceinline__ int xor_lane(int v) {
  static_assert(J == 1 || J == 2 || J == 4 || J == 8, "xor_lane spans a row");
  if constexpr (J == 1) return dpp_i<kDppQuadXor1>(v);
  else if constexpr (J == 2) return dpp_i<kDppQuadXor2>(v);
  else if constexpr (J == 4) return __builtin_amdgcn_ds_swizzle(v, 0x1F | (4 << 10));
  else return dpp_i<kDppRowRor8>(v);
}

__device__ __forceinline__ int lo32(double v) { return (int)(__double_as_longlong(v) & 0xffffffffll); }
__device__ __forceinline__ int hi32(double v) { return (int)(__double_as_longlong(v) >> 32); }
__device__ __forceinline__ double mk_double(int lo, int hi) {
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Compare-exchange of the keys of lanes l and l ^ J: lanes with `keep_min`
// keep the smaller key, the others the larger.  One comparison decides both
// sides (equal keys are identical, so taking either is the same).
template <int J>
__device__ __forceinline__ void cmpx(double &d, int &id, bool keep_min) {
  if constexpr (J >= 16) {
    int al, bl, ah, bh, ai, bi;
    lane_pair<J>(lo32(d), al, bl);
    lane_pair<J>(hi32(d), ah, bh);
    lane_pair<J>(id, ai, bi);
    const double ad = mk_double(al, ah), bd = mk_double(bl, bh);
    const bool b_lt = key_lt(bd, bi, ad, ai);  // the upper lane's key is the smaller
    const bool take_b = keep_min == b_lt;
    d = take_b ? bd : ad;
    id = take_b ? bi : ai;
  } else {
    const double od = mk_double(xor_lane<J>(lo32(d)), xor_lane<J>(hi32(d)));
    const int oid = xor_lane<J>(id);
    const bool o_lt = key_lt(od, oid, d, id);
    if (keep_min == o_lt) {
      d = od;
      id = oid;
    }
  }
}

template <bool Desc, int Size, int J>
__device__ __forceinline__ void sort_stage(double &d, int &id, int l) {
  const bool asc = ((l & Size) == 0) != Desc;
  const bool lower = (l & J) == 0;
  cmpx<J>(d, id, lower == asc);
  if constexpr (J > 1) sort_stage<Desc, Size, J / 2>(d, id, l);
}

template <bool Desc, int Size>
__device__ __forceinline__ void sort_upto(double &d, int &id, int l) {
  if constexpr (Size > 2) sort_upto<Desc, Size / 2>(d, id, l);
  sort_stage<Desc, Size, Size / 2>(d, id, l);
}

// Bitonic sort of 64 keys by lane, ascending (Desc = false) or descending.
template <bool Desc = false>
__device__ __forceinline__ void sort64(double &d, int &id) {
  sort_upto<Desc, 64>(d, id, lane_id());
}

template <int J>
__device__ __forceinline__ void merge_stage(double &d, int &id, int l) {
  cmpx<J>(d, id, (l & J) == 0);
  if constexpr (J > 1) merge_stage<J / 2>(d, id, l);
}

// Sort a bitonic sequence of 64 keys ascending.
__device__ __forceinline__ void merge64(double &d, int &id) { merge_stage<32>(d, id, lane_id()); }

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
    // keys of lane l - 1 (whole-wave shift; lane 0 reads nothing useful)
    const double up = mk_double(dpp_i<kDppWaveShr1>(lo32(d)), dpp_i<kDppWaveShr1>(hi32(d)));
    const int upid = dpp_i<kDppWaveShr1>(id);
    const bool prev_before = dpp_i<kDppWaveShr1>((int)before) != 0 && l > 0;
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
      if (!(readlane_d(d, 0) < inf_)) {  // empty top-k: the sorted batch is the result
        sort64<false>(cd, cid);
        d = cd;
        id = cid;
      } else {
        // descending batch against the ascending top-k: the lane-wise
        // smaller keys form a bitonic sequence holding the 64 smallest
        sort64<true>(cd, cid);
        if (key_lt(cd, cid, d, id)) {
          d = cd;
          id = cid;
        }
        merge64(d, id);
      }
    }
    refresh();
  }
};

}  // namespace tnn
