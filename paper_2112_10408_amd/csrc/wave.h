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

// This lane's bit of a wave-uniform lane mask (the mask itself serves as the
// per-lane condition: no shift or compare).
__device__ __forceinline__ bool lane_in(uint64_t mask) {
  return __builtin_amdgcn_inverse_ballot_w64(mask);
}

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

// Wave-wide minimum / maximum of non-negative floats (or +inf) as a
// wave-uniform value.  Non-negative floats order like their bit patterns as
// int32, so integer min / max does the comparisons.  DPP steps reduce each
// row of 16 lanes (lanes a step does not write read the identity of the
// operation, which lets the compiler fold each step into one min / max), row
// broadcasts carry the row results into lane 63, and reading that lane makes
// the result uniform.
constexpr int kDppRowBcast15 = 0x142;  // lane 15 of each row to the next row
constexpr int kDppRowBcast31 = 0x143;  // lane 31 to rows 2 and 3

template <bool Max, int Ctrl, int RowMask = 0xF>
__device__ __forceinline__ int ext_step(int v) {
  constexpr int ident = Max ? (int)0x80000000 : 0x7fffffff;
  const int o = __builtin_amdgcn_update_dpp(ident, v, Ctrl, RowMask, 0xF, false);
  return Max ? max(v, o) : min(v, o);
}

template <bool Max>
__device__ __forceinline__ int wave_ext_bits(int v) {
  v = ext_step<Max, kDppQuadXor1>(v);
  v = ext_step<Max, kDppQuadXor2>(v);
  v = ext_step<Max, kDppRowRor4>(v);
  v = ext_step<Max, kDppRowRor8>(v);
  v = ext_step<Max, kDppRowBcast15, 0xA>(v);
  v = ext_step<Max, kDppRowBcast31, 0xC>(v);
  return __builtin_amdgcn_readlane(v, 63);
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

// The lane holding the smallest of the non-negative floats `v` of the lanes
// set in `mask` (wave-uniform, non-zero; the lowest such lane on ties) and
// that value.  A single candidate needs no reduction.
__device__ __forceinline__ int pick_min(uint64_t mask, float v, float &vmin) {
  if ((mask & (mask - 1)) == 0) {
    const int l = __ffsll((long long)mask) - 1;
    vmin = readlane_f(v, l);
    return l;
  }
  return wave_argmin_lane(lane_in(mask) ? v : __builtin_huge_valf(), vmin);
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

// A (distance, index) key as three words: the distance's high and low halves
// and the index.  Distances handed to the sorting network are +0 .. +inf and
// indices are non-negative, so the unsigned lexicographic order of (hi, lo,
// index) is the order of key_lt, and a 96-bit subtraction's borrow decides a
// comparison in three carry-chained instructions.
struct Key3 {
  unsigned h, l, i;
};

__device__ __forceinline__ Key3 key3(double d, int id) {
  return Key3{(unsigned)hi32(d), (unsigned)lo32(d), (unsigned)id};
}

// Lanes that keep the smaller key of their pair in the stage (Size, J) of a
// bitonic sort over 64 lanes (ascending blocks of Size alternate with
// descending ones; Desc flips them all).
constexpr uint64_t keep_min_mask(int size, int j, bool desc) {
  uint64_t m = 0;
  for (int l = 0; l < 64; ++l) {
    const bool asc = ((l & size) == 0) != desc;
    if (((l & j) == 0) == asc) m |= 1ull << l;
  }
  return m;
}

// One compare-exchange stage with the partner lane read through a DPP
// control.  vcc first gets (partner < mine), then is flipped in the lanes
// that keep the smaller key, so that it is set exactly where a lane keeps its
// own key; the selects read the partner through the same control.  Each
// stage starts with two wait states: a DPP read of a register written by the
// previous vector instruction needs them.
#define TNN_CX_DPP(CTRL)                                                                   \
  "s_nop 1\n\t"                                                                            \
  "v_sub_co_u32_dpp %[t], vcc, %[i], %[i] " CTRL " row_mask:0xf bank_mask:0xf\n\t"         \
  "v_subb_co_u32_dpp %[t], vcc, %[l], %[l], vcc " CTRL " row_mask:0xf bank_mask:0xf\n\t"   \
  "v_subb_co_u32_dpp %[t], vcc, %[h], %[h], vcc " CTRL " row_mask:0xf bank_mask:0xf\n\t"   \
  "s_xor_b32 vcc_lo, vcc_lo, %[mlo]\n\t"                                                   \
  "s_xor_b32 vcc_hi, vcc_hi, %[mhi]\n\t"                                                   \
  "v_cndmask_b32_dpp %[i], %[i], %[i], vcc " CTRL " row_mask:0xf bank_mask:0xf\n\t"        \
  "v_cndmask_b32_dpp %[l], %[l], %[l], vcc " CTRL " row_mask:0xf bank_mask:0xf\n\t"        \
  "v_cndmask_b32_dpp %[h], %[h], %[h], vcc " CTRL " row_mask:0xf bank_mask:0xf"

// Keeps `k` where the mask bit of the lane says so given (o < k), else takes
// `o` (the partner's key, already in registers).
template <uint64_t M>
__device__ __forceinline__ void cx_with(Key3 &k, const Key3 &o) {
  unsigned t;
  asm volatile(
      "v_sub_co_u32 %[t], vcc, %[oi], %[i]\n\t"
      "v_subb_co_u32 %[t], vcc, %[ol], %[l], vcc\n\t"
      "v_subb_co_u32 %[t], vcc, %[oh], %[h], vcc\n\t"
      "s_xor_b32 vcc_lo, vcc_lo, %[mlo]\n\t"
      "s_xor_b32 vcc_hi, vcc_hi, %[mhi]\n\t"
      "v_cndmask_b32 %[i], %[oi], %[i], vcc\n\t"
      "v_cndmask_b32 %[l], %[ol], %[l], vcc\n\t"
      "v_cndmask_b32 %[h], %[oh], %[h], vcc"
      : [h] "+v"(k.h), [l] "+v"(k.l), [i] "+v"(k.i), [t] "=&v"(t)
      : [oh] "v"(o.h), [ol] "v"(o.l), [oi] "v"(o.i), [mlo] "i"((unsigned)M),
        [mhi] "i"((unsigned)(M >> 32))
      : "vcc");
}

// Compare-exchange of the keys of lanes l and l ^ J: lanes whose bit is set
// in M keep the smaller key, the others the larger.  Equal keys are
// identical, so either choice is the same.
template <int J, uint64_t M>
__device__ __forceinline__ void cmpx(Key3 &k) {
  constexpr unsigned mlo = (unsigned)M, mhi = (unsigned)(M >> 32);
  unsigned t;
  if constexpr (J == 1) {
    asm volatile(TNN_CX_DPP("quad_perm:[1,0,3,2]")
                 : [h] "+v"(k.h), [l] "+v"(k.l), [i] "+v"(k.i), [t] "=&v"(t)
                 : [mlo] "i"(mlo), [mhi] "i"(mhi)
                 : "vcc");
  } else if constexpr (J == 2) {
    asm volatile(TNN_CX_DPP("quad_perm:[2,3,0,1]")
                 : [h] "+v"(k.h), [l] "+v"(k.l), [i] "+v"(k.i), [t] "=&v"(t)
                 : [mlo] "i"(mlo), [mhi] "i"(mhi)
                 : "vcc");
  } else if constexpr (J == 8) {
    asm volatile(TNN_CX_DPP("row_ror:8")
                 : [h] "+v"(k.h), [l] "+v"(k.l), [i] "+v"(k.i), [t] "=&v"(t)
                 : [mlo] "i"(mlo), [mhi] "i"(mhi)
                 : "vcc");
  } else if constexpr (J == 4) {
    // no single DPP control swaps lanes 4 apart: an LDS swizzle
    const Key3 o{(unsigned)xor_lane<4>((int)k.h), (unsigned)xor_lane<4>((int)k.l),
                 (unsigned)xor_lane<4>((int)k.i)};
    cx_with<M>(k, o);
  } else {
    // 16 or 32 lanes apart: permlane swaps give the lower lane's key (a) and
    // the upper lane's key (b) in both lanes; keep a where (b < a) differs
    // from the mask, else take b
    int ah, bh, al, bl, ai, bi;
    lane_pair<J>((int)k.h, ah, bh);
    lane_pair<J>((int)k.l, al, bl);
    lane_pair<J>((int)k.i, ai, bi);
    k = Key3{(unsigned)ah, (unsigned)al, (unsigned)ai};
    cx_with<M>(k, Key3{(unsigned)bh, (unsigned)bl, (unsigned)bi});
  }
  (void)t;
}

template <bool Desc, int Size, int J>
__device__ __forceinline__ void sort_stage(Key3 &k) {
  cmpx<J, keep_min_mask(Size, J, Desc)>(k);
  if constexpr (J > 1) sort_stage<Desc, Size, J / 2>(k);
}

template <bool Desc, int Size>
__device__ __forceinline__ void sort_upto(Key3 &k) {
  if constexpr (Size > 2) sort_upto<Desc, Size / 2>(k);
  sort_stage<Desc, Size, Size / 2>(k);
}

// Bitonic sort of 64 keys by lane, ascending (Desc = false) or descending.
// A DPP read needs five wait states after a write of EXEC, which the code
// before a network may end with.
__device__ __forceinline__ void dpp_entry() { asm volatile("s_nop 4"); }

template <bool Desc = false>
__device__ __forceinline__ void sort64(Key3 &k) {
  dpp_entry();
  sort_upto<Desc, 64>(k);
}

// Sort a bitonic sequence of 64 keys ascending.
__device__ __forceinline__ void merge64(Key3 &k) {
  dpp_entry();
  sort_stage<false, 64, 32>(k);
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

  // Offer one key per lane; lanes outside the lane mask `gm` offer nothing.
  // Returns nothing; updates the threshold.
  __device__ __forceinline__ void offer(uint64_t gm, double nd, int nid) {
    nd += 0.0;  // -0.0 becomes +0.0, which the word order of the merge needs
    const int n = __popcll(gm);
    if (n <= kInsertMax) {
      while (gm) {
        const int l = __ffsll((long long)gm) - 1;
        gm &= gm - 1;
        insert_one(readlane_d(nd, l), readlane_i(nid, l));
      }
    } else {
      const bool in = lane_in(gm);
      Key3 c = key3(in ? nd : inf_, in ? nid : kNoId);
      if (!(readlane_d(d, 0) < inf_)) {  // empty top-k: the sorted batch is the result
        sort64<false>(c);
      } else {
        // descending batch against the ascending top-k: the lane-wise
        // smaller keys form a bitonic sequence holding the 64 smallest
        sort64<true>(c);
        Key3 m = key3(d, id);
        cx_with<~0ull>(m, c);
        c = m;
        merge64(c);
      }
      d = mk_double((int)c.l, (int)c.h);
      id = (int)c.i;
    }
    refresh();
  }
};

}  // namespace tnn
