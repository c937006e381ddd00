// Query kernels: per-call segment preparation, TNN search (plain and
// learned-radius seeded), linear search, and the bound export for tests.
#include <mutex>

#include "bounds.h"
#include "gka.h"
#include "query.h"
#include "radius_infer.h"

namespace tnn {

constexpr size_t kLdsBoxBytes = 48 * 1024;  // stage block boxes in LDS up to this size
#ifndef TNN_BRUTE_Q
#define TNN_BRUTE_Q 4
#endif
constexpr int kBruteQ = TNN_BRUTE_Q;  // queries per wave of the linear search

#ifndef TNN_QUERY_QUEUES
#define TNN_QUERY_QUEUES 16
#endif
// Queries a wave takes from a work queue at a time (0: fixed grid stride).
// The atomics on a counter serialise: with 8 counters, tickets of 2 queries
// cost 8 % of the 1M-point learned search against tickets of 8.  (The largest
// ticket; small query counts take smaller ones.)
#ifndef TNN_QUERY_CHUNK
#define TNN_QUERY_CHUNK 8
#endif
// The queries are split into kQueues contiguous slices with one counter
// each (one counter for all would serialise the atomics); a workgroup starts
// on slice blockIdx mod kQueues (dispatch is round-robin over the 8 dies, so
// each die's workgroups share two slices) and moves on to the next slice
// once its own is used up.
constexpr int kQueues = TNN_QUERY_QUEUES;
// The batched search splits its queue into 8 slices: with 16 its throughput
// was 2 % lower and the median per-airspace latency 15 % higher.
constexpr int kBatchQueues = 8;
constexpr int kTicketStride = 32;  // counters 256 bytes apart
// Resident workgroups (of 4 waves) per CU for the search: with its 68 VGPRs
// 7 would fit, but on the 1M-point learned search 5 ran fastest (7: 0.221 ms,
// 6: 0.205, 5: 0.202, 4: 0.213, 3: 0.240; L2 hit rate 81 % at both 4 and
// 7): more concurrent queries only add contention.
constexpr int kMaxSearchBlocksPerCu = 5;
static_assert(kQueues >= 1 && kQueues <= 16, "the query workspace holds 16 counters");

// ---------------------------------------------------------------------------
// Per-call preparation (depends on the scales): the segment records the
// search reads, with 1/|AB|_s^2, the radius R = sqrt(sum_f s_f e_f^2) rounded
// up, and the projection slack.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void prep_one(const IndexDesc &ix, const QueryArgs &a, float4 *rec,
                                         int64_t s, bool raw = false) {
  const float ax = ix.ax[s], ay = ix.ay[s], az = ix.az[s];
  const float bx = ix.bx[s], by = ix.by[s], bz = ix.bz[s];
  // AB as the bound computes it (float32 differences), norms in binary64
  const float fx = bx - ax, fy = by - ay, fz = bz - az;
  const double abx = (double)fx, aby = (double)fy, abz = (double)fz;
  const double n2 = a.s[0] * abx * abx + a.s[1] * aby * aby + a.s[2] * abz * abz;
  const float inv_n2 = n2 > 0.0 ? (float)(1.0 / n2) : 0.0f;
  const double ex = ix.ex[s], ey = ix.ey[s], ez = ix.ez[s];
  const float rad = __double2float_ru(sqrt(a.s[0] * ex * ex + a.s[1] * ey * ey + a.s[2] * ez * ez) *
                                      (1.0 + 0x1p-40));
  // exact AB and its norm bound the float32 errors of the bound
  const double tx = (double)bx - (double)ax;
  const double ty = (double)by - (double)ay;
  const double tz = (double)bz - (double)az;
  const double nt = sqrt(a.s[0] * tx * tx + a.s[1] * ty * ty + a.s[2] * tz * tz);
  const float slack = __double2float_ru(0x1p-17 * (nt + sqrt(n2)) * 0.5 * (1.0 + 0x1p-30));
  const int64_t S = ix.n_seg;
  rec[s] = make_float4(ax, ay, az, ix.tmin[s]);
  rec[S + s] = make_float4(fx, fy, fz, ix.tmax[s]);
  // with per-query scales the search forms these constants per query
  // (seg_lb_q) from the deviation bounds
  rec[2 * S + s] = raw ? make_float4(ix.ex[s], ix.ey[s], ix.ez[s], 0.0f)
                       : make_float4(inv_n2, rad, slack, 0.0f);
  reinterpret_cast<int2 *>(rec + 3 * S)[s] = make_int2(ix.pstart[s], ix.pcount[s]);
}

__global__ void prep_kernel(IndexDesc ix, QueryArgs a, float4 *rec, unsigned long long *ticket,
                            bool raw) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // the search kernel that follows starts its queues at 0
  if (s < kQueues && ticket) ticket[s * kTicketStride] = 0;
  if (s >= ix.n_seg) return;
  prep_one(ix, a, rec, s, raw);
}

// The preparation (workgroups below prep_blocks) and the radius prediction of
// every query (the others, one tile loop each), in one launch: the two are
// independent, and the search needs both.
__global__ __launch_bounds__(64 * radius::kInferWaves) void prep_infer_kernel(
    IndexDesc ix, QueryArgs a, float4 *rec, unsigned long long *ticket, bool raw,
    int64_t prep_blocks, tnn_points q, float *radius2, int64_t infer_groups) {
  if ((int64_t)blockIdx.x < prep_blocks) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < kQueues && ticket) ticket[s * kTicketStride] = 0;
    if (s < ix.n_seg) prep_one(ix, a, rec, s, raw);
    return;
  }
  radius::infer_tiles(a.model, q, a.alpha, radius2, nullptr, (int64_t)blockIdx.x - prep_blocks,
                      infer_groups);
}

// Copy n float4 from global memory to LDS with this workgroup's threads, four
// loads of a thread in flight before its first store (a rolled loop would wait
// out one global-load latency per element).  The loads are unconditional (an
// index past the end reads the last element; n >= 1 inside the loop) so that
// no branch makes the compiler wait for each one.
__device__ __forceinline__ void stage_to_lds(float4 *dst, const float4 *src, int n) {
  const int bs = (int)blockDim.x;
  for (int i0 = threadIdx.x; i0 < n; i0 += 4 * bs) {
    const int i1 = i0 + bs, i2 = i0 + 2 * bs, i3 = i0 + 3 * bs;
    const float4 a0 = src[i0];
    const float4 a1 = src[i1 < n ? i1 : n - 1];
    const float4 a2 = src[i2 < n ? i2 : n - 1];
    const float4 a3 = src[i3 < n ? i3 : n - 1];
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the stores
    dst[i0] = a0;
    if (i1 < n) dst[i1] = a1;
    if (i2 < n) dst[i2] = a2;
    if (i3 < n) dst[i3] = a3;
  }
}

// ---------------------------------------------------------------------------
// One wavefront answers one query.
// ---------------------------------------------------------------------------
// Per-wave work counters for the statistics output.  With On = false every
// update compiles to nothing, so searches run without statistics carry no
// counter registers or instructions.
template <bool On>
struct Counter {
  uint32_t v = 0;
  __device__ __forceinline__ void operator+=(uint32_t x) { v += x; }
  __device__ __forceinline__ void operator++() { ++v; }
  __device__ __forceinline__ void set(uint32_t x) { v = x; }
};
template <>
struct Counter<false> {
  __device__ __forceinline__ void operator+=(uint32_t) {}
  __device__ __forceinline__ void operator++() {}
  __device__ __forceinline__ void set(uint32_t) {}
};

template <bool On>
struct WaveStats {
  Counter<On> blocks, segs, points, merges, rounds, fallback;
};

template <bool PerQ, bool Stats>
struct Searcher {
  const IndexDesc &ix;
  const Prep &pr;
  const QueryArgs &a;
  QueryPoint q;
  TopK tk;
  WaveStats<Stats> st;
  int lane;
  int spi_shift;  // log2(kpad): lanes per segment when scanning points
  const float *box;   // block boxes (global memory or an LDS copy)
  const float *sbox;  // superblock boxes (global memory or an LDS copy)

  __device__ Searcher(const IndexDesc &ix_, const Prep &pr_, const QueryArgs &a_)
      : ix(ix_), pr(pr_), a(a_) {}

  // cylinder bound of a segment for this query's metric
  __device__ __forceinline__ float seg_bound(const SegView &sv) const {
    if constexpr (PerQ)
      return seg_lb_q(sv, q, a.s, a.sf);
    else
      return seg_lb(sv, q, a.sf);
  }

  // Scan the member points of the segments of block `bb` whose lanes are set
  // in `cm`, feeding the top-k, nearest key first.  Several segments share one
  // 64-lane pass; after each pass the segments whose key now exceeds the k-th
  // distance are dropped.  (ps_l, pc_l, key_l): this lane's segment's first
  // point slot, member count and key (non-negative float).
  __device__ void scan(uint64_t cm, int bb, int ps_l, int pc_l, float key_l) {
    const int kpad = 1 << spi_shift;
    const int spi = kWave >> spi_shift;
    const int slot = lane >> spi_shift;
    const int off = lane & (kpad - 1);
    while (cm) {
      int my_l = -1;
      for (int i = 0; i < spi && cm; ++i) {
        int l;
        if (__popcll(cm) <= spi - i) {
          // every remaining segment gets a slot in this pass: order is moot
          l = __ffsll((long long)cm) - 1;
        } else {
          float kmin;
          l = wave_argmin_lane(lane_in(cm) ? key_l : __builtin_huge_valf(), kmin);
        }
        cm &= ~(1ull << l);
        if (slot == i) my_l = l;
      }
      const bool has = my_l >= 0;
      // every lane must take part in the cross-lane reads: a lane that is
      // switched off does not supply its register
      const int src = has ? my_l : 0;
      const int ps = __shfl(ps_l, src, 64);
      const int pc_src = __shfl(pc_l, src, 64);
      const int pc = has ? pc_src : 0;
      const bool ok = has && off < pc;
      const int p = ps + off;
      float4 pv = make_float4(0.f, 0.f, 0.f, 0.f);
      int pid = kNoId;
      if (ok) {
        pv = ix.pt4[p];
        pid = ix.pid[p];
      }
      const double d = exact_dist(a.s, q.x, q.y, q.z, q.t, pv.x, pv.y, pv.z, pv.w);
      const bool valid = ok && pv.w < q.thrf;
      st.points += (uint32_t)__popcll(ballot(ok));
      const bool gate = valid && tk.admits(d, pid);
      const uint64_t gm = ballot(gate);
      if (gm) {
        tk.offer(gm, d, pid);
        ++st.merges;
        cm &= ballot((double)key_l <= tk.kd);
      }
    }
  }

  // This lane's segment record of block bb (an empty view past the end).
  __device__ __forceinline__ SegView fetch_block(int bb) const {
    const int64_t s = (int64_t)bb * kBlockSegs + lane;
    SegView sv{};
    if (s < ix.n_seg) sv = load_seg(pr, s);
    return sv;
  }

  // Scan the segments of block bb (bound bmin, this lane's record sv) whose
  // key lies in (prev, tau_cur], seeded segments excluded.  A segment's key
  // is the larger of its cylinder bound and its block's bound: both hold for
  // every member.
  __device__ __forceinline__ void visit_block(int bb, float bmin, const SegView &sv,
                                              double tau_cur, double prev, int seed_block,
                                              uint64_t seed_mask) {
    const int64_t S = ix.n_seg;
    const int64_t s = (int64_t)bb * kBlockSegs + lane;
    const float key_f = fmaxf(s < S ? seg_bound(sv) : __builtin_huge_valf(), bmin);
    const double key = (double)key_f;
    st.segs += (uint32_t)min((int64_t)kBlockSegs, S - (int64_t)bb * kBlockSegs);
    const bool seeded = bb == seed_block && lane_in(seed_mask);
    // a masked segment (infinite key) holds no candidate
    const bool cand = s < S && key < kInf && key <= tau_cur && key > prev && !seeded;
    const uint64_t cm = ballot(cand);
    if (cm) scan(cm, bb, sv.ps, sv.pc, key_f);
  }

  // One expansion round.  A segment's key is the larger of its cylinder
  // bound and its block's bound; every segment with prev < key <= min(tau,
  // k-th) is scanned (seeded segments excluded).  Rounds use increasing tau,
  // so a segment is scanned in the first round whose tau reaches its key, or
  // never when its key already exceeded the k-th distance then.  Returns, per
  // lane, the largest finite block or superblock bound that lane saw (the
  // caller reduces it only in the rare round that found fewer than k points).
  __device__ float round(double prev, double tau, int seed_block, uint64_t seed_mask) {
    const int nb = ix.n_blocks;
    const int ns = ix.n_super;
    const float finf = __builtin_huge_valf();
    float maxfin = 0.0f;
    // superblock level: 64 superblock bounds per pass
    for (int sbase = 0; sbase < ns; sbase += kWave) {
      const int sb = sbase + lane;
      const float lbs = sb < ns ? block_lb(sbox, sb, q, a.sf) : finf;
      st.blocks += (uint32_t)min(kWave, ns - sbase);
      if (lbs < finf) maxfin = fmaxf(maxfin, lbs);
      uint64_t ms = ballot(lbs < finf && (double)lbs <= fmin(tau, tk.kd));
      // superblocks, then blocks, in ascending order of their bounds: the
      // nearest points arrive first, so the k-th distance prunes the rest
      // early; once the next bound exceeds min(tau, k-th) so do all later ones
      while (ms) {
        float smin;
        const int sl = pick_min(ms, lbs, smin);
        ms &= ~(1ull << sl);
        if ((double)smin > fmin(tau, tk.kd)) break;
        // block level: the superblock's 64 blocks, one per lane
        const int b0 = (sbase + sl) * kSuperBlocks;
        const int b = b0 + lane;
        const float lbb = b < nb ? block_lb(box, b, q, a.sf) : finf;
        st.blocks += (uint32_t)min(kSuperBlocks, nb - b0);
        if (lbb < finf) maxfin = fmaxf(maxfin, lbb);
        uint64_t m = ballot(lbb < finf && (double)lbb <= fmin(tau, tk.kd));
        while (m) {
          float bmin;
          const int bl = pick_min(m, lbb, bmin);
          m &= ~(1ull << bl);
          const double tau_cur = fmin(tau, tk.kd);
          if ((double)bmin > tau_cur) break;
          const int bb = b0 + bl;
          visit_block(bb, bmin, fetch_block(bb), tau_cur, prev, seed_block, seed_mask);
        }
      }
    }
    return maxfin;
  }
};

template <bool On>
__device__ __forceinline__ void flush_stats(unsigned long long *stats, const WaveStats<On> &st) {
  if constexpr (On) {
    if (!stats || lane_id() != 0) return;
    atomicAdd(stats + TNN_STAT_QUERIES, 1ull);
    atomicAdd(stats + TNN_STAT_BLOCKS, (unsigned long long)st.blocks.v);
    atomicAdd(stats + TNN_STAT_SEGMENTS, (unsigned long long)st.segs.v);
    atomicAdd(stats + TNN_STAT_POINTS, (unsigned long long)st.points.v);
    atomicAdd(stats + TNN_STAT_MERGES, (unsigned long long)st.merges.v);
    atomicAdd(stats + TNN_STAT_ROUNDS, (unsigned long long)st.rounds.v);
    atomicAdd(stats + TNN_STAT_FALLBACKS, (unsigned long long)st.fallback.v);
  }
}

// Answer query `qi` with one wavefront (Algorithm 2 in radius form).
//  plain   : seed = the F segments with the smallest bounds inside the block
//            with the smallest block bound; then expand with tau = k-th.
//  learned : tau = predicted k-th distance; one round settles the query when
//            at least k candidates lie within it, otherwise expansion
//            continues from the k-th found (or a 16x larger radius).
// Rounds only widen tau; a segment is scanned in the first round whose
// radius reaches its bound, so no point enters the top-k twice.
// A query's inputs: its point and (learned radius) predicted k-th distance,
// read ahead of its search so that the loads of the next query of a ticket
// are in flight while the current one runs.
struct QueryIn {
  float x, y, z, t, r2;
};

__device__ __forceinline__ QueryIn load_query_in(const float *qx, const float *qy,
                                                 const float *qz, const float *qt,
                                                 const QueryArgs &a, int64_t qi) {
  QueryIn in;
  in.x = qx[qi];
  in.y = qy[qi];
  in.z = qz[qi];
  in.t = qt[qi];
  in.r2 = (a.flags & TNN_LEARNED) ? a.radius2[qi] : 0.0f;
  return in;
}

template <bool PerQ, bool Stats, bool Gka>
__device__ __forceinline__ void answer_query_with(const IndexDesc &ix, const Prep &pr,
                                                  const QueryArgs &a, const QueryIn &in,
                                                  int64_t qi, int32_t *out_idx, double *out_dist,
                                                  const float *box, const float *sbox) {
  Searcher<PerQ, Stats> se(ix, pr, a);
  se.lane = lane_id();
  se.box = box;
  se.sbox = sbox;
  se.spi_shift = 31 - __clz(ix.kpad);
  se.q = make_query(in.x, in.y, in.z, in.t, a.t_window);
  se.tk.init(a.k, a.inf);
  se.st = WaveStats<Stats>{};
  const int nb = ix.n_blocks;
  const int64_t S = ix.n_seg;
  // scale of the data, used to grow the radius when nothing is known yet
  // (set by the host for the shared scales)
  const double floor_tau = PerQ ? radius_floor(ix.lo, ix.hi, a.s) : a.floor_tau;

  int seed_block = -1;
  uint64_t seed_mask = 0;
  double tau;
  bool learned = (a.flags & TNN_LEARNED) != 0;
  double r2 = learned ? (double)in.r2 : 0.0;
  if (learned && !(r2 > 0.0 && r2 < kInf)) learned = false;  // no usable prediction
  // with TNN_LEARNED_SEED a learned query also takes the plain seed and starts
  // from the smaller of the two radii
  if (learned && !(a.flags & TNN_LEARNED_SEED)) {
    tau = r2;
  } else {
    // nearest block by its bound: best-first over superblocks (a superblock
    // bound never exceeds the bounds of its blocks, so once the nearest
    // unvisited superblock is no closer than the best block the argmin is
    // exact)
    float best = __builtin_huge_valf();
    int bestb = kNoId;
    {
      const int ns = ix.n_super;
      for (int sbase = 0; sbase < ns; sbase += kWave) {
        const int sb = sbase + se.lane;
        float lbs = sb < ns ? block_lb(se.sbox, sb, se.q, a.sf) : __builtin_huge_valf();
        se.st.blocks += (uint32_t)min(kWave, ns - sbase);
        for (;;) {
          float v;
          const int vl = wave_argmin_lane(lbs, v);
          if (!(v < best)) break;
          if (se.lane == vl) lbs = __builtin_huge_valf();
          const int b0 = (sbase + vl) * kSuperBlocks;
          const int b = b0 + se.lane;
          const float bv_l = b < nb ? block_lb(se.box, b, se.q, a.sf) : __builtin_huge_valf();
          se.st.blocks += (uint32_t)min(kSuperBlocks, nb - b0);
          float bv;
          const int bl = wave_argmin_lane(bv_l, bv);
          const int bi = b0 + bl;
          if (bv < best || (bv == best && bi < bestb)) {
            best = bv;
            bestb = bi;
          }
        }
      }
    }
    if (!(best < __builtin_huge_valf())) {  // nothing early enough anywhere
      tau = kInf;
      se.st.rounds.set(0);
      goto write_out;
    }
    seed_block = bestb;
    {
      const int64_t s = (int64_t)bestb * kBlockSegs + se.lane;
      SegView sv{};
      if (s < S) sv = load_seg(pr, s);
      const int ps_l = sv.ps, pc_l = sv.pc;
      const float v0 = s < S ? se.seg_bound(sv) : __builtin_huge_valf();
      float v = v0;
      se.st.segs += (uint32_t)min((int64_t)kBlockSegs, S - (int64_t)bestb * kBlockSegs);
      const int F = a.seed_segments;
      for (int i = 0; i < F; ++i) {
        float mv;
        const int ml = wave_argmin_lane(v, mv);
        if (!(mv < __builtin_huge_valf())) break;
        seed_mask |= 1ull << ml;
        if (se.lane == ml) v = __builtin_huge_valf();
      }
      if (seed_mask) se.scan(seed_mask, bestb, ps_l, pc_l, fmaxf(v0, best));
    }
    if (se.tk.kd < kInf) {
      tau = se.tk.kd;
    } else {
      // fewer than k candidates so far: start from the largest distance seen
      double far = se.tk.d < kInf ? se.tk.d : 0.0;
      for (int m = 32; m > 0; m >>= 1) far = fmax(far, __shfl_xor(far, m, 64));
      tau = fmax(fmax(far, (double)best) * 16.0, floor_tau);
    }
    if (learned) tau = fmin(tau, r2);
  }
  {
    double prev = -1.0;
    for (;;) {
      ++se.st.rounds;
      const float maxfin = se.round(prev, tau, seed_block, seed_mask);
      if (se.tk.kd <= tau || !(tau < kInf)) break;
      if (learned) se.st.fallback.set(1);
      prev = tau;
      if (se.tk.kd < kInf) {
        tau = se.tk.kd;
      } else {
        tau = fmax(tau * 16.0, floor_tau);
        if (tau >= (double)wave_max_nonneg(maxfin)) tau = kInf;
      }
    }
  }
write_out:
  if (se.lane < a.k) {
    out_idx[qi * a.k + se.lane] = se.tk.id == kNoId ? -1 : se.tk.id;
    out_dist[qi * a.k + se.lane] = se.tk.d;
  }
  // Gaussian kernel averaging straight from the registers of the top-k (the
  // batched search's instances that average; the single-call path averages
  // with a kernel of its own after the search)
  if constexpr (Gka)
    gka_context_average(se.lane < a.k && se.tk.id != kNoId && se.tk.d < kInf, se.tk.id, se.tk.d,
                        a.gka_values, a.gka_comp, a.gka_out + qi * a.gka_comp);
  flush_stats(a.stats, se.st);
}

// The query's own scales (wave-uniform), rounded toward zero to float32 for
// the float bounds.  False when one is negative or not finite, or (with
// `box`, for the float32 bounds) when the scaled index box leaves their range.
__device__ __forceinline__ bool load_query_scales(const double *qscale, int64_t qi, QueryArgs &aq,
                                                  const IndexDesc *box) {
  bool ok = true;
  for (int f = 0; f < 4; ++f) {
    const double v = qscale[4 * qi + f];
    ok = ok && v >= 0.0 && v < kInf;
    aq.s[f] = v;
    aq.sf[f] = __double2float_rz(v);
  }
  return ok && (!box || scaled_box_ok(box->lo, box->hi, aq.s));
}

// A query whose scales are invalid: (-1, NaN) in every slot.
__device__ __forceinline__ void write_bad_scale_row(const QueryArgs &a, int64_t qi,
                                                    int32_t *out_idx, double *out_dist) {
  const int lane = lane_id();
  if (lane < a.k) {
    out_idx[qi * a.k + lane] = -1;
    out_dist[qi * a.k + lane] = a.inf - a.inf;  // NaN (no 64-bit literal)
  }
  if (a.gka_values)  // no context: the averaging's NaN row
    gka_context_average(false, 0, 0.0, a.gka_values, a.gka_comp, a.gka_out + qi * a.gka_comp);
  // (cold path: the scale check fails before any search state exists)
  if (a.stats && lane == 0) atomicAdd(a.stats + TNN_STAT_QUERIES, 1ull);
}

template <bool PerQ, bool Stats, bool Gka>
__device__ __forceinline__ void answer_query(const IndexDesc &ix, const Prep &pr,
                                             const QueryArgs &a, const QueryIn &in, int64_t qi,
                                             int32_t *out_idx, double *out_dist,
                                             const float *box, const float *sbox,
                                             const double *qscale) {
  if constexpr (PerQ) {
    QueryArgs aq = a;
    if (!load_query_scales(qscale, qi, aq, &ix)) {
      write_bad_scale_row(a, qi, out_idx, out_dist);
      return;
    }
    answer_query_with<true, Stats, Gka>(ix, pr, aq, in, qi, out_idx, out_dist, box, sbox);
  } else {
    answer_query_with<false, Stats, Gka>(ix, pr, a, in, qi, out_idx, out_dist, box, sbox);
  }
}

// qscale (last, so the other arguments keep their places): per-query scales
// when PerQ, else unused.  Stats: the call collects statistics (a.stats set).
// (An averaging the call asks for runs as a kernel of its own afterwards.)
template <bool PerQ, bool Stats>
__global__ __launch_bounds__(512) void tnn_query_kernel(IndexDesc ix, Prep pr, QueryArgs a,
                                                        const float *qx, const float *qy,
                                                        const float *qz, const float *qt,
                                                        int64_t nq, int32_t *out_idx,
                                                        double *out_dist, const double *qscale) {
  const int64_t qi = (int64_t)blockIdx.x * (blockDim.x >> 6) + uniform_i((int)(threadIdx.x >> 6));
  if (qi >= nq) return;
  answer_query<PerQ, Stats, false>(ix, pr, a, load_query_in(qx, qy, qz, qt, a, qi), qi, out_idx,
                                   out_dist, ix.box, ix.sbox, qscale);
}

// Same search with the block boxes staged once per workgroup in LDS (small
// indexes): the grid is exactly what stays resident, and each wave takes
// TNN_QUERY_CHUNK queries at a time from a counter (query costs vary by
// orders of magnitude, so a fixed share per wave leaves a long tail).
// BoxesInLds: the block boxes fit in LDS too (the superblock boxes always
// do); a template argument so that every box read is a plain LDS or global
// access rather than a generic one.  PerQ: every query has its own scales.
// Stats: the call collects statistics (a.stats set).  The per-query-scale
// instances are compiled for 5 waves per SIMD (96 VGPRs; 113 and 4 waves
// otherwise); the shared-scale ones fit 7 as they are (67 VGPRs).
template <bool BoxesInLds, bool PerQ, bool Stats>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(PerQ ? 5 : 1))) void
tnn_query_lds_kernel(
    IndexDesc ix, Prep pr, QueryArgs a, const float *qx, const float *qy, const float *qz,
    const float *qt, int64_t nq, int32_t *out_idx, double *out_dist, const double *qscale) {
  extern __shared__ float4 s_box4[];
  // superblock boxes first, then (when they fit) the block boxes
  const int nsbox = 2 * ix.n_super;
  const float4 *g_sbox = reinterpret_cast<const float4 *>(ix.sbox);
  const float4 *g_box = reinterpret_cast<const float4 *>(ix.box);
  stage_to_lds(s_box4, g_sbox, nsbox);
  const int nbox = BoxesInLds ? 2 * ix.n_blocks : 0;
  stage_to_lds(s_box4 + nsbox, g_box, nbox);
  __syncthreads();
  const float *s_box = reinterpret_cast<const float *>(s_box4);
  const float *box = BoxesInLds ? reinterpret_cast<const float *>(s_box4 + nsbox) : ix.box;
#if TNN_QUERY_CHUNK > 0
  const int lane = lane_id();
  // Ticket size: TNN_QUERY_CHUNK queries, fewer when that would leave less
  // than two tickets per resident wave (a small query count would otherwise
  // gather on a few waves).
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t fit = nq / (2 * waves);
  const int step = (int)(fit < 1 ? 1 : fit > TNN_QUERY_CHUNK ? TNN_QUERY_CHUNK : fit);
  const int first = (int)(blockIdx.x % kQueues);
  for (int j = 0; j < kQueues; ++j) {
    const int qn = (first + j) % kQueues;
    const int64_t lo = nq * qn / kQueues, hi = nq * (qn + 1) / kQueues;
    unsigned long long *ctr = pr.ticket + qn * kTicketStride;
    for (;;) {
      unsigned long long b = 0;
      if (lane == 0) b = atomicAdd(ctr, (unsigned long long)step);
      const int64_t base = lo + (int64_t)uniform_u64(b);
      if (base >= hi) break;
      const int64_t end = base + step < hi ? base + step : hi;
      for (int64_t qi = base; qi < end; ++qi)
        answer_query<PerQ, Stats, false>(ix, pr, a, load_query_in(qx, qy, qz, qt, a, qi), qi,
                                         out_idx, out_dist, box, s_box, qscale);
    }
  }
#else
  const int wpb = blockDim.x >> 6;
  const int64_t stride = (int64_t)gridDim.x * wpb;
  for (int64_t qi = (int64_t)blockIdx.x * wpb + uniform_i((int)(threadIdx.x >> 6)); qi < nq;
       qi += stride)
    answer_query<PerQ, Stats, false>(ix, pr, a, load_query_in(qx, qy, qz, qt, a, qi), qi, out_idx,
                                     out_dist, box, s_box, qscale);
#endif
}

// ---------------------------------------------------------------------------
// Linear search (the paper's baseline, Sec. 3.6): every point, binary64
// distances, same top-k.  One wavefront answers Q consecutive queries, so
// each 64-point pass loads and converts its points once for all of them
// (Q = 1 with per-query scales).
// ---------------------------------------------------------------------------
template <int Q>
__global__ __launch_bounds__(512) void brute_kernel(IndexDesc ix, QueryArgs a, const float *qxp,
                                                    const float *qyp, const float *qzp,
                                                    const float *qtp, int64_t nq,
                                                    int32_t *out_idx, double *out_dist,
                                                    const double *qscale) {
  const int64_t q0 =
      ((int64_t)blockIdx.x * (blockDim.x >> 6) + uniform_i((int)(threadIdx.x >> 6))) * Q;
  if (q0 >= nq) return;
  const int lane = lane_id();
  double s[4] = {a.s[0], a.s[1], a.s[2], a.s[3]};
  if constexpr (Q == 1) {
    if (qscale) {
      QueryArgs aq = a;
      if (!load_query_scales(qscale, q0, aq, nullptr)) {
        write_bad_scale_row(a, q0, out_idx, out_dist);
        return;
      }
      for (int f = 0; f < 4; ++f) s[f] = aq.s[f];
    }
  }
  // queries past the end repeat the last one and are not written
  QueryPoint q[Q];
  TopK tk[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int64_t qi = q0 + j < nq ? q0 + j : nq - 1;
    q[j] = make_query(qxp[qi], qyp[qi], qzp[qi], qtp[qi], a.t_window);
    tk[j].init(a.k, a.inf);
  }
  uint32_t merges = 0;
  const int64_t n = ix.n_points;
  for (int64_t p0 = 0; p0 < n; p0 += kWave) {
    const int64_t p = p0 + lane;
    const bool ok = p < n;
    float4 pv = make_float4(0.f, 0.f, 0.f, 0.f);
    int pid = kNoId;
    if (ok) {
      pv = ix.pt4[p];
      pid = ix.pid[p];
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const double d = exact_dist(s, q[j].x, q[j].y, q[j].z, q[j].t, pv.x, pv.y, pv.z, pv.w);
      // bitwise, not short-circuit: no divergent branch in the inner loop
      const bool gate = ok & (pv.w < q[j].thrf) & tk[j].admits(d, pid);
      const uint64_t gm = ballot(gate);
      if (gm) {
        tk[j].offer(gm, d, pid);
        ++merges;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int64_t qi = q0 + j;
    if (qi < nq && lane < a.k) {
      out_idx[qi * a.k + lane] = tk[j].id == kNoId ? -1 : tk[j].id;
      out_dist[qi * a.k + lane] = tk[j].d;
    }
  }
  if (a.stats && lane == 0) {
    const int nmine = (int)(nq - q0 < Q ? nq - q0 : Q);
    atomicAdd(a.stats + TNN_STAT_QUERIES, (unsigned long long)nmine);
    atomicAdd(a.stats + TNN_STAT_POINTS, (unsigned long long)n * nmine);
    atomicAdd(a.stats + TNN_STAT_MERGES, (unsigned long long)merges);
  }
}

// ---------------------------------------------------------------------------
// Test export of the bounds, one thread per (query, segment) / (query, block).
// With per-query scales (qscale) the records hold the deviation bounds and
// each cylinder bound is formed for the query's own metric, as the
// per-query-scale search forms it; a row the search refuses gets NaN.
// ---------------------------------------------------------------------------
__global__ void debug_lb_kernel(IndexDesc ix, Prep pr, QueryArgs a, const float *qx,
                                const float *qy, const float *qz, const float *qt, int64_t nq,
                                double *seg_lb_out, float *block_lb_out, const double *qscale) {
  const int64_t S = ix.n_seg, nb = ix.n_blocks;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per_q = S + nb;
  if (i >= nq * per_q) return;
  const int64_t qi = i / per_q, j = i % per_q;
  const QueryPoint q = make_query(qx[qi], qy[qi], qz[qi], qt[qi], a.t_window);
  QueryArgs aq = a;
  bool ok = true;
  if (qscale) ok = load_query_scales(qscale, qi, aq, &ix);
  if (j < S) {
    if (!seg_lb_out) return;
    const SegView v = load_seg(pr, j);
    double lb = a.inf - a.inf;  // NaN (no 64-bit literal)
    if (ok) lb = qscale ? (double)seg_lb_q(v, q, aq.s, aq.sf) : (double)seg_lb(v, q, aq.sf);
    seg_lb_out[qi * S + j] = lb;
  } else if (block_lb_out) {
    block_lb_out[qi * nb + (j - S)] =
        ok ? block_lb(ix.box, (int)(j - S), q, aq.sf) : __int_as_float(0x7fc00000);
  }
}

// ---------------------------------------------------------------------------
// Batched ragged serving: one persistent launch over many indexes.
// ---------------------------------------------------------------------------
__global__ void batch_reset_kernel(unsigned long long *counter, unsigned *done, int n,
                                   unsigned long long *ticks) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kBatchQueues) counter[i * kTicketStride] = 0;
  if (i == 0) ticks[0] = wall_clock64();
  if (i < n) {
    done[i] = 0;
    ticks[i + 1] = 0;
  }
}

// Largest position p in [0, n) with prefix[p] <= g (prefix non-decreasing,
// prefix[0] = 0 <= g < prefix[n]).
__device__ __forceinline__ int find_item(const int64_t *prefix, int n, int64_t g) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void batch_prep_kernel(const BatchItemDev *items, const int64_t *seg_prefix, int n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= seg_prefix[n]) return;
  const int i = find_item(seg_prefix, n, g);
  const BatchItemDev &it = items[i];
  prep_one(it.ix, it.a, it.pr.rec, g - seg_prefix[i]);
}

// Waves pull `chunk` queries at a time from work-queue counters over the
// queries of all items laid end to end in the order given by `order`
// (longest first), split into kBatchQueues contiguous slices as in the
// single-index search; each query is answered exactly as by tnn_query.
// Completion is counted once per item run of a chunk; the wave that completes
// an item stamps its tick.  Every wave leaves once every slice is used up.
// Stats: some item collects statistics.  Compiled for 5 waves per SIMD (96
// VGPRs, no spills; left to itself the compiler takes 102 and 4 waves).
template <bool Stats, bool Gka>
__global__ __launch_bounds__(512, 5) void batch_kernel(const BatchItemDev *items,
                                                    const int64_t *qprefix, const int32_t *order,
                                                    int n, int chunk,
                                                    unsigned long long *counter, unsigned *done,
                                                    unsigned long long *ticks) {
  const int lane = lane_id();
  const int64_t total = qprefix[n];
  const int first = (int)(blockIdx.x % kBatchQueues);
  for (int j = 0; j < kBatchQueues; ++j) {
    const int qn = (first + j) % kBatchQueues;
    const int64_t lo = total * qn / kBatchQueues, hi = total * (qn + 1) / kBatchQueues;
    unsigned long long *ctr = counter + qn * kTicketStride;
    for (;;) {
      unsigned long long b = 0;
      if (lane == 0) b = atomicAdd(ctr, (unsigned long long)chunk);
      const int64_t base = lo + (int64_t)uniform_u64(b);
      if (base >= hi) break;
      const int64_t end = base + chunk < hi ? base + chunk : hi;
      int64_t gq = base;
      while (gq < end) {
        const int pos = find_item(qprefix, n, gq);
        const int64_t item_end = qprefix[pos + 1] < end ? qprefix[pos + 1] : end;
        const int item = order[pos];
        const BatchItemDev &it = items[item];
        const int64_t run = item_end - gq;
        for (; gq < item_end; ++gq)
          answer_query<false, Stats, Gka>(
              it.ix, it.pr, it.a,
              load_query_in(it.qx, it.qy, it.qz, it.qt, it.a, gq - qprefix[pos]),
              gq - qprefix[pos], it.out_idx, it.out_dist, it.ix.box, it.ix.sbox, nullptr);
        if (lane == 0) {
          const unsigned d = atomicAdd(&done[item], (unsigned)run) + (unsigned)run;
          if ((int64_t)d == it.nq) ticks[item + 1] = wall_clock64();
        }
      }
    }
  }
}

hipError_t launch_batch(const BatchLaunch &bl, hipStream_t st) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3((unsigned)((bl.n + 1 + 255) / 256)), dim3(256), 0, st,
                     bl.counter, bl.done, bl.n, bl.ticks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (bl.total_seg > 0) {
    hipLaunchKernelGGL(batch_prep_kernel, dim3((unsigned)((bl.total_seg + 255) / 256)), dim3(256),
                       0, st, bl.items, bl.seg_prefix, bl.n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (bl.total_q > 0) {
    using BK = decltype(&batch_kernel<true, true>);
    static const BK bkerns[4] = {batch_kernel<false, false>, batch_kernel<true, false>,
                                 batch_kernel<false, true>, batch_kernel<true, true>};
    hipLaunchKernelGGL(bkerns[(bl.stats ? 1 : 0) + (bl.gka ? 2 : 0)], dim3((unsigned)bl.grid),
                       dim3(bl.waves_per_block * kWave), 0, st, bl.items, bl.qprefix, bl.order,
                       bl.n, bl.chunk, bl.counter, bl.done, bl.ticks);
    e = hipGetLastError();
  }
  return e;
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
hipError_t launch_prep(const IndexDesc &ix, const QueryArgs &a, const Prep &pr, hipStream_t st,
                       bool per_query_scales) {
  const int tpb = 256;
  const int64_t grid = ix.n_seg > 0 ? (ix.n_seg + tpb - 1) / tpb : 1;
  hipLaunchKernelGGL(prep_kernel, dim3((unsigned)grid), dim3(tpb), 0, st, ix, a, pr.rec,
                     pr.ticket, per_query_scales);
  return hipGetLastError();
}

hipError_t launch_prep_infer(const IndexDesc &ix, const QueryArgs &a, const Prep &pr,
                             const tnn_points &qs, hipStream_t st, bool per_query_scales) {
  constexpr int tpb = 64 * radius::kInferWaves;
  const int64_t prep_blocks = ix.n_seg > 0 ? (ix.n_seg + tpb - 1) / tpb : 1;
  const int64_t per_group = (int64_t)radius::kInferTile * radius::kInferWaves;
  const int64_t groups = (qs.n + per_group - 1) / per_group;
  const int64_t infer_groups = groups < 1024 ? groups : 1024;
  hipLaunchKernelGGL(prep_infer_kernel, dim3((unsigned)(prep_blocks + infer_groups)), dim3(tpb), 0,
                     st, ix, a, pr.rec, pr.ticket, per_query_scales, prep_blocks, qs, pr.radius2,
                     infer_groups);
  return hipGetLastError();
}

static int cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
      c = 256;
    cached[dev] = c;
  }
  return cached[dev];
}

// Workgroups of the resident search kernel that fit on one CU, cached per
// (device, variant, waves per workgroup, LDS bytes): the occupancy query costs
// host time comparable to a small search.
template <class Query>
static int resident_per_cu(int variant, int wpb, size_t lds, Query query) {
  struct Entry {
    int dev, variant, wpb;
    size_t lds;
    int per_cu;
  };
  static Entry cache[32];
  static int used = 0;
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  std::lock_guard<std::mutex> lock(mu);
  for (int i = 0; i < used; ++i)
    if (cache[i].dev == dev && cache[i].variant == variant && cache[i].wpb == wpb &&
        cache[i].lds == lds)
      return cache[i].per_cu;
  int n = 0;
  if (query(&n) != hipSuccess || n <= 0) n = 1;
  if (used < 32) cache[used++] = Entry{dev, variant, wpb, lds, n};
  return n;
}

hipError_t launch_query(const IndexDesc &ix, const Prep &pr, const QueryArgs &a,
                        const tnn_points &qs, int waves_per_block, int32_t *out_idx,
                        double *out_dist, hipStream_t st, const double *query_scale) {
  if (qs.n == 0) return hipSuccess;
  const int64_t grid = (qs.n + waves_per_block - 1) / waves_per_block;
  const size_t sl = (size_t)ix.n_super * 8 * sizeof(float);
  const size_t bl = (size_t)ix.n_blocks * 8 * sizeof(float);
  if (sl <= kLdsBoxBytes) {
    const int in_lds = sl + bl <= kLdsBoxBytes ? 1 : 0;
    const size_t lds = in_lds ? sl + bl : sl;
    const bool perq = query_scale != nullptr;
    using Kern = decltype(&tnn_query_lds_kernel<true, true, true>);
    static const Kern kerns[8] = {
        tnn_query_lds_kernel<false, false, false>, tnn_query_lds_kernel<true, false, false>,
        tnn_query_lds_kernel<false, true, false>,  tnn_query_lds_kernel<true, true, false>,
        tnn_query_lds_kernel<false, false, true>,  tnn_query_lds_kernel<true, false, true>,
        tnn_query_lds_kernel<false, true, true>,   tnn_query_lds_kernel<true, true, true>};
    const int variant = in_lds + (perq ? 2 : 0) + (a.stats ? 4 : 0);
    const Kern kern = kerns[variant];
    const int per_cu = resident_per_cu(variant, waves_per_block, lds, [&](int *n) {
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, kern, waves_per_block * kWave, lds);
    });
    const int blocks_per_cu = per_cu < kMaxSearchBlocksPerCu ? per_cu : kMaxSearchBlocksPerCu;
    const int64_t resident = (int64_t)cu_count() * blocks_per_cu;
    const int64_t g = grid < resident ? grid : resident;
    hipLaunchKernelGGL(kern, dim3((unsigned)g), dim3(waves_per_block * kWave), lds, st, ix, pr, a,
                       qs.x, qs.y, qs.z, qs.t, qs.n, out_idx, out_dist, query_scale);
    return hipGetLastError();
  }
  using GKern = decltype(&tnn_query_kernel<true, true>);
  static const GKern gkerns[4] = {tnn_query_kernel<false, false>, tnn_query_kernel<true, false>,
                                  tnn_query_kernel<false, true>, tnn_query_kernel<true, true>};
  const GKern kern = gkerns[(query_scale ? 1 : 0) + (a.stats ? 2 : 0)];
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(waves_per_block * kWave), 0, st, ix, pr, a,
                     qs.x, qs.y, qs.z, qs.t, qs.n, out_idx, out_dist, query_scale);
  return hipGetLastError();
}

hipError_t launch_brute(const IndexDesc &ix, const QueryArgs &a, const tnn_points &qs,
                        int waves_per_block, int32_t *out_idx, double *out_dist, hipStream_t st,
                        const double *query_scale) {
  if (qs.n == 0) return hipSuccess;
  // queries per wave: kBruteQ sharing every point pass when that still gives
  // about 8 waves per SIMD, else one; one with per-query scales (each query's
  // scales would take scalar registers)
  const bool tiled = !query_scale && qs.n >= (int64_t)32 * cu_count() * kBruteQ;
  const int qpw = tiled ? kBruteQ : 1;
  const int64_t waves = (qs.n + qpw - 1) / qpw;
  const int64_t grid = (waves + waves_per_block - 1) / waves_per_block;
  hipLaunchKernelGGL(tiled ? brute_kernel<kBruteQ> : brute_kernel<1>, dim3((unsigned)grid),
                     dim3(waves_per_block * kWave), 0, st, ix, a, qs.x, qs.y, qs.z, qs.t, qs.n,
                     out_idx, out_dist, query_scale);
  return hipGetLastError();
}

hipError_t launch_debug_lb(const IndexDesc &ix, const Prep &pr, const QueryArgs &a,
                           const tnn_points &qs, double *seg_lb_out, float *block_lb_out,
                           hipStream_t st, const double *query_scale) {
  const int64_t total = qs.n * (ix.n_seg + ix.n_blocks);
  if (total == 0) return hipSuccess;
  const int tpb = 256;
  hipLaunchKernelGGL(debug_lb_kernel, dim3((unsigned)((total + tpb - 1) / tpb)), dim3(tpb), 0, st,
                     ix, pr, a, qs.x, qs.y, qs.z, qs.t, qs.n, seg_lb_out, block_lb_out,
                     query_scale);
  return hipGetLastError();
}

}  // namespace tnn
