// C ABI of the trajectory nearest-neighbour library (declared in tnn.h):
// argument checks, buffer layouts and kernel launches.  No allocation.
#include <algorithm>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "gka.h"
#include "host.h"
#include "kdorder.h"
#include "query.h"

using namespace tnn;
using host::BuildLayout;
using host::count_segments;
using host::offsets_ok;

static BuildLayout build_layout(int64_t n, int64_t S) {
  return host::build_layout(n, S, kBlockSegs, kSuperBlocks);
}

namespace {

const IndexDesc *desc_of(const tnn_index *index) {
  if (!index) return nullptr;
  const IndexDesc *d = reinterpret_cast<const IndexDesc *>(index);
  return d->magic == kIndexMagic ? d : nullptr;
}

bool points_ok(const tnn_points &p) {
  if (p.n < 0) return false;
  if (p.n == 0) return true;
  return p.x && p.y && p.z && p.t && p.n <= INT32_MAX;
}

tnn_status check_params(const tnn_query_params *p, int64_t n_queries = 1) {
  if (!p) return TNN_E_ARG;
  for (int f = 0; f < 4; ++f)
    if (!(p->scale[f] >= 0.0) || !std::isfinite(p->scale[f])) return TNN_E_ARG;
  if (!(p->t_window >= 0.0) || !std::isfinite(p->t_window)) return TNN_E_ARG;
  if (p->k < 1 || p->k > kMaxK) return TNN_E_ARG;
  if (p->flags & ~(TNN_BRUTE | TNN_MIXED_BF16 | TNN_LEARNED | TNN_LEARNED_SEED)) return TNN_E_ARG;
  if ((p->flags & TNN_LEARNED_SEED) && !(p->flags & TNN_LEARNED)) return TNN_E_ARG;
  if ((p->flags & TNN_LEARNED) && !p->d_radius2 && !p->radius_model && n_queries > 0)
    return TNN_E_ARG;
  if (p->radius_model) {
    if (p->d_radius2 || !(p->flags & TNN_LEARNED)) return TNN_E_ARG;
    if (!(p->radius_alpha > 0.0f) || !std::isfinite(p->radius_alpha)) return TNN_E_ARG;
    if (p->flags & TNN_BRUTE) return TNN_E_UNSUPPORTED;
  }
  if ((p->flags & TNN_MIXED_BF16) && !(p->flags & TNN_BRUTE)) return TNN_E_UNSUPPORTED;
  // the BF16 operands carry the scales: one metric per call
  if ((p->flags & TNN_MIXED_BF16) && p->d_query_scale) return TNN_E_UNSUPPORTED;
  if (p->seed_segments < 0 || p->seed_segments > 64) return TNN_E_ARG;
  if (p->d_gka_values &&
      (p->gka_comp < 1 || p->gka_comp > kGkaMaxComp || (n_queries > 0 && !p->d_gka_out)))
    return TNN_E_ARG;
  const int w = p->waves_per_block;
  if (!(w == 0 || w == 1 || w == 2 || w == 4 || w == 8)) return TNN_E_ARG;
  return TNN_OK;
}

QueryArgs make_args(const tnn_query_params *p) {
  QueryArgs a;
  a.inf = INFINITY;
  for (int f = 0; f < 4; ++f) {
    a.s[f] = p->scale[f];
    float v = (float)p->scale[f];
    if ((double)v > p->scale[f]) v = std::nextafter(v, 0.0f);  // round toward zero
    a.sf[f] = v;
  }
  a.t_window = p->t_window;
  a.k = p->k;
  a.flags = p->flags;
  a.seed_segments = p->seed_segments ? p->seed_segments : 4;
  a.floor_tau = 1e-300;  // set from the index by the callers that search
  a.radius2 = p->d_radius2;
  a.model = static_cast<const tnn_radius_model *>(p->radius_model);
  a.alpha = p->radius_alpha;
  a.stats = p->d_stats;
  a.gka_values = p->d_gka_values;
  a.gka_comp = p->d_gka_values ? p->gka_comp : 0;
  a.gka_out = p->d_gka_values ? p->d_gka_out : nullptr;
  return a;
}

// kSegRec planes of one float4 per segment, then 16 work-queue counters 256
// bytes apart,
// then (in-call radius prediction) one float per query
size_t prep_bytes(int64_t S, int64_t n_radius = 0) {
  return align_up(16 * kSegRec * (size_t)S) + 16 * 256 + align_up(4 * (size_t)n_radius);
}

Prep prep_view(void *scratch, int64_t S, bool radius = false) {
  char *b = static_cast<char *>(scratch);
  Prep p;
  p.rec = reinterpret_cast<float4 *>(b);
  p.ticket = reinterpret_cast<unsigned long long *>(b + align_up(16 * kSegRec * (size_t)S));
  p.radius2 = radius ? reinterpret_cast<float *>(b + align_up(16 * kSegRec * (size_t)S) + 16 * 256)
                     : nullptr;
  p.n_seg = S;
  return p;
}

}  // namespace

extern "C" {

const char *tnn_status_string(tnn_status s) {
  switch (s) {
    case TNN_OK: return "ok";
    case TNN_E_ARG: return "invalid argument";
    case TNN_E_UNSORTED: return "trajectory times decrease";
    case TNN_E_NONFINITE: return "non-finite coordinate";
    case TNN_E_WORKSPACE: return "workspace too small";
    case TNN_E_HIP: return "HIP runtime error";
    case TNN_E_UNSUPPORTED: return "unsupported request";
    case TNN_E_FORMAT: return "not a valid checkpoint for this library version";
    default: return "unknown status";
  }
}

tnn_status tnn_build_segments_workspace(const int64_t *h_traj_offsets, int64_t n_traj,
                                        int32_t seg_len, size_t *bytes) {
  if (!bytes || seg_len < 1 || seg_len > kMaxSegLen || !offsets_ok(h_traj_offsets, n_traj))
    return TNN_E_ARG;
  const int64_t n = h_traj_offsets[n_traj];
  if (n > INT32_MAX) return TNN_E_UNSUPPORTED;
  *bytes = build_layout(n, count_segments(h_traj_offsets, n_traj, seg_len)).total;
  return TNN_OK;
}

tnn_status tnn_build_segments(tnn_points pts, const int64_t *h_traj_offsets, int64_t n_traj,
                              int32_t seg_len, const double *order_scale, void *d_mem,
                              size_t bytes, void *stream, tnn_index *out) {
  if (!out || !d_mem || seg_len < 1 || seg_len > kMaxSegLen || !points_ok(pts) ||
      !offsets_ok(h_traj_offsets, n_traj) || h_traj_offsets[n_traj] != pts.n)
    return TNN_E_ARG;
  if (order_scale)
    for (int f = 0; f < 4; ++f)
      if (!(order_scale[f] >= 0.0) || !std::isfinite(order_scale[f])) return TNN_E_ARG;
  const int64_t n = pts.n;
  const int64_t S = count_segments(h_traj_offsets, n_traj, seg_len);
  const int64_t nb = (S + kBlockSegs - 1) / kBlockSegs;
  const BuildLayout L = build_layout(n, S);
  if (bytes < L.total) return TNN_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *m = static_cast<char *>(d_mem);
  auto F = [&](size_t off) { return reinterpret_cast<float *>(m + off); };
  auto I = [&](size_t off) { return reinterpret_cast<int32_t *>(m + off); };

  // segment table in trajectory order (host)
  std::vector<int32_t> tstart(S), tcf(S);
  {
    int64_t s = 0;
    for (int64_t j = 0; j < n_traj; ++j) {
      bool first = true;
      for (int64_t p = h_traj_offsets[j]; p < h_traj_offsets[j + 1]; p += seg_len) {
        const int64_t c = std::min<int64_t>(seg_len, h_traj_offsets[j + 1] - p);
        tstart[s] = (int32_t)p;
        tcf[s] = (int32_t)c | (first ? (1 << 16) : 0);
        first = false;
        ++s;
      }
    }
  }
  float osc_h[4];
  const float *osc_d = nullptr;
  if (order_scale)
    for (int f = 0; f < 4; ++f) osc_h[f] = (float)std::sqrt(order_scale[f]);
  if (S > 0) {
    TNN_HIP_CHECK(hipMemcpyAsync(I(L.tstart), tstart.data(), 4 * S, hipMemcpyHostToDevice, st));
    TNN_HIP_CHECK(hipMemcpyAsync(I(L.tcf), tcf.data(), 4 * S, hipMemcpyHostToDevice, st));
  }
  // status word at +0, order scales at +16 of the status slot
  uint32_t zero[4] = {0, 0, 0, 0};
  TNN_HIP_CHECK(hipMemcpyAsync(m + L.status, zero, 16, hipMemcpyHostToDevice, st));
  if (order_scale && S > 0) {
    TNN_HIP_CHECK(hipMemcpyAsync(m + L.status + 16, osc_h, 16, hipMemcpyHostToDevice, st));
    osc_d = reinterpret_cast<const float *>(m + L.status + 16);
  }
  uint32_t *status = reinterpret_cast<uint32_t *>(m + L.status);
  TNN_HIP_CHECK(launch_seg_stats(pts, I(L.tstart), I(L.tcf), S, osc_d, F(L.tf[0]), F(L.tf[1]),
                                 F(L.tf[2]), F(L.tf[3]), F(L.tf[4]), F(L.tf[5]), F(L.tf[6]),
                                 F(L.tf[7]), F(L.tf[8]), F(L.tf[9]), F(L.tf[10]), F(L.keys), status,
                                 st));
  // the kd order of the segments (identity without order scales) and each
  // segment's first point slot in that order, on the device: the splits
  // depend on S alone, so the host lists them without reading anything back
  TNN_HIP_CHECK(launch_iota(I(L.perm), S, st));
  std::vector<host::KdSplit> splits;
  if (order_scale && S > 0) {
    int64_t level_begin[host::kKdMaxLevels + 1];
    int n_levels = 0;
    splits.resize((size_t)host::kd_splits(S, kBlockSegs, nullptr, nullptr, nullptr));
    host::kd_splits(S, kBlockSegs, splits.data(), level_begin, &n_levels);
    auto *d_splits = reinterpret_cast<host::KdSplit *>(m + L.kdsplits);
    if (!splits.empty())
      TNN_HIP_CHECK(hipMemcpyAsync(d_splits, splits.data(), sizeof(host::KdSplit) * splits.size(),
                                   hipMemcpyHostToDevice, st));
    // dpstart serves as the partition's staging area until it is written
    for (int lv = 0; lv < n_levels; ++lv)
      TNN_HIP_CHECK(launch_kd_level(F(L.keys), I(L.perm), I(L.dpstart), d_splits + level_begin[lv],
                                    level_begin[lv + 1] - level_begin[lv], st));
    TNN_HIP_CHECK(launch_kd_leaves(F(L.keys), I(L.perm), S, st));
  }
  TNN_HIP_CHECK(launch_point_offsets(I(L.perm), I(L.tcf), S, I(L.dpstart), st));
  const float *src_f[11];
  float *dst_f[11];
  for (int i = 0; i < 11; ++i) {
    src_f[i] = F(L.tf[i]);
    dst_f[i] = F(L.f[i]);
  }
  TNN_HIP_CHECK(launch_seg_scatter(pts, S, I(L.perm), I(L.tstart), I(L.tcf), I(L.dpstart), src_f,
                                   dst_f, I(L.pstart), I(L.pcount), I(L.sorig), I(L.sfirst),
                                   reinterpret_cast<float4 *>(F(L.pt4)), I(L.pid), st));

  IndexDesc d;
  std::memset(&d, 0, sizeof(d));
  d.magic = kIndexMagic;
  d.seg_len = seg_len;
  int kp = 1;
  while (kp < seg_len) kp <<= 1;
  d.kpad = kp;
  d.n_blocks = (int32_t)nb;
  d.n_points = n;
  d.n_seg = S;
  d.pt4 = reinterpret_cast<const float4 *>(F(L.pt4));
  d.pid = I(L.pid);
  d.ax = F(L.f[0]);
  d.ay = F(L.f[1]);
  d.az = F(L.f[2]);
  d.bx = F(L.f[3]);
  d.by = F(L.f[4]);
  d.bz = F(L.f[5]);
  d.tmin = F(L.f[6]);
  d.tmax = F(L.f[7]);
  d.ex = F(L.f[8]);
  d.ey = F(L.f[9]);
  d.ez = F(L.f[10]);
  d.pstart = I(L.pstart);
  d.pcount = I(L.pcount);
  d.sorig = I(L.sorig);
  d.sfirst = I(L.sfirst);
  d.box = F(L.box);
  TNN_HIP_CHECK(launch_block_box(d, F(L.box), st));
  // the one read-back: the data checks and the block boxes (the kernels
  // above are safe on rejected data; nothing is returned from it)
  uint32_t status_h = 0;
  std::vector<float> box(8 * (size_t)nb);
  if (nb > 0)
    TNN_HIP_CHECK(hipMemcpyAsync(box.data(), F(L.box), 32 * nb, hipMemcpyDeviceToHost, st));
  TNN_HIP_CHECK(hipMemcpyAsync(&status_h, status, 4, hipMemcpyDeviceToHost, st));
  TNN_HIP_CHECK(hipStreamSynchronize(st));
  if (status_h & 2u) return TNN_E_NONFINITE;
  if (status_h & 1u) return TNN_E_UNSORTED;
  const int64_t ns = (nb + kSuperBlocks - 1) / kSuperBlocks;
  std::vector<float> sbox(8 * (size_t)ns);
  for (int64_t sb = 0; sb < ns; ++sb)
    for (int f = 0; f < 4; ++f) {
      float lo = INFINITY, hi = -INFINITY;
      for (int64_t b = sb * kSuperBlocks; b < std::min<int64_t>(nb, (sb + 1) * kSuperBlocks); ++b) {
        lo = std::min(lo, box[8 * b + f]);
        hi = std::max(hi, box[8 * b + 4 + f]);
      }
      sbox[8 * sb + f] = lo;
      sbox[8 * sb + 4 + f] = hi;
    }
  if (ns > 0) {
    TNN_HIP_CHECK(hipMemcpyAsync(F(L.sbox), sbox.data(), 32 * ns, hipMemcpyHostToDevice, st));
    TNN_HIP_CHECK(hipStreamSynchronize(st));
  }
  d.sbox = F(L.sbox);
  d.n_super = (int32_t)ns;
  for (int f = 0; f < 4; ++f) {
    d.lo[f] = 0.0f;
    d.hi[f] = 0.0f;
    if (nb == 0) continue;
    float lo = INFINITY, hi = -INFINITY;
    for (int64_t b = 0; b < nb; ++b) {
      lo = std::min(lo, box[8 * b + f]);
      hi = std::max(hi, box[8 * b + 4 + f]);
    }
    d.lo[f] = lo;
    d.hi[f] = hi;
  }
  std::memset(out, 0, sizeof(*out));
  std::memcpy(out, &d, sizeof(d));
  return TNN_OK;
}

tnn_status tnn_index_info(const tnn_index *index, int64_t *n_points, int64_t *n_segments,
                          int64_t *n_blocks, int32_t *seg_len) {
  const IndexDesc *d = desc_of(index);
  if (!d) return TNN_E_ARG;
  if (n_points) *n_points = d->n_points;
  if (n_segments) *n_segments = d->n_seg;
  if (n_blocks) *n_blocks = d->n_blocks;
  if (seg_len) *seg_len = d->seg_len;
  return TNN_OK;
}

tnn_status tnn_query_workspace(const tnn_index *index, int64_t n_queries,
                               const tnn_query_params *params, size_t *bytes) {
  const IndexDesc *d = desc_of(index);
  if (!d || !bytes || n_queries < 0) return TNN_E_ARG;
  const tnn_status c = check_params(params, n_queries);
  if (c != TNN_OK) return c;
  if (params->flags & TNN_MIXED_BF16)
    *bytes = mixed_scratch_bytes(d->n_points, n_queries, params->k);
  else
    *bytes = (params->flags & TNN_BRUTE)
                 ? 256
                 : prep_bytes(d->n_seg, params->radius_model ? n_queries : 0);
  return TNN_OK;
}

tnn_status tnn_query(const tnn_index *index, tnn_points queries, const tnn_query_params *params,
                     int32_t *d_out_idx, double *d_out_dist, void *d_scratch,
                     size_t scratch_bytes, void *stream) {
  const IndexDesc *d = desc_of(index);
  if (!d || !points_ok(queries)) return TNN_E_ARG;
  const tnn_status c = check_params(params, queries.n);
  if (c != TNN_OK) return c;
  if (queries.n > 0 && (!d_out_idx || !d_out_dist)) return TNN_E_ARG;
  size_t need = 0;
  tnn_query_workspace(index, queries.n, params, &need);
  const bool plain_brute = (params->flags & TNN_BRUTE) && !(params->flags & TNN_MIXED_BF16);
  if (scratch_bytes < need || (need > 0 && !d_scratch && !plain_brute)) return TNN_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const QueryArgs a = make_args(params);
  const int wpb = params->waves_per_block ? params->waves_per_block : 4;
  // float32 bounds and tiles: the scaled index box must stay in range (the
  // binary64 linear search has no such limit)
  const bool float_path = !(params->flags & TNN_BRUTE) || (params->flags & TNN_MIXED_BF16);
  if (float_path && !params->d_query_scale && !scaled_box_ok(d->lo, d->hi, params->scale))
    return TNN_E_UNSUPPORTED;
  // The averaging (Sec. 3.2, Eq. gka), when asked for, runs as a kernel of
  // its own right after the search, on the outputs the search has just
  // written: computed inside the search kernel instead, it took longer (its
  // exponentials and wave sums compete with the search for the vector units).
  QueryArgs as = a;
  as.gka_values = nullptr;
  as.gka_out = nullptr;
  as.gka_comp = 0;
  if (params->flags & TNN_BRUTE) {
    if (params->flags & TNN_MIXED_BF16)
      TNN_HIP_CHECK(launch_mixed_brute(*d, as, queries, d_out_idx, d_out_dist, d_scratch, st));
    else
      TNN_HIP_CHECK(launch_brute(*d, as, queries, wpb, d_out_idx, d_out_dist, st,
                                 params->d_query_scale));
  } else {
    const Prep pr = prep_view(d_scratch, d->n_seg, a.model != nullptr);
    QueryArgs at = as;
    at.floor_tau = radius_floor(d->lo, d->hi, a.s);
    if (a.model && queries.n > 0) {
      // the radius prediction shares the preparation's launch
      at.radius2 = pr.radius2;
      TNN_HIP_CHECK(launch_prep_infer(*d, at, pr, queries, st, params->d_query_scale != nullptr));
    } else {
      TNN_HIP_CHECK(launch_prep(*d, at, pr, st, params->d_query_scale != nullptr));
    }
    TNN_HIP_CHECK(launch_query(*d, pr, at, queries, wpb, d_out_idx, d_out_dist, st,
                               params->d_query_scale));
  }
  if (a.gka_values)
    TNN_HIP_CHECK(launch_gka(d_out_idx, d_out_dist, queries.n, a.k, a.gka_values, a.gka_comp,
                             d->n_points, a.gka_out, st));
  return TNN_OK;
}

tnn_status tnn_debug_export_index(const tnn_index *index, float *d_seg_f32, int32_t *d_seg_i32,
                                  int32_t *d_point_id, float *d_block_box, void *stream) {
  const IndexDesc *d = desc_of(index);
  if (!d) return TNN_E_ARG;
  TNN_HIP_CHECK(launch_export(*d, d_seg_f32, d_seg_i32, d_point_id, d_block_box,
                              static_cast<hipStream_t>(stream)));
  return TNN_OK;
}

tnn_status tnn_debug_lower_bounds(const tnn_index *index, tnn_points queries,
                                  const double *h_scale, double t_window,
                                  const double *d_query_scale, double *d_seg_lb,
                                  float *d_block_lb, void *d_scratch, size_t scratch_bytes,
                                  void *stream) {
  const IndexDesc *d = desc_of(index);
  if (!d || !points_ok(queries) || !h_scale) return TNN_E_ARG;
  tnn_query_params p;
  std::memset(&p, 0, sizeof(p));
  for (int f = 0; f < 4; ++f) p.scale[f] = h_scale[f];
  p.t_window = t_window;
  p.k = 1;
  const tnn_status c = check_params(&p);
  if (c != TNN_OK) return c;
  if (scratch_bytes < prep_bytes(d->n_seg) || (d->n_seg > 0 && !d_scratch)) return TNN_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const QueryArgs a = make_args(&p);
  const Prep pr = prep_view(d_scratch, d->n_seg);
  TNN_HIP_CHECK(launch_prep(*d, a, pr, st, d_query_scale != nullptr));
  TNN_HIP_CHECK(launch_debug_lb(*d, pr, a, queries, d_seg_lb, d_block_lb, st, d_query_scale));
  return TNN_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched ragged serving.
// ---------------------------------------------------------------------------
namespace {

struct BatchLayout {
  size_t items, qprefix, order, seg_prefix, counter, done, ticks, prep0, total;
  std::vector<size_t> prep;  // per item
};

BatchLayout batch_layout(const tnn_batch_item *items, int32_t n) {
  BatchLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  L.items = take(sizeof(BatchItemDev) * (size_t)n);
  L.qprefix = take(8 * (size_t)(n + 1));
  L.order = take(4 * (size_t)n);
  L.seg_prefix = take(8 * (size_t)(n + 1));
  L.counter = take(16 * 256);  // work-queue counters, 256 bytes apart
  L.done = take(4 * (size_t)n);
  L.ticks = take(8 * (size_t)(n + 1));
  L.prep0 = o;
  L.prep.resize(n);
  for (int32_t i = 0; i < n; ++i) {
    const IndexDesc *d = desc_of(items[i].index);
    L.prep[i] = take(prep_bytes(d ? d->n_seg : 0));
  }
  L.total = o;
  return L;
}

tnn_status check_items(const tnn_batch_item *items, int32_t n) {
  if (!items || n < 1 || n > TNN_MAX_BATCH_ITEMS) return TNN_E_ARG;
  for (int32_t i = 0; i < n; ++i) {
    const tnn_batch_item &it = items[i];
    if (!desc_of(it.index) || !points_ok(it.queries)) return TNN_E_ARG;
    const tnn_status c = check_params(&it.params, it.queries.n);
    if (c != TNN_OK) return c;
    if (it.params.flags & (TNN_BRUTE | TNN_MIXED_BF16)) return TNN_E_UNSUPPORTED;
    if (it.params.d_query_scale || it.params.radius_model) return TNN_E_UNSUPPORTED;
    const IndexDesc *d = desc_of(it.index);
    if (!scaled_box_ok(d->lo, d->hi, it.params.scale)) return TNN_E_UNSUPPORTED;
    if (it.queries.n > 0 && (!it.d_out_idx || !it.d_out_dist)) return TNN_E_ARG;
  }
  return TNN_OK;
}

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return cus;
}

}  // namespace

extern "C" {

tnn_status tnn_batch_workspace(const tnn_batch_item *items, int32_t n_items, size_t *bytes) {
  if (!bytes) return TNN_E_ARG;
  const tnn_status c = check_items(items, n_items);
  if (c != TNN_OK) return c;
  *bytes = batch_layout(items, n_items).total;
  return TNN_OK;
}

tnn_status tnn_batch_prepare(const tnn_batch_item *items, int32_t n_items,
                             const tnn_batch_config *config, void *d_scratch, size_t bytes,
                             void *stream, tnn_batch_plan *plan) {
  if (!plan || !d_scratch) return TNN_E_ARG;
  const tnn_status c = check_items(items, n_items);
  if (c != TNN_OK) return c;
  tnn_batch_config cfg = {8, 4, 4, 0};
  if (config) {
    if (config->chunk) cfg.chunk = config->chunk;
    if (config->waves_per_block) cfg.waves_per_block = config->waves_per_block;
    if (config->blocks_per_cu) cfg.blocks_per_cu = config->blocks_per_cu;
  }
  const int w = cfg.waves_per_block;
  if (cfg.chunk < 1 || cfg.chunk > 64 || !(w == 1 || w == 2 || w == 4 || w == 8) ||
      cfg.blocks_per_cu < 1 || cfg.blocks_per_cu > 16)
    return TNN_E_ARG;
  const BatchLayout L = batch_layout(items, n_items);
  if (bytes < L.total) return TNN_E_WORKSPACE;
  const int cus = device_cus();
  if (cus <= 0) return TNN_E_HIP;
  char *m = static_cast<char *>(d_scratch);
  const int32_t n = n_items;
  std::vector<BatchItemDev> dev(n);
  std::vector<int64_t> seg_prefix(n + 1, 0), qprefix(n + 1, 0);
  std::vector<double> cost(n);
  bool stats = false;
  for (int32_t i = 0; i < n; ++i) {
    const tnn_batch_item &it = items[i];
    const IndexDesc *d = desc_of(it.index);
    BatchItemDev &b = dev[i];
    b.ix = *d;
    b.a = make_args(&it.params);
    b.a.floor_tau = radius_floor(d->lo, d->hi, b.a.s);
    stats = stats || b.a.stats != nullptr;
    b.pr = prep_view(m + L.prep[i], d->n_seg);
    b.qx = it.queries.x;
    b.qy = it.queries.y;
    b.qz = it.queries.z;
    b.qt = it.queries.t;
    b.nq = it.queries.n;
    b.out_idx = it.d_out_idx;
    b.out_dist = it.d_out_dist;
    seg_prefix[i + 1] = seg_prefix[i] + d->n_seg;
    // per-query work grows with the blocks every round visits
    cost[i] = (double)it.queries.n * (double)(d->n_blocks + kBlockSegs);
  }
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
  for (int32_t p = 0; p < n; ++p) qprefix[p + 1] = qprefix[p] + dev[order[p]].nq;
  hipStream_t st = static_cast<hipStream_t>(stream);
  TNN_HIP_CHECK(hipMemcpyAsync(m + L.items, dev.data(), sizeof(BatchItemDev) * n, hipMemcpyHostToDevice, st));
  TNN_HIP_CHECK(hipMemcpyAsync(m + L.qprefix, qprefix.data(), 8 * (n + 1), hipMemcpyHostToDevice, st));
  TNN_HIP_CHECK(hipMemcpyAsync(m + L.order, order.data(), 4 * n, hipMemcpyHostToDevice, st));
  TNN_HIP_CHECK(hipMemcpyAsync(m + L.seg_prefix, seg_prefix.data(), 8 * (n + 1), hipMemcpyHostToDevice, st));
  TNN_HIP_CHECK(hipStreamSynchronize(st));
  BatchLaunch bl;
  std::memset(&bl, 0, sizeof(bl));
  bl.magic = kBatchMagic;
  bl.n = n;
  bl.chunk = cfg.chunk;
  bl.waves_per_block = w;
  bl.stats = stats ? 1 : 0;
  bool gka = false;
  for (int32_t i = 0; i < n; ++i) gka = gka || dev[i].a.gka_values != nullptr;
  bl.gka = gka ? 1 : 0;
  bl.grid = (int64_t)cus * cfg.blocks_per_cu;
  bl.total_q = qprefix[n];
  bl.total_seg = seg_prefix[n];
  bl.items = reinterpret_cast<const BatchItemDev *>(m + L.items);
  bl.qprefix = reinterpret_cast<const int64_t *>(m + L.qprefix);
  bl.order = reinterpret_cast<const int32_t *>(m + L.order);
  bl.seg_prefix = reinterpret_cast<const int64_t *>(m + L.seg_prefix);
  bl.counter = reinterpret_cast<unsigned long long *>(m + L.counter);
  bl.done = reinterpret_cast<unsigned *>(m + L.done);
  bl.ticks = reinterpret_cast<unsigned long long *>(m + L.ticks);
  std::memset(plan, 0, sizeof(*plan));
  std::memcpy(plan, &bl, sizeof(bl));
  return TNN_OK;
}

tnn_status tnn_query_batched(const tnn_batch_plan *plan, void *stream) {
  if (!plan) return TNN_E_ARG;
  const BatchLaunch *bl = reinterpret_cast<const BatchLaunch *>(plan);
  if (bl->magic != kBatchMagic) return TNN_E_ARG;
  TNN_HIP_CHECK(launch_batch(*bl, static_cast<hipStream_t>(stream)));
  return TNN_OK;
}

tnn_status tnn_batch_ticks(const tnn_batch_plan *plan, const uint64_t **d_ticks) {
  if (!plan || !d_ticks) return TNN_E_ARG;
  const BatchLaunch *bl = reinterpret_cast<const BatchLaunch *>(plan);
  if (bl->magic != kBatchMagic) return TNN_E_ARG;
  *d_ticks = reinterpret_cast<const uint64_t *>(bl->ticks);
  return TNN_OK;
}

tnn_status tnn_wall_clock_rate_khz(int64_t *khz) {
  if (!khz) return TNN_E_ARG;
  int dev = 0, rate = 0;
  TNN_HIP_CHECK(hipGetDevice(&dev));
  TNN_HIP_CHECK(hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev));
  *khz = rate;
  return TNN_OK;
}

tnn_status tnn_autotune_batched(const tnn_batch_item *items, int32_t n_items, void *d_scratch,
                                size_t bytes, void *stream, const char *cache_path,
                                tnn_batch_config *best) {
  if (!best) return TNN_E_ARG;
  const tnn_status c = check_items(items, n_items);
  if (c != TNN_OK) return c;
  int64_t total_q = 0, total_p = 0;
  for (int32_t i = 0; i < n_items; ++i) {
    total_q += items[i].queries.n;
    total_p += desc_of(items[i].index)->n_points;
  }
  int dev = 0;
  TNN_HIP_CHECK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  TNN_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
  char key[256];
  if (!host::cache_key(key, sizeof(key), prop.gcnArchName, n_items, (long long)total_q,
                       (long long)total_p))
    cache_path = nullptr;  // no key: tune without the cache
  if (cache_path) {
    if (FILE *f = std::fopen(cache_path, "r")) {
      char line[512];
      while (std::fgets(line, sizeof(line), f)) {
        int cfg[3];
        if (host::cache_parse_line(line, key, cfg)) {
          std::fclose(f);
          *best = tnn_batch_config{cfg[0], cfg[1], cfg[2], 0};
          return TNN_OK;
        }
      }
      std::fclose(f);
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  TNN_HIP_CHECK(hipEventCreate(&e0));
  TNN_HIP_CHECK(hipEventCreate(&e1));
  float best_ms = INFINITY;
  tnn_status rc = TNN_OK;
  for (int chunk : {1, 4, 16})
    for (int w : {2, 4, 8})
      for (int bpc : {2, 4, 8}) {
        tnn_batch_config cfg = {chunk, w, bpc, 0};
        tnn_batch_plan plan;
        rc = tnn_batch_prepare(items, n_items, &cfg, d_scratch, bytes, stream, &plan);
        if (rc != TNN_OK) goto done;
        rc = tnn_query_batched(&plan, stream);  // warm-up
        if (rc != TNN_OK) goto done;
        if (hipEventRecord(e0, st) != hipSuccess) { rc = TNN_E_HIP; goto done; }
        for (int r = 0; r < 3; ++r) {
          rc = tnn_query_batched(&plan, stream);
          if (rc != TNN_OK) goto done;
        }
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          rc = TNN_E_HIP;
          goto done;
        }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = TNN_E_HIP; goto done; }
        if (ms < best_ms) {
          best_ms = ms;
          *best = cfg;
        }
      }
  if (cache_path) {
    if (FILE *f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "%s %d %d %d\n", key, best->chunk, best->waves_per_block, best->blocks_per_cu);
      std::fclose(f);
    }
  }
done:
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
