"""Python binding of the C ABI: the same entry points, taking torch device
tensors.  Argument marshalling only -- every step runs in libtnn's kernels;
torch supplies device memory and the current stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import capi
from .capi import TnnIndex, TnnPoints, TnnQueryParams, check


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _f32(t):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 CUDA tensor")
    return t


def points(x, y, z, t):
    """tnn_points view of four float32 device tensors (kept alive by caller)."""
    n = x.shape[0]
    for a in (x, y, z, t):
        _f32(a)
        if a.shape[0] != n:
            raise ValueError("x, y, z, t must have the same length")
    return TnnPoints(_ptr(x), _ptr(y), _ptr(z), _ptr(t), n)


def to_device(*arrays, device="cuda"):
    return tuple(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device) for a in arrays)


@dataclass
class Index:
    mem: torch.Tensor
    c: TnnIndex
    n_points: int
    n_segments: int
    n_blocks: int
    seg_len: int

    @property
    def ref(self):
        return ctypes.byref(self.c)


def tnn_build_segments(x, y, z, t, traj_offsets, seg_len, order_scale=(1.0, 1.0, 10.0, 0.05)):
    L = capi.lib()
    off = np.ascontiguousarray(traj_offsets, dtype=np.int64)
    n_traj = off.shape[0] - 1
    nbytes = ctypes.c_size_t(0)
    check(L.tnn_build_segments_workspace(off.ctypes.data_as(ctypes.c_void_p), n_traj, seg_len,
                                         ctypes.byref(nbytes)), "tnn_build_segments_workspace")
    mem = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=x.device)
    idx = TnnIndex()
    osc = None
    if order_scale is not None:
        osc = (ctypes.c_double * 4)(*[float(v) for v in order_scale])
    check(L.tnn_build_segments(points(x, y, z, t), off.ctypes.data_as(ctypes.c_void_p), n_traj,
                               seg_len, osc, _ptr(mem), nbytes.value, _stream(), ctypes.byref(idx)),
          "tnn_build_segments")
    n_p, n_s, n_b, sl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    check(L.tnn_index_info(ctypes.byref(idx), ctypes.byref(n_p), ctypes.byref(n_s), ctypes.byref(n_b),
                           ctypes.byref(sl)), "tnn_index_info")
    return Index(mem, idx, n_p.value, n_s.value, n_b.value, sl.value)


def make_params(scale, t_window, k, flags=0, seed_segments=0, waves_per_block=0, radius2=None,
                stats=None, query_scale=None, gka_values=None, gka_out=None, radius_model=None,
                radius_alpha=1.0):
    p = TnnQueryParams()
    for i in range(4):
        p.scale[i] = float(scale[i])
    p.t_window = float(t_window)
    p.k = int(k)
    p.flags = int(flags)
    p.seed_segments = int(seed_segments)
    p.waves_per_block = int(waves_per_block)
    p.d_radius2 = _ptr(radius2) if radius2 is not None else None
    p.d_stats = _ptr(stats) if stats is not None else None
    if query_scale is not None:
        if query_scale.dtype != torch.float64 or query_scale.dim() != 2 or query_scale.shape[1] != 4:
            raise ValueError("query_scale must be a float64 [n_queries, 4] device tensor")
        if not query_scale.is_contiguous():
            raise ValueError("query_scale must be contiguous")
    p.d_query_scale = _ptr(query_scale) if query_scale is not None else None
    if gka_values is not None:
        if gka_values.dtype != torch.float32 or gka_values.dim() != 2 or not gka_values.is_contiguous():
            raise ValueError("gka_values must be a contiguous float32 [n_points, n_comp] device tensor")
        if gka_out is None or gka_out.dtype != torch.float64 or not gka_out.is_contiguous() or \
                gka_out.dim() != 2 or gka_out.shape[1] != gka_values.shape[1]:
            raise ValueError("gka_out must be a contiguous float64 [n_queries, n_comp] device tensor")
        p.d_gka_values = _ptr(gka_values)
        p.d_gka_out = _ptr(gka_out)
        p.gka_comp = int(gka_values.shape[1])
    if radius_model is not None:
        p.radius_model = _ptr(radius_model)
        p.radius_alpha = float(radius_alpha)
    return p


def tnn_query_workspace(index, n_queries, params):
    nbytes = ctypes.c_size_t(0)
    check(capi.lib().tnn_query_workspace(index.ref, n_queries, ctypes.byref(params), ctypes.byref(nbytes)),
          "tnn_query_workspace")
    return nbytes.value


def new_stats(device="cuda"):
    return torch.zeros(capi.TNN_STAT_COUNT, dtype=torch.int64, device=device)


def stats_dict(stats):
    v = stats.cpu().numpy().astype(np.uint64)
    out = {name: int(v[i]) for i, name in enumerate(capi.STAT_NAMES)}
    out["max_err"] = float(v[8:9].view(np.float64)[0])
    del out["max_err_bits"]
    return out


def tnn_query(index, qx, qy, qz, qt, scale, t_window, k, flags=0, seed_segments=0,
              waves_per_block=0, radius2=None, stats=None, out=None, scratch=None,
              query_scale=None, gka_values=None, gka_out=None, radius_model=None,
              radius_alpha=1.0):
    """Returns (idx int32 [nq, k], dist float64 [nq, k]) device tensors.
    query_scale: optional float64 [nq, 4] device tensor of per-query scales
    (replaces `scale`, which must still be valid).  gka_values (float32
    [n_points, n_comp]) with gka_out (float64 [nq, n_comp]): also the Gaussian
    kernel average of the values over each query's neighbours.  radius_model
    (with TNN_LEARNED, radius2 None): the library predicts the radius itself,
    scaled by radius_alpha, in the launch of its per-call preparation."""
    L = capi.lib()
    nq = qx.shape[0]
    if query_scale is not None and query_scale.shape[0] != nq:
        raise ValueError("query_scale needs one row per query")
    if gka_values is not None and gka_values.dim() == 1:
        gka_values = gka_values.view(-1, 1)
    if gka_values is not None and gka_out is None:
        gka_out = torch.empty((nq, gka_values.shape[1]), dtype=torch.float64, device=qx.device)
    params = make_params(scale, t_window, k, flags, seed_segments, waves_per_block, radius2, stats,
                         query_scale, gka_values, gka_out, radius_model, radius_alpha)
    need = tnn_query_workspace(index, nq, params)
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(max(need, 256), dtype=torch.uint8, device=qx.device)
    if out is None:
        out = (torch.empty((nq, k), dtype=torch.int32, device=qx.device),
               torch.empty((nq, k), dtype=torch.float64, device=qx.device))
    check(L.tnn_query(index.ref, points(qx, qy, qz, qt), ctypes.byref(params), _ptr(out[0]),
                      _ptr(out[1]), _ptr(scratch), scratch.numel(), _stream()), "tnn_query")
    return out


def tnn_query_noalloc(index, qx, qy, qz, qt, scale, t_window, k, flags=0, seed_segments=0,
                      waves_per_block=0, radius2=None, stats=None, out=None, query_scale=None,
                      gka_values=None, gka_out=None, radius_model=None, radius_alpha=1.0):
    """tnn_query with the library's own per-device scratch (no scratch
    argument; the library allocates nothing).  Returns (idx, dist); `out`
    supplies them preallocated."""
    L = capi.lib()
    nq = qx.shape[0]
    if query_scale is not None and query_scale.shape[0] != nq:
        raise ValueError("query_scale needs one row per query")
    params = make_params(scale, t_window, k, flags, seed_segments, waves_per_block, radius2, stats,
                         query_scale, gka_values, gka_out, radius_model, radius_alpha)
    if out is None:
        out = (torch.empty((nq, k), dtype=torch.int32, device=qx.device),
               torch.empty((nq, k), dtype=torch.float64, device=qx.device))
    check(L.tnn_query_noalloc(index.ref, points(qx, qy, qz, qt), ctypes.byref(params),
                              _ptr(out[0]), _ptr(out[1]), _stream()), "tnn_query_noalloc")
    return out


def tnn_debug_export_index(index):
    L = capi.lib()
    dev = index.mem.device
    seg_f = torch.empty((index.n_segments, 12), dtype=torch.float32, device=dev)
    seg_i = torch.empty((index.n_segments, 4), dtype=torch.int32, device=dev)
    pid = torch.empty(index.n_points, dtype=torch.int32, device=dev)
    box = torch.empty((index.n_blocks, 8), dtype=torch.float32, device=dev)
    check(L.tnn_debug_export_index(index.ref, _ptr(seg_f), _ptr(seg_i), _ptr(pid), _ptr(box), _stream()),
          "tnn_debug_export_index")
    return dict(seg_f32=seg_f, seg_i32=seg_i, point_id=pid, block_box=box)


def tnn_debug_lower_bounds(index, qx, qy, qz, qt, scale, t_window, query_scale=None,
                           block_bounds=True):
    """(seg_lb float64 [nq, S], blk_lb float32 [nq, nb] or None).  query_scale:
    optional float64 [nq, 4] device tensor of per-query scales."""
    L = capi.lib()
    nq = qx.shape[0]
    dev = qx.device
    seg_lb = torch.empty((nq, index.n_segments), dtype=torch.float64, device=dev)
    blk_lb = torch.empty((nq, index.n_blocks), dtype=torch.float32, device=dev) if block_bounds else None
    params = make_params(scale, t_window, 1)
    need = tnn_query_workspace(index, nq, params)
    scratch = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    sc = (ctypes.c_double * 4)(*[float(v) for v in scale])
    if query_scale is not None:
        if query_scale.dtype != torch.float64 or tuple(query_scale.shape) != (nq, 4) or \
                not query_scale.is_contiguous():
            raise ValueError("query_scale must be a contiguous float64 [n_queries, 4] device tensor")
    check(L.tnn_debug_lower_bounds(index.ref, points(qx, qy, qz, qt), sc, float(t_window),
                                   _ptr(query_scale), _ptr(seg_lb), _ptr(blk_lb), _ptr(scratch),
                                   scratch.numel(), _stream()), "tnn_debug_lower_bounds")
    return seg_lb, blk_lb


# --------------------------------------------------------------------------
# Learned k-th radius
# --------------------------------------------------------------------------
def tnn_radius_model_bytes():
    n = ctypes.c_size_t(0)
    check(capi.lib().tnn_radius_model_bytes(ctypes.byref(n)), "tnn_radius_model_bytes")
    return n.value


def tnn_radius_model_init(index, seed=1):
    m = torch.empty(tnn_radius_model_bytes(), dtype=torch.uint8, device=index.mem.device)
    check(capi.lib().tnn_radius_model_init(index.ref, _ptr(m), int(seed), _stream()),
          "tnn_radius_model_init")
    return m


def radius_params(model):
    """float32 view of the parameter vector inside a model blob."""
    return model[: capi.RADIUS_NPARAMS * 4].view(torch.float32)


def radius_box(model):
    off = (capi.RADIUS_NPARAMS + 3) * 4
    v = model[off: off + 32].view(torch.float32)
    return v[:4], v[4:]


def radius_grid(model):
    off = (capi.RADIUS_NPARAMS + 3) * 4 + 32
    g = capi.RADIUS_GRID
    return model[off: off + 4 * g ** 3].view(torch.int32).view(g, g, g)


def radius_starts(model):
    """Trajectory starts around each start-grid cell [x][y][t] (the feature's
    neighbourhood sum; uint16 values, widened to int32)."""
    off = (capi.RADIUS_NPARAMS + 3) * 4 + 32 + 4 * capi.RADIUS_GRID ** 3
    sxy, st = capi.RADIUS_START_XY, capi.RADIUS_START_T
    raw = model[off: off + 2 * sxy * sxy * st].view(torch.int16).to(torch.int32) & 0xFFFF
    return raw.view(sxy, sxy, st)


def tnn_radius_train_workspace(batch):
    n = ctypes.c_size_t(0)
    check(capi.lib().tnn_radius_train_workspace(int(batch), ctypes.byref(n)),
          "tnn_radius_train_workspace")
    return n.value


def tnn_radius_shuffle(n, seed, out=None, device="cuda"):
    """Device permutation of 0 .. n-1 (int32) drawn from `seed`."""
    if out is None:
        out = torch.empty(max(int(n), 1), dtype=torch.int32, device=device)
    check(capi.lib().tnn_radius_shuffle(int(n), int(seed) & (2 ** 64 - 1), _ptr(out), _stream()),
          "tnn_radius_shuffle")
    return out[:n]


def tnn_radius_grad(model, sx, sy, sz, st, dist, k, first, batch, scratch=None, order=None):
    dev = sx.device
    grad = torch.empty(capi.RADIUS_NPARAMS, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    need = tnn_radius_train_workspace(batch)
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(need, dtype=torch.uint8, device=dev)
    check(capi.lib().tnn_radius_grad(_ptr(model), points(sx, sy, sz, st), _ptr(dist), _ptr(order),
                                     int(k), int(first), int(batch), _ptr(grad), _ptr(loss),
                                     _ptr(scratch), scratch.numel(), _stream()), "tnn_radius_grad")
    return grad, loss


def tnn_radius_train_step(model, adam, sx, sy, sz, st, dist, k, first, batch, step, lr,
                          loss=None, scratch=None, order=None):
    dev = sx.device
    need = tnn_radius_train_workspace(batch)
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(need, dtype=torch.uint8, device=dev)
    check(capi.lib().tnn_radius_train_step(_ptr(model), _ptr(adam), points(sx, sy, sz, st), _ptr(dist),
                                           _ptr(order), int(k), int(first), int(batch), int(step),
                                           float(lr), _ptr(loss), _ptr(scratch), scratch.numel(),
                                           _stream()),
          "tnn_radius_train_step")
    return scratch


def tnn_radius_calibrate(model, sx, sy, sz, st, dist, k, quantile, out=None, scratch=None):
    """Safety factor alpha (device float32 [1]) for quantile q of the
    log-residuals of the labelled samples."""
    dev = sx.device
    n = ctypes.c_size_t(0)
    check(capi.lib().tnn_radius_calibrate_workspace(int(sx.shape[0]), ctypes.byref(n)),
          "tnn_radius_calibrate_workspace")
    if scratch is None or scratch.numel() < n.value:
        scratch = torch.empty(max(n.value, 256), dtype=torch.uint8, device=dev)
    if out is None:
        out = torch.empty(1, dtype=torch.float32, device=dev)
    check(capi.lib().tnn_radius_calibrate(_ptr(model), points(sx, sy, sz, st), _ptr(dist), int(k),
                                          float(quantile), _ptr(out), _ptr(scratch), scratch.numel(),
                                          _stream()), "tnn_radius_calibrate")
    return out


def tnn_radius_checkpoint_bytes():
    n = ctypes.c_size_t(0)
    check(capi.lib().tnn_radius_checkpoint_bytes(ctypes.byref(n)), "tnn_radius_checkpoint_bytes")
    return n.value


def tnn_radius_model_save(model):
    """Checkpoint bytes (numpy uint8) of a device model."""
    buf = np.empty(tnn_radius_checkpoint_bytes(), dtype=np.uint8)
    check(capi.lib().tnn_radius_model_save(_ptr(model), buf.ctypes.data_as(ctypes.c_void_p),
                                           buf.nbytes, _stream()), "tnn_radius_model_save")
    return buf


def tnn_radius_model_load(buf, model=None, device="cuda"):
    """Device model from checkpoint bytes (TnnError TNN_E_FORMAT if invalid)."""
    buf = np.ascontiguousarray(np.frombuffer(buf, dtype=np.uint8) if isinstance(buf, (bytes, bytearray))
                               else buf, dtype=np.uint8)
    if model is None:
        model = torch.empty(tnn_radius_model_bytes(), dtype=torch.uint8, device=device)
    check(capi.lib().tnn_radius_model_load(buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes,
                                           _ptr(model), _stream()), "tnn_radius_model_load")
    return model


def tnn_radius_features(model, qx, qy, qz, qt):
    f = torch.empty((qx.shape[0], capi.RADIUS_INPUTS), dtype=torch.float32, device=qx.device)
    check(capi.lib().tnn_radius_features(_ptr(model), points(qx, qy, qz, qt), _ptr(f), _stream()),
          "tnn_radius_features")
    return f


def tnn_radius_infer(model, qx, qy, qz, qt, alpha=1.0, out=None, logr=None):
    if out is None:
        out = torch.empty(qx.shape[0], dtype=torch.float32, device=qx.device)
    check(capi.lib().tnn_radius_infer(_ptr(model), points(qx, qy, qz, qt), float(alpha), _ptr(out),
                                      _ptr(logr), _stream()), "tnn_radius_infer")
    return out


def tnn_gka_average(idx, dist, values, out=None):
    """Gaussian kernel averaging of `values` (float32 [n_points, n_comp] on the
    device, caller point order) over each query's context (idx, dist from
    tnn_query).  Returns binary64 [n_queries, n_comp]."""
    nq, k = idx.shape
    vals = values if values.dim() == 2 else values.view(-1, 1)
    n_comp = vals.shape[1]
    if out is None:
        out = torch.empty((nq, n_comp), dtype=torch.float64, device=idx.device)
    check(capi.lib().tnn_gka_average(_ptr(idx), _ptr(dist), nq, k, _ptr(vals), n_comp,
                                     vals.shape[0], _ptr(out), _stream()), "tnn_gka_average")
    return out


# --------------------------------------------------------------------------
# Batched ragged serving
# --------------------------------------------------------------------------
class Batch:
    """A prepared batch: the C item array, its plan and every tensor the
    device descriptors point to (kept alive here)."""

    def __init__(self, items, keep, scratch, plan):
        self.items = items
        self.keep = keep
        self.scratch = scratch
        self.plan = plan


def _batch_items(entries):
    """entries: list of dicts with index, q (x, y, z, t tensors), scale,
    t_window, k, flags, radius2 (opt), stats (opt), out (opt)."""
    n = len(entries)
    arr = (capi.TnnBatchItem * n)()
    keep = []
    outs = []
    for i, e in enumerate(entries):
        qx, qy, qz, qt = e["q"]
        k = int(e["k"])
        out = e.get("out")
        if out is None:
            out = (torch.empty((qx.shape[0], k), dtype=torch.int32, device=qx.device),
                   torch.empty((qx.shape[0], k), dtype=torch.float64, device=qx.device))
        arr[i].index = ctypes.pointer(e["index"].c)
        arr[i].queries = points(qx, qy, qz, qt)
        gv = e.get("gka_values")
        if gv is not None and gv.dim() == 1:
            gv = gv.view(-1, 1)
        if gv is not None and e.get("gka_out") is None:
            e["gka_out"] = torch.empty((qx.shape[0], gv.shape[1]), dtype=torch.float64,
                                       device=qx.device)
        arr[i].params = make_params(e["scale"], e.get("t_window", 0.0), k, e.get("flags", 0),
                                    e.get("seed_segments", 0), 0, e.get("radius2"), e.get("stats"),
                                    None, gv, e.get("gka_out"))
        arr[i].d_out_idx = _ptr(out[0])
        arr[i].d_out_dist = _ptr(out[1])
        keep.append((e, out))
        outs.append(out)
    return arr, keep, outs


def tnn_batch_workspace(items, n):
    b = ctypes.c_size_t(0)
    check(capi.lib().tnn_batch_workspace(items, n, ctypes.byref(b)), "tnn_batch_workspace")
    return b.value


def tnn_batch_prepare(entries, config=None, scratch=None):
    arr, keep, outs = _batch_items(entries)
    n = len(entries)
    need = tnn_batch_workspace(arr, n)
    dev = entries[0]["q"][0].device
    if scratch is None or scratch.numel() < need:
        scratch = torch.empty(need, dtype=torch.uint8, device=dev)
    plan = capi.TnnBatchPlan()
    cfg = None
    if config is not None:
        cfg = capi.TnnBatchConfig(*[int(v) for v in config], 0) if not isinstance(config, capi.TnnBatchConfig) else config
    check(capi.lib().tnn_batch_prepare(arr, n, ctypes.byref(cfg) if cfg is not None else None,
                                       _ptr(scratch), scratch.numel(), _stream(), ctypes.byref(plan)),
          "tnn_batch_prepare")
    b = Batch(arr, keep, scratch, plan)
    b.outs = outs
    return b


def tnn_query_batched(batch):
    check(capi.lib().tnn_query_batched(ctypes.byref(batch.plan), _stream()), "tnn_query_batched")
    return batch.outs


def tnn_batch_ticks(batch):
    """int64 view (device) of the tick array [n_items + 1] inside the scratch."""
    p = ctypes.c_void_p(0)
    check(capi.lib().tnn_batch_ticks(ctypes.byref(batch.plan), ctypes.byref(p)), "tnn_batch_ticks")
    off = p.value - batch.scratch.data_ptr()
    n = len(batch.outs)
    return batch.scratch[off: off + 8 * (n + 1)].view(torch.int64)


def tnn_wall_clock_rate_khz():
    v = ctypes.c_int64(0)
    check(capi.lib().tnn_wall_clock_rate_khz(ctypes.byref(v)), "tnn_wall_clock_rate_khz")
    return v.value


def tnn_autotune_batched(entries, cache_path=None):
    arr, keep, outs = _batch_items(entries)
    n = len(entries)
    need = tnn_batch_workspace(arr, n)
    scratch = torch.empty(need, dtype=torch.uint8, device=entries[0]["q"][0].device)
    best = capi.TnnBatchConfig()
    check(capi.lib().tnn_autotune_batched(arr, n, _ptr(scratch), scratch.numel(), _stream(),
                                          cache_path.encode() if cache_path else None, ctypes.byref(best)),
          "tnn_autotune_batched")
    return (best.chunk, best.waves_per_block, best.blocks_per_cu)
