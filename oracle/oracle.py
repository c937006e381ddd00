"""Oracle functions (binary64, plain and slow).  TEST INFRASTRUCTURE ONLY.

Pieces and the passage each follows:

* ``knn``            -- brute-force masked scaled k-NN (C, OpenMP).  The scaled
                        metric and its space/time split (Sec. 3.4), the strict
                        time mask t_i < t_q - t_w (Sec. 3.4 masked temporal
                        part, Sec. 3.5), ties by caller index.  The paper states
                        the trajectory search is exact (Sec. 4.2), so this is
                        the result it must reach.
* ``knn`` with one scale row per query -- the same search when the scale
                        vector is a function of position (Sec. 3.2), each
                        query under its own metric.
* ``segments``       -- partition into runs of K points, segment AB from first to
                        last point, per-axis approximation error from the
                        Euclidean clamped projection (Sec. 3.4).
* ``lower_bound``    -- cylinder lower bound from a query to a segment:
                        projection in the scaled metric, radius subtracted in
                        non-squared units, masked time gap (Sec. 3.4 masked
                        distance and pruning criterion, Algorithm 1), in the
                        corrected reading (printed form is not a lower bound).
* ``gka_average``    -- Gaussian kernel averaging of measured values over the
                        context of each query (Sec. 3.2, Eq. gka), the context
                        being the k nearest past points; the exponent read as
                        decaying, exp(-d) with d the scaled squared distance.
* ``radius_*``/``mlp_*``/``adam_step`` -- the learned k-th radius predictor
                        (not in the paper): feature map, a 6-64-64-1 ReLU MLP,
                        squared-error loss on log r_k, its gradient by
                        backpropagation, Adam (Kingma & Ba 2015, Alg. 1), and
                        the safety factor's quantile of log-residuals.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build_oracle

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = build_oracle.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(build_oracle.SRC):
            build_oracle.build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.oracle_knn.argtypes = [i64, P, P, P, P, i64, P, P, P, P, P, f64, i32, P, P]
        lib.oracle_knn.restype = ctypes.c_int
        lib.oracle_knn_qscale.argtypes = [i64, P, P, P, P, i64, P, P, P, P, P, f64, i32, P, P]
        lib.oracle_knn_qscale.restype = ctypes.c_int
        lib.oracle_pair_dist.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, P]
        lib.oracle_pair_dist.restype = ctypes.c_int
        lib.oracle_pair_dist_qscale.argtypes = [i64, P, P, P, P, P, P, P, P, P, P, P, P]
        lib.oracle_pair_dist_qscale.restype = ctypes.c_int
        lib.oracle_segment_count.argtypes = [P, i64, i32]
        lib.oracle_segment_count.restype = i64
        lib.oracle_segments.argtypes = [P, P, P, P, P, i64, i32, i64, P, P, P, P, P, P, P]
        lib.oracle_segments.restype = i64
        _lib = lib
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def knn(points, queries, scale, t_window: float, k: int):
    """points/queries: (x, y, z, t) float32 arrays.  Returns (idx int64 [nq,k],
    dist float64 [nq,k]); empty slots are (-1, +inf).  `scale` is one vector of
    4 scales, or one row of 4 per query (per-query metric; a row with a
    negative or non-finite scale gives (-1, NaN) slots)."""
    lib = _load()
    px, py, pz, pt = (_f32(a) for a in points)
    qx, qy, qz, qt = (_f32(a) for a in queries)
    n, nq = px.shape[0], qx.shape[0]
    s = np.ascontiguousarray(scale, dtype=np.float64)
    idx = np.empty((nq, k), dtype=np.int64)
    dist = np.empty((nq, k), dtype=np.float64)
    if s.ndim == 2:
        if s.shape != (nq, 4):
            raise ValueError("per-query scales must be [n_queries, 4]")
        fn = lib.oracle_knn_qscale
    else:
        fn = lib.oracle_knn
    rc = fn(n, _ptr(px), _ptr(py), _ptr(pz), _ptr(pt), nq, _ptr(qx), _ptr(qy), _ptr(qz), _ptr(qt),
            _ptr(s), float(t_window), int(k), _ptr(idx), _ptr(dist))
    if rc != 0:
        raise ValueError("oracle_knn: bad argument")
    return idx, dist


def pair_dist(points, queries, qi, pi, scale):
    """Binary64 scaled squared distance of each pair (queries[qi[j]],
    points[pi[j]]) with the k-NN's arithmetic.  `scale`: one vector of 4, or
    one row of 4 per query (each pair under its query's metric)."""
    lib = _load()
    px, py, pz, pt = (_f32(a) for a in points)
    qx, qy, qz, qt = (_f32(a) for a in queries)
    qi = np.ascontiguousarray(qi, dtype=np.int64)
    pi = np.ascontiguousarray(pi, dtype=np.int64)
    s = np.ascontiguousarray(scale, dtype=np.float64)
    out = np.empty(qi.shape[0], dtype=np.float64)
    if s.ndim == 2:
        if s.shape != (qx.shape[0], 4):
            raise ValueError("per-query scales must be [n_queries, 4]")
        fn = lib.oracle_pair_dist_qscale
    else:
        fn = lib.oracle_pair_dist
    rc = fn(qi.shape[0], _ptr(qi), _ptr(pi), _ptr(qx), _ptr(qy), _ptr(qz),
                              _ptr(qt), _ptr(px), _ptr(py), _ptr(pz), _ptr(pt), _ptr(s), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_pair_dist: bad argument")
    return out


def segments(points, offsets, seg_len: int):
    """Segment table in trajectory order (dict of arrays)."""
    lib = _load()
    x, y, z, t = (_f32(a) for a in points)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    n_traj = off.shape[0] - 1
    cap = lib.oracle_segment_count(_ptr(off), n_traj, seg_len)
    if cap < 0:
        raise ValueError("bad offsets or seg_len")
    start = np.empty(cap, np.int64)
    count = np.empty(cap, np.int32)
    a = np.empty((cap, 3), np.float64)
    b = np.empty((cap, 3), np.float64)
    tmin = np.empty(cap, np.float64)
    tmax = np.empty(cap, np.float64)
    e = np.empty((cap, 3), np.float64)
    s = lib.oracle_segments(_ptr(x), _ptr(y), _ptr(z), _ptr(t), _ptr(off), n_traj, seg_len, cap,
                            _ptr(start), _ptr(count), _ptr(a), _ptr(b), _ptr(tmin), _ptr(tmax), _ptr(e))
    if s != cap:
        raise ValueError("oracle_segments failed")
    return dict(start=start, count=count, a=a, b=b, tmin=tmin, tmax=tmax, e=e)


def lower_bound(seg, queries, scale, t_window: float):
    """Cylinder lower bound lb[q, j] (binary64) for every query and segment.

    Mask (Sec. 3.4 masked temporal part): lb = +inf when t_min >= t_q - t_w,
    since then no member is strictly earlier than t_q - t_w.
    Otherwise, with the projection taken in the scaled metric,
        delta = clamp(<AP, AB>_s / |AB|_s^2, 0, 1)   (0 if |AB|_s = 0)
        D     = |AP - delta AB|_s                     (distance to segment)
        R     = sqrt(sum_f s_f e_f^2)                 (radius covering members)
        gap   = max(0, t_q - t_max, t_w)              (time gap to any valid member)
        lb    = max(0, D - R)^2 + s_t gap^2.
    The error is subtracted from the non-squared distance (the printed
    subtraction of squared quantities is not a lower bound), and the time gap
    is t_q - t_max (the printed t_B - t has the wrong sign).
    Plain numpy over a [nq, S] grid: small cases only.
    """
    s = np.asarray(scale, dtype=np.float64)
    qx, qy, qz, qt = (np.asarray(a, dtype=np.float64)[:, None] for a in queries)
    A = seg["a"][None]
    B = seg["b"][None]
    AB = B - A
    AP = np.stack([qx - A[..., 0], qy - A[..., 1], qz - A[..., 2]], axis=-1)
    n2 = (s[:3] * AB * AB).sum(-1)
    dot = (s[:3] * AP * AB).sum(-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        delta = np.where(n2 > 0, np.clip(dot / np.where(n2 > 0, n2, 1.0), 0.0, 1.0), 0.0)
    res = AP - delta[..., None] * AB
    D = np.sqrt((s[:3] * res * res).sum(-1))
    R = np.sqrt((s[:3] * seg["e"] ** 2).sum(-1))[None]
    gap = np.maximum(np.maximum(qt - seg["tmax"][None], 0.0), float(t_window))
    lb = np.maximum(D - R, 0.0) ** 2 + s[3] * gap * gap
    masked = seg["tmin"][None] >= qt - float(t_window)
    return np.where(masked, np.inf, lb)


# ----------------------------------------------------------------------------
# Learned k-th radius (not in the paper).
# ----------------------------------------------------------------------------
HIDDEN = 64
N_IN = 6
GRID = 32
START_XY = 128   # trajectory-start grid: cells along x and y
START_T = 512    # ... and along t
# parameter vector order: W1[64x6] b1[64] W2[64x64] b2[64] W3[64] b3[1]
PARAM_SHAPES = [("W1", (HIDDEN, N_IN)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)),
                ("b2", (HIDDEN,)), ("W3", (HIDDEN,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(sh)) for _, sh in PARAM_SHAPES)


def unpack_params(vec):
    vec = np.asarray(vec, dtype=np.float64)
    out, o = {}, 0
    for name, sh in PARAM_SHAPES:
        m = int(np.prod(sh))
        out[name] = vec[o:o + m].reshape(sh)
        o += m
    return out


def pack_params(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in PARAM_SHAPES])


def _cell(v, l, h, g):
    """min(g-1, max(0, trunc((v - l) * (g / (h - l))))) evaluated in float32
    exactly as written (0 for an empty span or a non-finite product)."""
    v = np.asarray(v, dtype=np.float32)
    l32, h32 = np.float32(l), np.float32(h)
    span = h32 - l32
    cs = np.float32(g) / span if span > 0 else np.float32(0.0)
    c = ((v - l32) * cs).astype(np.float32)
    c = np.where(np.isfinite(c), c, np.float32(0.0))
    return np.clip(np.trunc(c), 0, g - 1).astype(np.int64)


def radius_cells(px, py, pt, lo, hi):
    """Cell of the (x, y, t) density grid, decided in float32 exactly as
    written: c = min(G-1, max(0, trunc((v - lo) * (G / (hi - lo)))))."""
    return [_cell(v, l, h, GRID) for v, l, h in ((px, lo[0], hi[0]), (py, lo[1], hi[1]),
                                                (pt, lo[3], hi[3]))]


def radius_start_cells(px, py, pt, lo, hi):
    """Cell of the finer trajectory-start grid (START_XY x START_XY x START_T)."""
    return (_cell(px, lo[0], hi[0], START_XY), _cell(py, lo[1], hi[1], START_XY),
            _cell(pt, lo[3], hi[3], START_T))


def radius_start_grid(first_x, first_y, first_t, lo, hi):
    """Number of trajectories whose first point falls in each cell."""
    cx, cy, ct = radius_start_cells(first_x, first_y, first_t, lo, hi)
    grid = np.zeros((START_XY, START_XY, START_T), dtype=np.int64)
    np.add.at(grid, (cx, cy, ct), 1)
    return grid


def radius_start_count(qx, qy, qt, lo, hi, starts):
    """Trajectory starts in the query's start-grid cell, its eight spatial
    neighbours, and the same nine cells one time step earlier (cells outside
    the grid contribute nothing)."""
    cx, cy, ct = radius_start_cells(qx, qy, qt, lo, hi)
    total = np.zeros(cx.shape, dtype=np.int64)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dt in (-1, 0):
                x, y, t = cx + dx, cy + dy, ct + dt
                inside = (x >= 0) & (x < START_XY) & (y >= 0) & (y < START_XY) & (t >= 0)
                total += np.where(inside, starts[np.clip(x, 0, START_XY - 1),
                                                 np.clip(y, 0, START_XY - 1),
                                                 np.clip(t, 0, START_T - 1)], 0)
    return total


def radius_density_grid(seg_a, seg_b, seg_tmin, seg_tmax, lo, hi):
    """Segment count per (x, y, t) cell, by segment midpoint computed in
    float32 as 0.5 * (first + last)."""
    a = np.asarray(seg_a, dtype=np.float32)
    b = np.asarray(seg_b, dtype=np.float32)
    mx = np.float32(0.5) * (a[:, 0] + b[:, 0])
    my = np.float32(0.5) * (a[:, 1] + b[:, 1])
    mt = np.float32(0.5) * (np.asarray(seg_tmin, np.float32) + np.asarray(seg_tmax, np.float32))
    cx, cy, ct = radius_cells(mx, my, mt, lo, hi)
    grid = np.zeros((GRID, GRID, GRID), dtype=np.int64)
    np.add.at(grid, (cx, cy, ct), 1)
    return grid


def radius_features(qx, qy, qz, qt, lo, hi, grid, starts):
    """Feature map: the four coordinates mapped to [-1, 1] over the data's
    bounding box, 0.25 log1p of the segment count of the query's grid cell,
    and 0.5 log1p of the trajectory starts around the query in space and
    recent time (radius_start_count): a query near the start of its own
    trajectory has few earlier points of it, so its k-th distance is larger."""
    cols = []
    for v, l, h in zip((qx, qy, qz, qt), lo, hi):
        v = np.asarray(v, dtype=np.float64)
        span = float(h) - float(l)
        g = 2.0 / span if span > 0 else 1.0
        cols.append((v - 0.5 * (float(l) + float(h))) * g)
    cx, cy, ct = radius_cells(qx, qy, qt, lo, hi)
    cols.append(0.25 * np.log1p(grid[cx, cy, ct].astype(np.float64)))
    cols.append(0.5 * np.log1p(radius_start_count(qx, qy, qt, lo, hi, starts).astype(np.float64)))
    return np.stack(cols, axis=1)


def mlp_forward(params, X):
    """Returns (out[n], cache).  out = W3 relu(W2 relu(W1 x + b1) + b2) + b3."""
    p = params if isinstance(params, dict) else unpack_params(params)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    out = h2 @ p["W3"] + p["b3"][0]
    return out, (X, z1, h1, z2, h2)


def mlp_loss(params, X, y):
    """Mean squared error over samples with a finite label."""
    out, _ = mlp_forward(params, X)
    m = np.isfinite(y)
    n = max(int(m.sum()), 1)
    r = np.where(m, out - np.where(m, y, 0.0), 0.0)
    return float((r * r).sum() / n)


def mlp_loss_grad(params, X, y):
    """Backpropagation of ``mlp_loss``; returns (loss, flat gradient)."""
    p = params if isinstance(params, dict) else unpack_params(params)
    out, (X, z1, h1, z2, h2) = mlp_forward(p, X)
    m = np.isfinite(y)
    n = max(int(m.sum()), 1)
    r = np.where(m, out - np.where(m, y, 0.0), 0.0)
    loss = float((r * r).sum() / n)
    g_out = 2.0 * r / n                       # dL/dout
    g = {"W3": h2.T @ g_out, "b3": np.array([g_out.sum()])}
    g_h2 = np.outer(g_out, p["W3"])
    g_z2 = g_h2 * (z2 > 0)
    g["W2"] = g_z2.T @ h1
    g["b2"] = g_z2.sum(0)
    g_h1 = g_z2 @ p["W2"]
    g_z1 = g_h1 * (z1 > 0)
    g["W1"] = g_z1.T @ X
    g["b1"] = g_z1.sum(0)
    return loss, pack_params(g)


def adam_step(theta, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); step counts from 1.
    Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def radius_calibrate(logr, kth_dist, quantile):
    """Safety factor of the predicted radius: alpha = exp(x_q), x_q the
    q-quantile of the log-residuals 0.5 log d_k - logr over the samples whose
    k-th distance d_k is finite and positive and whose residual is finite.
    The quantile interpolates linearly between the order statistics at
    position (m - 1) q of the m sorted residuals: x_lo + (h - lo)(x_hi - x_lo)
    with h = (m - 1) q, lo = floor(h).  No such sample: alpha = 1."""
    d = np.asarray(kth_dist, dtype=np.float64)
    lr = np.asarray(logr, dtype=np.float32).astype(np.float64)
    ok = np.isfinite(d) & (d > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = 0.5 * np.log(np.where(ok, d, 1.0)) - lr
    r = np.sort(r[ok & np.isfinite(r)])
    m = r.shape[0]
    if m == 0:
        return 1.0
    h = float(m - 1) * float(quantile)
    lo = int(math.floor(h))
    x_lo = r[lo]
    x_hi = r[lo + 1] if lo + 1 < m else x_lo
    return math.exp(x_lo + (h - lo) * (x_hi - x_lo))


def radius_label(kth_dist):
    """Training target: log of the k-th neighbour radius, r_k = sqrt(d_k);
    +inf distance (fewer than k candidates) gives a non-finite label."""
    d = np.asarray(kth_dist, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(np.isfinite(d) & (d > 0), 0.5 * np.log(np.where(d > 0, d, 1.0)), np.nan)


def finite_difference_grad(params, X, y, h=1e-6, which=None):
    """Central differences of ``mlp_loss`` (independent of the backprop code)."""
    theta = np.array(params, dtype=np.float64)
    idx = range(theta.shape[0]) if which is None else which
    g = np.zeros(theta.shape[0])
    for i in idx:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        g[i] = (mlp_loss(tp, X, y) - mlp_loss(tm, X, y)) / (2.0 * h)
    return g


# ----------------------------------------------------------------------------
# Gaussian kernel averaging over the k-NN context (Sec. 3.2, Eq. gka).
# ----------------------------------------------------------------------------
def gka_average(idx, dist, values):
    """Forecast per query: sum_c w_c v_c / sum_c w_c over the context slots c
    with idx >= 0, w_c = exp(-d_c) where d_c = sum_f s_f (q_f - p_f)^2 is the
    scaled squared distance the k-NN search returns (the printed exponent
    carries no minus sign; only a decaying kernel gives an average weighted
    towards the nearer measurements, Sec. 3.2).  The weights are taken
    relative to the nearest slot, exp(-(d_c - d_0)), which leaves the ratio
    unchanged and keeps far contexts from underflowing to 0/0.  A query
    without context gets NaN.  idx [Q, k], dist [Q, k], values [N, C] ->
    [Q, C] binary64."""
    idx = np.asarray(idx, dtype=np.int64)
    dist = np.asarray(dist, dtype=np.float64)
    values = np.asarray(values, dtype=np.float64).reshape(len(values), -1)
    nq, k = idx.shape
    out = np.full((nq, values.shape[1]), np.nan)
    for q in range(nq):
        used = [r for r in range(k) if idx[q, r] >= 0 and math.isfinite(dist[q, r])]
        if not used:
            continue
        d0 = dist[q, used[0]]
        num = np.zeros(values.shape[1])
        den = 0.0
        for r in used:
            w = math.exp(-(dist[q, r] - d0))
            num += w * values[idx[q, r]]
            den += w
        out[q] = num / den
    return out
