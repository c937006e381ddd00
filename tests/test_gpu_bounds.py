"""The bound invariant at scale (Sec. 3.4 pruning criterion, Algorithm 1):
every cylinder bound and block bound the search uses is at most the exact
binary64 distance (oracle arithmetic) of every candidate member, over about
1e7 (query, segment) pairs per case, with adversarial queries: on the
segment, at both end caps and just beyond them, at distance R from the axis
(where max(0, D - R) is 0 up to rounding), at, just after and inside a
segment's time span, climbing segments under a large z scale, and
coordinates offset to about 1e4 km (float32 spacing near 1 m).  The mask is
exact: a bound is finite iff some member is a candidate.  The per-query-scale
variant checks the bounds each query forms for its own metric."""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_util import build, dev_points, say
from paper_2112_10408_amd import synth
from paper_2112_10408_amd import tnn as T

pytestmark = pytest.mark.gpu

K = 11


def _climbing(seed, offset, n_traj=80, n_pts=300):
    """Trajectories that climb and wiggle (z and y vary within a segment), so
    that anisotropic scales matter for the projection and radius."""
    rng = np.random.default_rng(seed)
    ps = synth.trajectories(n_traj, n_pts, 400.0, 3600.0, seed)
    ps.z = (ps.z + np.cumsum(rng.normal(0, 0.3, ps.n))).astype(np.float32)
    ps.y = (ps.y + rng.normal(0, 0.4, ps.n) + offset).astype(np.float32)
    ps.x = (ps.x + offset).astype(np.float32)
    return ps


def _adversarial_queries(ps, scale, n, seed):
    """n queries, each built against one random segment (trajectory order)."""
    rng = np.random.default_rng(seed)
    seg = oracle.segments(ps.soa(), ps.offsets, K)
    S = seg["start"].shape[0]
    s3 = np.asarray(scale[:3], dtype=np.float64)
    js = rng.integers(0, S, n)
    out = np.empty((n, 4), dtype=np.float64)
    for i, j in enumerate(js):
        A, B = seg["a"][j], seg["b"][j]
        AB = B - A
        tmin, tmax = seg["tmin"][j], seg["tmax"][j]
        kind = i % 6
        if kind == 0:    # on the segment
            P = A + rng.uniform(0, 1) * AB
        elif kind == 1:  # an end cap
            P = A.copy() if rng.uniform() < 0.5 else B.copy()
        elif kind == 2:  # just beyond an end cap along the axis
            P = A - 1e-3 * AB if rng.uniform() < 0.5 else B + 1e-3 * AB
        elif kind == 3:  # at distance R(s) from the axis, perpendicular in the s metric
            R = math.sqrt(float((s3 * seg["e"][j] ** 2).sum()))
            v = rng.normal(size=3)
            n2 = float((s3 * AB * AB).sum())
            if n2 > 0:
                v = v - (float((s3 * v * AB).sum()) / n2) * AB
            nv = math.sqrt(float((s3 * v * v).sum()))
            P = A + rng.uniform(0, 1) * AB + (R / nv if nv > 0 else 0.0) * v
        elif kind == 4:  # off the segment by a few radii
            P = A + rng.uniform(-0.2, 1.2) * AB + rng.normal(0, 0.5, 3)
        else:            # a random point near the data
            P = np.array([rng.uniform(ps.x.min(), ps.x.max()), rng.uniform(ps.y.min(), ps.y.max()),
                          rng.uniform(ps.z.min(), ps.z.max())])
        tk = rng.integers(0, 4)
        if tk == 0:
            t = tmax                                        # last member masked
        elif tk == 1:
            t = float(np.nextafter(np.float32(tmax), np.float32(np.inf)))  # every member valid
        elif tk == 2:
            t = rng.uniform(tmin, tmax)                     # inside the span
        else:
            t = tmax + rng.uniform(0, 40)
        out[i, :3] = P
        out[i, 3] = t
    qs = synth.PointSet(*(out[:, c].astype(np.float32) for c in range(4)),
                        np.array([0, n], dtype=np.int64))
    return qs


def _check_bounds(ps, qs, ix, scale, t_window, qscale=None, chunk=192):
    """lb <= min candidate distance for every (query, segment); block bounds
    likewise; masks exact.  Returns the number of pairs checked."""
    q = dev_points(qs)
    qsc = torch.from_numpy(qscale).cuda() if qscale is not None else None
    seg_lb, blk_lb = T.tnn_debug_lower_bounds(ix, *q, scale, t_window, query_scale=qsc)
    ex = T.tnn_debug_export_index(ix)
    torch.cuda.synchronize()
    seg_lb = seg_lb.cpu().numpy()
    blk_lb = blk_lb.cpu().numpy().astype(np.float64)
    si = ex["seg_i32"].cpu().numpy()
    pid = ex["point_id"].cpu().numpy().astype(np.int64)
    S, nb = ix.n_segments, ix.n_blocks
    starts = si[:, 1]
    assert np.array_equal(starts, np.concatenate([[0], np.cumsum(si[:-1, 2])]))
    pt_slot = ps.t[pid].astype(np.float64)
    sc = np.asarray(scale if qscale is None else qscale, dtype=np.float64)
    for c0 in range(0, qs.n, chunk):
        c1 = min(qs.n, c0 + chunk)
        QQ = np.repeat(np.arange(c0, c1, dtype=np.int64), ps.n)
        PP = np.tile(pid, c1 - c0)
        d = oracle.pair_dist(ps.soa(), qs.soa(), QQ, PP, sc).reshape(c1 - c0, ps.n)
        thr = qs.t[c0:c1].astype(np.float64)[:, None] - t_window
        d = np.where(pt_slot[None, :] < thr, d, np.inf)
        dmin = np.minimum.reduceat(d, starts, axis=1)           # [chunk, S]
        lb = seg_lb[c0:c1]
        assert not np.isnan(lb).any()
        bad = ~(lb <= dmin)
        assert not bad.any(), (f"cylinder bound above a member's distance at "
                               f"{np.argwhere(bad)[:5].tolist()}: lb {lb[bad][:5]} d {dmin[bad][:5]}")
        assert np.array_equal(np.isfinite(lb), np.isfinite(dmin)), "mask differs"
        bmin = np.minimum.reduceat(dmin, np.arange(0, S, 64), axis=1)  # [chunk, nb]
        assert bmin.shape[1] == nb
        assert np.all(blk_lb[c0:c1] <= bmin), "block bound above a member's distance"
    return qs.n * S


@pytest.mark.parametrize("offset", [0.0, 1.0e4])
@pytest.mark.parametrize("scale,t_window", [((1.0, 1.0, 10.0, 0.05), 0.0),
                                            ((1.0, 1.0, 100.0, 0.05), 25.0),
                                            ((0.3, 2.0, 100.0, 0.5), 0.0)])
def test_bound_invariant_at_scale(offset, scale, t_window):
    ps = _climbing(21, offset)
    ix = build(ps, K, order_scale=scale)
    qs = _adversarial_queries(ps, scale, 4800, seed=22)
    say(f"bound invariant: offset {offset}, scale {scale}, t_w {t_window}: "
        f"{qs.n} queries x {ix.n_segments} segments")
    pairs = _check_bounds(ps, qs, ix, scale, t_window)
    assert pairs >= 1e7


@pytest.mark.parametrize("offset", [0.0, 1.0e4])
def test_bound_invariant_per_query_scales(offset):
    """Every query under its own scales (a smooth field around (1, 1, 10,
    0.05) plus rows with sigma_z = 100, zero and tiny scales): the bounds the
    per-query-scale search forms (1/|AB|^2_s, R and the slack computed per
    query) hold for every candidate member."""
    ps = _climbing(23, offset)
    ix = build(ps, K)
    base = (1.0, 1.0, 10.0, 0.05)
    qs = _adversarial_queries(ps, base, 4800, seed=24)
    rows = synth.scale_field(qs.x - np.float32(offset), qs.y - np.float32(offset), qs.z, 400.0,
                             seed=25)
    rows = np.ascontiguousarray(rows, dtype=np.float64)
    rows[1::7, 2] = 100.0
    rows[2::7, 3] = 0.0
    rows[3::7, :3] = 0.0
    rows[4::7, 0] = 1e-6
    say(f"per-query-scale bounds: offset {offset}: {qs.n} queries x {ix.n_segments} segments")
    pairs = _check_bounds(ps, qs, ix, base, 0.0, qscale=rows)
    assert pairs >= 1e7


def test_per_query_bounds_equal_shared_bounds_for_equal_rows():
    """With every row equal to the shared scales, the per-query bounds are
    valid and no tighter than allowed: within float32 rounding of the shared
    ones (they differ only in how the slack is formed)."""
    ps = _climbing(26, 0.0, n_traj=20, n_pts=120)
    ix = build(ps, K)
    base = (1.0, 1.0, 10.0, 0.05)
    qs = _adversarial_queries(ps, base, 600, seed=27)
    q = dev_points(qs)
    rows = torch.tensor([base] * qs.n, dtype=torch.float64, device="cuda")
    a, _ = T.tnn_debug_lower_bounds(ix, *q, base, 0.0)
    b, _ = T.tnn_debug_lower_bounds(ix, *q, base, 0.0, query_scale=rows)
    torch.cuda.synchronize()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(np.isinf(a), np.isinf(b))
    fin = np.isfinite(a)
    assert np.allclose(np.sqrt(b[fin]), np.sqrt(a[fin]), rtol=1e-5, atol=1e-3)
    # an invalid row gets NaN bounds
    rows[5, 1] = -1.0
    c, _ = T.tnn_debug_lower_bounds(ix, *q, base, 0.0, query_scale=rows)
    torch.cuda.synchronize()
    c = c.cpu().numpy()
    assert np.isnan(c[5]).all() and not np.isnan(np.delete(c, 5, axis=0)).any()
