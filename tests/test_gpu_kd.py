"""The kd order of the index build, made on the device level by level: the
segment order it produces equals a numpy rendering of the same splits (a
range longer than a block splits along its widest key axis into its m
smallest entries by key, ties by segment number, and the rest, each part
keeping its order; m = n/2 rounded up to a multiple of the block; inside
each block the splits go on, m = n/2, down to single segments).  Sizes
from a single split to ranges of tens of thousands of segments (several
partition chunks per workgroup), with tied keys, zero order scales and one
point per segment."""
import math

import numpy as np
import pytest
import torch

from gpu_util import build, say
from paper_2112_10408_amd import synth
from paper_2112_10408_amd import tnn as T

pytestmark = pytest.mark.gpu
BLOCK = 64


def _segment_keys(ps, seg_len, order_scale):
    """Per segment in trajectory order: (float32 centroid of first and last
    point) x float32 sqrt(scale), the time key from the run's min and max."""
    osc = np.array([math.sqrt(s) for s in order_scale], dtype=np.float64).astype(np.float32)
    rows = []
    for j in range(len(ps.offsets) - 1):
        for p in range(int(ps.offsets[j]), int(ps.offsets[j + 1]), seg_len):
            q = min(p + seg_len, int(ps.offsets[j + 1])) - 1
            tt = ps.t[p:q + 1].astype(np.float32)
            c = [0.5 * (float(a[p]) + float(a[q])) for a in (ps.x, ps.y, ps.z)]
            c.append(0.5 * (float(tt.min()) + float(tt.max())))
            rows.append(np.array(c, dtype=np.float64).astype(np.float32) * osc)
    return np.array(rows, dtype=np.float32).reshape(-1, 4)


def _split(idx, keys, s, n, m):
    """idx[s:s+n] into its m smallest by (key on the range's widest axis,
    segment number) and the rest, each part keeping its order."""
    r = idx[s:s + n].copy()
    k = keys[r]
    ext = k.max(axis=0) - k.min(axis=0)
    ax = 0
    for f in range(1, 4):
        if ext[f] > ext[ax]:
            ax = f
    order = np.lexsort((r, k[:, ax] + np.float32(0.0)))  # -0 as +0
    left = np.zeros(n, dtype=bool)
    left[order[:m]] = True
    idx[s:s + n] = np.concatenate([r[left], r[~left]])


def _levels(ranges, idx, keys, m_of):
    while True:
        nxt, split = [], False
        for s, n in ranges:
            m = m_of(n)
            if m is None:
                nxt.append((s, n))
                continue
            _split(idx, keys, s, n, m)
            nxt += [(s, m), (s + m, n - m)]
            split = True
        ranges = nxt
        if not split:
            return


def _block_m(n):
    if n <= BLOCK:
        return None
    m = ((n // 2 + BLOCK - 1) // BLOCK) * BLOCK
    return (n - 1) // BLOCK * BLOCK if m >= n else m


def _kd_reference(keys):
    S = keys.shape[0]
    idx = np.arange(S, dtype=np.int64)
    _levels([(0, S)], idx, keys, _block_m)
    # inside each block the splits go on down to single entries, m = n // 2
    _levels([(b, min(BLOCK, S - b)) for b in range(0, S, BLOCK)], idx, keys,
            lambda n: n // 2 if n >= 2 else None)
    return idx


@pytest.mark.parametrize("n_traj,n_pts,seg_len,order_scale,dups", [
    (4, 40, 1, synth.SCALE, 0),                  # 160 segments: one split level
    (60, 90, 8, synth.SCALE, 10),                # tied keys from duplicated trajectories
    (300, 200, 4, (1.0, 1.0, 0.0, 0.0), 0),      # zero scales: only x and y split
    (2000, 200, 8, synth.SCALE, 40),             # 50k segments
    (500, 400, 1, (1.0, 4.0, 10.0, 0.05), 0),    # 200k one-point segments
])
def test_kd_order_matches_reference(n_traj, n_pts, seg_len, order_scale, dups):
    ps = synth.trajectories(n_traj, n_pts, 500.0, 6 * 3600.0, seed=71 + n_traj)
    if dups:
        # the first trajectories repeated at the end: equal keys, resolved
        # by segment number
        take = np.arange(int(ps.offsets[dups]))
        ps = synth.PointSet(np.concatenate([ps.x, ps.x[take]]), np.concatenate([ps.y, ps.y[take]]),
                            np.concatenate([ps.z, ps.z[take]]), np.concatenate([ps.t, ps.t[take]]),
                            np.concatenate([ps.offsets, ps.offsets[1:dups + 1] + ps.offsets[-1]]))
    say("kd order", n_traj, n_pts, seg_len, ps.n)
    ix = build(ps, seg_len, order_scale)
    got = T.tnn_debug_export_index(ix)["seg_i32"][:, 0].cpu().numpy().astype(np.int64)
    want = _kd_reference(_segment_keys(ps, seg_len, order_scale))
    assert got.shape == want.shape
    assert np.array_equal(got, want)
