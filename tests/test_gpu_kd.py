"""The kd order of the index build, made on the device level by level: the
segment order it produces equals a numpy rendering of the same splits (a
range longer than a block splits along its widest key axis into its m
smallest entries by key, ties by segment number, and the rest, each part
keeping its order; m = n/2 rounded up to a multiple of the block; inside
each block the splits go on, m = n/2, down to single segments).  Sizes
from a single split to ranges of tens of thousands of segments (several
partition chunks per workgroup), with tied keys, zero order scales and one
point per segment."""
import numpy as np
import pytest
import torch

from gpu_util import build, say
from kd_reference import kd_reference, segment_keys
from paper_2112_10408_amd import synth
from paper_2112_10408_amd import tnn as T

pytestmark = pytest.mark.gpu


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
    want = kd_reference(segment_keys(ps, seg_len, order_scale))
    assert got.shape == want.shape
    assert np.array_equal(got, want)


def test_no_order_scale_keeps_trajectory_order():
    """Without order scales the segments stay in trajectory order (no kd
    order), and the searches still return the oracle's neighbours."""
    import oracle
    from gpu_util import assert_same, dev_points

    ps = synth.trajectories(50, 130, 300.0, 3 * 3600.0, seed=77)
    ix = build(ps, 8, None)
    got = T.tnn_debug_export_index(ix)["seg_i32"][:, 0].cpu().numpy()
    assert np.array_equal(got, np.arange(ix.n_segments))
    qs, _ = synth.sample_queries(ps, 200, seed=78)
    gi, gd = T.tnn_query(ix, *dev_points(qs), synth.SCALE, 0.0, 16)
    torch.cuda.synchronize()
    oi, od = oracle.knn(ps.soa(), qs.soa(), synth.SCALE, 0.0, 16)
    assert_same(gi.cpu().numpy(), gd.cpu().numpy(), oi, od, "trajectory order")
