"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the oracle."""
import functools
import sys

import numpy as np
import torch

import oracle
from paper_2112_10408_amd import synth
from paper_2112_10408_amd import tnn as T


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev_points(ps):
    return T.to_device(ps.x, ps.y, ps.z, ps.t)


def build(ps, seg_len, order_scale=synth.SCALE):
    x, y, z, t = dev_points(ps)
    idx = T.tnn_build_segments(x, y, z, t, ps.offsets, seg_len, order_scale)
    idx._keep = (x, y, z, t)
    return idx


def gpu_query(index, qs, scale, t_window, k, **kw):
    qx, qy, qz, qt = dev_points(qs)
    i, d = T.tnn_query(index, qx, qy, qz, qt, scale, t_window, k, **kw)
    torch.cuda.synchronize()
    return i.cpu().numpy(), d.cpu().numpy()


def assert_same(gi, gd, oi, od, what=""):
    """Indices bit-exact; distances bit-identical (the binary64 formula and
    its order are the same on both sides)."""
    gi = np.asarray(gi, dtype=np.int64)
    bad = np.argwhere(gi != oi)
    if bad.size:
        q = bad[0][0]
        raise AssertionError(f"{what}: index mismatch at query {q}: gpu {gi[q].tolist()} "
                             f"oracle {oi[q].tolist()} gpu_d {gd[q].tolist()} oracle_d {od[q].tolist()}")
    same = (gd == od) | (np.isinf(gd) & np.isinf(od))
    if not same.all():
        q = np.argwhere(~same)[0][0]
        rel = np.max(np.abs(gd[q] - od[q]) / np.maximum(np.abs(od[q]), 1e-300))
        assert rel <= 1e-12, f"{what}: distance mismatch at query {q}: rel {rel}"


@functools.lru_cache(maxsize=None)
def config_data(name):
    ps, qs, qidx, cfg = synth.make_config(name)
    return ps, qs, qidx, cfg
