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


def assert_same(gi, gd, oi, od, what="", rtol=1e-12):
    """Indices bit-exact on every slot; every distance equal to the oracle's
    (both +inf, or both NaN for a row without a metric) or, where not
    bit-identical, within `rtol` relative of it -- checked on every slot of
    every query, not only the first that differs."""
    gi = np.asarray(gi, dtype=np.int64)
    oi = np.asarray(oi, dtype=np.int64)
    gd = np.asarray(gd, dtype=np.float64)
    od = np.asarray(od, dtype=np.float64)
    assert gi.shape == oi.shape and gd.shape == od.shape, f"{what}: shape {gi.shape} vs {oi.shape}"
    bad = np.argwhere(gi != oi)
    if bad.size:
        q = bad[0][0]
        raise AssertionError(f"{what}: index mismatch in {len(np.unique(bad[:, 0]))} queries, first "
                             f"{q}: gpu {gi[q].tolist()} oracle {oi[q].tolist()} "
                             f"gpu_d {gd[q].tolist()} oracle_d {od[q].tolist()}")
    same = (gd == od) | (np.isinf(gd) & np.isinf(od) & (np.sign(gd) == np.sign(od))) | \
        (np.isnan(gd) & np.isnan(od))
    if not same.all():
        diff = ~same
        with np.errstate(invalid="ignore", divide="ignore"):
            rel = np.abs(gd[diff] - od[diff]) / np.maximum(np.abs(od[diff]), 1e-300)
        worst = np.nanargmax(np.where(np.isnan(rel), np.inf, rel))
        q = np.argwhere(diff)[worst][0]
        ok = np.isfinite(rel) & (rel <= rtol)
        assert ok.all(), (f"{what}: {int((~ok).sum())} distances beyond rtol {rtol} in "
                          f"{len(np.unique(np.argwhere(diff)[~ok][:, 0]))} queries; worst "
                          f"query {q}: rel {rel[worst]}")


@functools.lru_cache(maxsize=None)
def config_data(name):
    ps, qs, qidx, cfg = synth.make_config(name)
    return ps, qs, qidx, cfg
