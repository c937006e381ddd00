"""GPU parity of the batched persistent launch (ragged airspaces, k, flags)
against the oracle, HIP-graph replay, device ticks and the autotuner."""
import os

import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_same, build, dev_points, say
from paper_2112_10408_amd import capi, synth
from paper_2112_10408_amd import tnn as T

pytestmark = pytest.mark.gpu
SCALE = synth.SCALE


def _airspaces(seed=3, n_air=9):
    rng = np.random.default_rng(seed)
    out = []
    for a in range(n_air):
        n_traj = int(rng.integers(5, 60))
        n_pts = int(rng.integers(20, 120))
        ps = synth.trajectories(n_traj, n_pts, 300.0, 3600.0, seed=seed * 100 + a)
        nq = 0 if a == 4 else int(rng.integers(1, 400))
        qs, _ = synth.sample_queries(ps, min(nq, ps.n), seed=a) if nq else (ps.take(np.arange(0)), None)
        k = int(rng.choice([1, 8, 32, 64]))
        seg_len = int(rng.choice([8, 16, 32]))
        flags = capi.TNN_LEARNED if a % 3 == 1 else capi.TNN_PLAIN
        out.append(dict(ps=ps, qs=qs, k=k, seg_len=seg_len, flags=flags))
    return out


def _entries(airs):
    entries = []
    for a in airs:
        ix = build(a["ps"], a["seg_len"])
        q = dev_points(a["qs"])
        e = dict(index=ix, q=q, scale=SCALE, k=a["k"], flags=a["flags"])
        if a["flags"] & capi.TNN_LEARNED:
            rng = np.random.default_rng(a["k"])
            r2 = np.exp(rng.normal(5, 2, a["qs"].n)).astype(np.float32)  # any guess
            e["radius2"] = torch.from_numpy(r2).cuda()
        entries.append(e)
    return entries


def _check(airs, outs):
    for a, (oi_t, od_t) in zip(airs, outs):
        if a["qs"].n == 0:
            continue
        oi, od = oracle.knn(a["ps"].soa(), a["qs"].soa(), SCALE, 0.0, a["k"])
        assert_same(oi_t.cpu().numpy(), od_t.cpu().numpy(), oi, od, "batched")


@pytest.mark.parametrize("config", [None, (1, 2, 1), (16, 8, 2)])
def test_batched_matches_oracle(config):
    airs = _airspaces()
    entries = _entries(airs)
    say("batched", config)
    b = T.tnn_batch_prepare(entries, config)
    outs = T.tnn_query_batched(b)
    torch.cuda.synchronize()
    _check(airs, outs)
    ticks = T.tnn_batch_ticks(b).cpu().numpy()
    for i, a in enumerate(airs):
        if a["qs"].n:
            assert ticks[i + 1] >= ticks[0] > 0
        else:
            assert ticks[i + 1] == 0


def test_batched_graph_replay_equals_eager():
    airs = _airspaces(seed=5, n_air=6)
    entries = _entries(airs)
    b = T.tnn_batch_prepare(entries)
    outs = T.tnn_query_batched(b)
    torch.cuda.synchronize()
    ref = [(i.clone(), d.clone()) for i, d in outs]
    _check(airs, ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        T.tnn_query_batched(b)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        T.tnn_query_batched(b)
    for rep in range(3):
        for i, d in outs:  # eager work between replays
            i.fill_(-7)
            d.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (i, d), (ri, rd) in zip(outs, ref):
            assert torch.equal(i, ri) and torch.equal(d, rd), rep


def test_autotuner_picks_and_caches(tmp_path):
    airs = _airspaces(seed=9, n_air=4)
    entries = _entries(airs)
    cache = str(tmp_path / "tune.txt")
    best = T.tnn_autotune_batched(entries, cache)
    assert os.path.exists(cache)
    line = open(cache).read().strip().split()
    assert tuple(int(v) for v in line[-3:]) == best
    assert T.tnn_autotune_batched(entries, cache) == best  # served from the cache
    b = T.tnn_batch_prepare(entries, best)
    outs = T.tnn_query_batched(b)
    torch.cuda.synchronize()
    _check(airs, outs)


def test_full_size_64_airspaces_sampled_against_the_oracle():
    """The 64-airspace serving workload at full size (about 7.4M points and
    873k queries, k in {8, 32, 64}), learned radius from each airspace's own
    (untrained) model: one persistent launch; a seeded sample of 64 queries
    per airspace (plus its earliest query) checked against the oracle, every
    query against the airspace's own plain search, and a second launch
    byte-identical to the first (the work queue's atomics only reorder work)."""
    airs = synth.airspaces(64)
    entries, samples = [], []
    for i, a in enumerate(airs):
        ps, qs = a["points"], a["queries"]
        ix = build(ps, a["seg_len"])
        q = dev_points(qs)
        model = T.tnn_radius_model_init(ix, seed=i + 1)
        r2 = T.tnn_radius_infer(model, *q, alpha=2.0)
        entries.append(dict(index=ix, q=q, scale=SCALE, k=a["k"], flags=capi.TNN_LEARNED,
                            radius2=r2))
        rng = np.random.default_rng(500 + i)
        smp = np.sort(rng.choice(qs.n, min(64, qs.n), replace=False))
        samples.append(np.unique(np.concatenate([smp, [int(np.argmin(qs.t))]])))
    say("full-size batch:", sum(a["points"].n for a in airs), "points,",
        sum(a["queries"].n for a in airs), "queries")
    b = T.tnn_batch_prepare(entries)
    outs = T.tnn_query_batched(b)
    torch.cuda.synchronize()
    first = [(i.cpu().numpy().copy(), d.cpu().numpy().copy()) for i, d in outs]
    T.tnn_query_batched(b)
    torch.cuda.synchronize()
    for (i, d), (fi, fd) in zip(outs, first):
        assert i.cpu().numpy().tobytes() == fi.tobytes() and d.cpu().numpy().tobytes() == fd.tobytes()
    for n_a, (a, e, smp, (gi, gd)) in enumerate(zip(airs, entries, samples, first)):
        oi, od = oracle.knn(a["points"].soa(), a["queries"].take(smp).soa(), SCALE, 0.0, a["k"])
        assert_same(gi[smp], gd[smp], oi, od, f"airspace {n_a} sample")
        pi, pd = T.tnn_query(e["index"], *e["q"], SCALE, 0.0, a["k"])
        torch.cuda.synchronize()
        assert np.array_equal(pi.cpu().numpy(), gi) and np.array_equal(pd.cpu().numpy(), gd), n_a
