"""GPU parity: the HIP path (through the C ABI) against the CPU oracle."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_same, build, config_data, dev_points, gpu_query, say
from paper_2112_10408_amd import capi, synth
from paper_2112_10408_amd import tnn as T

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SCALE = synth.SCALE


def _soa(rows):
    a = np.array([[float(Fraction(str(v))) for v in r] for r in rows], dtype=np.float64)
    return synth.PointSet(*(a[:, i].astype(np.float32) for i in range(4)),
                          offsets=np.array([0, a.shape[0]], dtype=np.int64))


def _golden():
    with open(os.path.join(GOLDEN, "knn_cases.json")) as f:
        return json.load(f)["cases"]


MIXED = capi.TNN_BRUTE | capi.TNN_MIXED_BF16
ALL_PATHS = [capi.TNN_PLAIN, capi.TNN_BRUTE, MIXED]


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c["name"])
@pytest.mark.parametrize("flags", ALL_PATHS)
def test_golden_cases(case, flags):
    say("golden", case["name"], flags)
    ps = _soa(case["points"])
    ps.offsets = np.array(case["offsets"], dtype=np.int64)
    qs = _soa(case["queries"])
    ix = build(ps, seg_len=2)
    gi, gd = gpu_query(ix, qs, case["scale"], case["t_window"], case["k"], flags=flags)
    assert gi.tolist() == case["idx"]
    want = np.array([[math.inf if v == "inf" else float(Fraction(v)) for v in r] for r in case["dist"]])
    assert np.array_equal(gd, want)


def _tie_points():
    """3 trajectories of 100 points around (100, 100, 10) at offsets whose
    scaled squared distance is exact in binary64: 0, 1 or 25 under unit
    spatial scales, so most keys tie on the distance and the index decides."""
    offs = [(0, 0), (1, 0), (0, 1), (3, 4), (4, 3), (-3, 4), (-4, -3), (5, 0), (0, -5), (-1, 0)]
    n_traj, per = 3, 100
    x, y = [], []
    for j in range(n_traj * per):
        dx, dy = offs[(7 * j + j // per) % len(offs)]
        x.append(100.0 + dx)
        y.append(100.0 + dy)
    t = np.tile(np.arange(per, dtype=np.float32) * 4.0, n_traj)
    return synth.PointSet(np.array(x, np.float32), np.array(y, np.float32),
                          np.full(n_traj * per, 10.0, np.float32), t,
                          offsets=np.arange(0, n_traj * per + 1, per, dtype=np.int64))


@pytest.mark.parametrize("flags", ALL_PATHS)
@pytest.mark.parametrize("scale", [(1.0, 1.0, 1.0, 0.0), (0.0, 0.0, 0.0, 0.0), (-0.0, -0.0, -0.0, -0.0)],
                         ids=["unit", "zero", "negzero"])
def test_exact_ties_and_signed_zero_distances(flags, scale):
    """Keys that tie on the distance are ordered by index, through the one-by-one
    insertion (few newcomers) and the sorting network (many), k up to 64; with
    all scales -0.0 every distance is a signed zero, which the result reports
    as +0.0 (equal to the oracle's -0.0)."""
    say("ties", flags, scale)
    ps = _tie_points()
    ix = build(ps, seg_len=8)
    qt = np.array([1000.0, 200.0, 41.0, 4.5, 0.0], np.float32)
    qs = synth.PointSet(np.full(5, 100.0, np.float32), np.full(5, 100.0, np.float32),
                        np.full(5, 10.0, np.float32), qt, offsets=np.array([0, 5], dtype=np.int64))
    for k in (5, 32, 64):
        gi, gd = gpu_query(ix, qs, scale, 0.0, k, flags=flags)
        oi, od = oracle.knn(ps.soa(), qs.soa(), scale, 0.0, k)
        assert_same(gi, gd, oi, od, f"ties k={k}")
        assert not np.signbit(gd[np.isfinite(gd)]).any()


def test_linear_search_query_tiles_and_tail():
    """Enough queries that the binary64 linear search answers several per
    wave (from 32 x CUs x queries-per-wave on), and a count that leaves a
    partial last tile: every row against the oracle."""
    ps, qs0, _, cfg = config_data("c1")
    say("linear search tiles")
    n = 40003
    reps = -(-n // qs0.x.shape[0])
    cols = []
    for a, step in ((qs0.x, 0.37), (qs0.y, -0.21), (qs0.z, 0.0), (qs0.t, 11.0)):
        cols.append(np.concatenate([a + np.float32(step * r) for r in range(reps)])[:n].astype(np.float32))
    qs = synth.PointSet(*cols, offsets=np.array([0, n], dtype=np.int64))
    ix = build(ps, cfg["seg_len"])
    gi, gd = gpu_query(ix, qs, SCALE, 0.0, cfg["k"], flags=capi.TNN_BRUTE)
    oi, od = oracle.knn(ps.soa(), qs.soa(), SCALE, 0.0, cfg["k"])
    assert_same(gi, gd, oi, od, "linear search tiles")


@pytest.mark.parametrize("flags", ALL_PATHS)
def test_c1_all_queries(flags):
    """10k points (200 x 50), K=16, every point a query, k=8."""
    ps, qs, _, cfg = config_data("c1")
    say("c1", flags)
    ix = build(ps, cfg["seg_len"])
    gi, gd = gpu_query(ix, qs, SCALE, 0.0, cfg["k"], flags=flags)
    oi, od = oracle.knn(ps.soa(), qs.soa(), SCALE, 0.0, cfg["k"])
    assert_same(gi, gd, oi, od, "c1")


def _climbing(seed, n_traj=40, n_pts=77):
    rng = np.random.default_rng(seed)
    ps = synth.trajectories(n_traj, n_pts, 120.0, 900.0, seed)
    ps.z = (ps.z + np.cumsum(rng.normal(0, 0.3, ps.n))).astype(np.float32)
    ps.y = (ps.y + rng.normal(0, 0.4, ps.n)).astype(np.float32)
    return ps


@pytest.mark.parametrize("seg_len", [1, 5, 16, 64])
def test_segments_match_oracle(seg_len):
    ps = _climbing(3)
    say("segments", seg_len)
    ix = build(ps, seg_len)
    ex = T.tnn_debug_export_index(ix)
    torch.cuda.synchronize()
    seg = oracle.segments(ps.soa(), ps.offsets, seg_len)
    S = seg["start"].shape[0]
    assert ix.n_segments == S
    f = ex["seg_f32"].cpu().numpy().astype(np.float64)
    i = ex["seg_i32"].cpu().numpy()
    pid = ex["point_id"].cpu().numpy()
    order = i[:, 0]
    assert sorted(order.tolist()) == list(range(S))
    # integer fields bit-exact
    assert np.array_equal(pid[i[:, 1]], seg["start"][order])
    assert np.array_equal(i[:, 2], seg["count"][order])
    assert np.array_equal(np.sort(pid), np.arange(ps.n))
    for s in range(0, S, max(1, S // 50)):
        c = i[s, 2]
        assert np.array_equal(pid[i[s, 1]:i[s, 1] + c], np.arange(seg["start"][order[s]], seg["start"][order[s]] + c))
    # endpoints and times are copies of float32 inputs: exact
    assert np.array_equal(f[:, 0:3], seg["a"][order])
    assert np.array_equal(f[:, 3:6], seg["b"][order])
    assert np.array_equal(f[:, 6], seg["tmin"][order])
    assert np.array_equal(f[:, 7], seg["tmax"][order])
    # errors: rounded up, never below the oracle's, within a float32 ulp + slack
    e_o = seg["e"][order]
    e_g = f[:, 8:11]
    assert np.all(e_g >= e_o)
    mag = np.abs(seg["a"][order]) + np.abs(seg["b"][order]) + 1.0
    assert np.all(e_g - e_o <= np.spacing(e_g.astype(np.float32)).astype(np.float64) + 1e-9 * mag)


@pytest.mark.parametrize("scale", [SCALE, (1.0, 3.0, 100.0, 0.5), (0.2, 1.0, 1.0, 0.0)])
@pytest.mark.parametrize("t_window", [0.0, 25.0])
def test_lower_bounds_hold_and_are_tight(scale, t_window):
    ps = _climbing(5)
    ix = build(ps, 11)
    say("lower bounds", scale, t_window)
    rng = np.random.default_rng(8)
    qi = rng.choice(ps.n, 64, replace=False)
    qs = ps.take(qi)
    qs.t = (qs.t + rng.uniform(-3, 30, qs.n)).astype(np.float32)
    qx, qy, qz, qt = dev_points(qs)
    seg_lb, blk_lb = T.tnn_debug_lower_bounds(ix, qx, qy, qz, qt, scale, t_window)
    ex = T.tnn_debug_export_index(ix)
    torch.cuda.synchronize()
    seg_lb = seg_lb.cpu().numpy()
    blk_lb = blk_lb.cpu().numpy().astype(np.float64)
    i = ex["seg_i32"].cpu().numpy()
    pid = ex["point_id"].cpu().numpy()
    S = ix.n_segments
    # exact distance of every (query, point) pair, oracle arithmetic
    QQ, PP = np.meshgrid(np.arange(qs.n), np.arange(ps.n), indexing="ij")
    d = oracle.pair_dist(ps.soa(), qs.soa(), QQ.ravel(), PP.ravel(), scale).reshape(qs.n, ps.n)
    valid = ps.t[None, :].astype(np.float64) < (qs.t.astype(np.float64)[:, None] - t_window)
    dm = np.where(valid, d, np.inf)
    seg_o = oracle.segments(ps.soa(), ps.offsets, 11)
    lb_o = oracle.lower_bound(seg_o, qs.soa(), scale, t_window)[:, i[:, 0]]
    for s in range(S):
        members = pid[i[s, 1]:i[s, 1] + i[s, 2]]
        dmin = dm[:, members].min(1)
        assert np.all(seg_lb[:, s] <= dmin), s
        b = s // 64
        assert np.all(blk_lb[:, b] <= dmin), s
    # masks agree exactly with the oracle's; finite bounds within rounding slack
    assert np.array_equal(np.isinf(seg_lb), np.isinf(lb_o))
    fin = np.isfinite(lb_o)
    assert np.all(seg_lb[fin] <= lb_o[fin] * (1 + 1e-9) + 1e-12)
    # float32 bound: within its proven slack of the binary64 definition
    assert np.all(np.sqrt(seg_lb[fin]) >= np.sqrt(lb_o[fin]) * (1 - 1e-5) - 1e-3)


@pytest.mark.parametrize("k", [1, 7, 32, 64])
@pytest.mark.parametrize("seg_len", [1, 3, 32, 64])
def test_shapes_and_ragged(k, seg_len):
    """Several blocks, ragged trajectories, k up to 64, K from 1 to 64."""
    rng = np.random.default_rng(k * 100 + seg_len)
    counts = rng.integers(1, 150, 60)
    ps = synth.trajectories(60, counts, 150.0, 1200.0, seed=k + seg_len)
    qs, _ = synth.sample_queries(ps, 300, seed=1)
    say("shapes", k, seg_len, ps.n)
    ix = build(ps, seg_len)
    oi, od = oracle.knn(ps.soa(), qs.soa(), SCALE, 0.0, k)
    for flags in ALL_PATHS:
        gi, gd = gpu_query(ix, qs, SCALE, 0.0, k, flags=flags)
        assert_same(gi, gd, oi, od, f"k={k} K={seg_len} flags={flags}")


@pytest.mark.parametrize("scale,t_window", [((1, 1, 10, 0.05), 60.0), ((1, 1, 10, 0.0), 0.0),
                                            ((0, 0, 0, 1), 0.0), ((1, 1, 1, 1), 0.0),
                                            ((1, 2, 3, 4e-4), 1000.0)])
def test_scales_windows_and_off_data_queries(scale, t_window):
    ps = synth.trajectories(80, 60, 200.0, 1800.0, seed=21)
    rng = np.random.default_rng(22)
    qs = synth.PointSet(rng.uniform(-20, 220, 400).astype(np.float32),
                        rng.uniform(-20, 220, 400).astype(np.float32),
                        rng.uniform(7, 13, 400).astype(np.float32),
                        rng.uniform(-100, 2300, 400).astype(np.float32), np.array([0, 400]))
    say("scales", scale, t_window)
    ix = build(ps, 16)
    oi, od = oracle.knn(ps.soa(), qs.soa(), scale, t_window, 10)
    for flags in ALL_PATHS:
        gi, gd = gpu_query(ix, qs, scale, t_window, 10, flags=flags)
        assert_same(gi, gd, oi, od, f"scale={scale} tw={t_window} flags={flags}")


@pytest.mark.parametrize("flags", ALL_PATHS)
def test_empty_and_tiny_inputs(flags):
    ps = synth.trajectories(3, 4, 10.0, 100.0, seed=1)
    ix = build(ps, 16)
    empty = synth.PointSet(*(np.zeros(0, np.float32) for _ in range(4)), np.array([0, 0]))
    gi, gd = gpu_query(ix, empty, SCALE, 0.0, 5, flags=flags)
    assert gi.shape == (0, 5)
    qs = ps.take(np.arange(ps.n))
    gi, gd = gpu_query(ix, qs, SCALE, 0.0, 64, flags=flags)  # k far above the data
    oi, od = oracle.knn(ps.soa(), qs.soa(), SCALE, 0.0, 64)
    assert_same(gi, gd, oi, od, "k>N")


@pytest.mark.parametrize("seeded", [False, True], ids=["unseeded", "seeded"])
@pytest.mark.parametrize("kind", ["zero", "inf", "nan", "tiny", "huge", "exact", "under", "noisy"])
def test_learned_radius_never_changes_results(kind, seeded):
    """Any prediction gives the oracle's result, with or without the plain
    seed (TNN_LEARNED_SEED)."""
    ps, qs, _, cfg = config_data("c1")
    ix = build(ps, cfg["seg_len"])
    k = cfg["k"]
    oi, od = oracle.knn(ps.soa(), qs.soa(), SCALE, 0.0, k)
    kth = od[:, k - 1]
    rng = np.random.default_rng(4)
    r2 = {"zero": np.zeros(qs.n), "inf": np.full(qs.n, np.inf), "nan": np.full(qs.n, np.nan),
          "tiny": np.full(qs.n, 1e-30), "huge": np.full(qs.n, 1e30),
          "exact": kth, "under": kth * 0.999,
          "noisy": kth * np.exp(rng.normal(0, 1.0, qs.n))}[kind]
    say("learned radius", kind)
    r2t = torch.from_numpy(np.asarray(r2, dtype=np.float32)).cuda()
    fl = capi.TNN_LEARNED | (capi.TNN_LEARNED_SEED if seeded else 0)
    gi, gd = gpu_query(ix, qs, SCALE, 0.0, k, flags=fl, radius2=r2t)
    assert_same(gi, gd, oi, od, f"learned {kind} seeded {seeded}")


def test_c2_full_size_sampled_parity():
    """1M points (5000 x 200), K=32, 100k sampled queries, k=32: every query
    on the GPU (plain TNN and linear search agree everywhere); a seeded sample
    of queries checked against the oracle."""
    ps, qs, _, cfg = config_data("c2")
    k = cfg["k"]
    say("c2 build")
    ix = build(ps, cfg["seg_len"])
    stats = T.new_stats()
    say("c2 plain")
    gi, gd = gpu_query(ix, qs, SCALE, 0.0, k, stats=stats)
    say("c2 stats", T.stats_dict(stats))
    say("c2 brute")
    bi, bd = gpu_query(ix, qs, SCALE, 0.0, k, flags=capi.TNN_BRUTE)
    assert_same(gi, gd, bi.astype(np.int64), bd, "c2 plain vs brute")
    say("c2 mixed")
    mi, md = gpu_query(ix, qs, SCALE, 0.0, k, flags=MIXED)
    assert_same(gi, gd, mi.astype(np.int64), md, "c2 plain vs mixed brute")
    rng = np.random.default_rng(2112)
    sample = np.sort(rng.choice(qs.n, 256, replace=False))
    sample = np.concatenate([sample, np.argsort(qs.t)[:8]])  # the earliest queries
    oi, od = oracle.knn(ps.soa(), qs.take(sample).soa(), SCALE, 0.0, k)
    assert_same(gi[sample], gd[sample], oi, od, "c2 sample")
    # properties on every query: ascending keys, valid, caller indices
    assert np.all((np.diff(gd, axis=1) >= 0) | np.isinf(gd[:, 1:]))
    ok = gi >= 0
    assert np.all(ps.t[np.where(ok, gi, 0)][ok] < qs.t[:, None].repeat(k, 1)[ok])


@pytest.mark.parametrize("flags", [0, capi.TNN_LEARNED, MIXED], ids=["plain", "learned", "bf16"])
def test_repeat_runs_are_bitwise_identical(flags):
    """Work-queue atomics (the search's tickets, the BF16 search's items)
    change only which wave does what: two runs give the same bytes."""
    ps, qs, _, cfg = config_data("c1")
    ix = build(ps, cfg["seg_len"])
    kw = {}
    if flags & capi.TNN_LEARNED:
        model = T.tnn_radius_model_init(ix, seed=4)
        kw["radius2"] = T.tnn_radius_infer(model, *dev_points(qs), alpha=1.0)
    a = gpu_query(ix, qs, SCALE, 0.0, cfg["k"], flags=flags, **kw)
    b = gpu_query(ix, qs, SCALE, 0.0, cfg["k"], flags=flags, **kw)
    assert a[0].tobytes() == b[0].tobytes() and a[1].tobytes() == b[1].tobytes()


def test_mixed_precision_error_is_within_the_proven_margin():
    """BF16 tiles: the largest |approximate - binary64| distance over every
    rescored pair stays below gamma (|u|^2 + |v|^2) with gamma = 2^-16, and
    the indices are bit-exact."""
    ps, qs, _, cfg = config_data("c1")
    k = cfg["k"]
    ix = build(ps, cfg["seg_len"])
    stats = T.new_stats()
    gi, gd = gpu_query(ix, qs, SCALE, 0.0, k, flags=MIXED, stats=stats)
    oi, od = oracle.knn(ps.soa(), qs.soa(), SCALE, 0.0, k)
    assert_same(gi, gd, oi, od, "mixed c1")
    st = T.stats_dict(stats)
    say("mixed stats", st)
    pts = np.stack([a.astype(np.float64) for a in ps.soa()], 1)
    lo, hi = pts.min(0), pts.max(0)
    c = 0.5 * (lo + hi)
    s = np.asarray(SCALE)
    n_max = (s * np.maximum((lo - c) ** 2, (hi - c) ** 2)).sum()
    assert st["rescored"] >= qs.n * 1  # every query rescored at least its neighbours
    assert 0.0 < st["max_err"] <= 2.0 ** -16 * 2 * n_max


def _workload(kind):
    if kind == "random":
        ps = synth.random_points(20_000, 300.0, 3600.0, 32, seed=41)
    elif kind == "routes":
        ps = synth.routes(100, 200, 300.0, 3600.0, 6, seed=42)
    else:
        ps = synth.trajectories(100, 200, 300.0, 3600.0, seed=43)
    qs, _ = synth.sample_queries(ps, 1500, seed=44)
    return ps, qs


@pytest.mark.parametrize("kind", ["random", "routes", "trajectories"])
@pytest.mark.parametrize("t_window", [0.0, 1800.0])
@pytest.mark.parametrize("flags", ALL_PATHS + [capi.TNN_LEARNED])
def test_second_workloads_and_window(kind, t_window, flags):
    """Random points (Sec. 4.2: no structure to prune with), traffic along a few
    airways, and the 30-minute context window, every query against the oracle."""
    ps, qs = _workload(kind)
    say("workload", kind, t_window, flags)
    ix = build(ps, 32)
    kw = {}
    if flags == capi.TNN_LEARNED:
        rng = np.random.default_rng(7)
        kw["radius2"] = torch.from_numpy(np.exp(rng.normal(6, 2, qs.n)).astype(np.float32)).cuda()
    gi, gd = gpu_query(ix, qs, SCALE, t_window, 32, flags=flags, **kw)
    oi, od = oracle.knn(ps.soa(), qs.soa(), SCALE, t_window, 32)
    assert_same(gi, gd, oi, od, f"{kind} tw={t_window}")


@pytest.mark.parametrize("k,n_comp", [(1, 1), (8, 2), (32, 3), (64, 8)])
def test_gka_average_matches_oracle(k, n_comp):
    """Gaussian kernel averaging (Sec. 3.2, Eq. gka) over the context the
    search returns, against the oracle on the same context; queries early in
    the data have empty or short contexts."""
    ps = synth.trajectories(60, 90, 40.0, 900.0, seed=21)
    _, qi = synth.sample_queries(ps, 700, seed=22)
    qs = ps.take(np.concatenate([qi, np.argsort(ps.t)[:3]]))  # the earliest have no past
    ix = build(ps, 16)
    scale = (0.5, 0.5, 4.0, 0.02)
    q = dev_points(qs)
    gi, gd = T.tnn_query(ix, *q, scale, 0.0, k)
    rng = np.random.default_rng(k)
    vals = rng.normal(0.0, 10.0, (ps.n, n_comp)).astype(np.float32)
    out = T.tnn_gka_average(gi, gd, torch.from_numpy(vals).cuda())
    torch.cuda.synchronize()
    want = oracle.gka_average(gi.cpu().numpy(), gd.cpu().numpy(), vals)
    got = out.cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(want))
    assert np.isnan(want).any() and not np.isnan(want).all()
    ok = ~np.isnan(want)
    assert np.allclose(got[ok], want[ok], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("flags", [capi.TNN_PLAIN, capi.TNN_LEARNED, capi.TNN_BRUTE, MIXED],
                         ids=["plain", "learned", "brute", "bf16"])
@pytest.mark.parametrize("k,n_comp", [(1, 1), (8, 2), (32, 3), (64, 8)])
def test_gka_asked_of_the_search(flags, k, n_comp):
    """The averaging requested with the search (the averaging kernel run on
    the call's stream right after the search) equals tnn_gka_average on the
    returned context bit for bit, and the oracle's average within 1e-12; the
    neighbours are unchanged."""
    ps = synth.trajectories(60, 90, 40.0, 900.0, seed=23)
    _, qi = synth.sample_queries(ps, 600, seed=24)
    qs = ps.take(np.concatenate([qi, np.argsort(ps.t)[:3]]))
    ix = build(ps, 16)
    scale = (0.5, 0.5, 4.0, 0.02)
    q = dev_points(qs)
    kw = {}
    if flags & capi.TNN_LEARNED:
        model = T.tnn_radius_model_init(ix, seed=2)
        kw["radius2"] = T.tnn_radius_infer(model, *q, alpha=1.0)
    vals = torch.from_numpy(np.random.default_rng(k).normal(0.0, 10.0, (ps.n, n_comp))
                            .astype(np.float32)).cuda()
    gi, gd = T.tnn_query(ix, *q, scale, 0.0, k, flags=flags, **kw)
    fi, fd = T.tnn_query(ix, *q, scale, 0.0, k, flags=flags, gka_values=vals,
                         gka_out=(g := torch.empty((qs.n, n_comp), dtype=torch.float64,
                                                   device="cuda")), **kw)
    sep = T.tnn_gka_average(gi, gd, vals)
    torch.cuda.synchronize()
    assert torch.equal(gi, fi) and torch.equal(gd, fd)
    got, ref = g.cpu().numpy(), sep.cpu().numpy()
    assert got.tobytes() == ref.tobytes()
    want = oracle.gka_average(gi.cpu().numpy(), gd.cpu().numpy(), vals.cpu().numpy())
    assert np.array_equal(np.isnan(got), np.isnan(want)) and np.isnan(want).any()
    ok = ~np.isnan(want)
    assert np.allclose(got[ok], want[ok], rtol=1e-12, atol=1e-12)


def test_gka_asked_per_query_scales_and_batched():
    """The averaging asked under per-query scales (a row without a metric
    gets a NaN average) and in a batched launch (the search's epilogue, each
    item its own values)."""
    ps = synth.trajectories(40, 80, 40.0, 900.0, seed=25)
    qs, _ = synth.sample_queries(ps, 300, seed=26)
    ix = build(ps, 16)
    q = dev_points(qs)
    vals = torch.from_numpy(np.random.default_rng(5).normal(0, 3, (ps.n, 2)).astype(np.float32)).cuda()
    rows = synth.scale_field(qs.x, qs.y, qs.z, 40.0, seed=27)
    rows[7, 1] = -1.0
    qsc = torch.from_numpy(np.ascontiguousarray(rows)).cuda()
    gi, gd = T.tnn_query(ix, *q, SCALE, 0.0, 8, query_scale=qsc)
    g = torch.empty((qs.n, 2), dtype=torch.float64, device="cuda")
    T.tnn_query(ix, *q, SCALE, 0.0, 8, query_scale=qsc, gka_values=vals, gka_out=g)
    sep = T.tnn_gka_average(gi, gd, vals)
    torch.cuda.synchronize()
    assert g.cpu().numpy().tobytes() == sep.cpu().numpy().tobytes()
    assert np.isnan(g[7].cpu().numpy()).all()
    ps2 = synth.trajectories(30, 70, 30.0, 900.0, seed=28)
    qs2, _ = synth.sample_queries(ps2, 200, seed=29)
    ix2 = build(ps2, 8)
    vals2 = torch.from_numpy(np.random.default_rng(6).normal(0, 3, ps2.n).astype(np.float32)).cuda()
    entries = [dict(index=ix, q=q, scale=SCALE, k=8, gka_values=vals),
               dict(index=ix2, q=dev_points(qs2), scale=SCALE, k=32, gka_values=vals2)]
    b = T.tnn_batch_prepare(entries)
    outs = T.tnn_query_batched(b)
    torch.cuda.synchronize()
    for e, (bi, bd) in zip(entries, outs):
        sep = T.tnn_gka_average(bi, bd, e["gka_values"].view(-1, e["gka_out"].shape[1]))
        torch.cuda.synchronize()
        assert e["gka_out"].cpu().numpy().tobytes() == sep.cpu().numpy().tobytes()


PERQ_PATHS = [capi.TNN_PLAIN, capi.TNN_LEARNED, capi.TNN_BRUTE]


def _perq_query(ix, qs, rows, tw, k, flags, model=None):
    q = dev_points(qs)
    qscale = torch.from_numpy(np.ascontiguousarray(rows)).cuda()
    r2 = None
    if flags & capi.TNN_LEARNED:
        r2 = T.tnn_radius_infer(model, *q, alpha=1.0)
    i, d = T.tnn_query(ix, *q, SCALE, tw, k, flags=flags, radius2=r2, query_scale=qscale)
    torch.cuda.synchronize()
    return i.cpu().numpy(), d.cpu().numpy()


@pytest.mark.parametrize("flags", PERQ_PATHS)
@pytest.mark.parametrize("tw", [0.0, 1800.0])
def test_per_query_scales_match_oracle(flags, tw):
    """Scales varying over space (Sec. 3.2), one row per query: every path
    against the oracle under each query's own metric; rows with zero scales,
    wide factors, and invalid rows (negative, NaN, inf) -> (-1, NaN)."""
    ps = synth.trajectories(300, 80, 800.0, 4 * 3600.0, seed=41)
    ix = build(ps, 16)
    rng = np.random.default_rng(7)
    qs = ps.take(rng.choice(ps.n, 700, replace=False))
    rows = synth.scale_field(qs.x, qs.y, qs.z, 800.0, seed=3)
    rows[0] = 0.0                                   # every point at distance 0
    rows[1, 3] = 0.0                                # time ignored
    rows[2, :3] = 0.0                               # time only
    rows[3] *= np.array([1e-3, 1e-3, 1e3, 1e2])     # far from the shared metric
    rows[4] *= 1e6
    rows[10, 1] = -0.5                              # invalid rows
    rows[11, 2] = np.nan
    rows[12, 0] = np.inf
    model = T.tnn_radius_model_init(ix, seed=5) if flags & capi.TNN_LEARNED else None
    for k in (1, 8, 64):
        say("per-query scales", flags, tw, k)
        gi, gd = _perq_query(ix, qs, rows, tw, k, flags, model)
        oi, od = oracle.knn(ps.soa(), qs.soa(), rows, tw, k)
        bad = np.array([10, 11, 12])
        assert (gi[bad] == -1).all() and np.isnan(gd[bad]).all()
        keep = np.setdiff1d(np.arange(qs.n), bad)
        assert_same(gi[keep], gd[keep], oi[keep], od[keep], f"per-query scales k={k}")


def test_per_query_scales_equal_rows_match_shared_metric():
    """Equal rows reproduce the shared-scale search bit for bit."""
    ps, qs, _, cfg = config_data("c1")
    ix = build(ps, cfg["seg_len"])
    k = cfg["k"]
    rows = np.tile(np.array(SCALE, dtype=np.float64), (qs.n, 1))
    gi, gd = _perq_query(ix, qs, rows, 0.0, k, capi.TNN_PLAIN)
    si, sd = gpu_query(ix, qs, SCALE, 0.0, k)
    assert np.array_equal(gi, si) and np.array_equal(gd, sd)


def test_per_query_scales_refused_where_unsupported():
    ps = synth.trajectories(20, 30, 300.0, 3600.0, seed=2)
    ix = build(ps, 16)
    q = dev_points(ps)
    qscale = torch.ones((ps.n, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(capi.TnnError) as e:
        T.tnn_query(ix, *q, SCALE, 0.0, 4, flags=MIXED, query_scale=qscale)
    assert e.value.code == capi.TNN_E_UNSUPPORTED


@pytest.mark.parametrize("path", ["plain", "learned", "mixed", "brute", "per_query"])
def test_single_query_call_graph_replay_equals_eager(path):
    """tnn_query allocates nothing and launches only kernels (no memsets), so
    a call captured in a HIP graph replays to the eager result, with eager
    work between replays."""
    ps = synth.trajectories(120, 60, 500.0, 7200.0, seed=13)
    ix = build(ps, 16)
    qs, _ = synth.sample_queries(ps, 900, seed=14)
    q = dev_points(qs)
    k = 16
    flags = {"plain": capi.TNN_PLAIN, "learned": capi.TNN_LEARNED, "mixed": MIXED,
             "brute": capi.TNN_BRUTE, "per_query": capi.TNN_PLAIN}[path]
    r2 = None
    if path == "learned":
        model = T.tnn_radius_model_init(ix, seed=2)
        r2 = T.tnn_radius_infer(model, *q, alpha=1.0)
    qscale = None
    if path == "per_query":
        qscale = torch.from_numpy(synth.scale_field(qs.x, qs.y, qs.z, 500.0, seed=4)).cuda()
    params = T.make_params(SCALE, 0.0, k, flags, radius2=r2, query_scale=qscale)
    scratch = torch.empty(max(T.tnn_query_workspace(ix, qs.n, params), 256), dtype=torch.uint8,
                          device="cuda")
    out = (torch.empty((qs.n, k), dtype=torch.int32, device="cuda"),
           torch.empty((qs.n, k), dtype=torch.float64, device="cuda"))

    def call():
        T.tnn_query(ix, *q, SCALE, 0.0, k, flags=flags, radius2=r2, out=out, scratch=scratch,
                    query_scale=qscale)

    call()
    torch.cuda.synchronize()
    ref = (out[0].clone(), out[1].clone())
    rows = qscale.cpu().numpy() if qscale is not None else SCALE
    oi, od = oracle.knn(ps.soa(), qs.soa(), rows, 0.0, k)
    assert_same(ref[0].cpu().numpy(), ref[1].cpu().numpy(), oi, od, f"eager {path}")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        call()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    for rep in range(3):
        out[0].fill_(-7)
        out[1].fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]), (path, rep)


def test_huge_scales_and_far_queries():
    """Scales whose scaled index box leaves float32 range are refused by the
    float paths (TNN, BF16) and answered by the binary64 linear search; large
    scales inside the range and far-out queries stay exact on TNN (its bounds
    saturate instead of overflowing to the "masked" +inf); the BF16 tiles
    report queries beyond their range as (-1, NaN)."""
    ps = synth.trajectories(60, 40, 300.0, 3600.0, seed=17)
    ix = build(ps, 16)
    rng = np.random.default_rng(18)
    qs = ps.take(rng.choice(ps.n, 200, replace=False))
    huge = (1e34, 1e34, 1e35, 1e30)
    oi, od = oracle.knn(ps.soa(), qs.soa(), huge, 0.0, 8)
    gi, gd = gpu_query(ix, qs, huge, 0.0, 8, flags=capi.TNN_BRUTE)
    assert_same(gi, gd, oi, od, "huge scales, binary64 linear search")
    for flags in (capi.TNN_PLAIN, capi.TNN_LEARNED, MIXED):
        with pytest.raises(capi.TnnError) as e:
            q = dev_points(qs)
            r2 = torch.ones(qs.n, dtype=torch.float32, device="cuda")
            T.tnn_query(ix, *q, huge, 0.0, 8, flags=flags, radius2=r2)
        assert e.value.code == capi.TNN_E_UNSUPPORTED, flags
    # just inside the range: float32 bounds still exact
    edge = tuple(v * 1e24 for v in SCALE)
    oi, od = oracle.knn(ps.soa(), qs.soa(), edge, 0.0, 8)
    for flags in (capi.TNN_PLAIN, capi.TNN_BRUTE, MIXED):
        gi, gd = gpu_query(ix, qs, edge, 0.0, 8, flags=flags)
        assert_same(gi, gd, oi, od, f"large scales flags={flags}")
    far = qs.take(np.arange(qs.n))
    far.x = far.x.copy()
    far.x[::7] = np.float32(3e16)  # scaled squared norm ~1e33
    oi, od = oracle.knn(ps.soa(), far.soa(), SCALE, 0.0, 8)
    gi, gd = gpu_query(ix, far, SCALE, 0.0, 8, flags=MIXED)
    bad = np.arange(0, far.n, 7)
    assert (gi[bad] == -1).all() and np.isnan(gd[bad]).all()
    keep = np.setdiff1d(np.arange(far.n), bad)
    assert_same(gi[keep], gd[keep], oi[keep], od[keep], "far queries, BF16")
    for flags in (capi.TNN_PLAIN, capi.TNN_BRUTE):
        gi, gd = gpu_query(ix, far, SCALE, 0.0, 8, flags=flags)
        assert_same(gi, gd, oi, od, f"far queries flags={flags}")
