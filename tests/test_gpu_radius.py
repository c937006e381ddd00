"""GPU parity of the learned k-th radius kernels (features, inference,
forward/backward, Adam) against the oracle, and what training gains."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_same, build, config_data, dev_points, gpu_query, say
from paper_2112_10408_amd import capi, radius, synth
from paper_2112_10408_amd import tnn as T

pytestmark = pytest.mark.gpu
SCALE = synth.SCALE


@pytest.fixture(scope="module")
def setup():
    ps = synth.trajectories(400, 120, 800.0, 4 * 3600.0, seed=31)
    ix = build(ps, 16)
    model = T.tnn_radius_model_init(ix, seed=5)
    torch.cuda.synchronize()
    seg = oracle.segments(ps.soa(), ps.offsets, 16)
    lo = np.array([a.min() for a in ps.soa()], dtype=np.float32)
    hi = np.array([a.max() for a in ps.soa()], dtype=np.float32)
    grid = oracle.radius_density_grid(seg["a"], seg["b"], seg["tmin"], seg["tmax"], lo, hi)
    f0 = ps.offsets[:-1]
    starts = oracle.radius_start_grid(ps.x[f0], ps.y[f0], ps.t[f0], lo, hi)
    return ps, ix, model, lo, hi, (grid, starts)


def test_box_and_density_grid_match_oracle(setup):
    ps, ix, model, lo, hi, (grid, starts) = setup
    glo, ghi = T.radius_box(model)
    assert np.array_equal(glo.cpu().numpy(), lo) and np.array_equal(ghi.cpu().numpy(), hi)
    g = T.radius_grid(model).cpu().numpy()
    assert g.sum() == ix.n_segments
    assert np.array_equal(g, grid)
    # the model stores, per cell, the start count of the feature's neighbourhood
    st = T.radius_starts(model).cpu().numpy()
    sxy, stt = oracle.START_XY, oracle.START_T
    cx, cy, ct = np.meshgrid(np.arange(sxy), np.arange(sxy), np.arange(stt), indexing="ij")
    want = np.zeros_like(starts)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dt in (-1, 0):
                x, y, t = cx + dx, cy + dy, ct + dt
                inside = (x >= 0) & (x < sxy) & (y >= 0) & (y < sxy) & (t >= 0)
                want += np.where(inside, starts[np.clip(x, 0, sxy - 1), np.clip(y, 0, sxy - 1),
                                                np.clip(t, 0, stt - 1)], 0)
    assert starts.sum() == len(ps.offsets) - 1
    assert np.array_equal(st, want)


def test_features_match_oracle(setup):
    ps, ix, model, lo, hi, grids = setup
    rng = np.random.default_rng(3)
    qs = ps.take(rng.choice(ps.n, 2000, replace=False))
    f = T.tnn_radius_features(model, *dev_points(qs)).cpu().numpy().astype(np.float64)
    fo = oracle.radius_features(*qs.soa(), lo, hi, *grids)
    assert np.allclose(f, fo, rtol=1e-6, atol=2e-6)


def test_inference_matches_oracle_forward(setup):
    ps, ix, model, lo, hi, grids = setup
    qs = ps.take(np.arange(0, ps.n, 7))
    q = dev_points(qs)
    logr = torch.empty(qs.n, dtype=torch.float32, device="cuda")
    r2 = T.tnn_radius_infer(model, *q, alpha=1.5, logr=logr)
    theta = T.radius_params(model).cpu().numpy().astype(np.float64)
    out, _ = oracle.mlp_forward(theta, oracle.radius_features(*qs.soa(), lo, hi, *grids))
    lg = logr.cpu().numpy().astype(np.float64)
    assert np.allclose(lg, out, rtol=1e-5, atol=1e-5)
    assert np.allclose(r2.cpu().numpy(), (1.5 * np.exp(lg)) ** 2, rtol=1e-5)


@pytest.mark.parametrize("batch", [1, 63, 64, 1000, 1100])
def test_gradient_matches_oracle_backprop(setup, batch):
    ps, ix, model, lo, hi, grids = setup
    k = 8
    rng = np.random.default_rng(batch)
    qs = ps.take(rng.choice(ps.n, batch + 10, replace=False))
    _, dist = oracle.knn(ps.soa(), qs.soa(), SCALE, 0.0, k)
    q = dev_points(qs)
    dd = torch.from_numpy(dist).cuda()
    first = 10
    say("grad", batch)
    g, loss = T.tnn_radius_grad(model, *q, dd, k, first, batch)
    g = g.cpu().numpy().astype(np.float64)
    theta = T.radius_params(model).cpu().numpy().astype(np.float64)
    sub = qs.take(np.arange(first, first + batch))
    X = oracle.radius_features(*sub.soa(), lo, hi, *grids)
    y = oracle.radius_label(dist[first:first + batch, k - 1])
    lo_, go = oracle.mlp_loss_grad(theta, X, y)
    assert float(loss.item()) == pytest.approx(lo_, rel=1e-4, abs=1e-6)
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go) + 1e-7


def test_adam_step_matches_oracle(setup):
    ps, ix, model0, lo, hi, grids = setup
    model = model0.clone()
    k = 8
    qs = ps.take(np.arange(0, ps.n, 11)[:2048])
    _, dist = oracle.knn(ps.soa(), qs.soa(), SCALE, 0.0, k)
    q = dev_points(qs)
    dd = torch.from_numpy(dist).cuda()
    theta0 = T.radius_params(model).cpu().numpy().astype(np.float64)
    adam = torch.zeros(2 * capi.RADIUS_NPARAMS, dtype=torch.float32, device="cuda")
    m = np.zeros_like(theta0)
    v = np.zeros_like(theta0)
    th = theta0
    for step in (1, 2, 3):
        g_step, _ = T.tnn_radius_grad(model, *q, dd, k, 0, qs.n)
        gs = g_step.cpu().numpy().astype(np.float64)
        T.tnn_radius_train_step(model, adam, *q, dd, k, 0, qs.n, step, 1e-3)
        th, m, v = oracle.adam_step(th, gs, m, v, step, 1e-3)
        got = T.radius_params(model).cpu().numpy().astype(np.float64)
        assert np.allclose(got, th, rtol=1e-5, atol=1e-6), step
        th = got  # follow the device weights so rounding does not accumulate


def test_training_learns_more_than_a_constant():
    """Trained on the method's own k-th radii, the MLP predicts held-out
    radii better than the best constant, and the learned search stays exact
    while comparing fewer points than plain TNN."""
    ps, qs, _, cfg = config_data("c1")
    k = cfg["k"]
    ix = build(ps, cfg["seg_len"])
    rng = np.random.default_rng(17)
    perm = rng.permutation(ps.n)
    tr, te = ps.take(perm[:6000]), ps.take(perm[6000:])
    say("train radius")
    model, loss, pdist, ptr = radius.train(ix, *dev_points(tr), SCALE, 0.0, k, epochs=40, batch=512,
                                           lr=3e-3)
    te_q = dev_points(te)
    logr = torch.empty(te.n, dtype=torch.float32, device="cuda")
    T.tnn_radius_infer(model, *te_q, 1.0, logr=logr)
    _, od = oracle.knn(ps.soa(), te.soa(), SCALE, 0.0, k)
    y = oracle.radius_label(od[:, k - 1])
    ok = np.isfinite(y)
    pred = logr.cpu().numpy()[ok]
    mse_model = float(np.mean((pred - y[ok]) ** 2))
    mse_const = float(np.var(y[ok]))
    say("held-out mse", mse_model, "constant", mse_const)
    # the radius depends mostly on how far along its own trajectory a query
    # lies, which the trajectory-start feature exposes
    assert mse_model < 0.6 * mse_const
    alpha = radius.calibrate(model, *ptr, pdist, k, quantile=0.9)
    r2 = T.tnn_radius_infer(model, *te_q, alpha)
    st_l = T.new_stats()
    gi, gd = gpu_query(ix, te, SCALE, 0.0, k, flags=capi.TNN_LEARNED, radius2=r2, stats=st_l)
    oi, _ = oracle.knn(ps.soa(), te.soa(), SCALE, 0.0, k)
    assert_same(gi, gd, oi, od, "learned c1")
    st_p = T.new_stats()
    gpu_query(ix, te, SCALE, 0.0, k, stats=st_p)
    sl, sp = T.stats_dict(st_l), T.stats_dict(st_p)
    say("learned", sl, "plain", sp)
    assert sl["blocks"] < sp["blocks"]
    assert sl["fallbacks"] < 0.35 * te.n


@pytest.mark.parametrize("n", [1, 2, 3, 17, 4096, 100_000])
def test_shuffle_is_a_seeded_permutation(n):
    """The training order is a permutation of 0 .. n-1, the same for the same
    seed, different for another seed (n > 3)."""
    a = T.tnn_radius_shuffle(n, 7).cpu().numpy()
    b = T.tnn_radius_shuffle(n, 7).cpu().numpy()
    c = T.tnn_radius_shuffle(n, 8).cpu().numpy()
    assert np.array_equal(np.sort(a), np.arange(n))
    assert np.array_equal(a, b)
    if n > 3:
        assert not np.array_equal(a, c)
        assert not np.array_equal(a, np.arange(n))


def test_gradient_in_a_given_order_matches_oracle(setup):
    """A batch taken through an order array: the samples order[first + b]
    (the order here comes from numpy, and is the same input on both sides)."""
    ps, ix, model, lo, hi, grids = setup
    k = 8
    rng = np.random.default_rng(9)
    qs = ps.take(rng.choice(ps.n, 700, replace=False))
    _, dist = oracle.knn(ps.soa(), qs.soa(), SCALE, 0.0, k)
    order = rng.permutation(qs.n).astype(np.int32)
    first, batch = 100, 300
    g, loss = T.tnn_radius_grad(model, *dev_points(qs), torch.from_numpy(dist).cuda(), k, first,
                                batch, order=torch.from_numpy(order).cuda())
    g = g.cpu().numpy().astype(np.float64)
    theta = T.radius_params(model).cpu().numpy().astype(np.float64)
    sel = order[first:first + batch]
    X = oracle.radius_features(*qs.take(sel).soa(), lo, hi, *grids)
    y = oracle.radius_label(dist[sel, k - 1])
    lo_, go = oracle.mlp_loss_grad(theta, X, y)
    assert float(loss.item()) == pytest.approx(lo_, rel=1e-4, abs=1e-6)
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go) + 1e-7


def test_gradient_skips_unlabelled_samples(setup):
    """Samples whose k-th distance is +inf (fewer than k earlier points) or 0
    carry no label and add nothing to the gradient or the loss, wherever they
    sit: first and last rows of each 32-sample tile, in both workgroups of a
    ragged batch of 97."""
    ps, ix, model, lo, hi, grids = setup
    k = 8
    rng = np.random.default_rng(12)
    qs = ps.take(rng.choice(ps.n, 97, replace=False))
    _, dist = oracle.knn(ps.soa(), qs.soa(), SCALE, 0.0, k)
    dist = np.ascontiguousarray(dist)
    dist[[0, 31, 32, 63, 64, 96], k - 1] = np.inf
    dist[[5, 40, 70], k - 1] = 0.0
    g, loss = T.tnn_radius_grad(model, *dev_points(qs), torch.from_numpy(dist).cuda(), k, 0, qs.n)
    g = g.cpu().numpy().astype(np.float64)
    theta = T.radius_params(model).cpu().numpy().astype(np.float64)
    X = oracle.radius_features(*qs.soa(), lo, hi, *grids)
    y = oracle.radius_label(dist[:, k - 1])
    assert np.isnan(y).sum() >= 9
    lo_, go = oracle.mlp_loss_grad(theta, X, y)
    assert float(loss.item()) == pytest.approx(lo_, rel=1e-4, abs=1e-6)
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go) + 1e-7


@pytest.mark.parametrize("quantile", [0.0, 0.5, 0.9, 0.99, 1.0])
def test_calibration_matches_oracle_quantile(setup, quantile):
    """The safety factor computed on the device (inference, log-residuals,
    radix selection of the two order statistics) against the oracle's
    quantile of the same model outputs and k-th distances, including samples
    without a label."""
    ps, ix, model, lo, hi, grids = setup
    k = 8
    rng = np.random.default_rng(11)
    # the earliest points have fewer than k points in their past: no label
    sel = np.unique(np.concatenate([rng.choice(ps.n, 5000, replace=False), np.argsort(ps.t)[:20]]))
    qs = ps.take(sel)
    _, dist = oracle.knn(ps.soa(), qs.soa(), SCALE, 0.0, k)
    assert np.isinf(dist[:, k - 1]).any()
    q = dev_points(qs)
    dd = torch.from_numpy(dist).cuda()
    alpha = float(T.tnn_radius_calibrate(model, *q, dd, k, quantile).item())
    logr = torch.empty(qs.n, dtype=torch.float32, device="cuda")
    T.tnn_radius_infer(model, *q, 1.0, logr=logr)
    want = oracle.radius_calibrate(logr.cpu().numpy(), dist[:, k - 1], quantile)
    assert alpha == pytest.approx(want, rel=2e-7)


def test_calibration_without_labels_is_one(setup):
    ps, ix, model, lo, hi, grids = setup
    qs = ps.take(np.arange(10))
    dd = torch.full((10, 8), float("inf"), dtype=torch.float64, device="cuda")
    assert float(T.tnn_radius_calibrate(model, *dev_points(qs), dd, 8, 0.9).item()) == 1.0


def test_checkpoint_round_trip_gives_identical_radii(setup, tmp_path):
    """A trained model saved to a versioned checkpoint and loaded back into a
    fresh buffer predicts bit-identical radii; a damaged, truncated or
    foreign file is refused with TNN_E_FORMAT."""
    ps, ix, _, lo, hi, grids = setup
    rng = np.random.default_rng(12)
    tr = ps.take(rng.choice(ps.n, 4000, replace=False))
    model, _, _, _ = radius.train(ix, *dev_points(tr), SCALE, 0.0, 8, epochs=3, batch=512)
    path = str(tmp_path / "radius.ckpt")
    radius.save(model, path)
    loaded = radius.load(path)
    assert loaded.data_ptr() != model.data_ptr()
    assert torch.equal(loaded, model)
    te = ps.take(rng.choice(ps.n, 3000, replace=False))
    q = dev_points(te)
    a = T.tnn_radius_infer(model, *q, 1.7)
    b = T.tnn_radius_infer(loaded, *q, 1.7)
    torch.cuda.synchronize()
    assert a.cpu().numpy().tobytes() == b.cpu().numpy().tobytes()
    raw = bytearray(open(path, "rb").read())
    for bad in (raw[:-1], raw[:100], bytes(b"x") + raw[1:]):
        with pytest.raises(capi.TnnError) as e:
            T.tnn_radius_model_load(bytes(bad))
        assert e.value.code == capi.TNN_E_FORMAT
    flipped = bytearray(raw)
    flipped[64 + 1234] ^= 1  # one payload bit
    with pytest.raises(capi.TnnError) as e:
        T.tnn_radius_model_load(bytes(flipped))
    assert e.value.code == capi.TNN_E_FORMAT


def test_learned_radius_gains_time_on_one_million_points():
    """The gain in time: on the 1M-point workload (100k queries, k = 32) the
    learned step (radius inference + learned search) beats plain TNN's search,
    median of 5 timings of 5 calls each, and returns the same bytes."""
    ps, qs, qidx, cfg = config_data("c2")
    k = cfg["k"]
    ix = build(ps, cfg["seg_len"])
    # trained as the benchmark trains it: 100k labelled queries, 8 epochs
    tq, _ = synth.sample_queries(ps, 100_000, cfg["seed"] + 2000, exclude=qidx)
    model, _, pdist, ptr = radius.train(ix, *dev_points(tq), SCALE, 0.0, k, epochs=8, batch=4096,
                                        lr=3e-3)
    alpha = radius.calibrate(model, *ptr, pdist, k, quantile=0.99)
    q = dev_points(qs)
    out = (torch.empty((qs.n, k), dtype=torch.int32, device="cuda"),
           torch.empty((qs.n, k), dtype=torch.float64, device="cuda"))
    scr = torch.empty(T.tnn_query_workspace(ix, qs.n, T.make_params(SCALE, 0.0, k)),
                      dtype=torch.uint8, device="cuda")
    r2 = torch.empty(qs.n, dtype=torch.float32, device="cuda")

    def plain():
        T.tnn_query(ix, *q, SCALE, 0.0, k, out=out, scratch=scr)

    def learned():
        T.tnn_radius_infer(model, *q, alpha, out=r2)
        T.tnn_query(ix, *q, SCALE, 0.0, k, flags=capi.TNN_LEARNED, radius2=r2, out=out,
                    scratch=scr)

    def median_ms(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 5)
        return float(np.median(ts))

    mp = median_ms(plain)
    ref = (out[0].clone(), out[1].clone())
    ml = median_ms(learned)
    say(f"plain {mp:.4f} ms, learned step {ml:.4f} ms, gain {mp / ml:.3f}x")
    assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])
    assert ml < mp


@pytest.mark.parametrize("seeded", [False, True], ids=["unseeded", "seeded"])
def test_radius_predicted_inside_the_call(setup, seeded):
    """With the model passed to tnn_query the library predicts the radius in
    its preparation launch: the same bytes and the same work counters as
    predicting first with tnn_radius_infer, and the oracle's result; argument
    checks of the combination."""
    ps, ix, model, lo, hi, grids = setup
    rng = np.random.default_rng(21)
    qs = ps.take(np.sort(rng.choice(ps.n, 3000, replace=False)))
    q = dev_points(qs)
    k = 16
    fl = capi.TNN_LEARNED | (capi.TNN_LEARNED_SEED if seeded else 0)
    r2 = T.tnn_radius_infer(model, *q, alpha=2.5)
    st_a, st_b = T.new_stats(), T.new_stats()
    ai, ad = T.tnn_query(ix, *q, SCALE, 0.0, k, flags=fl, radius2=r2, stats=st_a)
    bi, bd = T.tnn_query(ix, *q, SCALE, 0.0, k, flags=fl, radius_model=model, radius_alpha=2.5,
                         stats=st_b)
    torch.cuda.synchronize()
    assert torch.equal(ai, bi) and torch.equal(ad, bd)
    assert T.stats_dict(st_a) == T.stats_dict(st_b)
    oi, od = oracle.knn(ps.soa(), qs.soa(), SCALE, 0.0, k)
    assert_same(bi.cpu().numpy(), bd.cpu().numpy(), oi, od, "in-call radius")
    bad = [dict(radius2=r2, radius_model=model, radius_alpha=2.5),   # both
           dict(radius_model=model, radius_alpha=0.0),               # alpha not positive
           dict(radius_model=model, radius_alpha=float("nan"))]
    for kw in bad:
        with pytest.raises(capi.TnnError) as e:
            T.tnn_query(ix, *q, SCALE, 0.0, k, flags=fl, **kw)
        assert e.value.code == capi.TNN_E_ARG
    with pytest.raises(capi.TnnError) as e:
        T.tnn_query(ix, *q, SCALE, 0.0, k, flags=capi.TNN_LEARNED | capi.TNN_BRUTE,
                    radius_model=model, radius_alpha=2.5)
    assert e.value.code == capi.TNN_E_UNSUPPORTED
