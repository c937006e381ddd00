"""Pins for the CPU oracle: hand-worked values, exact-rational brute force,
invariants and planted mistakes.  CPU only."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact_rational import exact_knn
from paper_2112_10408_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _val(s):
    if s is None:
        return None
    if isinstance(s, (int, float)):
        return float(s)
    if s == "inf":
        return math.inf
    return float(Fraction(s))


def _soa(rows):
    a = np.array([[float(Fraction(str(v))) for v in r] for r in rows], dtype=np.float64)
    return tuple(a[:, i].astype(np.float32) for i in range(4))


def _cases(name, key):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)[key]


@pytest.mark.parametrize("case", _cases("knn_cases.json", "cases"), ids=lambda c: c["name"])
def test_knn_golden(case):
    pts = _soa(case["points"])
    qs = _soa(case["queries"])
    idx, dist = oracle.knn(pts, qs, case["scale"], case["t_window"], case["k"])
    assert idx.tolist() == case["idx"]
    want = np.array([[_val(v) for v in row] for row in case["dist"]])
    assert np.array_equal(dist, want)


def _dyadic(rng, n, lo=-64, hi=64, den=8):
    return (rng.integers(lo * den, hi * den, n) / den).astype(np.float32)


@pytest.mark.parametrize("seed", range(12))
def test_knn_equals_exact_rational_on_dyadic(seed):
    rng = np.random.default_rng(seed)
    n, nq, k = 40, 12, int(rng.integers(1, 9))
    pts = tuple(_dyadic(rng, n) for _ in range(3)) + (_dyadic(rng, n, 0, 32, 4),)
    qs = tuple(_dyadic(rng, nq) for _ in range(3)) + (_dyadic(rng, nq, 0, 32, 4),)
    scale = [1.0, 1.0, 2.0, 0.25] if seed % 2 else [0.5, 0.5, 4.0, 0.125]
    tw = [0.0, 0.5, 2.0][seed % 3]
    idx, dist = oracle.knn(pts, qs, scale, tw, k)
    ei, ed = exact_knn(pts, qs, scale, tw, k)
    assert np.array_equal(idx, ei)
    # dyadic inputs with a few bits: every binary64 operation is exact
    assert np.array_equal(dist, np.array([[float(v) for v in row] for row in ed]))


@pytest.mark.parametrize("seed", range(4))
def test_knn_ranks_by_exact_distance_on_float_data(seed):
    """On general float data the oracle's order may differ from the exact
    real order only between distances within a few binary64 ulps."""
    rng = np.random.default_rng(100 + seed)
    n, nq, k = 60, 8, 6
    pts = tuple(rng.uniform(0, 50, n).astype(np.float32) for _ in range(4))
    qs = tuple(rng.uniform(0, 50, nq).astype(np.float32) for _ in range(4))
    scale = [1.0, 1.0, 10.0, 0.05]
    idx, dist = oracle.knn(pts, qs, scale, 0.0, k)
    ei, ed = exact_knn(pts, qs, scale, 0.0, k)
    for q in range(nq):
        for r in range(k):
            if ei[q, r] < 0:
                assert idx[q, r] == -1
                continue
            assert abs(dist[q, r] - float(ed[q][r])) <= 1e-14 * float(ed[q][r])


def test_knn_invariants_translation_and_scale():
    rng = np.random.default_rng(7)
    n, nq, k = 80, 16, 5
    pts = tuple(_dyadic(rng, n) for _ in range(3)) + (_dyadic(rng, n, 0, 32, 4),)
    qs = tuple(_dyadic(rng, nq) for _ in range(3)) + (_dyadic(rng, nq, 0, 32, 4),)
    s = [1.0, 1.0, 2.0, 0.25]
    i0, d0 = oracle.knn(pts, qs, s, 0.0, k)
    # translation of every coordinate (dyadic shift keeps arithmetic exact)
    sh = (np.float32(256.0), np.float32(-128.0), np.float32(64.0), np.float32(512.0))
    i1, d1 = oracle.knn(tuple(p + c for p, c in zip(pts, sh)), tuple(q + c for q, c in zip(qs, sh)), s, 0.0, k)
    assert np.array_equal(i0, i1) and np.array_equal(d0, d1)
    # multiplying every scale by 4 multiplies every distance by 4
    i2, d2 = oracle.knn(pts, qs, [4 * v for v in s], 0.0, k)
    assert np.array_equal(i0, i2) and np.array_equal(d2, 4 * d0)
    # swapping x and y together with their scales changes nothing
    i3, d3 = oracle.knn((pts[1], pts[0], pts[2], pts[3]), (qs[1], qs[0], qs[2], qs[3]), [1.0, 1.0, 2.0, 0.25], 0.0, k)
    assert np.array_equal(i0, i3) and np.array_equal(d0, d3)


def test_knn_properties_on_trajectories():
    ps = synth.trajectories(30, 40, 200.0, 1800.0, seed=11)
    qs, _ = synth.sample_queries(ps, 200, seed=12)
    k = 12
    s = synth.SCALE
    idx, dist = oracle.knn(ps.soa(), qs.soa(), s, 0.0, k)
    P = np.stack([a.astype(np.float64) for a in ps.soa()], 1)
    Q = np.stack([a.astype(np.float64) for a in qs.soa()], 1)
    for q in range(qs.n):
        valid = P[:, 3] < Q[q, 3]
        diff = Q[q][None] - P
        d = (((s[0] * diff[:, 0] ** 2 + s[1] * diff[:, 1] ** 2) + s[2] * diff[:, 2] ** 2) + s[3] * diff[:, 3] ** 2)
        order = np.lexsort((np.arange(ps.n), d))
        order = order[valid[order]][:k]
        m = len(order)
        assert idx[q, :m].tolist() == order.tolist()
        assert np.array_equal(dist[q, :m], d[order])
        assert np.all(idx[q, m:] == -1) and np.all(np.isinf(dist[q, m:]))


def test_planted_mistake_is_caught():
    """A dropped time term (a plausible slip) disagrees with T1's hand values."""
    case = _cases("knn_cases.json", "cases")[0]
    pts = _soa(case["points"])
    qs = _soa(case["queries"])
    idx, dist = oracle.knn(pts, qs, [1, 1, 1, 0], 0, 3)  # time term dropped
    want = np.array([[_val(v) for v in row] for row in case["dist"]])
    assert not np.array_equal(dist, want)


# ---------------------------------------------------------------- segments --
@pytest.mark.parametrize("case", _cases("segment_cases.json", "segments"), ids=lambda c: c["name"])
def test_segments_golden(case):
    pts = _soa(case["points"])
    seg = oracle.segments(pts, np.array(case["offsets"]), case["seg_len"])
    assert seg["start"].tolist() == case["start"]
    assert seg["count"].tolist() == case["count"]
    for key in ("a", "b", "tmin", "tmax", "e"):
        assert np.array_equal(seg[key], np.array(case[key], dtype=np.float64)), key


def _dist_to_segment_dense(P, A, B, s):
    """Minimum over the segment by bounded scalar minimisation of the convex
    distance along it (no projection formula involved)."""
    from scipy.optimize import minimize_scalar
    f = lambda u: float(np.sqrt((((P - (A + u * (B - A))) ** 2) * s).sum()))
    r = minimize_scalar(f, bounds=(0.0, 1.0), method="bounded", options={"xatol": 1e-12})
    return min(r.fun, f(0.0), f(1.0))


def test_segment_radius_covers_members():
    ps = synth.trajectories(6, 70, 500.0, 3600.0, seed=3)
    seg = oracle.segments(ps.soa(), ps.offsets, 16)
    P = np.stack([a.astype(np.float64) for a in ps.soa()], 1)
    s = np.array([1.0, 1.0, 10.0])
    assert seg["count"].sum() == ps.n
    for j in range(seg["start"].shape[0]):
        R = math.sqrt((s * seg["e"][j] ** 2).sum())
        for i in range(seg["start"][j], seg["start"][j] + seg["count"][j]):
            assert _dist_to_segment_dense(P[i, :3], seg["a"][j], seg["b"][j], s) <= R + 1e-9
            assert seg["tmin"][j] <= P[i, 3] <= seg["tmax"][j]


# ------------------------------------------------------------ lower bounds --
def _printed_bound(seg, q, scale):
    """The bound as printed in Algorithm 1 (Euclidean unit vector, squared
    error subtracted, time gap t_B - t): a planted alternative reading."""
    A, B = seg["a"][0], seg["b"][0]
    AB = B - A
    P = np.array(q[:3], dtype=np.float64)
    n2 = (AB * AB).sum()
    u = 0.0 if n2 == 0 else min(max(((P - A) * AB).sum() / n2, 0.0), 1.0)
    Ps = A + u * AB
    s = np.array(scale, dtype=np.float64)
    D = (s[:3] * (Ps - P) ** 2).sum() + s[3] * max(seg["tmax"][0] - q[3], 0.0) ** 2
    E = s[:3].max() * (seg["e"][0] ** 2).sum()
    return max(D - E, 0.0)


@pytest.mark.parametrize("case", _cases("segment_cases.json", "lower_bounds"), ids=lambda c: c["name"])
def test_lower_bound_golden(case):
    pts = _soa(case["points"])
    seg = oracle.segments(pts, np.array(case["offsets"]), case["seg_len"])
    q = tuple(np.array([v], dtype=np.float32) for v in case["query"])
    lb = oracle.lower_bound(seg, q, case["scale"], case["t_window"])[0, 0]
    want = _val(case["lb"])
    if math.isinf(want):
        assert math.isinf(lb)
    else:
        assert lb == pytest.approx(want, rel=1e-14, abs=1e-14)
    _, d = oracle.knn(pts, q, case["scale"], case["t_window"], 1)
    assert d[0, 0] == _val(case["nearest_member_dist"])
    assert lb <= d[0, 0]
    if case["printed_form"] is not None:
        pb = _printed_bound(seg, case["query"], case["scale"])
        assert pb == pytest.approx(_val(case["printed_form"]), rel=1e-14)
        assert pb > d[0, 0]  # the printed reading would prune the true neighbour


def _climbing(seed, n_traj=12, n_pts=45):
    """Trajectories that also move in z and wiggle, so that anisotropic scales
    matter for the projection."""
    rng = np.random.default_rng(seed)
    ps = synth.trajectories(n_traj, n_pts, 80.0, 600.0, seed)
    ps.z = (ps.z + np.cumsum(rng.normal(0, 0.3, ps.n))).astype(np.float32)
    ps.y = (ps.y + rng.normal(0, 0.4, ps.n)).astype(np.float32)
    return ps


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("scale", [(1, 1, 10, 0.05), (1, 3, 100, 0.5), (0.2, 1, 1, 0.0)])
@pytest.mark.parametrize("t_window", [0.0, 25.0, 200.0, 1800.0])
def test_lower_bound_never_exceeds_member_distance(seed, scale, t_window):
    """lb <= every candidate member's distance, and the mask is exact, also
    with a window (candidates t_i < t_q - t_w; gap at least t_w).  The
    trajectories span about 800 s, so t_w = 1800 masks every segment."""
    ps = _climbing(seed)
    seg = oracle.segments(ps.soa(), ps.offsets, 11)
    rng = np.random.default_rng(seed + 50)
    # queries: data points, points on segments, and random points nearby
    qi = rng.choice(ps.n, 60, replace=False)
    qx = np.concatenate([ps.x[qi], rng.uniform(-5, 90, 40).astype(np.float32)])
    qy = np.concatenate([ps.y[qi], rng.uniform(-5, 90, 40).astype(np.float32)])
    qz = np.concatenate([ps.z[qi], rng.uniform(0, 20, 40).astype(np.float32)])
    qt = np.concatenate([ps.t[qi] + 0.5, rng.uniform(0, 700, 40)]).astype(np.float32)
    lb = oracle.lower_bound(seg, (qx, qy, qz, qt), scale, t_window)
    P = np.stack([a.astype(np.float64) for a in ps.soa()], 1)
    s = np.array(scale, dtype=np.float64)
    for j in range(seg["start"].shape[0]):
        mem = slice(seg["start"][j], seg["start"][j] + seg["count"][j])
        diff = np.stack([qx, qy, qz, qt], 1).astype(np.float64)[:, None, :] - P[None, mem]
        d = (s * diff ** 2).sum(-1)
        valid = P[None, mem, 3] < qt.astype(np.float64)[:, None] - t_window
        dmin = np.where(valid, d, np.inf).min(1)
        assert np.all(lb[:, j] <= dmin * (1 + 1e-12))
        # mask is exact: finite bound iff some member is valid
        assert np.array_equal(np.isfinite(lb[:, j]), valid.any(1))


def test_lower_bound_tight_for_exact_segments():
    """Collinear, evenly timed points: R = 0, and a query on the line after
    the last point has the last point's distance as its bound."""
    x = np.arange(8, dtype=np.float32)
    z = np.zeros(8, np.float32)
    t = np.arange(8, dtype=np.float32) * 2
    seg = oracle.segments((x, z, z, t), np.array([0, 8]), 8)
    q = (np.array([10.0], np.float32), np.zeros(1, np.float32), np.zeros(1, np.float32), np.array([20.0], np.float32))
    lb = oracle.lower_bound(seg, q, (1, 1, 1, 1), 0.0)[0, 0]
    assert lb == 9.0 + 36.0


# --------------------------------------------------------- learned radius --
def test_mlp_backprop_matches_finite_differences():
    rng = np.random.default_rng(5)
    theta = rng.normal(0, 0.3, oracle.N_PARAMS)
    X = rng.normal(0, 1, (17, oracle.N_IN))
    y = rng.normal(1, 0.5, 17)
    y[3] = np.nan  # unlabeled sample is ignored
    loss, g = oracle.mlp_loss_grad(theta, X, y)
    which = list(rng.choice(oracle.N_PARAMS, 120, replace=False)) + [oracle.N_PARAMS - 1]
    fd = oracle.finite_difference_grad(theta, X, y, h=1e-6, which=which)
    assert np.allclose(g[which], fd[which], rtol=1e-5, atol=1e-8)
    assert loss == pytest.approx(oracle.mlp_loss(theta, X, y))


def test_mlp_closed_form_constant_network():
    """All weights zero: out = b3 everywhere, loss = mean (b3 - y)^2 and
    only b3 has a gradient, 2 mean(b3 - y)."""
    theta = np.zeros(oracle.N_PARAMS)
    theta[-1] = 1.5
    X = np.ones((4, oracle.N_IN))
    y = np.array([1.0, 2.0, 3.0, 4.0])
    loss, g = oracle.mlp_loss_grad(theta, X, y)
    assert loss == pytest.approx(((1.5 - y) ** 2).mean())
    assert g[-1] == pytest.approx(2 * (1.5 - y).mean())
    assert np.all(g[:-1] == 0)


def _mlp_golden():
    with open(os.path.join(GOLDEN, "mlp_cases.json")) as f:
        g = json.load(f)
    w = g["weights"]
    p = {name: np.zeros(sh) for name, sh in oracle.PARAM_SHAPES}
    for r, c, v in w["W1"]:
        p["W1"][r, c] = v
    for r, c, v in w["W2"]:
        p["W2"][r, c] = v
    for key in ("b1", "b2", "W3"):
        for u, v in w[key]:
            p[key][u] = v
    p["b3"][0] = w["b3"]
    X = np.array([c["x"] for c in g["cases"]], dtype=np.float64)
    want = np.array([c["out"] for c in g["cases"]], dtype=np.float64)
    return p, X, want


def test_mlp_forward_hand_worked_cases():
    """Hand-worked forward passes (tests/golden/mlp_cases.json): dyadic
    weights and inputs, so the binary64 output is exact."""
    p, X, want = _mlp_golden()
    out, _ = oracle.mlp_forward(p, X)
    assert np.array_equal(out, want)
    # the flat parameter order of the device layout gives the same network
    out_flat, _ = oracle.mlp_forward(oracle.pack_params(p), X)
    assert np.array_equal(out_flat, want)


def test_mlp_forward_pins_catch_planted_mistakes(monkeypatch):
    """Plausible slips in the forward pass each miss a hand-worked value:
    W2 read transposed, a feature column swapped, and the ReLUs dropped
    (planted in the oracle module by replacing np.maximum)."""
    p, X, want = _mlp_golden()
    pt = dict(p)
    pt["W2"] = p["W2"].T.copy()
    assert not np.array_equal(oracle.mlp_forward(pt, X)[0], want)
    ps = dict(p)
    ps["W1"] = p["W1"][:, [0, 1, 2, 4, 3, 5]].copy()
    assert not np.array_equal(oracle.mlp_forward(ps, X)[0], want)

    class NoRelu:
        def __getattr__(self, name):
            return getattr(np, name)

        @staticmethod
        def maximum(a, b):
            return a

    import oracle.oracle as om
    monkeypatch.setattr(om, "np", NoRelu())
    assert not np.array_equal(om.mlp_forward(p, X)[0], want)


def test_adam_steps_two_and_three_closed_form():
    """Adam (Kingma & Ba 2015, Alg. 1) beyond the first step.
    Constant gradient g: m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the
    bias-corrected m_hat = g and v_hat = g^2 at every step and each update is
    lr g / (|g| + eps).
    Gradient g, -g, g: m_1 = g/10, m_2 = 0.09 g - 0.1 g = -g/100,
    m_3 = -0.009 g + 0.1 g = 0.091 g; m_hat_2 = (-1/100)/(19/100) g = -g/19,
    m_hat_3 = 0.091/0.271 g = 91/271 g; |g| constant gives v_hat_t = g^2."""
    lr, eps = 0.01, 1e-8
    g = np.array([0.5, -2.0, 1e-3, 3.0])
    th, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for step in (1, 2, 3):
        th, m, v = oracle.adam_step(th, g, m, v, step, lr=lr)
        assert np.allclose(th, -step * lr * g / (np.abs(g) + eps), rtol=1e-12)
    # sign-flipping gradient
    th, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    ups = []
    for step, sgn in ((1, 1.0), (2, -1.0), (3, 1.0)):
        before = th.copy()
        th, m, v = oracle.adam_step(th, sgn * g, m, v, step, lr=lr)
        ups.append(before - th)
    assert np.allclose(m, 0.091 * g, rtol=1e-12)
    assert np.allclose(v, (0.999 ** 2 * 0.001 + 0.999 * 0.001 + 0.001) * g * g, rtol=1e-12)
    assert np.allclose(ups[0], lr * g / (np.abs(g) + eps), rtol=1e-12)
    assert np.allclose(ups[1], lr * (-g / 19.0) / (np.abs(g) + eps), rtol=1e-10)
    assert np.allclose(ups[2], lr * (91.0 / 271.0) * g / (np.abs(g) + eps), rtol=1e-10)


def test_adam_pin_catches_bias_correction_slip():
    """Bias correction by beta instead of beta^step (a plausible slip: the
    step count ignored) misses the step-2 closed form: planted by giving the
    oracle step 1 where it should see step 2."""
    lr, eps = 0.01, 1e-8
    g = np.array([0.5, -2.0, 3.0])
    th, m, v = oracle.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=lr)
    th_bad, _, _ = oracle.adam_step(th, g, m, v, 1, lr=lr)
    assert not np.allclose(th_bad, -2 * lr * g / (np.abs(g) + eps), rtol=1e-6)


def test_lower_bound_window_pins_catch_a_dropped_window():
    """The golden bounds with t_w > 0 reject a bound that ignores the
    window in the time gap or in the mask (planted by calling the oracle
    with t_w = 0)."""
    cases = [c for c in _cases("segment_cases.json", "lower_bounds") if c["t_window"] > 0]
    assert len(cases) >= 4
    for case in cases:
        pts = _soa(case["points"])
        seg = oracle.segments(pts, np.array(case["offsets"]), case["seg_len"])
        q = tuple(np.array([v], dtype=np.float32) for v in case["query"])
        lb0 = oracle.lower_bound(seg, q, case["scale"], 0.0)[0, 0]
        assert lb0 != _val(case["lb"]), case["name"]


def test_adam_first_step_closed_form():
    """First Adam step: bias correction gives m_hat = g, v_hat = g^2, so the
    update is -lr g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th, m, v = oracle.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_radius_cells_and_label():
    lo = np.array([0.0, 0.0, 0.0, 0.0], np.float32)
    hi = np.array([32.0, 64.0, 1.0, 3200.0], np.float32)
    cx, cy, ct = oracle.radius_cells(np.array([0.0, 31.999, 32.0, -5.0], np.float32),
                                     np.array([63.99, 2.0, 1.0, 70.0], np.float32),
                                     np.array([100.0, 3199.0, 3200.0, 0.0], np.float32), lo, hi)
    assert cx.tolist() == [0, 31, 31, 0]
    assert cy.tolist() == [31, 1, 0, 31]
    assert ct.tolist() == [1, 31, 31, 0]
    lab = oracle.radius_label(np.array([4.0, np.inf, 0.0]))
    assert lab[0] == pytest.approx(math.log(2.0)) and np.isnan(lab[1]) and np.isnan(lab[2])


def test_generator_is_seeded_and_sorted():
    a = synth.trajectories(20, 33, 100.0, 600.0, seed=9)
    b = synth.trajectories(20, 33, 100.0, 600.0, seed=9)
    for u, v in zip(a.soa(), b.soa()):
        assert u.tobytes() == v.tobytes()
    for j in range(20):
        tt = a.t[a.offsets[j]:a.offsets[j + 1]]
        assert np.all(np.diff(tt) > 0)
        step = np.hypot(np.diff(a.x[a.offsets[j]:a.offsets[j + 1]]), np.diff(a.y[a.offsets[j]:a.offsets[j + 1]]))
        assert np.all((step > 0.6) & (step < 1.3))  # ~230 m/s over 4 s


def test_radius_density_grid_and_features_hand_case():
    """Three segments with hand-placed midpoints in a box [0, 32]^2 x [0, 320]:
    cell width 1 in x and y, 10 in t."""
    lo = np.array([0.0, 0.0, 8.0, 0.0], np.float32)
    hi = np.array([32.0, 32.0, 12.0, 320.0], np.float32)
    a = np.array([[0.0, 0.0, 9.0], [3.0, 4.0, 9.0], [3.0, 4.0, 9.0]])
    b = np.array([[1.0, 1.0, 9.0], [4.0, 5.0, 9.0], [4.0, 5.0, 9.0]])
    tmin = np.array([0.0, 100.0, 104.0])
    tmax = np.array([10.0, 110.0, 114.0])
    g = oracle.radius_density_grid(a, b, tmin, tmax, lo, hi)
    # midpoints (0.5, 0.5, 5) -> cell (0, 0, 0); (3.5, 4.5, 105) and (3.5, 4.5, 109) -> (3, 4, 10)
    assert g.sum() == 3 and g[0, 0, 0] == 1 and g[3, 4, 10] == 2
    no_starts = np.zeros((oracle.START_XY, oracle.START_XY, oracle.START_T), np.int64)
    f = oracle.radius_features(np.array([16.0, 3.9], np.float32), np.array([0.0, 4.2], np.float32),
                               np.array([10.0, 12.0], np.float32), np.array([160.0, 107.0], np.float32),
                               lo, hi, g, no_starts)
    # centre maps to 0, edges to -1 / +1; density feature 0.25 log1p(count)
    assert np.allclose(f[0, :4], [0.0, -1.0, 0.0, 0.0])
    assert f[0, 4] == 0.0
    assert f[1, 4] == pytest.approx(0.25 * math.log(3.0))
    assert f[1, 2] == pytest.approx(1.0)


def test_radius_start_grid_and_feature_hand_case():
    """Trajectory starts in a box [0, 128]^2 x [0, 5120]: start-grid cells are
    1 wide in x and y and 10 in t.  The feature counts starts in the query's
    cell, its 8 spatial neighbours, and those 9 cells one time step earlier."""
    lo = np.array([0.0, 0.0, 8.0, 0.0], np.float32)
    hi = np.array([128.0, 128.0, 12.0, 5120.0], np.float32)
    fx = np.array([5.5, 6.5, 0.2, 127.9, 8.0, 5.7], np.float32)
    fy = np.array([5.5, 4.2, 0.7, 127.9, 5.0, 5.2], np.float32)
    ft = np.array([105.0, 99.0, 3.0, 5119.0, 105.0, 109.9], np.float32)
    st = oracle.radius_start_grid(fx, fy, ft, lo, hi)
    # (5, 5, 10) twice, (6, 4, 9), (0, 0, 0), (127, 127, 511), (8, 5, 10)
    assert st.sum() == 6 and st[5, 5, 10] == 2 and st[6, 4, 9] == 1 and st[0, 0, 0] == 1
    assert st[127, 127, 511] == 1 and st[8, 5, 10] == 1
    qx = np.array([5.1, 0.1, 5.1, 127.5, 5.1, 128.0], np.float32)
    qy = np.array([5.9, 0.1, 5.9, 127.5, 5.9, 128.0], np.float32)
    qt = np.array([101.0, 1.0, 89.0, 5119.0, 115.0, 5120.0], np.float32)
    cnt = oracle.radius_start_count(qx, qy, qt, lo, hi, st)
    # q0 cell (5,5,10): (5,5,10) x2 and (6,4,9); (8,5,10) is two cells away
    # q1 cell (0,0,0): only (0,0,0) (neighbours below 0 do not exist)
    # q2 cell (5,5,8): the starts at t-cells 9 and 10 lie in its future
    # q3 cell (127,127,511): (127,127,511)
    # q4 cell (5,5,11): (5,5,10) x2; (6,4,9) is two time cells back
    # q5 on the upper edge: clamped into cell (127,127,511)
    assert cnt.tolist() == [3, 1, 0, 1, 2, 1]
    g = np.zeros((oracle.GRID,) * 3, np.int64)
    f = oracle.radius_features(qx, qy, np.full(6, 10.0, np.float32), qt, lo, hi, g, st)
    assert np.allclose(f[:, 5], 0.5 * np.log1p(np.array([3, 1, 0, 1, 2, 1], np.float64)))
    assert np.all(f[:, 4] == 0.0)


def test_gka_average_closed_forms():
    """Gaussian kernel averaging over the k-NN context (Sec. 3.2, Eq. gka):
    closed-form cases of exp(-d) weights."""
    vals = np.array([[1.0, -2.0], [3.0, 5.0], [10.0, 0.5], [7.0, 7.0]])
    # one neighbour: its value
    out = oracle.gka_average(np.array([[2, -1]]), np.array([[4.0, np.inf]]), vals)
    assert np.array_equal(out, [[10.0, 0.5]])
    # d1 - d0 = ln 2: weights 1 and 1/2
    d0 = 3.0
    out = oracle.gka_average(np.array([[0, 1]]), np.array([[d0, d0 + math.log(2.0)]]), vals)
    want = (vals[0] + 0.5 * vals[1]) / 1.5
    assert np.allclose(out[0], want, rtol=1e-15)
    # equal distances: the plain mean, whatever the distance (no underflow)
    out = oracle.gka_average(np.array([[0, 1, 3]]), np.array([[1e6, 1e6, 1e6]]), vals)
    assert np.allclose(out[0], vals[[0, 1, 3]].mean(axis=0), rtol=1e-15)
    # no context: NaN
    out = oracle.gka_average(np.array([[-1, -1]]), np.array([[np.inf, np.inf]]), vals)
    assert np.all(np.isnan(out))
    # constant values stay constant; a common shift of the distances changes nothing
    c = np.full((4, 2), 2.5)
    d = np.array([[0.3, 1.7, 2.2, 9.0]])
    i4 = np.array([[3, 0, 2, 1]])
    assert np.allclose(oracle.gka_average(i4, d, c), 2.5, rtol=1e-15)
    a = oracle.gka_average(i4, d, vals)
    b = oracle.gka_average(i4, d + 123.0, vals)
    assert np.allclose(a, b, rtol=1e-14)
    # far neighbours barely count: exp(-50) relative weight
    out = oracle.gka_average(np.array([[1, 2]]), np.array([[0.0, 50.0]]), vals)
    assert np.allclose(out[0], vals[1], rtol=1e-20, atol=1e-19 * 10)


def test_per_query_scales_hand_case():
    """Two queries at the same place under different metrics (Sec. 3.2: the
    scales may vary over space).  Query point (0, 0, 0, 10); A = (1, 0, 0, 0),
    B = (0, 0, 0.5, 0), C = (0, 0, 0, 20) (after the query: masked).
    s = (1, 1, 1, 0): d_A = 1, d_B = 0.25 -> B, A.
    s = (1, 1, 10, 0): d_A = 1, d_B = 2.5 -> A, B.
    s = (0, 0, 0, 1): d_A = d_B = 100 -> tie, lower index A first."""
    pts = tuple(np.array(v, dtype=np.float32) for v in
                ([1.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.5, 0.0], [0.0, 0.0, 20.0]))
    q = tuple(np.array([v] * 3, dtype=np.float32) for v in (0.0, 0.0, 0.0, 10.0))
    s = np.array([[1, 1, 1, 0], [1, 1, 10, 0], [0, 0, 0, 1]], dtype=np.float64)
    idx, dist = oracle.knn(pts, q, s, 0.0, 3)
    assert idx.tolist() == [[1, 0, -1], [0, 1, -1], [0, 1, -1]]
    assert dist[:, :2].tolist() == [[0.25, 1.0], [1.0, 2.5], [100.0, 100.0]]
    assert np.isinf(dist[:, 2]).all()


def test_per_query_scales_reduce_to_the_shared_metric():
    """Equal rows give the shared-scale result; each row alone gives that
    query's shared-scale result; a power-of-two factor on a row scales its
    distances exactly and keeps its indices; a bad row is (-1, NaN) and leaves
    the others alone."""
    ps = synth.trajectories(30, 40, 300.0, 3600.0, seed=8)
    rng = np.random.default_rng(4)
    qs = ps.take(rng.choice(ps.n, 40, replace=False))
    base = np.array(synth.SCALE)
    k = 7
    i0, d0 = oracle.knn(ps.soa(), qs.soa(), base, 0.0, k)
    i1, d1 = oracle.knn(ps.soa(), qs.soa(), np.tile(base, (qs.n, 1)), 0.0, k)
    assert np.array_equal(i0, i1) and np.array_equal(d0, d1)
    rows = base * rng.uniform(0.25, 4.0, size=(qs.n, 4))
    iq, dq = oracle.knn(ps.soa(), qs.soa(), rows, 0.0, k)
    for j in range(0, qs.n, 5):
        one = qs.take(np.array([j]))
        ij, dj = oracle.knn(ps.soa(), one.soa(), rows[j], 0.0, k)
        assert np.array_equal(iq[j], ij[0]) and np.array_equal(dq[j], dj[0])
    scaled = rows.copy()
    scaled[::2] *= 8.0
    i2, d2 = oracle.knn(ps.soa(), qs.soa(), scaled, 0.0, k)
    assert np.array_equal(i2, iq)
    fin = np.isfinite(dq)
    assert np.array_equal(d2[::2][fin[::2]], 8.0 * dq[::2][fin[::2]])
    assert np.array_equal(d2[1::2], dq[1::2])
    bad = rows.copy()
    bad[3, 2] = -1.0
    bad[5, 0] = np.nan
    bad[6, 3] = np.inf
    i3, d3 = oracle.knn(ps.soa(), qs.soa(), bad, 0.0, k)
    for j in (3, 5, 6):
        assert (i3[j] == -1).all() and np.isnan(d3[j]).all()
    keep = np.setdiff1d(np.arange(qs.n), [3, 5, 6])
    assert np.array_equal(i3[keep], iq[keep]) and np.array_equal(d3[keep], dq[keep])


@pytest.mark.parametrize("seed", range(4))
def test_per_query_scales_equal_exact_rational_on_dyadic(seed):
    """Dyadic data and dyadic per-query scales: every binary64 operation is
    exact, so each row equals the exact rational k-NN under its own metric."""
    rng = np.random.default_rng(100 + seed)
    n, nq, k = 40, 10, int(rng.integers(1, 9))
    pts = tuple(_dyadic(rng, n) for _ in range(3)) + (_dyadic(rng, n, 0, 32, 4),)
    qs = tuple(_dyadic(rng, nq) for _ in range(3)) + (_dyadic(rng, nq, 0, 32, 4),)
    choices = np.array([0.0, 0.125, 0.25, 0.5, 1.0, 2.0, 4.0])
    rows = rng.choice(choices, size=(nq, 4))
    tw = [0.0, 0.5][seed % 2]
    idx, dist = oracle.knn(pts, qs, rows, tw, k)
    for j in range(nq):
        one = tuple(a[j:j + 1] for a in qs)
        ei, ed = exact_knn(pts, one, list(rows[j]), tw, k)
        assert np.array_equal(idx[j], ei[0]), j
        assert np.array_equal(dist[j], np.array([float(v) for v in ed[0]])), j


def test_pair_dist_with_query_rows_reduces_to_the_shared_metric():
    """One scale row per query: equal rows give the shared-metric distances,
    and a row scaled by a power of two scales exactly its pairs; every pair
    equals the k-NN's own distance for that pair (k = n on one query)."""
    ps = synth.trajectories(5, 20, 100.0, 600.0, seed=2)
    qs = ps.take(np.array([99, 50, 7]))
    QQ, PP = np.meshgrid(np.arange(3), np.arange(ps.n), indexing="ij")
    QQ, PP = QQ.ravel(), PP.ravel()
    base = np.array(synth.SCALE)
    d0 = oracle.pair_dist(ps.soa(), qs.soa(), QQ, PP, base)
    rows = np.tile(base, (3, 1))
    assert np.array_equal(oracle.pair_dist(ps.soa(), qs.soa(), QQ, PP, rows), d0)
    rows[1] *= 4.0
    d1 = oracle.pair_dist(ps.soa(), qs.soa(), QQ, PP, rows)
    m = QQ == 1
    assert np.array_equal(d1[m], 4.0 * d0[m]) and np.array_equal(d1[~m], d0[~m])
    # against the k-NN: every point of the earliest-to-latest order, no mask
    qt = tuple(a.copy() for a in qs.soa())
    qt[3][:] = np.float32(1e9)
    idx, dist = oracle.knn(ps.soa(), qt, rows, 0.0, ps.n)
    late = synth.PointSet(*qt, np.array([0, 3]))
    d2 = oracle.pair_dist(ps.soa(), late.soa(), QQ, PP, rows).reshape(3, ps.n)
    for q in range(3):
        assert np.array_equal(dist[q], d2[q][idx[q]])


def test_radius_calibrate_closed_forms_and_numpy_quantile():
    """The safety factor's quantile: hand cases, then np.quantile's default
    (linear) method on random residuals; unlabelled and non-finite samples
    are left out, and no labelled sample gives alpha = 1."""
    # residuals 0, 1, ..., 9 (logr = 0, d_k = e^(2 i)): median position 4.5
    d = np.exp(2.0 * np.arange(10))
    lr = np.zeros(10, np.float32)
    assert oracle.radius_calibrate(lr, d, 0.5) == pytest.approx(math.exp(4.5), rel=1e-14)
    assert oracle.radius_calibrate(lr, d, 0.0) == pytest.approx(1.0, rel=1e-14)
    assert oracle.radius_calibrate(lr, d, 1.0) == pytest.approx(math.exp(9.0), rel=1e-14)
    # q = 0.9 over 10 values: position 8.1 -> 8.1
    assert oracle.radius_calibrate(lr, d, 0.9) == pytest.approx(math.exp(8.1), rel=1e-13)
    # unlabelled samples (inf, 0, NaN distance) are skipped
    d2 = np.concatenate([d, [np.inf, 0.0, np.nan]])
    lr2 = np.zeros(13, np.float32)
    assert oracle.radius_calibrate(lr2, d2, 0.5) == pytest.approx(math.exp(4.5), rel=1e-14)
    # a non-finite prediction is skipped too
    lr3 = lr2.copy()
    lr3[0] = np.inf
    assert oracle.radius_calibrate(lr3, d2, 0.0) == pytest.approx(math.exp(1.0), rel=1e-14)
    assert oracle.radius_calibrate(lr2[:3], np.array([np.inf, 0.0, np.nan]), 0.5) == 1.0
    rng = np.random.default_rng(3)
    lr = rng.normal(0, 1, 5001).astype(np.float32)
    d = np.exp(rng.normal(2, 3, 5001))
    r = 0.5 * np.log(d) - lr.astype(np.float64)
    for q in (0.0, 0.37, 0.9, 0.99, 1.0):
        want = math.exp(float(np.quantile(r, q)))
        assert oracle.radius_calibrate(lr, d, q) == pytest.approx(want, rel=1e-13)
