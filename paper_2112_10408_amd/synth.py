"""Seeded synthetic aircraft-trajectory workloads.

This module only draws inputs: point clouds laid out along flight paths and
query sets sampled from them.  It holds none of the nearest-neighbour
arithmetic, so both the CPU oracle and the GPU path can be fed from it.

The paper evaluates on Mode-S recordings (Sec. 3.1: about one million points
per day over European airspace, sampled every 4 s by the secondary
surveillance radars) and on a smoothed random walk (Sec. 4.2).  Neither is
available here; the generator below stands in for them with the same shape:
time-sorted trajectories of (x, y, z km, t s) points, 4 s apart, with smooth
heading drift.

Recipe per trajectory (all draws from one ``numpy.random.default_rng``):
  start (x0, y0) ~ U[0, L]^2 km, altitude z ~ U[8, 12] km (constant),
  start time t0 ~ U[0, T] s, heading h0 ~ U[0, 2 pi), speed v ~ N(230, 15) m/s;
  per 4 s step: h += N(0, 0.5 deg), x += 4 v cos(h) / 1000, y += 4 v sin(h) / 1000,
  t += 4.  No clipping to the box.
Output: float32 structure-of-arrays, trajectory-contiguous, int64 offsets.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 2112104080
SCALE = (1.0, 1.0, 10.0, 0.05)  # (sigma_x, sigma_y, sigma_z, sigma_t)


@dataclasses.dataclass
class PointSet:
    x: np.ndarray  # float32 [N]
    y: np.ndarray
    z: np.ndarray
    t: np.ndarray
    offsets: np.ndarray  # int64 [n_traj + 1]

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def take(self, idx: np.ndarray) -> "PointSet":
        idx = np.asarray(idx)
        return PointSet(self.x[idx], self.y[idx], self.z[idx], self.t[idx],
                        np.array([0, idx.shape[0]], dtype=np.int64))

    def soa(self):
        return self.x, self.y, self.z, self.t


def trajectories(n_traj: int, n_pts, box_km: float, span_s: float,
                 seed: int) -> PointSet:
    """Draw ``n_traj`` trajectories.  ``n_pts`` is an int or an int array."""
    rng = np.random.default_rng(seed)
    counts = np.broadcast_to(np.asarray(n_pts, dtype=np.int64), (n_traj,)).copy()
    x0 = rng.uniform(0.0, box_km, n_traj)
    y0 = rng.uniform(0.0, box_km, n_traj)
    z0 = rng.uniform(8.0, 12.0, n_traj)
    t0 = rng.uniform(0.0, span_s, n_traj)
    h0 = rng.uniform(0.0, 2.0 * math.pi, n_traj)
    v = rng.normal(230.0, 15.0, n_traj)
    offsets = np.zeros(n_traj + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    n = int(offsets[-1])
    steps = np.maximum(counts - 1, 0)
    dh = rng.normal(0.0, math.radians(0.5), int(steps.sum()))
    x = np.empty(n, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    z = np.empty(n, dtype=np.float64)
    t = np.empty(n, dtype=np.float64)
    # Vectorised per trajectory: headings are cumulative drifts.
    traj_of_step = np.repeat(np.arange(n_traj), steps)
    step_first = np.zeros(n_traj + 1, dtype=np.int64)
    np.cumsum(steps, out=step_first[1:])
    h = np.cumsum(dh)
    h -= np.repeat(np.concatenate(([0.0], h))[step_first[:-1]], steps)
    h += h0[traj_of_step]
    vx = 4.0 * v[traj_of_step] * np.cos(h) / 1000.0
    vy = 4.0 * v[traj_of_step] * np.sin(h) / 1000.0
    cx = np.cumsum(vx)
    cy = np.cumsum(vy)
    cx -= np.repeat(np.concatenate(([0.0], cx))[step_first[:-1]], steps)
    cy -= np.repeat(np.concatenate(([0.0], cy))[step_first[:-1]], steps)
    first = offsets[:-1]
    x[first] = x0
    y[first] = y0
    rest = np.ones(n, dtype=bool)
    rest[first] = False
    x[rest] = x0[traj_of_step] + cx
    y[rest] = y0[traj_of_step] + cy
    tr = np.repeat(np.arange(n_traj), counts)
    local = np.arange(n) - offsets[tr]
    z[:] = z0[tr]
    t[:] = t0[tr] + 4.0 * local
    f = np.float32
    return PointSet(x.astype(f), y.astype(f), z.astype(f), t.astype(f), offsets)


def random_points(n: int, box_km: float, span_s: float, seg_len: int,
                  seed: int) -> PointSet:
    """The paper's pathological set (Sec. 4.2): points drawn uniformly and
    grouped at random into 'trajectories' of ``seg_len`` points, each group
    sorted by time so that it is a valid time-sorted trajectory."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, box_km, n)
    y = rng.uniform(0.0, box_km, n)
    z = rng.uniform(8.0, 12.0, n)
    t = rng.uniform(0.0, span_s, n)
    n_traj = (n + seg_len - 1) // seg_len
    offsets = np.minimum(np.arange(n_traj + 1, dtype=np.int64) * seg_len, n)
    for j in range(n_traj):
        a, b = offsets[j], offsets[j + 1]
        o = np.argsort(t[a:b], kind="stable")
        x[a:b], y[a:b], z[a:b], t[a:b] = x[a:b][o], y[a:b][o], z[a:b][o], t[a:b][o]
    f = np.float32
    return PointSet(x.astype(f), y.astype(f), z.astype(f), t.astype(f), offsets)


def routes(n_traj: int, n_pts: int, box_km: float, span_s: float, n_routes: int,
           seed: int) -> PointSet:
    """Route-clustered traffic, closer to recorded flights than uniform
    headings: ``n_routes`` straight airways cross the box (a random point and
    direction each); every trajectory follows one of them in either
    direction, starting at a uniform position along it, with a lateral offset
    ~ N(0, 5) km, a flight level in {9, 10, 11, 12} km plus N(0, 0.02) km,
    speed ~ N(230, 15) m/s and heading drift ~ N(0, 0.1 deg) per 4 s step.
    Start times ~ U[0, T] s."""
    rng = np.random.default_rng(seed)
    rx = rng.uniform(0.0, box_km, n_routes)
    ry = rng.uniform(0.0, box_km, n_routes)
    rh = rng.uniform(0.0, math.pi, n_routes)
    r = rng.integers(0, n_routes, n_traj)
    back = rng.random(n_traj) < 0.5
    along = rng.uniform(-0.5 * box_km, 0.5 * box_km, n_traj)
    lateral = rng.normal(0.0, 5.0, n_traj)
    h0 = rh[r] + np.where(back, math.pi, 0.0)
    x0 = rx[r] + along * np.cos(rh[r]) - lateral * np.sin(rh[r])
    y0 = ry[r] + along * np.sin(rh[r]) + lateral * np.cos(rh[r])
    z0 = rng.integers(9, 13, n_traj) + rng.normal(0.0, 0.02, n_traj)
    t0 = rng.uniform(0.0, span_s, n_traj)
    v = rng.normal(230.0, 15.0, n_traj)
    dh = rng.normal(0.0, math.radians(0.1), (n_traj, n_pts - 1))
    h = h0[:, None] + np.concatenate([np.zeros((n_traj, 1)), np.cumsum(dh, axis=1)], axis=1)
    step = 4.0 * v[:, None] / 1000.0
    dx = np.concatenate([np.zeros((n_traj, 1)), (step * np.cos(h))[:, :-1]], axis=1)
    dy = np.concatenate([np.zeros((n_traj, 1)), (step * np.sin(h))[:, :-1]], axis=1)
    x = x0[:, None] + np.cumsum(dx, axis=1)
    y = y0[:, None] + np.cumsum(dy, axis=1)
    z = np.repeat(z0[:, None], n_pts, axis=1)
    t = t0[:, None] + 4.0 * np.arange(n_pts)[None, :]
    offsets = np.arange(n_traj + 1, dtype=np.int64) * n_pts
    f = np.float32
    return PointSet(x.ravel().astype(f), y.ravel().astype(f), z.ravel().astype(f),
                    t.ravel().astype(f), offsets)


def sample_queries(ps: PointSet, n_queries: int | None, seed: int,
                   exclude: np.ndarray | None = None) -> tuple[PointSet, np.ndarray]:
    """Queries are data points, sampled uniformly without replacement
    (``None`` = every point, in order).  Returns (queries, point indices)."""
    if n_queries is None:
        idx = np.arange(ps.n, dtype=np.int64)
    else:
        rng = np.random.default_rng(seed)
        pool = np.arange(ps.n, dtype=np.int64)
        if exclude is not None:
            keep = np.ones(ps.n, dtype=bool)
            keep[exclude] = False
            pool = pool[keep]
        idx = rng.choice(pool, size=n_queries, replace=False)
    return ps.take(idx), idx


# Workloads.  c1..c5 follow the five evaluation configurations: 10k points
# (k=8, K=16), 1M points with 100k sampled queries (k=32, K=32), the same 1M
# points with every point a query, 8M points (k=64) with 200k training and 1M
# test queries, and 64 ragged airspaces.
CONFIGS = {
    "c1": dict(n_traj=200, n_pts=50, box_km=1000.0, span_s=4 * 3600.0,
               seg_len=16, k=8, n_queries=None, seed=SEED_BASE + 1),
    "c2": dict(n_traj=5000, n_pts=200, box_km=3000.0, span_s=12 * 3600.0,
               seg_len=32, k=32, n_queries=100_000, seed=SEED_BASE + 2),
    "c3": dict(n_traj=5000, n_pts=200, box_km=3000.0, span_s=12 * 3600.0,
               seg_len=32, k=32, n_queries=None, seed=SEED_BASE + 2),
    "c4": dict(n_traj=20000, n_pts=400, box_km=6000.0, span_s=24 * 3600.0,
               seg_len=32, k=64, n_queries=1_000_000, n_train=200_000,
               seed=SEED_BASE + 4),
    # the paper's production setting: only points at least 30 min old
    "c2w": dict(n_traj=5000, n_pts=200, box_km=3000.0, span_s=12 * 3600.0,
                seg_len=32, k=32, n_queries=100_000, seed=SEED_BASE + 2, t_window=1800.0),
    # Sec. 4.2's random points: TNN cannot prune, results must stay exact
    "rand": dict(kind="random", n=1_000_000, box_km=3000.0, span_s=12 * 3600.0,
                 seg_len=32, k=32, n_queries=100_000, seed=SEED_BASE + 6),
    # traffic along 40 airways
    "routes": dict(kind="routes", n_traj=5000, n_pts=200, box_km=3000.0, span_s=12 * 3600.0,
                   n_routes=40, seg_len=32, k=32, n_queries=100_000, seed=SEED_BASE + 7),
}


def scale_field(x, y, z, box_km: float, seed: int, base=SCALE, spread: float = 0.7):
    """Per-query scales that vary smoothly over space, the shape of the
    paper's proposal of the scale vector as a function of position (Sec. 3.2):
    s_xy, s_z and s_t each the base value times exp(spread * a smooth field
    in [-1, 1]) with random phases, so they range over about exp(+-spread).
    s_x = s_y (one horizontal scale).  Returns float64 [n, 4]."""
    rng = np.random.default_rng(seed)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=6)
    w = 2.0 * np.pi / box_km
    fxy = np.sin(w * 1.3 * x + ph[0]) * np.cos(w * 0.9 * y + ph[1])
    fz = np.sin(0.5 * z + ph[2]) * np.cos(w * 0.7 * x + ph[3])
    ft = np.cos(w * 1.1 * y + ph[4]) * np.sin(w * 0.6 * x + ph[5])
    out = np.empty((x.shape[0], 4), dtype=np.float64)
    out[:, 0] = base[0] * np.exp(spread * fxy)
    out[:, 1] = out[:, 0]
    out[:, 2] = base[2] * np.exp(spread * fz)
    out[:, 3] = base[3] * np.exp(spread * ft)
    return out


def make_config(name: str):
    """Return (points, queries, query point indices, cfg dict)."""
    cfg = dict(CONFIGS[name])
    cfg.setdefault("t_window", 0.0)
    kind = cfg.get("kind", "trajectories")
    if kind == "random":
        ps = random_points(cfg["n"], cfg["box_km"], cfg["span_s"], cfg["seg_len"], cfg["seed"])
    elif kind == "routes":
        ps = routes(cfg["n_traj"], cfg["n_pts"], cfg["box_km"], cfg["span_s"], cfg["n_routes"],
                    cfg["seed"])
    else:
        ps = trajectories(cfg["n_traj"], cfg["n_pts"], cfg["box_km"], cfg["span_s"], cfg["seed"])
    if name == "c4":
        rng = np.random.default_rng(cfg["seed"] + 1000)
        perm = rng.permutation(ps.n)
        tr_idx = perm[: cfg["n_train"]]
        te_idx = perm[cfg["n_train"]: cfg["n_train"] + cfg["n_queries"]]
        cfg["train_idx"] = tr_idx
        qs = ps.take(te_idx)
        return ps, qs, te_idx, cfg
    qs, qidx = sample_queries(ps, cfg["n_queries"], cfg["seed"] + 1000)
    return ps, qs, qidx, cfg


def airspaces(n_air: int = 64, seed: int = SEED_BASE + 5, pts_per_traj: int = 200,
              n_range=(10_000, 500_000), q_range=(1_000, 50_000), ks=(8, 32, 64)):
    """Ragged serving workload: independent airspaces with log-uniform point
    and query counts and k drawn from ``ks``.  Yields dicts."""
    rng = np.random.default_rng(seed)
    n_a = np.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1]), n_air))
    q_a = np.exp(rng.uniform(math.log(q_range[0]), math.log(q_range[1]), n_air))
    k_a = rng.choice(np.asarray(ks), n_air)
    out = []
    for a in range(n_air):
        n_traj = max(1, int(round(n_a[a] / pts_per_traj)))
        ps = trajectories(n_traj, pts_per_traj, 3000.0, 12 * 3600.0, seed * 131 + a)
        nq = min(int(round(q_a[a])), ps.n)
        qs, qidx = sample_queries(ps, nq, seed * 131 + a + 1000)
        out.append(dict(points=ps, queries=qs, qidx=qidx, k=int(k_a[a]), seg_len=32))
    return out
