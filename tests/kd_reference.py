"""numpy rendering of the index build's kd order of segments into blocks
(test infrastructure): a range longer than a block splits along its widest
key axis into its m smallest entries by (key, segment number) and the rest,
each part keeping its order, m = n/2 rounded up to a multiple of the block;
inside each block the halving goes on, m = n/2, down to single segments."""
import math

import numpy as np

BLOCK = 64


def segment_keys(ps, seg_len, order_scale):
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


def kd_reference(keys):
    S = keys.shape[0]
    idx = np.arange(S, dtype=np.int64)
    _levels([(0, S)], idx, keys, _block_m)
    # inside each block the splits go on down to single entries, m = n // 2
    _levels([(b, min(BLOCK, S - b)) for b in range(0, S, BLOCK)], idx, keys,
            lambda n: n // 2 if n >= 2 else None)
    return idx
