"""Exact-rational brute force used only to cross-check the oracle.

Every quantity is a ``fractions.Fraction``: no rounding anywhere, so on dyadic
inputs (where binary64 arithmetic is exact) the oracle must agree bit for bit,
and on general inputs it ranks by the exact real distance.
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr

import numpy as np


def exact_knn(points, queries, scale, t_window, k):
    px, py, pz, pt = points
    qx, qy, qz, qt = queries
    s = [Fr(float(v)) for v in scale]
    tw = Fr(float(t_window))
    res_i, res_d = [], []
    for q in range(len(qx)):
        cand = []
        for i in range(len(px)):
            if not (Fr(float(pt[i])) < Fr(float(qt[q])) - tw):
                continue
            d = (s[0] * (Fr(float(qx[q])) - Fr(float(px[i]))) ** 2
                 + s[1] * (Fr(float(qy[q])) - Fr(float(py[i]))) ** 2
                 + s[2] * (Fr(float(qz[q])) - Fr(float(pz[i]))) ** 2
                 + s[3] * (Fr(float(qt[q])) - Fr(float(pt[i]))) ** 2)
            cand.append((d, i))
        cand.sort()
        top = cand[:k]
        res_i.append([i for _, i in top] + [-1] * (k - len(top)))
        res_d.append([d for d, _ in top] + [math.inf] * (k - len(top)))
    return np.array(res_i, dtype=np.int64), res_d
