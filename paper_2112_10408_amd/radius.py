"""Host driver for the learned k-th radius: label, train, calibrate.

Labels are the k-th distances that plain TNN returns for a set of training
queries (the method's own output).  Training runs the library's forward /
backward and Adam kernels; this module only loops over epochs and batches.
"""
from __future__ import annotations

import math

import torch

from . import capi
from . import tnn as T


def train(index, sx, sy, sz, st, scale, t_window, k, epochs=20, batch=4096, lr=3e-3,
          seed=1, log=None):
    """Returns (model blob, final mean loss, labels' dist tensor)."""
    dev = sx.device
    n = sx.shape[0]
    # labels: plain TNN on the training queries
    _, dist = T.tnn_query(index, sx, sy, sz, st, scale, t_window, k)
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(n, generator=g).to(dev)
    px, py, pz, pt = (a[perm].contiguous() for a in (sx, sy, sz, st))
    pdist = dist[perm].contiguous()
    model = T.tnn_radius_model_init(index, seed)
    adam = torch.zeros(2 * capi.RADIUS_NPARAMS, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    scratch = None
    step = 0
    nb = max(1, n // batch) if n > 0 else 0
    for ep in range(epochs):
        for b in range(nb):
            step += 1
            first = b * batch
            size = min(batch, n - first) if b < nb - 1 else n - first
            scratch = T.tnn_radius_train_step(model, adam, px, py, pz, pt, pdist, k, first, size,
                                              step, lr, loss=loss, scratch=scratch)
        if log is not None:
            log(f"radius epoch {ep}: loss {float(loss.item()):.4f}")
    return model, float(loss.item()), pdist, (px, py, pz, pt)


def calibrate(model, sx, sy, sz, st, dist, k, quantile=0.9):
    """Safety factor alpha = exp(q-quantile of log r_k - prediction) over the
    labelled training queries: about (1 - q) of them fall back."""
    logr = torch.empty(sx.shape[0], dtype=torch.float32, device=sx.device)
    T.tnn_radius_infer(model, sx, sy, sz, st, 1.0, logr=logr)
    dk = dist[:, k - 1]
    ok = torch.isfinite(dk) & (dk > 0)
    resid = (0.5 * torch.log(dk[ok]) - logr[ok].double())
    if resid.numel() == 0:
        return 1.0
    return float(math.exp(torch.quantile(resid, quantile).item()))
