"""Host side of the learned k-th radius: label, train, calibrate, save.

Labels are the k-th distances that plain TNN returns for a set of training
queries (the method's own output).  Every arithmetic step runs in the
library's kernels (training order, forward / backward, Adam, the safety
factor's quantile); this module only loops over epochs and batches.
"""
from __future__ import annotations

import torch

from . import capi
from . import tnn as T


def train(index, sx, sy, sz, st, scale, t_window, k, epochs=20, batch=4096, lr=3e-3,
          seed=1, log=None):
    """Returns (model blob, final mean loss, the labels' dist tensor, the
    training samples).  Each epoch visits the samples in a fresh device
    permutation."""
    dev = sx.device
    n = sx.shape[0]
    # labels: plain TNN on the training queries
    _, dist = T.tnn_query(index, sx, sy, sz, st, scale, t_window, k)
    model = T.tnn_radius_model_init(index, seed)
    adam = torch.zeros(2 * capi.RADIUS_NPARAMS, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    order = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    scratch = None
    step = 0
    nb = max(1, n // batch) if n > 0 else 0
    for ep in range(epochs):
        if n > 0:
            T.tnn_radius_shuffle(n, seed * 1000003 + ep, out=order)
        for b in range(nb):
            step += 1
            first = b * batch
            size = min(batch, n - first) if b < nb - 1 else n - first
            scratch = T.tnn_radius_train_step(model, adam, sx, sy, sz, st, dist, k, first, size,
                                              step, lr, loss=loss, scratch=scratch, order=order)
        if log is not None:
            log(f"radius epoch {ep}: loss {float(loss.item()):.4f}")
    return model, float(loss.item()), dist, (sx, sy, sz, st)


def calibrate(model, sx, sy, sz, st, dist, k, quantile=0.9):
    """Safety factor alpha: exp of the q-quantile of the labelled samples'
    log-residuals (about 1 - q of them then fall back)."""
    return float(T.tnn_radius_calibrate(model, sx, sy, sz, st, dist, k, quantile).item())


def save(model, path):
    """Write a versioned checkpoint of the model to `path`."""
    buf = T.tnn_radius_model_save(model)
    with open(path, "wb") as f:
        f.write(buf.tobytes())


def load(path, device="cuda"):
    """Device model from a checkpoint file (TnnError TNN_E_FORMAT if the file
    is not an intact checkpoint of this library's model)."""
    with open(path, "rb") as f:
        data = f.read()
    return T.tnn_radius_model_load(data, device=device)
