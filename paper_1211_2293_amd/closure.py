"""Training the learned closure on the GPU through the C ABI.

The closure's network predicts, for a body and an accepted cell, the
normalised residual between the exact sum over the cell's bodies and the
cell's monopole.  Its training pairs come from the method itself
(tc_residuals: each target walks alone at theta and every accepted cell
gives one pair); each step is the library's forward, backward and Adam
kernels (tc_mlp_step).  This module only orders the minibatches and calls
the library.
"""
from __future__ import annotations

import numpy as np

from . import workloads


def residual_pairs(tc, theta, eps, targets):
    """(feat [P][10], y [P][3]) CUDA tensors for the int64/int32 original
    body indices in `targets` (numpy)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(targets, np.int32)).to(tc.stream.device)
    feat, y, _ = tc.residuals(theta, eps, t)
    return feat.clone(), y.clone()


def train(tc, feat, y, *, epochs=40, batch=4096, lr=3e-3, lr_final=3e-5, seed=0, init_seed=0,
          val=None, log=None):
    """Train from the seeded initial parameters: `epochs` passes over the
    pairs in seeded random minibatches of `batch`, Adam with the learning
    rate decaying geometrically from lr to lr_final.  Returns a dict with
    the first and last batch losses, the steps taken and, with val =
    (feat, y), the validation mean squared error and that of predicting
    zero."""
    import torch
    dev = tc.stream.device
    tc.mlp_load(torch.from_numpy(workloads.mlp_params(init_seed)).to(dev))
    npairs = feat.shape[0]
    steps = max(1, epochs * npairs // batch)
    order = torch.from_numpy(workloads.batch_order(npairs, steps, batch, seed)).to(dev)
    first = last = None
    for k in range(steps):
        idx = order[k * batch:(k + 1) * batch]
        rate = lr * (lr_final / lr) ** (k / max(steps - 1, 1))
        want = k == 0 or k == steps - 1 or (log is not None and k % 1000 == 0)
        loss = tc.mlp_step(feat, y, idx, lr=rate, want_loss=want)
        if k == 0:
            first = loss
        if k == steps - 1:
            last = loss
        if log is not None and k % 1000 == 0:
            log(f"  step {k}/{steps}: loss {loss:.3e}")
    out = {"pairs": int(npairs), "steps": int(steps), "batch": int(batch), "epochs": epochs,
           "loss_first": first, "loss_last": last}
    if val is not None:
        fv, yv = val
        pred = tc.mlp_forward(fv)
        out["val_mse"] = float(((pred - yv) ** 2).mean())
        out["val_mse_zero"] = float((yv ** 2).mean())
    return out
