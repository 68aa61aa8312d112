"""Training the learned closure on the GPU through the C ABI.

The closure's network predicts, for a body and an accepted cell, the
normalised residual between the exact sum over the cell's bodies and the
cell's monopole.  Its training pairs come from the method itself
(tc_residuals: each target walks alone at theta and every accepted cell
gives one pair); each step is the library's forward, backward and Adam
kernels (tc_mlp_step).  This module only orders the minibatches and calls
the library; the random draws (initial parameters, minibatch order) are
inputs from the caller.
"""
from __future__ import annotations

import numpy as np


def residual_pairs(tc, theta, eps, targets):
    """(feat [P][10], y [P][3]) CUDA tensors for the int64/int32 original
    body indices in `targets` (numpy)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(targets, np.int32)).to(tc.stream.device)
    feat, y, _ = tc.residuals(theta, eps, t)
    return feat.clone(), y.clone()


def steps_for(npairs, epochs, batch):
    """Adam steps of `epochs` passes over npairs pairs in batches of `batch`."""
    return max(1, epochs * int(npairs) // batch)


def train(tc, feat, y, params0, order, *, epochs=40, batch=4096, lr=3e-3, lr_final=3e-5, val=None, log=None):
    """Train from the initial parameters params0 (FP32 numpy, canonical
    order): steps_for(pairs, epochs, batch) Adam steps, step k on the
    samples order[k * batch:(k + 1) * batch] (int32 numpy, at least that
    long), the learning rate decaying geometrically from lr to lr_final.
    Returns a dict with the first and last batch losses, the steps taken
    and, with val = (feat, y), the validation mean squared error and that of
    predicting zero."""
    import torch
    dev = tc.stream.device
    npairs = feat.shape[0]
    steps = steps_for(npairs, epochs, batch)
    if len(order) < steps * batch:
        raise ValueError(f"order holds {len(order)} samples, {steps * batch} needed")
    tc.mlp_load(torch.from_numpy(np.ascontiguousarray(params0, np.float32)).to(dev))
    order = torch.from_numpy(np.ascontiguousarray(order[:steps * batch], np.int32)).to(dev)
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


def quadrupole_prediction(feat):
    """The analytic quadrupole term in the network's target units, from the
    same features: with u = (x - C)/s, uh = u/|u| and Qh = Q/(M s^2), the
    unsoftened quadrupole acceleration G [Q r / r^5 - (5/2)(r.Q r) r / r^7]
    (r = x - C) times |r|^4 / (G M s^2) is Qh uh - (5/2)(uh.Qh uh) uh.  The
    control the trained network is measured against (torch, on the
    features' device)."""
    import torch
    u = feat[:, 0:3].double()
    q = feat[:, 3:9].double()
    uh = u / torch.linalg.norm(u, dim=1, keepdim=True)
    x, y, z = uh[:, 0], uh[:, 1], uh[:, 2]
    qx = q[:, 0] * x + q[:, 3] * y + q[:, 4] * z
    qy = q[:, 3] * x + q[:, 1] * y + q[:, 5] * z
    qz = q[:, 4] * x + q[:, 5] * y + q[:, 2] * z
    uqu = qx * x + qy * y + qz * z
    out = torch.stack([qx, qy, qz], dim=1) - 2.5 * uqu[:, None] * uh
    return out.float()
