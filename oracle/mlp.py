"""FP64 reference of the learned closure's network: TEST INFRASTRUCTURE ONLY.

The closure predicts, for a body and an accepted cell, the normalised
residual between the exact sum over the cell's bodies and the cell's
monopole (a small multilayer perceptron 10-64-64-3 with GELU activations,
trained by mean squared error with Adam).  The paper's treecode stops at the
monopole (§3.1); the closure is this project's extension of it.

Network:  z1 = f W1 + b1, h1 = gelu(z1), z2 = h1 W2 + b2, h2 = gelu(z2),
          y = h2 W3 + b3,  gelu(z) = z (1 + erf(z / sqrt 2)) / 2.
Parameters, canonical flat order (5059 values): W1 [10][64], b1 [64],
W2 [64][64], b2 [64], W3 [64][3], b3 [3].

With ``bf16=True`` the matrix products take bfloat16-rounded operands (round
to nearest, ties to even, applied to an FP32 value) exactly where the GPU
kernels feed their BF16 matrix-core instructions; everything else is FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf as _erf

SHAPES = [("W1", (10, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 3)),
          ("b3", (3,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)          # 5059


def unflatten(theta):
    theta = np.asarray(theta, np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SHAPES])


def init_params(seed=0):
    """Seeded initial parameters (the shared input generator's draw):
    weights uniform in +-1/sqrt(fan_in), biases zero."""
    from paper_1211_2293_amd import workloads
    return workloads.mlp_params(seed)


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) from the FP32 value of x;
    returned as float64 holding the bfloat16 value."""
    f = np.array(x, np.float32, copy=True, ndmin=1)
    u = f.view(np.uint32)
    lsb = (u >> 16) & np.uint32(1)
    u += np.uint32(0x7FFF)                  # no wrap for finite values
    u += lsb
    u &= np.uint32(0xFFFF0000)
    r = f.astype(np.float64)
    return r.reshape(np.shape(x)) if np.ndim(x) else r[0]


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, f, bf16_ops=False):
    """Returns (y, cache).  f is [B][10]."""
    p = unflatten(theta)
    q = bf16 if bf16_ops else (lambda v: np.asarray(v, np.float64))
    f = np.asarray(f, np.float64)
    fi = q(f)
    z1 = fi @ q(p["W1"]) + p["b1"]
    h1 = gelu(z1)
    h1i = q(h1)
    z2 = h1i @ q(p["W2"]) + p["b2"]
    h2 = gelu(z2)
    h2i = q(h2)
    y = h2i @ q(p["W3"]) + p["b3"]
    return y, dict(fi=fi, z1=z1, h1i=h1i, z2=z2, h2i=h2i, p=p)


def loss_and_grad(theta, f, y_true, bf16_ops=False):
    """Mean squared error over all B x 3 outputs and its gradient with
    respect to the flat parameters (backward pass of the network above;
    with bf16_ops the backward products also take bfloat16 operands)."""
    y, c = forward(theta, f, bf16_ops)
    q = bf16 if bf16_ops else (lambda v: np.asarray(v, np.float64))
    p = c["p"]
    B = y.shape[0]
    diff = y - np.asarray(y_true, np.float64)
    loss = float((diff ** 2).sum() / (B * 3))
    dy = 2.0 * diff / (B * 3)
    dyi = q(dy)
    g = {}
    g["W3"] = c["h2i"].T @ dyi
    g["b3"] = dy.sum(0)
    dh2 = dyi @ q(p["W3"]).T
    dz2 = dh2 * gelu_grad(c["z2"])
    dz2i = q(dz2)
    g["W2"] = c["h1i"].T @ dz2i
    g["b2"] = dz2.sum(0)
    dh1 = dz2i @ q(p["W2"]).T
    dz1 = dh1 * gelu_grad(c["z1"])
    dz1i = q(dz1)
    g["W1"] = c["fi"].T @ dz1i
    g["b1"] = dz1.sum(0)
    return loss, flatten(g)


def adam(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba); step counts from 1.  Returns new
    (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def learned_corrections(tree, theta_l, theta_p, params, G=1.0, gs=64, cluster=1024, chunk=1 << 17,
                        groups=None):
    """The learned walk with no fallback: for every walk group, the cells
    accepted at theta_l but opened at theta_p (the opening test of §3.1 on
    the group's box, FP64) are its learned cells; each of the group's bodies
    gets the network's correction G M s^2 yhat / |x - C|^4 for each of them
    (bfloat16 operands as on the GPU).  Returns a dict: corr [n][3] in
    original order, per_group (learned cells per walk group), and per
    learned (group, cell) pair its group index and the largest predicted
    residual relative to the monopole, |yhat| s^2 / |x - C|^2, over the
    group's bodies (the fallback test's statistic).  `groups` restricts
    the work to those walk-group indices (the others get no corrections)."""
    n = tree.n
    c = tree.cells()
    _, size = tree.root()
    perm = tree.bodies()["perm"]
    xs = tree.pos[perm]
    rcp = tree.mac_radii(theta_p)
    mbar = c["M"][0] / n
    gb, gc = tree.groups(gs, cluster)
    per_group = np.zeros(len(gb), np.int64)
    pairs = []                                        # (group, cell)
    todo = range(len(gb)) if groups is None else sorted(int(g) for g in groups)
    for g in todo:
        b, k = gb[g], gc[g]
        items = tree.walk_items_range(theta_l, b, b + k)
        acc_cells = items[items >= 0]
        if len(acc_cells) == 0:
            continue
        lo, hi = xs[b:b + k].min(0), xs[b:b + k].max(0)
        com = c["com"][acc_cells]
        d = np.maximum(np.maximum(lo[None] - com, 0.0), com - hi[None])
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        lc = acc_cells[~(d2 > rcp[acc_cells])]
        per_group[g] = len(lc)
        pairs.extend((g, int(cl)) for cl in lc)
    corr = np.zeros((n, 3))
    pair_group = np.array([p[0] for p in pairs], np.int64)
    pair_gmax = np.zeros(len(pairs))
    rows, owners, weights, pidx, ratios = [], [], [], [], []

    def run():
        F = np.concatenate(rows)
        y, _ = forward(params, F, bf16_ops=True)
        W = np.concatenate(weights)
        np.add.at(corr, np.concatenate(owners), G * W[:, None] * y)
        nrm = np.sqrt((y * y).sum(1)) * np.concatenate(ratios)
        np.maximum.at(pair_gmax, np.concatenate(pidx), nrm)
        rows.clear(), owners.clear(), weights.clear(), pidx.clear(), ratios.clear()

    held = 0
    for j, (g, cl) in enumerate(pairs):
        b, k = gb[g], gc[g]
        x = xs[b:b + k]
        s = size / 2.0 ** c["level"][cl]
        M = c["M"][cl]
        f = np.zeros((k, 10))
        f[:, :3] = (x - c["com"][cl]) / s
        f[:, 3:9] = c["Q"][cl] / (M * s * s)
        f[:, 9] = math.log(M / mbar)
        rows.append(f.astype(np.float32))
        owners.append(perm[b:b + k])
        dd = x - c["com"][cl]
        d2 = (dd[:, 0] * dd[:, 0] + dd[:, 1] * dd[:, 1]) + dd[:, 2] * dd[:, 2]
        weights.append(M * s * s / (d2 * d2))
        ratios.append(s * s / d2)
        pidx.append(np.full(k, j))
        held += k
        if held >= chunk:
            run()
            held = 0
    if rows:
        run()
    return dict(corr=corr, per_group=per_group, pair_group=pair_group, pair_gmax=pair_gmax)
