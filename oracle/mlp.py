"""FP64 reference of the learned closure's network: TEST INFRASTRUCTURE ONLY.

The closure predicts, for a body and an accepted cell, the normalised
residual between the exact sum over the cell's bodies and the cell's
monopole (a small multilayer perceptron 10-64-64-3 with GELU activations,
trained by mean squared error with Adam).  The paper's treecode stops at the
monopole (§3.1); the closure is this project's extension of it.

Network:  z1 = f W1 + b1, h1 = gelu(z1), z2 = h1 W2 + b2, h2 = gelu(z2),
          y = h2 W3 + b3,
          gelu(z) = z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))) / 2,
the tanh form of the Gaussian error linear unit (Hendrycks and Gimpel,
2016), within 5e-4 of z Phi(z) everywhere.
Parameters, canonical flat order (5059 values): W1 [10][64], b1 [64],
W2 [64][64], b2 [64], W3 [64][3], b3 [3].

With ``bf16=True`` the matrix products take bfloat16-rounded operands (round
to nearest, ties to even, applied to an FP32 value) exactly where the GPU
kernels feed their BF16 matrix-core instructions; everything else is FP64.
"""
from __future__ import annotations

import math

import numpy as np

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
    import workloads
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


_GC = math.sqrt(2.0 / math.pi)
_GA = 0.044715


def gelu(z):
    z = np.asarray(z, np.float64)
    return 0.5 * z * (1.0 + np.tanh(_GC * (z + _GA * z ** 3)))


def gelu_grad(z):
    """d gelu / dz: (1 + t)/2 + z (1 - t^2) c (1 + 3 a z^2) / 2 with
    t = tanh(c (z + a z^3))."""
    z = np.asarray(z, np.float64)
    t = np.tanh(_GC * (z + _GA * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * _GC * (1.0 + 3.0 * _GA * z * z)


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


def _soft_sum(xt, ex, em, G, eps):
    """FP64 softened sums at the targets xt [k][3] over the entries (points
    ex [E][3], masses em [E]): acceleration G sum m d / (|d|^2 + eps^2)^(3/2)
    and potential -G sum m / (|d|^2 + eps^2)^(1/2), d = x_e - x_t.  An entry
    at the target itself adds nothing to the acceleration; its potential
    term is left in (the caller removes it)."""
    d = ex[None, :, :] - xt[:, None, :]
    r2 = (d * d).sum(-1) + eps * eps
    inv = 1.0 / np.sqrt(r2)
    w = em[None, :] * inv
    acc = G * ((w * inv * inv)[:, :, None] * d).sum(1)
    pot = -G * w.sum(1)
    return acc, pot


def learned_walk(tree, theta_l, theta_p, tau, params, G=1.0, eps=1e-2, gs=64, cluster=1024, groups=None,
                 chunk=1 << 17):
    """The learned walk with its per-cell fallback, step by step in FP64.

    For every walk group (runs of at most gs sorted bodies inside cluster
    cells of at most `cluster` bodies), the walk at theta_l (the opening test
    of §3.1 on the group's box) gives accepted cells and opened leaves.  An
    accepted cell that the test at theta_p would open is a learned cell: the
    network (bfloat16 operands as on the GPU) predicts yhat for each of the
    group's bodies, and the group's largest |yhat| s^2 / |x - C|^2 is the
    cell's statistic.  If it exceeds tau the cell falls back: its subtree is
    walked at theta_p, i.e. it is replaced by the items of the plain theta_p
    walk that lie in its subtree (every ancestor of a learned cell is opened
    at theta_p as well, since theta_p < theta_l widens the opening radius).
    Otherwise the cell stays a monopole and each body gets G M s^2 yhat /
    |x - C|^4 on top.  Cells accepted at both radii are monopoles, opened
    leaves give their bodies directly.  Forces are FP64 softened sums over
    these entries (self excluded); the potential keeps the monopoles only.

    Returns a dict: acc [n][3], pot [n] (original order; bodies outside
    `groups` zero), kept and fell [groups] (learned cells kept / fallen back
    per walk group), pair_group, pair_cell and pair_gmax per learned
    (group, cell) pair (in group order), and entries: per computed group
    (monopole cells, opened leaves) as pre-order index arrays."""
    n = tree.n
    c = tree.cells()
    _, size = tree.root()
    perm = tree.bodies()["perm"]
    xs = tree.pos[perm]
    ms = tree.mass[perm]
    rcp = tree.mac_radii(theta_p)
    mbar = c["M"][0] / n
    gb, gc = tree.groups(gs, cluster)
    todo = list(range(len(gb))) if groups is None else sorted(int(g) for g in groups)
    walks = {}
    pairs = []                                        # (group, cell), in group order
    for g in todo:
        b, k = int(gb[g]), int(gc[g])
        items_l = tree.walk_items_range(theta_l, b, b + k)
        acc_cells = items_l[items_l >= 0]
        lo, hi = xs[b:b + k].min(0), xs[b:b + k].max(0)
        com = c["com"][acc_cells]
        d = np.maximum(np.maximum(lo[None] - com, 0.0), com - hi[None])
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        learned = acc_cells[~(d2 > rcp[acc_cells])]
        walks[g] = (items_l, learned)
        pairs.extend((g, int(cl)) for cl in learned)
    pair_group = np.array([p[0] for p in pairs], np.int64)
    pair_cell = np.array([p[1] for p in pairs], np.int64)
    pair_gmax = np.zeros(len(pairs))
    pair_corr = {}
    rows, meta = [], []

    def run():
        F = np.concatenate([r[0] for r in rows])
        y, _ = forward(params, F, bf16_ops=True)
        o = 0
        for (_, w, ratio), (j, b, k) in zip(rows, meta):
            yy = y[o:o + k]
            o += k
            pair_gmax[j] = float((np.sqrt((yy * yy).sum(1)) * ratio).max())
            pair_corr[j] = G * w[:, None] * yy
        rows.clear(), meta.clear()

    held = 0
    for j, (g, cl) in enumerate(pairs):
        b, k = int(gb[g]), int(gc[g])
        x = xs[b:b + k]
        s = size / 2.0 ** c["level"][cl]
        M = c["M"][cl]
        f = np.zeros((k, 10))
        f[:, :3] = (x - c["com"][cl]) / s
        f[:, 3:9] = c["Q"][cl] / (M * s * s)
        f[:, 9] = math.log(M / mbar)
        dd = x - c["com"][cl]
        d2 = (dd[:, 0] * dd[:, 0] + dd[:, 1] * dd[:, 1]) + dd[:, 2] * dd[:, 2]
        rows.append((f.astype(np.float32), M * s * s / (d2 * d2), s * s / d2))
        meta.append((j, b, k))
        held += k
        if held >= chunk:
            run()
            held = 0
    if rows:
        run()

    acc = np.zeros((n, 3))
    pot = np.zeros(n)
    kept = np.zeros(len(gb), np.int64)
    fell = np.zeros(len(gb), np.int64)
    entries = {}
    first_pair = np.searchsorted(pair_group, todo)       # pairs are in group order
    for gi, g in enumerate(todo):
        b, k = int(gb[g]), int(gc[g])
        items_l, learned = walks[g]
        j0 = int(first_pair[gi])
        gm = pair_gmax[j0:j0 + len(learned)]
        falls = np.sort(learned[gm > tau])
        keep_j = j0 + np.flatnonzero(~(gm > tau))
        cells = items_l[items_l >= 0]
        cells = cells[~np.isin(cells, falls)]
        leaves = -1 - items_l[items_l < 0]
        if len(falls):
            items_p = tree.walk_items_range(theta_p, b, b + k)
            cc = np.where(items_p >= 0, items_p, -1 - items_p)
            slot = np.searchsorted(falls, cc, side="right") - 1
            inside = (slot >= 0) & (cc < c["skip"][falls[np.maximum(slot, 0)]])
            cells = np.concatenate([cells, items_p[inside & (items_p >= 0)]])
            leaves = np.concatenate([leaves, cc[inside & (items_p < 0)]])
        kept[g] = len(keep_j)
        fell[g] = len(falls)
        entries[g] = (cells, leaves)
        nb = c["count"][leaves]
        bodies = np.repeat(c["begin"][leaves] - np.cumsum(nb) + nb, nb) + np.arange(nb.sum())
        ex = np.concatenate([c["com"][cells], xs[bodies]])
        em = np.concatenate([c["M"][cells], ms[bodies]])
        a, p = _soft_sum(xs[b:b + k], ex, em, G, eps)
        p += G * ms[b:b + k] / eps                        # the body's own term
        for j in keep_j:
            a += pair_corr[j]
        acc[perm[b:b + k]] = a
        pot[perm[b:b + k]] = p
    return dict(acc=acc, pot=pot, kept=kept, fell=fell, pair_group=pair_group, pair_cell=pair_cell,
                pair_gmax=pair_gmax, entries=entries)
