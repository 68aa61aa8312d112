"""Pins of the learned-closure oracle: bfloat16 rounding against the
library cast, the analytic gradient against central finite differences,
GELU against its closed form, and the residual against special cases
(a one-body cell has no residual; two equal bodies approach the analytic
quadrupole term)."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp


def test_bf16_matches_library_cast():
    rng = np.random.default_rng(80)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.uniform(-5, 5, 4000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 3.0e38]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert mlp.bf16(np.float32(1.0 + 2 ** -8)) == 1.0


def test_gelu_closed_form():
    z = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    ref = np.array([0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in z])
    np.testing.assert_allclose(mlp.gelu(z), ref, rtol=1e-15)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15
    h = 1e-6
    for v in z:
        fd = (mlp.gelu(np.array([v + h]))[0] - mlp.gelu(np.array([v - h]))[0]) / (2 * h)
        assert abs(fd - mlp.gelu_grad(np.array([v]))[0]) < 1e-8


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(81)
    theta = mlp.init_params(seed=3).astype(np.float64)
    f = rng.normal(size=(37, 10))
    y = rng.normal(size=(37, 3)) * 0.1
    loss, g = mlp.loss_and_grad(theta, f, y)
    h = 1e-6
    idx = np.concatenate([rng.choice(mlp.NPARAM, 60, replace=False), [0, 639, 640, 4800, 5056, 5058]])
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, f, y)[0] - mlp.loss_and_grad(tm, f, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_forward_is_close_to_fp64():
    rng = np.random.default_rng(82)
    theta = mlp.init_params(seed=4)
    f = rng.normal(size=(100, 10))
    y64, _ = mlp.forward(theta, f, bf16_ops=False)
    y16, _ = mlp.forward(theta, f, bf16_ops=True)
    assert oracle.rel_l2(y16, y64) < 2e-2          # 8-bit mantissas
    assert oracle.rel_l2(y16, y64) > 0             # the emulation does round


def test_adam_first_step_moves_by_lr():
    theta = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 1e-3, 0.0])
    t1, m, v = mlp.adam(theta, g, np.zeros(5), np.zeros(5), 1, lr=1e-3)
    # bias-corrected first step: -lr * g / (|g| + eps)
    np.testing.assert_allclose(t1[:4], -1e-3 * np.sign(g[:4]), rtol=1e-4)
    assert t1[4] == 0.0


def _pair_tree(R, a=1e-3):
    # two equal bodies at C +- a x (a tight leaf) and a target at C + R x;
    # a few far bodies keep the tree non-trivial
    C = np.array([0.3, 0.3, 0.3])         # off the coarse subdivision planes
    pos = np.array([C - [a, 0, 0], C + [a, 0, 0], C + [R, 0, 0],
                    [0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.0, 1.0, 0.0]])
    mass = np.array([1.0, 1.0, 1e-9, 1e-9, 1e-9, 1e-9])
    return pos, mass


@pytest.mark.parametrize("R", [0.5, 0.6])
def test_two_body_cell_approaches_quadrupole(R):
    a = 1e-3
    pos, mass = _pair_tree(R, a)
    t = oracle.Tree(pos, mass, leaf_cap=2)
    r = t.residuals(0.9, 1e-9, np.array([2]))
    c = t.cells()
    # the accepted cell holding both heavy bodies
    k = [i for i, cl in enumerate(r["cell"]) if c["M"][cl] > 1.5]
    assert len(k) == 1
    y = r["y"][k[0]]
    # exact minus monopole along the axis: 6 G m a^2 / R^4 toward the pair,
    # in units of the quadrupole scale G M s^2 / R^4 with M = 2m: 3 a^2 / s^2,
    # pointing to -x
    lo, size = t.root()
    s = size / 2.0 ** c["level"][r["cell"][k[0]]]
    ref = 3.0 * a * a / (s * s)
    assert abs(-y[0] / ref - 1.0) < 1e-3 * (1 + (a / R) ** 2 * 1e3)
    assert abs(y[1]) < 1e-12 and abs(y[2]) < 1e-12


def test_one_body_cell_has_no_residual():
    rng = np.random.default_rng(83)
    pos = rng.uniform(0, 1, (300, 3))
    mass = rng.uniform(0.5, 1.5, 300)
    t = oracle.Tree(pos, mass, leaf_cap=1)
    r = t.residuals(0.7, 1e-2, np.arange(0, 300, 17))
    c = t.cells()
    single = c["count"][r["cell"]] == 1
    assert single.any()
    assert np.abs(r["y"][single]).max() < 1e-12


def test_pairs_are_the_per_body_walk():
    rng = np.random.default_rng(84)
    pos = rng.normal(size=(2000, 3))
    mass = rng.uniform(0.5, 1.5, 2000)
    t = oracle.Tree(pos, mass, leaf_cap=8)
    targets = np.array([0, 5, 1999, 777])
    r = t.residuals(0.8, 1e-2, targets)
    tpos = t.sorted_positions(targets)
    m2p, _ = t.walk_counts_groups(0.8, tpos, np.ones(len(tpos), np.int64))
    np.testing.assert_array_equal(r["count"], m2p)
    # features: displacement over the cell side and the mass ratio
    c = t.cells()
    lo, size = t.root()
    for k in range(0, len(r["cell"]), 97):
        cl = r["cell"][k]
        p = targets[r["target"][k]]
        s = size / 2.0 ** c["level"][cl]
        np.testing.assert_allclose(r["feat"][k, :3], (pos[p] - c["com"][cl]) / s, rtol=1e-6, atol=1e-7)
        assert abs(r["feat"][k, 9] - math.log(c["M"][cl] / (mass.sum() / 2000))) < 1e-5


def test_learned_corrections_with_a_constant_network():
    """With W3 = 0 and b3 = (1, 0, 0) every prediction is (1, 0, 0); with
    theta_p = 0 every cell the theta_l walk accepts is learned, so the x
    correction of a body is the sum of M s^2 / |x - C|^4 over the accepted
    cells of its group's walk (brute force from the walk items)."""
    from paper_1211_2293_amd import workloads
    w = workloads.plummer_sphere(1500, seed=85)
    t = oracle.Tree(w.pos, w.mass, 8)
    p = mlp.unflatten(mlp.init_params(seed=10).astype(np.float64))
    p["W3"][:] = 0.0
    p["b3"][:] = [1.0, 0.0, 0.0]
    r = mlp.learned_corrections(t, 0.7, 0.0, mlp.flatten(p), G=2.0)
    c = t.cells()
    perm = t.bodies()["perm"]
    gb, gc = t.groups(64, 1024)
    _, size = t.root()
    ref = np.zeros(w.n)
    gmax = []
    for g, (b, k) in enumerate(zip(gb, gc)):
        items = t.walk_items_range(0.7, b, b + k)
        acc_cells = items[items >= 0]
        assert r["per_group"][g] == len(acc_cells)
        s2 = (size / 2.0 ** c["level"][acc_cells]) ** 2
        ratio = np.zeros(len(acc_cells))
        for i in perm[b:b + k]:
            d = w.pos[i][None] - c["com"][acc_cells]
            d2 = (d * d).sum(1)
            ref[i] = 2.0 * (c["M"][acc_cells] * s2 / d2 ** 2).sum()
            ratio = np.maximum(ratio, s2 / d2)
        gmax.append(ratio)
    np.testing.assert_allclose(r["corr"][:, 0], ref, rtol=1e-12)
    assert np.all(r["corr"][:, 1:] == 0.0)
    # the fallback statistic: the largest |yhat| s^2 / d^2 over the group
    np.testing.assert_allclose(r["pair_gmax"], np.concatenate(gmax), rtol=1e-12)
    # theta_p close to theta_l leaves few learned cells, never more
    r2 = mlp.learned_corrections(t, 0.7, 0.69, mlp.flatten(p))
    assert np.all(r2["per_group"] <= r["per_group"]) and r2["per_group"].sum() < r["per_group"].sum()
