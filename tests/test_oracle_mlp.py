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
    """The tanh form of GELU: 0 and slope 1/2 at the origin, gelu(z) -
    gelu(-z) = z exactly (tanh is odd), the identity and zero far out,
    within the approximation's 5e-4 of the erf form z Phi(z), and the
    derivative equal to central differences."""
    z = np.linspace(-6.0, 6.0, 2401)
    g = mlp.gelu(z)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15
    np.testing.assert_allclose(g - mlp.gelu(-z), z, rtol=0, atol=1e-15)
    assert abs(mlp.gelu(np.array([12.0]))[0] - 12.0) < 1e-14 and abs(mlp.gelu(np.array([-12.0]))[0]) < 1e-14
    erf_form = np.array([0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in z])
    assert np.abs(g - erf_form).max() < 5e-4
    h = 1e-6
    for v in (-3.0, -1.0, -0.2, 0.5, 2.0):
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
    import workloads
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


def _walk_case():
    import workloads
    w = workloads.plummer_sphere(2500, seed=86)
    t = oracle.Tree(w.pos, w.mass, 16)
    p = mlp.unflatten(mlp.init_params(seed=11).astype(np.float64))
    p["W3"] *= 0.2
    return w, t, mlp.flatten(p)


def _covered_once(t, ent):
    c = t.cells()
    cover = np.zeros(t.n, np.int64)
    for i in np.concatenate(ent):
        cover[c["begin"][i]:c["begin"][i] + c["count"][i]] += 1
    return np.all(cover == 1)


def test_learned_walk_extremes_and_partition():
    """tau = 0: every learned cell falls back and the walk is the plain walk
    at theta_p (forces of the C oracle's group walk); tau = inf: every
    learned cell is kept, the walk is the plain theta_l walk plus the
    corrections of learned_corrections.  At any tau each group's entries
    cover every body exactly once (the fallback replaces a cell by its
    subtree's theta_p items, nothing more, nothing less)."""
    w, t, theta = _walk_case()
    gb, gc = t.groups(64, 1024)
    eps = 1e-2
    r0 = mlp.learned_walk(t, 0.9, 0.5, 0.0, theta, eps=eps)
    a_p, p_p = t.forces_groups(0.5, gb, gc, eps=eps)
    np.testing.assert_allclose(r0["acc"], a_p, rtol=1e-11, atol=1e-11 * np.abs(a_p).max())
    np.testing.assert_allclose(r0["pot"], p_p, rtol=1e-11)
    assert np.all(r0["kept"] == 0) and r0["fell"].sum() > 100
    ri = mlp.learned_walk(t, 0.9, 0.5, np.inf, theta, eps=eps)
    a_l, p_l = t.forces_groups(0.9, gb, gc, eps=eps)
    corr = mlp.learned_corrections(t, 0.9, 0.5, theta)
    np.testing.assert_allclose(ri["acc"], a_l + corr["corr"], rtol=1e-11, atol=1e-11 * np.abs(a_l).max())
    np.testing.assert_allclose(ri["pot"], p_l, rtol=1e-11)
    np.testing.assert_array_equal(ri["kept"], corr["per_group"])
    np.testing.assert_allclose(ri["pair_gmax"], corr["pair_gmax"], rtol=1e-12)
    tau = float(np.median(ri["pair_gmax"]))
    rm = mlp.learned_walk(t, 0.9, 0.5, tau, theta, eps=eps)
    np.testing.assert_array_equal(rm["kept"] + rm["fell"], corr["per_group"])
    fell_ref = np.bincount(ri["pair_group"][ri["pair_gmax"] > tau], minlength=len(gb))
    np.testing.assert_array_equal(rm["fell"], fell_ref)
    assert rm["kept"].sum() > 0 and rm["fell"].sum() > 0
    for r in (r0, ri, rm):
        for g, ent in r["entries"].items():
            assert _covered_once(t, ent), g
    # the mixed walk lies between the two plain walks in cost and error
    d, _ = oracle.direct(w.pos, w.mass, eps=eps)
    e0, em, ei = (oracle.rel_l2(r["acc"], d) for r in (r0, rm, ri))
    print(f"E vs direct: tau=0 {e0:.3e}, median tau {em:.3e}, tau=inf {ei:.3e}")


def test_learned_walk_fallback_of_a_leaf_gives_its_bodies():
    """A learned leaf that falls back contributes its bodies directly (its
    subtree's theta_p items are the opened leaf itself)."""
    w, t, theta = _walk_case()
    r = mlp.learned_walk(t, 0.9, 0.5, 0.0, theta, eps=1e-2)
    c = t.cells()
    leaves = [(g, cl) for g, cl in zip(r["pair_group"], r["pair_cell"]) if c["leaf"][cl]]
    assert leaves
    for g, cl in leaves[:50]:
        cells, opened = r["entries"][g]
        assert cl in opened and cl not in cells
