"""Parity at the full workload sizes, in the launch configuration the
benchmark times (build, moments, radii, fused walk + force through the C
ABI): trees, groups and interaction counts bit-exact against the oracle over
all bodies, forces on a seeded sample of walk groups within 1e-5 relative L2
(the oracle computes those groups one by one), and the learned walk at
tau = inf on sampled groups."""
import numpy as np
import pytest

import oracle
from oracle import mlp
import workloads
from tests.gpu_util import assert_tree_equal, gpu_tree, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _sampled_parity(w, theta, eps, ngroups=128, seed=300, counts_all=True):
    print(f"{w.name} n={w.n} theta={theta}: GPU", flush=True)
    g = gpu_tree(w.pos, w.mass, w.leaf_cap, theta=theta, G=w.G, eps=eps)
    assert g["status"] == 0
    print("  oracle tree", flush=True)
    t = oracle.Tree(w.pos, w.mass, w.leaf_cap)
    assert_tree_equal(g, t)
    gb, gc = g["gbeg"], g["gcnt"]
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(len(gb), size=min(ngroups, len(gb)), replace=False))
    if counts_all:
        m2p, p2p = t.walk_counts_groups(theta, gb, gc)
        np.testing.assert_array_equal(g["m2p"], m2p)
        np.testing.assert_array_equal(g["p2p"], p2p)
    else:
        m2p, p2p = t.walk_counts_groups(theta, gb[sel], gc[sel])
        np.testing.assert_array_equal(g["m2p"][sel], m2p)
        np.testing.assert_array_equal(g["p2p"][sel], p2p)
    print("  oracle forces on sampled groups", flush=True)
    a, p = t.forces_groups(theta, gb[sel], gc[sel], G=w.G, eps=eps)
    perm = t.bodies()["perm"]
    bodies = np.concatenate([perm[b:b + k] for b, k in zip(gb[sel], gc[sel])])
    ea = oracle.rel_l2(g["acc"][bodies], a[bodies])
    ep = oracle.rel_l2(g["pot"][bodies], p[bodies])
    print(f"  {len(bodies)} sampled bodies: acc {ea:.2e} pot {ep:.2e}", flush=True)
    assert ea < TOL and ep < TOL
    return g, t


@pytest.mark.timeout(300)
def test_plummer_1m():
    w = workloads.plummer_sphere()
    _sampled_parity(w, 0.5, w.eps)


def test_disk_2d_262k():
    w = workloads.gaussian_disk()
    _sampled_parity(w, 0.5, w.eps)


@pytest.mark.timeout(400)
@pytest.mark.parametrize("theta", [0.3, 0.7])
def test_two_plummer_4m(theta):
    w = workloads.two_plummer()
    _sampled_parity(w, theta, w.eps, ngroups=64, counts_all=False)


@pytest.mark.timeout(900)
def test_clustered_16m():
    w = workloads.clustered()
    _sampled_parity(w, 0.7, w.eps, ngroups=64, counts_all=False)


@pytest.mark.timeout(300)
def test_learned_walk_1m_sampled_groups():
    from paper_1211_2293_amd import treecode
    w = workloads.plummer_sphere()
    tc = treecode.Treecode(3, leaf_cap=16)
    keep = (to_dev(w.pos), to_dev(w.mass))
    tc.build(*keep)
    tc.moments()
    p = mlp.unflatten(mlp.init_params(seed=9).astype(np.float64))
    p["W3"] *= 0.2
    theta = mlp.flatten(p).astype(np.float32)
    tc.mlp_load(to_dev(theta))
    acc, _ = tc.forces_learned(0.8, 0.5, float("inf"), eps=w.eps)
    kept, fell = (v.cpu().numpy() for v in tc.learned_counts())
    gb, gc = (v.cpu().numpy() for v in tc.groups())
    t = oracle.Tree(w.pos, w.mass, 16)
    sel = np.sort(np.random.default_rng(301).choice(len(gb), size=24, replace=False))
    ref = mlp.learned_corrections(t, 0.8, 0.5, theta, groups=sel)
    np.testing.assert_array_equal(kept[sel], ref["per_group"][sel])
    assert np.all(fell == 0)
    a, _ = t.forces_groups(0.8, gb[sel], gc[sel], eps=w.eps)
    perm = t.bodies()["perm"]
    bodies = np.concatenate([perm[b:b + k] for b, k in zip(gb[sel], gc[sel])])
    g_acc = acc.cpu().numpy()[bodies]
    corr = oracle.rel_l2(g_acc - a[bodies], ref["corr"][bodies])
    total = oracle.rel_l2(g_acc, a[bodies] + ref["corr"][bodies])
    print(f"learned 1M, {len(bodies)} sampled bodies: corrections {corr:.2e}, total {total:.2e}", flush=True)
    assert corr < 1e-2 and total < 1e-4
