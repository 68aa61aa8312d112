"""GPU walk + force summation vs the oracle at the same theta and grouping:
interaction counts identical, accelerations and potentials within 1e-5
relative L2; theta = 0 reproduces the FP64 direct sum; results are
bit-reproducible run to run (§3.1 force law and walk)."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import gpu_tree

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _check_against_oracle(pos, mass, lc, theta, eps, G=1.0, split=None, t=None):
    tc = None
    if split is not None:
        from paper_1211_2293_amd import treecode
        tc = treecode.Treecode(pos.shape[1], leaf_cap=lc)
        tc.set_split(split)
    g = gpu_tree(pos, mass, lc, theta=theta, G=G, eps=eps, tc=tc)
    assert g["status"] == 0
    if t is None:
        t = oracle.Tree(pos.astype(np.float64), np.asarray(mass, np.float64), lc)
    gb, gc = t.groups(64, 1024)
    np.testing.assert_array_equal(g["gbeg"], gb)
    np.testing.assert_array_equal(g["gcnt"], gc)
    m2p, p2p = t.walk_counts_groups(theta, gb, gc)
    np.testing.assert_array_equal(g["m2p"], m2p)
    np.testing.assert_array_equal(g["p2p"], p2p)
    np.testing.assert_array_equal(g["tests"], t.walk_tests_groups(theta, gb, gc))
    a, p = t.forces_groups(theta, gb, gc, G=G, eps=eps)
    ea, ep = oracle.rel_l2(g["acc"], a), oracle.rel_l2(g["pot"], p)
    print(f"n={len(pos)} theta={theta}: acc {ea:.2e} pot {ep:.2e} "
          f"interactions/body {((m2p + p2p) * gc).sum() / len(pos):.0f}", flush=True)
    assert ea < TOL and ep < TOL
    return g, t


@pytest.mark.parametrize("theta", [0.0, 0.3, 0.5, 0.8, 1.0])
def test_uniform_cube_fp64_state(theta):
    w = workloads.uniform_cube(4096)
    _check_against_oracle(w.pos, w.mass, w.leaf_cap, theta, w.eps)


def test_disk_2d_fp64_state():
    """FP64 positions and masses in 2D (the FP64 key path and the bodies
    without an FP32 copy), as the FP64 cube does in 3D."""
    pos = np.random.default_rng(68).normal(0.0, 1.0, (5000, 2))      # FP64, not FP32-rounded
    _check_against_oracle(pos, np.full(5000, 1.0 / 5000), 8, 0.5, 1e-2)


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.7, 0.9])
def test_plummer(theta):
    w = workloads.plummer_sphere(30000, seed=60)
    _check_against_oracle(w.pos, w.mass, 16, theta, 1e-2)


@pytest.mark.parametrize("theta", [0.0, 0.5, 0.8])
def test_disk_2d(theta):
    w = workloads.gaussian_disk(10000, seed=61)
    _check_against_oracle(w.pos, w.mass, 16, theta, 1e-2)


@pytest.mark.parametrize("dim,lc", [(3, 1), (3, 3), (3, 32), (3, 64), (3, 100), (3, 256), (2, 1), (2, 64)])
def test_leaf_caps_in_both_walk_kernels(dim, lc):
    """Leaf sizes from 1 to the largest allowed: the walk copies the bodies of
    unaccepted leaves with the next power of two of leaf_cap lanes per leaf
    (at most 64), larger leaves in rounds of 64, and the list fills and
    flushes at other points.  Shared walks (the default at this size) and
    one wave per group (split mode 0) against the oracle."""
    w = workloads.plummer_sphere(20000, seed=66) if dim == 3 else workloads.gaussian_disk(20000, seed=67)
    t = oracle.Tree(w.pos.astype(np.float64), w.mass.astype(np.float64), lc)
    for split in (1, 0):
        _check_against_oracle(w.pos, w.mass, lc, 0.6, 1e-2, split=split, t=t)


def test_clustered_pareto_masses():
    w = workloads.clustered(40000, seed=62)
    _check_against_oracle(w.pos, w.mass, 16, 0.7, 1e-3)


def test_ragged_and_tiny_sizes():
    rng = np.random.default_rng(63)
    for n in (1, 2, 63, 64, 65, 130, 1000):
        pos = rng.uniform(0, 1, (n, 3)).astype(np.float32)
        mass = rng.uniform(0.5, 1.5, n).astype(np.float32)
        g = gpu_tree(pos, mass, 8, theta=0.6, eps=1e-2)
        a, p = oracle.direct(pos, mass, eps=1e-2) if n <= 2 else oracle.Tree(pos, mass, 8).walk_forces(0.6, eps=1e-2)
        if n == 1:
            assert np.all(g["acc"] == 0) and np.all(g["pot"] == 0)
            continue
        assert oracle.rel_l2(g["acc"], a) < TOL and oracle.rel_l2(g["pot"], p) < TOL


def test_theta_zero_is_direct_sum():
    w = workloads.plummer_sphere(12000, seed=64)
    g = gpu_tree(w.pos, w.mass, 16, theta=0.0, eps=1e-2)
    a, p = oracle.direct(w.pos, w.mass, eps=1e-2)
    assert oracle.rel_l2(g["acc"], a) < TOL
    assert oracle.rel_l2(g["pot"], p) < TOL
    # every group's list is all n bodies
    assert np.all(g["m2p"] == 0) and np.all(g["p2p"] == len(w.pos))
    assert g["gcnt"].sum() == len(w.pos)


def test_coincident_bodies_and_oversized_leaf():
    # 2000 identical keys: one level-L leaf larger than the LDS list
    n = 2000
    pos = np.full((n, 3), 0.25, np.float32)
    pos[:10] += np.linspace(0.1, 0.5, 10)[:, None].astype(np.float32)
    mass = np.ones(n, np.float32) / n
    g = gpu_tree(pos, mass, 8, theta=0.5, eps=1e-3)
    a, p = oracle.Tree(pos, mass, 8).walk_forces(0.5, eps=1e-3)
    assert np.abs(g["acc"] - a).max() <= 1e-5 * np.abs(a).max()
    assert oracle.rel_l2(g["pot"], p) < TOL


def test_bodies_on_cell_faces():
    rng = np.random.default_rng(65)
    pos = (rng.integers(0, 17, (3000, 3)) / 16.0).astype(np.float32)
    pos = np.unique(pos, axis=0)
    mass = np.ones(len(pos), np.float32)
    _check_against_oracle(pos, mass, 4, 0.5, 1e-2)


def test_deterministic():
    w = workloads.plummer_sphere(50000, seed=66)
    g1 = gpu_tree(w.pos, w.mass, 16, theta=0.5, eps=1e-2)
    g2 = gpu_tree(w.pos, w.mass, 16, theta=0.5, eps=1e-2)
    np.testing.assert_array_equal(g1["acc"], g2["acc"])
    np.testing.assert_array_equal(g1["pot"], g2["pot"])


@pytest.mark.parametrize("wl", ["plummer", "disk", "plummer-200k"])
def test_schedule_does_not_change_results(wl):
    """The persistent waves take the groups in an order set by the previous
    evaluation's per-body list lengths; a group's walk and sums do not depend
    on it, so results are bitwise the same whatever ran before: a fresh
    context (no costs yet), costs from the same problem, and stale costs
    from a permuted copy of it."""
    from paper_1211_2293_amd import treecode
    from tests.gpu_util import to_dev
    # (60,000 bodies: the shared walks; 200,000: one wave per group)
    w = (workloads.plummer_sphere(60000, seed=79) if wl == "plummer" else
         workloads.gaussian_disk(60000, seed=80) if wl == "disk" else workloads.plummer_sphere(200000, seed=82))
    tc = treecode.Treecode(w.dim, leaf_cap=16)

    def run(pos, mass):
        p, m = to_dev(pos), to_dev(mass)
        tc.build(p, m)
        tc.moments()
        tc.walk(0.5)
        acc, pot = tc.forces(1.0, 1e-2)
        m2p, p2p = tc.counts()
        return [v.cpu().numpy() for v in (acc, pot, m2p, p2p)]

    first = run(w.pos, w.mass)
    again = run(w.pos, w.mass)
    shuffle = np.random.default_rng(81).permutation(w.n)
    run(w.pos[shuffle], w.mass[shuffle])
    stale = run(w.pos, w.mass)
    for x, y, z in zip(first, again, stale):
        np.testing.assert_array_equal(x, y)
        np.testing.assert_array_equal(x, z)


def test_G_scales_linearly():
    w = workloads.plummer_sphere(5000, seed=67)
    g1 = gpu_tree(w.pos, w.mass, 16, theta=0.5, eps=1e-2, G=1.0)
    g2 = gpu_tree(w.pos, w.mass, 16, theta=0.5, eps=1e-2, G=2.5)
    np.testing.assert_allclose(g2["acc"], 2.5 * g1["acc"], rtol=1e-6, atol=0)


@pytest.mark.parametrize("theta", [0.5, 0.8])
def test_quadrupole_cells_match_oracle(theta):
    """Accepted cells with their quadrupole term (tc_set_multipole(2)):
    the same walk and counts, forces within 1e-5 of the oracle's second-order
    expansion, and closer to the direct sum than the monopole walk."""
    import torch
    from paper_1211_2293_amd import treecode
    from tests.gpu_util import to_dev
    w = workloads.plummer_sphere(30000, seed=65)
    tc = treecode.Treecode(3, leaf_cap=16)
    keep = (to_dev(w.pos), to_dev(w.mass))
    tc.build(*keep)
    tc.moments()
    tc.walk(theta)
    a1, _ = tc.forces(1.0, 1e-2)
    a1 = a1.cpu().numpy()
    tc.set_multipole(2)
    acc, pot = tc.forces(1.0, 1e-2)
    m2p, p2p = (v.cpu().numpy() for v in tc.counts())
    t = oracle.Tree(w.pos, w.mass, 16)
    gb, gc = t.groups(64, 1024)
    rm2p, rp2p = t.walk_counts_groups(theta, gb, gc)
    np.testing.assert_array_equal(m2p, rm2p)
    np.testing.assert_array_equal(p2p, rp2p)
    a, p = t.forces_groups(theta, gb, gc, eps=1e-2, order=2)
    ea, ep = oracle.rel_l2(acc.cpu().numpy(), a), oracle.rel_l2(pot.cpu().numpy(), p)
    s = workloads.sample_indices(w.n, 2000, seed=66)
    d, _ = oracle.direct(w.pos, w.mass, eps=1e-2, targets=s)
    e1, e2 = oracle.rel_l2(a1[s], d), oracle.rel_l2(acc.cpu().numpy()[s], d)
    print(f"theta={theta}: quadrupole vs oracle acc {ea:.2e} pot {ep:.2e}; E vs direct monopole {e1:.2e} "
          f"quadrupole {e2:.2e}", flush=True)
    assert ea < 1e-5 and ep < 1e-5
    assert e2 < 0.5 * e1
    tc.set_multipole(1)
    b1, _ = tc.forces(1.0, 1e-2)
    np.testing.assert_array_equal(b1.cpu().numpy(), a1)


@pytest.mark.parametrize("case", ["plummer", "disk", "disk-small", "root-leaf", "quadrupole", "plummer-mid",
                                  "disk-mid", "quadrupole-mid"])
def test_shared_walks_match_one_wave(case):
    """Walks spread over several waves against one wave per group: split
    walks (tc_set_split mode 2, small n: one task per level-1 cell and
    child) and walks shared by a block of waves (mode 1, the default: the
    cells of one level dealt out); the interactions and counts must equal
    the one-wave walk's and the forces agree to summation order."""
    from paper_1211_2293_amd import treecode
    from tests.gpu_util import to_dev
    # split walks exist up to 12,288 bodies in 3D and 24,576 in 2D; shared
    # walks up to 163,840, by eight waves per group up to 36,000 bodies
    # (without quadrupole lists) and by four above
    w = {"plummer": lambda: workloads.plummer_sphere(12000, seed=67),
         "disk": lambda: workloads.gaussian_disk(24000, seed=68),
         "disk-small": lambda: workloads.gaussian_disk(16000, seed=84),
         "root-leaf": lambda: workloads.plummer_sphere(12, seed=69),
         "quadrupole": lambda: workloads.plummer_sphere(12000, seed=67),
         "plummer-mid": lambda: workloads.plummer_sphere(100000, seed=82),
         "disk-mid": lambda: workloads.gaussian_disk(100000, seed=83),
         "quadrupole-mid": lambda: workloads.plummer_sphere(40000, seed=82)}[case]()
    tc = treecode.Treecode(w.pos.shape[1], leaf_cap=16)
    keep = (to_dev(w.pos), to_dev(w.mass))
    tc.build(*keep)
    tc.moments()
    tc.walk(0.6)
    if case.startswith("quadrupole"):
        tc.set_multipole(2)
    out = {}
    for mode in (0, 1, 2):
        tc.set_split(mode)
        acc, pot = tc.forces(1.0, 1e-2)
        m2p, p2p = (v.cpu().numpy() for v in tc.counts())
        if mode == 2 and w.n <= (12288 if w.dim == 3 else 24576):
            with pytest.raises(treecode.TcError):     # split walks keep no tested-cell counts
                tc.tests()
            tests = None
        else:
            tests = tc.tests().cpu().numpy()
        out[mode] = (acc.cpu().numpy(), pot.cpu().numpy(), m2p, p2p, tests)
    # cells tested: a shared walk's parts test each cell once between them
    np.testing.assert_array_equal(out[1][4], out[0][4])
    for mode in (1, 2):
        np.testing.assert_array_equal(out[mode][2], out[0][2])
        np.testing.assert_array_equal(out[mode][3], out[0][3])
        ea, ep = oracle.rel_l2(out[mode][0], out[0][0]), oracle.rel_l2(out[mode][1], out[0][1])
        print(f"{case}: mode {mode} vs one wave acc {ea:.2e} pot {ep:.2e}", flush=True)
        assert ea < 2e-6 and ep < 2e-6
        # run-to-run identical
        tc.set_split(mode)
        again, _ = tc.forces(1.0, 1e-2)
        np.testing.assert_array_equal(again.cpu().numpy(), out[mode][0])


@pytest.mark.parametrize("dim", [3, 2])
def test_plain_accumulation_in_shared_walks(dim):
    """The uncompensated running sums of the precision study, in the walk
    shared by a block of waves (the default below 163,840 bodies): counts
    as in the oracle, forces within the parity bound."""
    from paper_1211_2293_amd import treecode
    from tests.gpu_util import to_dev
    w = workloads.plummer_sphere(30000, seed=84) if dim == 3 else workloads.gaussian_disk(30000, seed=85)
    tc = treecode.Treecode(dim, leaf_cap=16)
    tc.build(to_dev(w.pos), to_dev(w.mass))
    tc.moments()
    tc.walk(0.6)
    tc.set_accumulation(False)
    acc, pot = tc.forces(1.0, 1e-2)
    m2p, p2p = (v.cpu().numpy() for v in tc.counts())
    gb, gc = (v.cpu().numpy() for v in tc.groups())
    t = oracle.Tree(w.pos.astype(np.float64), w.mass.astype(np.float64), 16)
    om, op = t.walk_counts_groups(0.6, gb, gc)
    np.testing.assert_array_equal(m2p, om)
    np.testing.assert_array_equal(p2p, op)
    a, p = t.forces_groups(0.6, gb, gc, G=1.0, eps=1e-2)
    ea, ep = oracle.rel_l2(acc.cpu().numpy(), a), oracle.rel_l2(pot.cpu().numpy(), p)
    print(f"dim={dim} plain accumulation: acc {ea:.2e} pot {ep:.2e}", flush=True)
    assert ea < TOL and ep < TOL


def test_shared_walk_at_its_largest_size():
    """163,840 bodies, the largest size that shares a group's walk among a
    block of waves: interaction counts equal to the oracle's and forces
    within the parity bound."""
    w = workloads.plummer_sphere(163840, seed=86)
    _check_against_oracle(w.pos, w.mass, 16, 0.5, w.eps)
