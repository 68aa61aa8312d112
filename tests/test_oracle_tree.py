"""Pins of the oracle's treecode (§3.1): keys, sort, subdivision, moments,
opening criterion and walk, each checked against something other than the
oracle itself (an independent construction, an invariant, a special case or
brute force)."""
import json
import os

import numpy as np
import pytest

import oracle


def deinterleave(key, dim, L):
    """Independent decoding of a Morton key: level l's digit carries one bit
    per axis, x in the most significant position."""
    q = [0] * dim
    key = int(key)
    for l in range(1, L + 1):
        digit = (key >> (dim * (L - l))) & ((1 << dim) - 1)
        for a in range(dim):
            bit = (digit >> (dim - 1 - a)) & 1
            q[a] |= bit << (L - l)
    return q


def clumps(n, dim, seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, 1, (4, dim))
    k = rng.integers(0, 4, n)
    return c[k] + rng.normal(0, 1e-3, (n, dim)) * (1 + k[:, None])


CASES = [
    ("uniform3", lambda: np.random.default_rng(1).uniform(0, 1, (1000, 3)), 8),
    ("uniform2", lambda: np.random.default_rng(2).uniform(-3, 5, (900, 2)), 4),
    ("clumps3", lambda: clumps(800, 3, 3), 8),
    ("clumps2", lambda: clumps(600, 2, 4), 16),
    ("gauss3_lc1", lambda: np.random.default_rng(5).normal(0, 1, (300, 3)), 1),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    name, gen, lc = request.param
    pos = gen()
    n, dim = pos.shape
    mass = np.random.default_rng(9).uniform(0.5, 1.5, n)
    t = oracle.Tree(pos, mass, lc)
    return pos, mass, lc, t


def test_root_cube_power_of_two(case):
    pos, _, _, t = case
    lo, size = t.root()
    np.testing.assert_array_equal(lo, pos.min(0))
    ext = (pos.max(0) - pos.min(0)).max()
    m, e = np.frexp(size)
    assert m == 0.5                       # a power of two
    assert size >= ext and size / 2 < ext


def test_keys_roundtrip_and_quantisation(case):
    pos, _, _, t = case
    b = t.bodies()
    lo, size = t.root()
    L = t.L
    scale = 2.0 ** L / size
    for i in range(0, t.n, 7):
        q = deinterleave(b["key_orig"][i], t.dim, L)
        for a in range(t.dim):
            off = (pos[i, a] - lo[a]) * scale
            # q is the integer cell of the offset, clamped into the cube
            assert q[a] == min(int(np.floor(off)), 2 ** L - 1)


def test_sort_is_stable_by_key_then_index(case):
    _, _, _, t = case
    b = t.bodies()
    ref = sorted(range(t.n), key=lambda i: (int(b["key_orig"][i]), i))
    np.testing.assert_array_equal(b["perm"], np.array(ref, np.uint32))
    np.testing.assert_array_equal(b["key"], b["key_orig"][b["perm"]])


def test_tree_equals_geometric_subdivision(case):
    pos, _, lc, t = case
    lo, size = t.root()
    geo = oracle.geometric_tree(pos, lc, lo, size, t.L)
    c = t.cells()
    perm = t.bodies()["perm"]
    mine = [(int(c["level"][k]), frozenset(perm[c["begin"][k]:c["begin"][k] + c["count"][k]].tolist()))
            for k in range(t.ncells)]
    assert mine == geo


def test_tree_invariants(case):
    _, mass, lc, t = case
    c = t.cells()
    Cn = t.ncells
    leaf = c["leaf"].astype(bool)
    # every body in exactly one leaf
    hit = np.zeros(t.n, int)
    for k in np.nonzero(leaf)[0]:
        hit[c["begin"][k]:c["begin"][k] + c["count"][k]] += 1
    assert np.all(hit == 1)
    # leaves hold at most leaf_cap bodies unless at the deepest level
    assert np.all((c["count"][leaf] <= lc) | (c["level"][leaf] == t.L))
    # internal cells hold more than leaf_cap bodies and sit above level L
    assert np.all(c["count"][~leaf] > lc) and np.all(c["level"][~leaf] < t.L)
    # children tile their parent, in order, one level deeper
    for k in np.nonzero(~leaf)[0]:
        ch = k + 1
        pos_ = c["begin"][k]
        nk = 0
        while ch < c["skip"][k]:
            assert c["parent"][ch] == k and c["level"][ch] == c["level"][k] + 1
            assert c["begin"][ch] == pos_
            pos_ += c["count"][ch]
            ch = c["skip"][ch]
            nk += 1
        assert pos_ == c["begin"][k] + c["count"][k] and nk == c["nch"][k]
        assert 1 <= nk <= 2 ** t.dim
    assert c["skip"][0] == Cn and c["parent"][0] == -1
    # total mass
    assert abs(c["M"][leaf].sum() - mass.sum()) <= 1e-15 * mass.sum() * 4


def test_moments_equal_direct_sums(case):
    pos, mass, _, t = case
    c = t.cells()
    perm = t.bodies()["perm"]
    for k in range(t.ncells):
        idx = perm[c["begin"][k]:c["begin"][k] + c["count"][k]]
        M = mass[idx].sum()
        com = (mass[idx, None] * pos[idx]).sum(0) / M
        assert abs(c["M"][k] - M) <= 1e-13 * M
        np.testing.assert_allclose(c["com"][k], com, rtol=0, atol=1e-12 * (1 + np.abs(com).max()))
        if t.dim == 3:
            d = pos[idx] - com
            r2 = (d * d).sum(1)
            full = 3 * np.einsum("i,ia,ib->ab", mass[idx], d, d) - np.eye(3) * (mass[idx] * r2).sum()
            ref = np.array([full[0, 0], full[1, 1], full[2, 2], full[0, 1], full[0, 2], full[1, 2]])
            scale = (mass[idx] * r2).sum() + 1e-300
            assert np.abs(c["Q"][k] - ref).max() <= 1e-11 * scale
    # root centre of mass is the global one
    np.testing.assert_allclose(c["com"][0], (mass[:, None] * pos).sum(0) / mass.sum(), atol=1e-13)


def test_single_body_cell_and_two_point_quadrupole(golden_dir):
    with open(os.path.join(golden_dir, "closed_forms.json")) as f:
        g = json.load(f)["two_point_quadrupole"]
    pos = np.array([[-0.5, 0.0, 0.0], [0.5, 0.0, 0.0]])
    t = oracle.Tree(pos, np.ones(2), leaf_cap=2)         # root is the only cell
    c = t.cells()
    assert t.ncells == 1
    np.testing.assert_allclose(c["Q"][0], g["Q"], atol=1e-15)
    t1 = oracle.Tree(pos, np.ones(2), leaf_cap=1)        # one body per leaf
    c1 = t1.cells()
    for k in np.nonzero(c1["count"] == 1)[0]:
        np.testing.assert_array_equal(c1["com"][k], pos[t1.bodies()["perm"][c1["begin"][k]]])
        assert np.all(c1["Q"][k] == 0)


def test_special_keys():
    # one body: key 0, a single leaf
    t = oracle.Tree(np.array([[0.3, 0.2, 0.1]]), np.ones(1), 8)
    assert t.ncells == 1 and t.bodies()["key"][0] == 0
    # the body on the far corner is clamped into the last cell
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    t = oracle.Tree(pos, np.ones(2), 1)
    k = t.bodies()["key_orig"]
    assert k[0] == 0 and k[1] == 2 ** 63 - 1
    # coincident bodies: a chain down to a level-L leaf holding all of them
    t = oracle.Tree(np.full((20, 3), 0.25), np.ones(20), 4)
    c = t.cells()
    assert t.ncells == t.L + 1
    assert c["leaf"][-1] == 1 and c["count"][-1] == 20 and c["level"][-1] == t.L


def test_cells_lie_in_their_cube(case):
    """The cell side s = size / 2^level and the centre used by the opening
    criterion describe a cube that holds every body of the cell."""
    pos, _, _, t = case
    c = t.cells()
    lo, size = t.root()
    perm = t.bodies()["perm"]
    theta = 0.5
    r2 = t.mac_radii(theta)
    for k in range(t.ncells):
        s = size / 2.0 ** c["level"][k]
        idx = perm[c["begin"][k]:c["begin"][k] + c["count"][k]]
        q = np.array([deinterleave(int(c["prefix"][k]) << (t.dim * (t.L - int(c["level"][k]))), t.dim, t.L)])
        origin = lo + q[0] / 2.0 ** t.L * size
        centre = origin + 0.5 * s
        assert np.all(pos[idx] >= origin - 1e-12) and np.all(pos[idx] <= origin + s + 1e-12)
        delta = np.linalg.norm(c["com"][k] - centre)
        assert abs(np.sqrt(r2[k]) - (s / theta + delta)) <= 1e-12 * (s / theta + delta)
    assert np.all(np.isinf(t.mac_radii(0.0)))


def _brute_walk(t, theta, g, gs):
    """Enumerate the opening test for every cell and keep the terminal cells
    whose ancestors are all opened, in pre-order."""
    c = t.cells()
    r2 = t.mac_radii(theta)
    perm = t.bodies()["perm"]
    sorted_pos = t.pos[perm]
    b, e = g * gs, min((g + 1) * gs, t.n)
    lo, hi = sorted_pos[b:e].min(0), sorted_pos[b:e].max(0)
    d = np.maximum(np.maximum(lo[None] - c["com"], 0), c["com"] - hi[None])
    acc = (d * d).sum(1) > r2
    items = []
    for k in range(t.ncells):
        a = c["parent"][k]
        blocked = False
        while a >= 0:
            if acc[a] or c["leaf"][a]:
                blocked = True
                break
            a = c["parent"][a]
        if blocked:
            continue
        if acc[k]:
            items.append(k)
        elif c["leaf"][k]:
            items.append(-1 - k)
    return items


@pytest.mark.parametrize("theta", [0.3, 0.7, 1.0])
def test_walk_matches_brute_force_and_partitions(case, theta):
    _, _, _, t = case
    c = t.cells()
    gs = 64
    G = (t.n + gs - 1) // gs
    m2p, p2p = t.walk_counts(theta, gs)
    for g in range(G):
        items = t.walk_items(theta, g, gs)
        assert list(items) == _brute_walk(t, theta, g, gs)
        cover = np.zeros(t.n, int)
        for it in items:
            k = it if it >= 0 else -1 - it
            cover[c["begin"][k]:c["begin"][k] + c["count"][k]] += 1
        assert np.all(cover == 1)         # every body exactly once
        assert m2p[g] == sum(1 for it in items if it >= 0)
        assert p2p[g] == sum(c["count"][-1 - it] for it in items if it < 0)


@pytest.mark.parametrize("theta", [0.0, 0.5, 0.9])
def test_walk_tests_are_the_terminal_items_and_their_ancestors(case, theta):
    """Cells tested by a group's walk (a work measure): every terminal item
    (accepted cell or opened leaf) and every cell opened on the way to it,
    which are exactly the items' ancestors; at theta = 0 nothing is accepted,
    so every group tests every cell."""
    _, _, _, t = case
    c = t.cells()
    gb, gc = t.groups(64, 1024)
    tests = t.walk_tests_groups(theta, gb, gc)
    if theta == 0.0:
        assert np.all(tests == t.ncells)
    for g in range(len(gb)):
        items = t.walk_items_range(theta, gb[g], gb[g] + gc[g])
        anc = set()
        for it in items:
            k = int(c["parent"][it if it >= 0 else -1 - it])
            while k >= 0 and k not in anc:
                anc.add(k)
                k = int(c["parent"][k])
        assert tests[g] == len(items) + len(anc)


@pytest.mark.parametrize("gs", [64, 1, 7])
def test_theta_zero_reproduces_direct_sum(case, gs):
    pos, mass, _, t = case
    a, p = t.forces(0.0, G=1.0, eps=1e-3, gs=gs)
    b, q = oracle.direct(pos, mass, G=1.0, eps=1e-3)
    assert oracle.rel_l2(a, b) < 1e-13
    assert oracle.rel_l2(p, q) < 1e-13


def test_treecode_error_grows_with_theta():
    """Statistical sanity, not a pin: the approximation error rises with
    theta and stays small at theta = 0.5."""
    rng = np.random.default_rng(21)
    pos = rng.normal(0, 1, (3000, 3))
    mass = np.full(3000, 1.0 / 3000)
    t = oracle.Tree(pos, mass, 8)
    b, _ = oracle.direct(pos, mass, eps=1e-2)
    errs = [oracle.rel_l2(t.forces(th, eps=1e-2)[0], b) for th in (0.2, 0.5, 0.9)]
    assert errs[0] < errs[1] < errs[2]
    assert errs[1] < 5e-3


def test_selected_groups_match_full_forces():
    rng = np.random.default_rng(22)
    pos = rng.uniform(0, 1, (2000, 3))
    mass = rng.uniform(0.5, 1.5, 2000)
    t = oracle.Tree(pos, mass, 8)
    a, p = t.forces(0.6, eps=1e-3)
    sel = [0, 5, 31]
    b, q = t.forces(0.6, eps=1e-3, groups=sel)
    idx = oracle.group_bodies(t, sel)
    np.testing.assert_array_equal(a[idx], b[idx])
    np.testing.assert_array_equal(p[idx], q[idx])


def _pair(R, a=1e-3):
    # two equal bodies at C -+ a x (one tight leaf) and a light target at
    # C + R x; light far bodies keep the tree non-trivial
    C = np.array([0.3, 0.3, 0.3])
    pos = np.array([C - [a, 0, 0], C + [a, 0, 0], C + [R, 0, 0],
                    [0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.0, 1.0, 0.0]])
    mass = np.array([1.0, 1.0, 1e-12, 1e-12, 1e-12, 1e-12])
    return pos, mass


@pytest.mark.parametrize("R", [0.5, 0.6])
def test_quadrupole_term_of_an_equal_pair(R):
    """Seen along its axis from R, a pair of equal masses m at -+a pulls with
    G m [1/(R-a)^2 + 1/(R+a)^2] = (2 G m / R^2)(1 + 3 a^2/R^2 + 5 a^4/R^4 + ...):
    the monopole misses the 3 a^2/R^2 term, the quadrupole expansion of the
    accepted cell recovers it up to O(a^4/R^4)."""
    a = 1e-3
    pos, mass = _pair(R, a)
    t = oracle.Tree(pos, mass, leaf_cap=2)
    p = t.sorted_positions(np.array([2]))
    exact = 1.0 / (R - a) ** 2 + 1.0 / (R + a) ** 2
    err = {}
    for order in (1, 2):
        acc, _ = t.forces_groups(0.9, p, np.array([1]), eps=1e-9, order=order)
        m2p, _ = t.walk_counts_groups(0.9, p, np.array([1]))
        assert m2p[0] >= 1                           # the pair's cell is accepted
        err[order] = (-acc[2, 0] - exact) / exact
    assert abs(err[1] / (-3 * a * a / R ** 2) - 1.0) < 1e-3
    assert abs(err[2]) < 1e-9


def test_quadrupole_force_is_minus_the_potential_gradient():
    """a = -grad phi for the expansion with quadrupole terms (central
    differences of the returned potential; the step is too small to change
    any list)."""
    rng = np.random.default_rng(122)
    pos = rng.normal(size=(800, 3))
    mass = rng.uniform(0.5, 1.5, 800)
    t = oracle.Tree(pos, mass, 8)
    k = 17
    x = pos[k].copy()
    h = 1e-6
    a0, _ = t.forces_groups(0.8, t.sorted_positions(np.array([k])), np.array([1]), eps=1e-2, order=2)
    grad = np.zeros(3)
    for q in range(3):
        ph = []
        for sgn in (1, -1):
            pp = pos.copy()
            pp[k, q] = x[q] + sgn * h
            tt = oracle.Tree(pp, mass, 8)
            _, pot = tt.forces_groups(0.8, tt.sorted_positions(np.array([k])), np.array([1]), eps=1e-2, order=2)
            ph.append(pot[k])
        grad[q] = (ph[0] - ph[1]) / (2 * h)
    np.testing.assert_allclose(a0[k], -grad, rtol=1e-6)


def test_quadrupole_order_leaves_bodies_and_theta_zero_alone():
    rng = np.random.default_rng(121)
    pos = rng.normal(size=(1500, 3))
    mass = rng.uniform(0.5, 1.5, 1500)
    t = oracle.Tree(pos, mass, 8)
    a0, p0 = t.walk_forces(0.0, eps=1e-2, order=2)
    d, dp = oracle.direct(pos, mass, eps=1e-2)
    assert oracle.rel_l2(a0, d) < 1e-12 and oracle.rel_l2(p0, dp) < 1e-12
    # quadrupoles improve the treecode at a fixed opening angle
    a1, _ = t.walk_forces(0.8, eps=1e-2)
    a2, _ = t.walk_forces(0.8, eps=1e-2, order=2)
    assert oracle.rel_l2(a2, d) < 0.5 * oracle.rel_l2(a1, d)
