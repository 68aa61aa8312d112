"""Pins of the oracle's walk groups (``orc_groups``): the bodies a walk
shares are runs of at most gs consecutive bodies in key order that never
leave one *cluster cell*, a maximal cell of at most K bodies (or a leaf
holding more, which only bodies with identical keys can form).  The group
walk is this project's reading of the per-body lists of §3.1/§3.2 (one list
per group of bodies); every GPU parity test compares against these groups,
so they are rebuilt here by two independent constructions:

* vectorised numpy from the cell arrays: the cluster cells are the cells
  that qualify and whose parent does not, taken in order of their first
  body and cut into runs from their start;
* for small systems, the naive geometric subdivision (no keys, no sort):
  the maximal qualifying subspaces as sets of bodies.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.test_oracle_tree import CASES


def numpy_groups(t, gs, K):
    c = t.cells()
    count, leaf, parent, begin = c["count"], c["leaf"].astype(bool), c["parent"], c["begin"]
    qual = (count <= K) | leaf
    par_qual = np.zeros_like(qual)
    has_par = parent >= 0
    par_qual[has_par] = qual[parent[has_par]]
    cl = np.flatnonzero(qual & ~par_qual)
    cl = cl[np.argsort(begin[cl], kind="stable")]
    nruns = (count[cl] + gs - 1) // gs
    first = np.repeat(begin[cl], nruns)
    k = np.arange(nruns.sum()) - np.repeat(np.cumsum(nruns) - nruns, nruns)
    gbeg = first + k * gs
    end = np.repeat(begin[cl] + count[cl], nruns)
    gcnt = np.minimum(gbeg + gs, end) - gbeg
    return gbeg, gcnt, cl


def check_groups(t, gs, K):
    gb, gc = t.groups(gs, K)
    nb, nc, cl = numpy_groups(t, gs, K)
    np.testing.assert_array_equal(gb, nb)
    np.testing.assert_array_equal(gc, nc)
    # a partition of the sorted bodies into consecutive runs
    assert gb[0] == 0 and np.all(gb[1:] == gb[:-1] + gc[:-1]) and gb[-1] + gc[-1] == t.n
    assert np.all((gc >= 1) & (gc <= gs))
    # no run straddles two cluster cells; only a cell's last run is short
    c = t.cells()
    lo, hi = c["begin"][cl], c["begin"][cl] + c["count"][cl]
    owner = np.searchsorted(lo, gb, side="right") - 1
    assert np.all(gb + gc <= hi[owner])
    short = gc < gs
    assert np.all(gb[short] + gc[short] == hi[owner[short]])
    # maximality: every cluster cell's parent holds more than K bodies
    par = c["parent"][cl]
    assert np.all((par < 0) | (c["count"][np.maximum(par, 0)] > K))
    return gb, gc


@pytest.mark.parametrize("gs,K", [(64, 1024), (64, 100), (7, 40), (1, 12)])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_groups_equal_numpy_construction(case, gs, K):
    _, gen, lc = case
    pos = gen()
    t = oracle.Tree(pos, np.ones(len(pos)), lc)
    check_groups(t, gs, K)


@pytest.mark.parametrize("gs,K", [(64, 1024), (64, 256), (32, 3000)])
def test_groups_on_a_clustered_mass_spectrum(gs, K):
    w = workloads.clustered(20000, seed=11)
    t = oracle.Tree(w.pos, w.mass, w.leaf_cap)
    gb, gc = check_groups(t, gs, K)
    assert len(gb) > (w.n + gs - 1) // gs          # clusters cut the runs short


@pytest.mark.parametrize("K", [30, 100, 400])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_groups_equal_geometric_cluster_cells(case, K):
    """The cluster cells of the naive subdivision (maximal subspaces of at
    most K bodies, or leaves) are exactly the bodies of consecutive groups."""
    _, gen, lc = case
    pos = gen()
    t = oracle.Tree(pos, np.ones(len(pos)), lc)
    lo, size = t.root()
    cells = oracle.geometric_tree(pos, lc, lo, size, t.L)
    kids = {}
    stack = []                                      # depth-first order: parents precede children
    for idx, (lev, members) in enumerate(cells):
        while stack and cells[stack[-1]][0] >= lev:
            stack.pop()
        kids.setdefault(stack[-1] if stack else -1, []).append(idx)
        stack.append(idx)

    def is_leaf(i):
        return i not in kids

    clusters = []

    def find(i):
        lev, members = cells[i]
        if len(members) <= K or is_leaf(i):
            clusters.append(members)
            return
        for j in kids[i]:
            find(j)

    find(0)
    gb, gc = t.groups(64, K)
    perm = t.bodies()["perm"]
    got = [frozenset(perm[b:b + k].tolist()) for b, k in zip(gb, gc)]
    # consecutive groups, merged while they fill one cluster cell, give the cells in order
    it = iter(got)
    for members in clusters:
        acc = set()
        while len(acc) < len(members):
            g = next(it)
            assert g <= members and not (g & acc)
            acc |= g
        assert acc == members
    assert next(it, None) is None
