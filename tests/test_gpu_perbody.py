"""Per-body interaction lists (the treecode as §3.1 states it: each body
builds its own list, which is then summed) against the oracle's per-body
walk: list lengths bit-exact per body, forces within 1e-5 relative L2, theta
= 0 reproducing the direct sum; and against the grouped walk, which accepts
more conservatively."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1211_2293_amd import treecode
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _run(w, theta, eps, lc=16):
    tc = treecode.Treecode(w.pos.shape[1], leaf_cap=lc)
    keep = (to_dev(w.pos), to_dev(w.mass))
    tc.build(*keep)
    tc.moments()
    tc.walk(theta)
    total, cnt = tc.lists_count(want_counts=True)
    acc, pot, lists = tc.lists_forces(1.0, eps)
    assert tc.status() == treecode.TC_OK
    return tc, total, cnt.cpu().numpy().view(np.uint32), acc.cpu().numpy(), pot.cpu().numpy(), keep


@pytest.mark.parametrize("gen,theta", [("plummer", 0.5), ("plummer", 0.8), ("disk", 0.5), ("clustered", 0.7)])
def test_per_body_lists_match_oracle(gen, theta):
    w = {"plummer": lambda: workloads.plummer_sphere(20000, seed=110),
         "disk": lambda: workloads.gaussian_disk(12000, seed=111),
         "clustered": lambda: workloads.clustered(30000, seed=112)}[gen]()
    eps = 1e-3 if gen == "clustered" else 1e-2
    tc, total, cnt, acc, pot, _ = _run(w, theta, eps)
    t = oracle.Tree(w.pos, w.mass, 16)
    ones = np.ones(w.n, np.int64)
    m2p, p2p = t.walk_counts_groups(theta, np.arange(w.n, dtype=np.int64), ones)
    np.testing.assert_array_equal(cnt.astype(np.int64), m2p + p2p)
    assert total == int((m2p + p2p).sum())
    a, p = t.forces_groups(theta, np.arange(w.n, dtype=np.int64), ones, eps=eps)
    ea, ep = oracle.rel_l2(acc, a), oracle.rel_l2(pot, p)
    # the grouped walk's lists are longer (its test is conservative)
    gb, gc = t.groups(64, 1024)
    gm, gp = t.walk_counts_groups(theta, gb, gc)
    print(f"{gen} theta={theta}: per-body {total / w.n:.0f} entries/body vs grouped "
          f"{((gm + gp) * gc).sum() / w.n:.0f}; acc {ea:.2e} pot {ep:.2e}", flush=True)
    assert ea < 1e-5 and ep < 1e-5
    assert total < ((gm + gp) * gc).sum()


def test_per_body_theta_zero_is_direct_sum():
    w = workloads.plummer_sphere(3000, seed=113)
    tc, total, cnt, acc, pot, _ = _run(w, 0.0, 1e-2)
    assert total == w.n * w.n and np.all(cnt == w.n)
    a, p = oracle.direct(w.pos, w.mass, eps=1e-2)
    assert oracle.rel_l2(acc, a) < 1e-5 and oracle.rel_l2(pot, p) < 1e-5


def test_lists_buffer_too_small_is_rejected():
    w = workloads.plummer_sphere(2000, seed=114)
    tc, total, *_ = _run(w, 0.6, 1e-2)
    small = torch.empty(total - 1, dtype=torch.int32, device="cuda")
    with pytest.raises(treecode.TcError):
        tc.lists_forces(1.0, 1e-2, lists=small)
    # a new walk invalidates the counts
    tc.walk(0.7)
    big = torch.empty(total * 2, dtype=torch.int32, device="cuda")
    with pytest.raises(treecode.TcError):
        tc.lists_forces(1.0, 1e-2, lists=big)
