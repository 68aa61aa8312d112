"""GPU fast multipole method vs the oracle's: the dual tree traversal's pairs
identical as sets (grouped by target on the GPU), accelerations and
potentials within 1e-5 relative L2, theta = 0 equal to the FP64 direct sum,
results bit-reproducible, and the degenerate trees (one body, coincident
bodies, a leaf wider than a wave)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1211_2293_amd import treecode

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _gpu_fmm(pos, mass, lc, theta, eps, G=1.0):
    dev = torch.device("cuda:0")
    dt = torch.float64 if pos.dtype == np.float64 else torch.float32
    p = torch.from_numpy(np.ascontiguousarray(pos)).to(dev, dt)
    m = torch.from_numpy(np.ascontiguousarray(mass)).to(dev, dt)
    tc = treecode.Treecode(3, leaf_cap=lc)
    tc.build(p, m)
    tc.moments()
    sizes = tc.fmm_plan(theta)
    acc, pot = tc.fmm_forces(G, eps)
    m2l, p2p = tc.fmm_pairs(sizes)
    torch.cuda.synchronize()
    assert tc.status() == 0
    return tc, sizes, acc.cpu().numpy(), pot.cpu().numpy(), m2l.cpu().numpy(), p2p.cpu().numpy()


def _sorted_pairs(a):
    a = np.asarray(a, np.int64)
    return a[np.lexsort((a[:, 1], a[:, 0]))] if len(a) else a.reshape(0, 2)


def _check(pos, mass, lc, theta, eps, G=1.0):
    print(f"case n={len(pos)} theta={theta} leaf_cap={lc}", flush=True)
    tc, sizes, acc, pot, m2l, p2p = _gpu_fmm(pos, mass, lc, theta, eps, G)
    t = oracle.Tree(np.asarray(pos, np.float64), np.asarray(mass, np.float64), lc)
    om, op = oracle.fmm_pairs(t, theta)
    # grouped by target on the GPU; the same sets
    assert np.all(np.diff(m2l[:, 0]) >= 0) and np.all(np.diff(p2p[:, 0]) >= 0)
    np.testing.assert_array_equal(_sorted_pairs(m2l), _sorted_pairs(om))
    np.testing.assert_array_equal(_sorted_pairs(p2p), _sorted_pairs(op))
    a, p = oracle.fmm_forces(t, theta, G=G, eps=eps)
    ea, ep = oracle.rel_l2(acc, a), oracle.rel_l2(pot, p)
    print(f"  m2l {sizes[1]} p2p {sizes[2]} widest level {sizes[0]}: acc {ea:.2e} pot {ep:.2e}", flush=True)
    assert ea < TOL and ep < TOL
    return tc, acc, pot


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.8])
def test_plummer(theta):
    w = workloads.plummer_sphere(20000, seed=70)
    _check(w.pos, w.mass, 16, theta, 1e-2)


def test_uniform_cube_fp64_state():
    w = workloads.uniform_cube(4096)
    _check(w.pos, w.mass, w.leaf_cap, 0.5, w.eps)


def test_clustered_pareto_masses():
    w = workloads.clustered(30000, seed=71)
    _check(w.pos, w.mass, 16, 0.6, 1e-3, G=2.0)


def test_long_partner_lists_are_split():
    # a dense clump and a few bodies spread around it: leaves with thousands
    # of direct partners, whose sums are cut into chunks on the GPU
    rng = np.random.default_rng(77)
    w = workloads.plummer_sphere(20000, seed=77)
    pos = np.concatenate([w.pos * 0.05, rng.uniform(0.5, 1.5, (6, 3))]).astype(np.float32)
    mass = np.full(len(pos), 1.0 / len(pos), np.float32)
    t = oracle.Tree(pos.astype(np.float64), mass.astype(np.float64), 16)
    _, op = oracle.fmm_pairs(t, 0.3)
    assert np.bincount(op[:, 0]).max() > 4 * 256      # several chunks for some leaves
    _check(pos, mass, 16, 0.3, 1e-3)


def test_theta_zero_is_the_direct_sum():
    w = workloads.plummer_sphere(5000, seed=72)
    _, sizes, acc, pot, m2l, _ = _gpu_fmm(w.pos, w.mass, 16, 0.0, 1e-2)
    assert sizes[1] == 0 and len(m2l) == 0
    a, p = oracle.direct(w.pos, w.mass, eps=1e-2)
    assert oracle.rel_l2(acc, a) < TOL and oracle.rel_l2(pot, p) < TOL


def test_reproducible_and_replanned():
    w = workloads.plummer_sphere(20000, seed=73)
    _, _, a1, p1, _, _ = _gpu_fmm(w.pos, w.mass, 16, 0.5, 1e-2)
    tc, _, a2, p2, _, _ = _gpu_fmm(w.pos, w.mass, 16, 0.5, 1e-2)
    np.testing.assert_array_equal(a1, a2)
    np.testing.assert_array_equal(p1, p2)
    # a new tree and a new theta in the same context and buffer
    dev = torch.device("cuda:0")
    pos2 = (w.pos * 1.5 + 0.25).astype(np.float32)
    tc.build(torch.from_numpy(pos2).to(dev), torch.from_numpy(w.mass).to(dev))
    tc.moments()
    with pytest.raises(treecode.TcError):
        tc.fmm_forces(1.0, 1e-2)            # the old plan died with the old tree
    tc.fmm_plan(0.7)
    acc, pot = tc.fmm_forces(1.0, 1e-2)
    t = oracle.Tree(pos2.astype(np.float64), w.mass.astype(np.float64), 16)
    a, p = oracle.fmm_forces(t, 0.7, eps=1e-2)
    assert oracle.rel_l2(acc.cpu().numpy(), a) < TOL and oracle.rel_l2(pot.cpu().numpy(), p) < TOL


def test_degenerate_trees():
    rng = np.random.default_rng(74)
    # one body: no force, no potential
    _, _, acc, pot, _, _ = _gpu_fmm(np.zeros((1, 3), np.float32), np.ones(1, np.float32), 16, 0.5, 1e-2)
    assert np.all(acc == 0.0) and np.all(pot == 0.0)
    # small and ragged sizes
    for n in (2, 17, 65, 300):
        pos = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
        _check(pos, np.full(n, 1.0 / n, np.float32), 4, 0.6, 1e-2)
    # 100 coincident bodies (one leaf at the deepest level, wider than a
    # wave) next to a few others
    pos = np.concatenate([np.full((100, 3), 0.25), rng.uniform(0, 1, (50, 3))]).astype(np.float32)
    _check(pos, np.full(150, 0.01, np.float32), 8, 0.5, 1e-2)


def test_rejects_2d_and_missing_plan():
    w = workloads.plummer_sphere(1000, seed=75)
    dev = torch.device("cuda:0")
    tc = treecode.Treecode(3, leaf_cap=16)
    tc.build(torch.from_numpy(w.pos).to(dev), torch.from_numpy(w.mass).to(dev))
    with pytest.raises(treecode.TcError):
        tc.fmm_plan(0.5)                    # before moments
    tc.moments()
    with pytest.raises(treecode.TcError):
        tc.fmm_forces(1.0, 1e-2)            # before a plan
    with pytest.raises(treecode.TcError):
        tc.fmm_plan(-1.0)
    d2 = workloads.gaussian_disk(1000, seed=76)
    t2 = treecode.Treecode(2, leaf_cap=16)
    t2.build(torch.from_numpy(d2.pos).to(dev), torch.from_numpy(d2.mass).to(dev))
    t2.moments()
    with pytest.raises(treecode.TcError):
        t2.fmm_plan(0.5)


def test_full_size_plummer_1m():
    # the 1,048,576-body Plummer sphere against the oracle's FMM on all bodies
    w = workloads.plummer_sphere()
    print(f"case n={w.n} theta=0.5", flush=True)
    _, sizes, acc, pot, _, _ = _gpu_fmm(w.pos, w.mass, 16, 0.5, w.eps)
    t = oracle.Tree(w.pos.astype(np.float64), w.mass.astype(np.float64), 16)
    a, p = oracle.fmm_forces(t, 0.5, eps=w.eps)
    ea, ep = oracle.rel_l2(acc, a), oracle.rel_l2(pot, p)
    print(f"  m2l {sizes[1]} p2p {sizes[2]}: acc {ea:.2e} pot {ep:.2e}", flush=True)
    assert ea < TOL and ep < TOL


def test_plan_capacities_and_retry():
    # through the C ABI: capacities of 1 are refused with lower bounds of
    # what is needed; growing them to those bounds converges, and the plan
    # then gives the binding's result bit for bit
    import ctypes as C
    w = workloads.plummer_sphere(20000, seed=78)
    dev = torch.device("cuda:0")
    tc = treecode.Treecode(3, leaf_cap=16)
    tc.build(torch.from_numpy(w.pos).to(dev), torch.from_numpy(w.mass).to(dev))
    tc.moments()
    L = treecode.lib()
    ncells = tc.num_cells()
    caps = [1, 1, 1]
    sizes = np.zeros(3, dtype=np.int64)
    refusals = 0
    while True:
        need = int(L.tc_fmm_buffer_bytes(ncells, *caps))
        assert need > 0
        buf = torch.empty(need, dtype=torch.uint8, device=dev)
        rc = L.tc_fmm_plan(tc._h, 0.6, C.c_void_p(buf.data_ptr()), need, *caps, sizes.ctypes.data_as(C.c_void_p))
        if rc == treecode.TC_OK:
            break
        assert rc == treecode.TC_EWORKSPACE
        refusals += 1
        assert refusals < 20
        grown = [max(c, int(z)) for c, z in zip(caps, sizes)]
        assert grown != caps                      # every refusal names a larger need
        caps = grown
    assert refusals >= 1
    acc = torch.empty((w.n, 3), dtype=torch.float32, device=dev)
    pot = torch.empty(w.n, dtype=torch.float32, device=dev)
    assert L.tc_fmm_forces(tc._h, 1.0, 1e-2, C.c_void_p(acc.data_ptr()), C.c_void_p(pot.data_ptr())) == 0
    del buf
    tc.fmm_plan(0.6)
    a2, p2 = tc.fmm_forces(1.0, 1e-2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(acc.cpu().numpy(), a2.cpu().numpy())
    np.testing.assert_array_equal(pot.cpu().numpy(), p2.cpu().numpy())
