"""GPU leapfrog step and FP64 diagnostics vs the oracle (§3.1: each body
updates its position and velocity from the computed forces)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1211_2293_amd import treecode
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _tree_force(mass, lc, theta, eps, G=1.0):
    return lambda x: oracle.Tree(x, mass, lc).walk_forces(theta, G=G, eps=eps)[0]


def test_uniform_cube_one_force_and_one_step():
    """One force evaluation plus one kick-drift-kick step of dt = 1e-3 on
    FP64 state, against the FP64 oracle with the same theta; both are also
    reported against the FP64 direct sum."""
    w = workloads.uniform_cube(4096)
    pos, vel, mass = to_dev(w.pos), to_dev(w.vel), to_dev(w.mass)
    tc = treecode.Treecode(3, leaf_cap=w.leaf_cap)
    tc.build(pos, mass)
    tc.moments()
    tc.walk(w.theta)
    acc0, pot0 = tc.forces(w.G, w.eps)
    a0 = acc0.cpu().numpy()
    t0 = oracle.Tree(w.pos, w.mass, w.leaf_cap)
    ra0, rp0 = t0.walk_forces(w.theta, eps=w.eps)
    d0, _ = oracle.direct(w.pos, w.mass, eps=w.eps)
    e_tree, e_direct = oracle.rel_l2(a0, ra0), oracle.rel_l2(a0, d0)
    print(f"force vs same-theta oracle {e_tree:.2e}, vs direct sum {e_direct:.2e}, "
          f"oracle treecode vs direct {oracle.rel_l2(ra0, d0):.2e}", flush=True)
    assert e_tree < 1e-5
    tc.leapfrog(w.dt, pos, vel)
    x1, v1, a1 = oracle.kdk(w.pos, w.vel, ra0, w.dt, _tree_force(w.mass, w.leaf_cap, w.theta, w.eps))
    gx, gv = pos.cpu().numpy(), vel.cpu().numpy()
    # x' - x = dt^2/2 a: a force error of at most 1e-5 of the largest
    # acceleration moves a body by at most dt^2/2 * 1e-5 * max|a|
    assert np.abs(gx - x1).max() <= 0.5 * w.dt ** 2 * 1e-5 * np.abs(ra0).max()
    assert oracle.rel_l2(gv, v1) < 1e-5
    # diagnostics of the new state: FP64 reductions of the GPU's own values
    # are exact to rounding; against the oracle's forces within 1e-5
    d = tc.diag(vel)
    # the enqueued form runs the same kernels on the same values
    d_dev = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    tc.diag_async(vel, d_dev)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(d_dev.cpu().numpy(), d)
    acc1 = torch.empty((4096, 3), dtype=torch.float32, device="cuda")
    pot1 = torch.empty(4096, dtype=torch.float32, device="cuda")
    # re-run the force call to fetch the kept results (same tree, same theta)
    tc.walk(w.theta)
    tc.forces(w.G, w.eps, acc1, pot1)
    ref = oracle.diagnostics(w.mass, gv, acc1.cpu().numpy(), pot1.cpu().numpy())
    np.testing.assert_allclose(d[:2], ref[:2], rtol=1e-12)
    np.testing.assert_allclose(d[2:], ref[2:], rtol=1e-9, atol=1e-15)
    ekin = 0.5 * np.sum(w.mass * np.sum(v1 * v1, axis=1))
    assert abs(d[0] - ekin) <= 1e-5 * abs(ekin)


def test_ten_steps_plummer_f32():
    w = workloads.plummer_sphere(20000, seed=70)
    pos, vel, mass = to_dev(w.pos), to_dev(w.vel), to_dev(w.mass)
    tc = treecode.Treecode(3, leaf_cap=16)
    tc.build(pos, mass)
    tc.moments()
    tc.walk(0.5)
    tc.forces(1.0, 1e-2)
    e0 = tc.diag(vel)
    for _ in range(10):
        tc.leapfrog(1e-3, pos, vel)
    assert tc.status() == 0
    e1 = tc.diag(vel)
    etot0, etot1 = e0[0] + e0[1], e1[0] + e1[1]
    print(f"energy {etot0:.8f} -> {etot1:.8f}, rel drift {abs(etot1 - etot0) / abs(etot0):.2e}", flush=True)
    assert abs(etot1 - etot0) < 1e-4 * abs(etot0)
    # oracle integration of the same 10 steps
    x, v = w.pos.astype(np.float64), w.vel.astype(np.float64)
    f = _tree_force(w.mass, 16, 0.5, 1e-2)
    a = f(x)
    for _ in range(10):
        x, v, a = oracle.kdk(x, v, a, 1e-3, f)
    assert oracle.rel_l2(pos.cpu().numpy(), x) < 1e-6
    assert oracle.rel_l2(vel.cpu().numpy(), v) < 1e-5


def test_disk_2d_steps_and_momentum():
    w = workloads.gaussian_disk(8000, seed=71)
    pos, vel, mass = to_dev(w.pos), to_dev(w.vel), to_dev(w.mass)
    tc = treecode.Treecode(2, leaf_cap=16)
    tc.build(pos, mass)
    tc.moments()
    tc.walk(0.5)
    tc.forces(1.0, 1e-2)
    for _ in range(3):
        tc.leapfrog(1e-3, pos, vel)
    d = tc.diag(vel)
    assert d[4] == 0.0 and d[7] == 0.0        # no z components in 2D
    x, v = w.pos.astype(np.float64), w.vel.astype(np.float64)
    f = _tree_force(w.mass, 16, 0.5, 1e-2)
    a = f(x)
    for _ in range(3):
        x, v, a = oracle.kdk(x, v, a, 1e-3, f)
    assert oracle.rel_l2(vel.cpu().numpy(), v) < 1e-5


def test_call_order_on_device():
    w = workloads.plummer_sphere(1000, seed=72)
    pos, vel, mass = to_dev(w.pos), to_dev(w.vel), to_dev(w.mass)
    tc = treecode.Treecode(3, leaf_cap=16)
    tc.build(pos, mass)
    with pytest.raises(treecode.TcError) as e:
        tc.walk(0.5)
    assert e.value.code == treecode.TC_ESTATE
    tc.moments()
    with pytest.raises(treecode.TcError):
        tc.forces(1.0, 1e-2)
    with pytest.raises(treecode.TcError):
        tc.leapfrog(1e-3, pos, vel)
    tc.walk(0.5)
    tc.forces(1.0, 1e-2)
    tc.leapfrog(1e-3, pos, vel)
    assert tc.status() == 0


@pytest.mark.parametrize("created_stream", [False, True])
def test_graph_replay_matches_eager_launches(created_stream):
    """Leapfrog steps with the pre-force part replayed as a graph give the
    same bits as launching every kernel; the graph is recorded again when
    the buffers or dt change, and eager work in between is ordered.  On the
    null stream the graph runs on a private stream behind events, on a
    created stream it is recorded and replayed on that stream."""
    w = workloads.plummer_sphere(30000, seed=71)
    stream = torch.cuda.Stream() if created_stream else torch.cuda.current_stream()

    def run(graph):
        with torch.cuda.stream(stream):
            return _run(graph)

    def _run(graph):
        pos_a, vel_a, mass = to_dev(w.pos), to_dev(w.vel), to_dev(w.mass)
        pos_b, vel_b = to_dev(w.pos), to_dev(w.vel)
        tc = treecode.Treecode(3, leaf_cap=16)
        tc.set_graph(graph)
        out = []
        for pos, vel in ((pos_a, vel_a), (pos_b, vel_b)):
            tc.build(pos, mass)
            tc.moments()
            tc.walk(0.6)
            tc.forces(1.0, 1e-2)
            for k in range(4):
                tc.leapfrog(1e-3 if k < 2 else 2e-3, pos, vel)
                pos.add_(0.0)                      # eager torch work on the same stream
            d = tc.diag(vel)
            out.append((pos.cpu().numpy(), vel.cpu().numpy(), d))
        assert tc.status() == treecode.TC_OK
        return out

    eager, graph = run(False), run(True)
    for (xe, ve, de), (xg, vg, dg) in zip(eager, graph):
        np.testing.assert_array_equal(xg, xe)
        np.testing.assert_array_equal(vg, ve)
        np.testing.assert_array_equal(dg, de)
    # both buffer pairs started from the same state
    np.testing.assert_array_equal(graph[0][0], graph[1][0])


def test_stage_timing_counts_every_stage_and_changes_nothing():
    """Per-stage timing brackets each stage of a leapfrog step once per step
    (the diagnostics once per call) and leaves the results bit for bit as
    they are without it."""
    w = workloads.plummer_sphere(30000, seed=73)

    def run(timed):
        pos, vel, mass = to_dev(w.pos), to_dev(w.vel), to_dev(w.mass)
        tc = treecode.Treecode(3, leaf_cap=16)
        tc.build(pos, mass)
        tc.moments()
        tc.walk(0.5)
        tc.forces(1.0, 1e-2)
        tc.set_stage_timing(timed)
        rec = torch.empty(8, dtype=torch.float64, device="cuda")
        for _ in range(3):
            tc.leapfrog(1e-3, pos, vel)
            tc.diag_async(vel, rec)
        st = tc.stage_timing() if timed else None
        tc.set_stage_timing(False)
        assert tc.status() == treecode.TC_OK
        return pos.cpu().numpy(), vel.cpu().numpy(), rec.cpu().numpy(), st

    x0, v0, d0, _ = run(False)
    x1, v1, d1, st = run(True)
    np.testing.assert_array_equal(x1, x0)
    np.testing.assert_array_equal(v1, v0)
    np.testing.assert_array_equal(d1, d0)
    for name, (ms, cnt) in st.items():
        assert cnt == 3, (name, cnt)
        assert ms > 0.0, name
    print("stage ms per step: " + ", ".join(f"{k} {v[0] / 3:.3f}" for k, v in st.items()), flush=True)
