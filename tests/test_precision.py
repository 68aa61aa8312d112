"""Precision study on the two-Plummer workload (4,194,304 bodies): for each
theta, the error of the GPU forces against the FP64 direct sum on 8192
seeded sample bodies, split into the approximation error of the method
(the FP64 treecode with the same walk groups against the direct sum) and
the arithmetic error of the FP32 force loop (GPU against that FP64
treecode), with compensated and with plain running-sum accumulation."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1211_2293_amd import treecode
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _E(a, ref):
    d = np.asarray(a, np.float64) - ref
    return float(np.sqrt((d * d).sum() / (ref * ref).sum()))


@pytest.mark.timeout(900)
def test_two_plummer_precision_split():
    w = workloads.two_plummer()
    tc = treecode.Treecode(3, leaf_cap=w.leaf_cap)
    keep = (to_dev(w.pos), to_dev(w.mass))
    tc.build(*keep)
    tc.moments()
    sample = workloads.sample_indices(w.n, 8192, seed=104)
    ref, _ = tc.direct(to_dev(sample.astype(np.int32)), G=w.G, eps=w.eps)
    ref = ref.cpu().numpy()
    gb, gc = (v.cpu().numpy() for v in tc.groups())
    print("oracle tree", flush=True)
    t = oracle.Tree(w.pos, w.mass, w.leaf_cap)
    inv = np.empty(w.n, np.int64)
    inv[t.bodies()["perm"]] = np.arange(w.n)
    gsel = np.unique(np.searchsorted(gb, inv[sample], side="right") - 1)
    rows = []
    for theta in (0.3, 0.5, 0.7):
        a64, _ = t.forces_groups(theta, gb[gsel], gc[gsel], G=w.G, eps=w.eps)
        a64 = a64[sample]
        approx = _E(a64, ref)
        res = {}
        for comp in (True, False):
            tc.set_accumulation(comp)
            tc.walk(theta)
            acc, _ = tc.forces(w.G, w.eps, want_pot=False)
            a = acc.cpu().numpy()[sample]
            res[comp] = (_E(a, ref), _E(a, a64))
        tc.set_accumulation(True)
        rows.append((theta, approx, res))
        print(f"theta={theta}: E vs direct {res[True][0]:.3e} (approximation {approx:.3e}); arithmetic "
              f"compensated {res[True][1]:.3e}, plain running sum {res[False][1]:.3e}", flush=True)
    for theta, approx, res in rows:
        assert res[True][1] < 1e-5                        # the parity bar
        assert res[False][1] < 1e-3
        # the approximation dominates; the arithmetic adds at most a little
        assert abs(res[True][0] - approx) <= res[True][1] + 1e-12
    # error grows with theta
    assert rows[0][1] < rows[1][1] < rows[2][1]
