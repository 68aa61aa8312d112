"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and fetch what the oracle is compared with.  Imports torch lazily so CPU-only
collection works."""
from __future__ import annotations

import numpy as np


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_tree(pos, mass, leaf_cap, theta=None, G=1.0, eps=None, moments=True, tc=None):
    """Build (and optionally walk + force) on the GPU, in a new context or in
    the given one; return numpy results."""
    import torch

    from paper_1211_2293_amd import treecode
    dim = pos.shape[1]
    if tc is None:
        tc = treecode.Treecode(dim, leaf_cap=leaf_cap)
    p = to_dev(pos)
    m = to_dev(mass)
    tc.build(p, m)
    out = {"tc": tc, "pos_t": p, "mass_t": m}
    if moments:
        tc.moments()
    if theta is not None:
        tc.walk(theta)
        acc, pot = tc.forces(G, eps)
        m2p, p2p = tc.counts()
        out.update(acc=acc.cpu().numpy(), pot=pot.cpu().numpy(), m2p=m2p.cpu().numpy(),
                   p2p=p2p.cpu().numpy(), tests=tc.tests().cpu().numpy())
    gb, gc = tc.groups()
    out["gbeg"], out["gcnt"] = gb.cpu().numpy(), gc.cpu().numpy()
    torch.cuda.synchronize()
    k, perm = tc.keys()
    out["key"] = k.cpu().numpy().view(np.uint64)
    out["perm"] = perm.cpu().numpy().view(np.uint32)
    cells = tc.cells(moments=moments)
    out["cells"] = {a: v.cpu().numpy() for a, v in cells.items()}
    out["cells"]["prefix"] = out["cells"]["prefix"].view(np.uint64)
    out["root"] = tc.root()
    out["status"] = tc.status()
    return out


def assert_tree_equal(g, t):
    """Bit-exact comparison of the GPU tree with an oracle.Tree."""
    b = t.bodies()
    lo, size = t.root()
    glo, gsize = g["root"]
    np.testing.assert_array_equal(glo, lo)
    assert gsize == size
    np.testing.assert_array_equal(g["key"], b["key"])
    np.testing.assert_array_equal(g["perm"], b["perm"])
    c = t.cells()
    gc = g["cells"]
    assert len(gc["level"]) == t.ncells
    for f in ("level", "prefix", "begin", "count", "parent", "skip", "nch", "leaf"):
        np.testing.assert_array_equal(gc[f].astype(np.int64) if f != "prefix" else gc[f],
                                      c[f].astype(np.int64) if f != "prefix" else c[f], err_msg=f)
    obeg, ocnt = t.groups(64, 1024)
    np.testing.assert_array_equal(g["gbeg"], obeg)
    np.testing.assert_array_equal(g["gcnt"], ocnt)
    if "M" in gc:
        np.testing.assert_array_equal(gc["M"], c["M"])
        np.testing.assert_array_equal(gc["com"], c["com"])
        if t.dim == 3:
            scale = np.abs(c["Q"]).max(axis=1, keepdims=True) + 1e-300
            assert np.all(np.abs(gc["Q"] - c["Q"]) <= 1e-12 * scale)
