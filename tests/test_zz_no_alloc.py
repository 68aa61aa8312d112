"""The allocation-free force evaluation (tc_forces_noalloc) against the
entry points it combines (tc_build, tc_moments, tc_walk, tc_forces with the
caller's workspace): the same bits, on two calls in a row, the second with
fewer bodies, through the C ABI."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads
from paper_1211_2293_amd import treecode as T

pytestmark = pytest.mark.gpu


def _reference(w, theta):
    tc = T.Treecode(3, leaf_cap=w.leaf_cap)
    pos, mass = torch.from_numpy(w.pos).cuda(), torch.from_numpy(w.mass).cuda()
    tc.build(pos, mass)
    tc.moments()
    tc.walk(theta)
    acc, pot = tc.forces(w.G, w.eps)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), pot.cpu().numpy()


def test_noalloc_matches_the_workspace_path_twice():
    L = T.lib()
    h = C.c_void_p()
    assert L.tc_create(C.byref(h), 3, C.c_void_p(torch.cuda.current_stream().cuda_stream)) == T.TC_OK
    L.tc_forces_noalloc.restype = C.c_int
    L.tc_forces_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_int,
                                    C.c_double, C.c_double, C.c_double, C.c_void_p, C.c_void_p]
    try:
        for n, seed, theta in ((40000, 31, 0.5), (7000, 32, 0.6)):
            w = workloads.plummer_sphere(n, seed=seed)
            ref_acc, ref_pot = _reference(w, theta)
            pos, mass = torch.from_numpy(w.pos).cuda(), torch.from_numpy(w.mass).cuda()
            acc = torch.full((n, 3), float("nan"), dtype=torch.float32, device="cuda")
            pot = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
            torch.cuda.synchronize()
            print(f"tc_forces_noalloc n={n} theta={theta}", flush=True)
            rc = L.tc_forces_noalloc(h, C.c_void_p(pos.data_ptr()), C.c_void_p(mass.data_ptr()), n, w.leaf_cap,
                                     T.TC_F32, theta, w.G, w.eps, C.c_void_p(acc.data_ptr()),
                                     C.c_void_p(pot.data_ptr()))
            assert rc == T.TC_OK, L.tc_strerror(rc)
            assert L.tc_status(h) == T.TC_OK
            np.testing.assert_array_equal(acc.cpu().numpy(), ref_acc)
            np.testing.assert_array_equal(pot.cpu().numpy(), ref_pot)
        # beyond the scratch: refused before anything is launched
        big = 1 << 20
        assert L.tc_workspace_bytes(big, 3, 16) > T.NOALLOC_SCRATCH_BYTES
        assert L.tc_forces_noalloc(h, C.c_void_p(pos.data_ptr()), C.c_void_p(mass.data_ptr()), big, 16, T.TC_F32,
                                   0.5, 1.0, 1e-2, None, None) == T.TC_EWORKSPACE
    finally:
        L.tc_destroy(h)
