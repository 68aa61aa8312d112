"""The C-ABI library loads, exports every function include/tc.h declares,
and rejects bad arguments and call orders on the host, before any launch
(so these run without a GPU)."""
import ctypes as C

import pytest

from paper_1211_2293_amd import treecode as T


@pytest.fixture(scope="module")
def L():
    return T.lib()


def test_exports_every_declared_symbol(L):
    names = T.header_functions()
    assert len(names) >= 19
    for nm in names:
        assert hasattr(L, nm), nm


def test_workspace_bytes(L):
    assert L.tc_workspace_bytes(0, 3, 8) == 0
    assert L.tc_workspace_bytes(100, 4, 8) == 0
    assert L.tc_workspace_bytes(100, 3, 0) == 0
    assert L.tc_workspace_bytes(100, 3, 257) == 0
    a = L.tc_workspace_bytes(1000, 3, 8)
    b = L.tc_workspace_bytes(2000, 3, 8)
    assert 0 < a < b
    # 2D trees may be deeper (31 levels), so their bound is larger per body
    assert L.tc_workspace_bytes(1000, 2, 8) > 0


def _ctx(L, dim=3):
    h = C.c_void_p()
    assert L.tc_create(C.byref(h), dim, None) == T.TC_OK
    return h


def test_create_rejects_bad_dim(L):
    h = C.c_void_p()
    assert L.tc_create(C.byref(h), 4, None) == T.TC_EINVAL
    assert L.tc_create(None, 3, None) == T.TC_EINVAL


def test_call_order_and_arguments(L):
    h = _ctx(L)
    fake = C.c_void_p(1 << 40)            # never dereferenced: every call below fails its checks
    # nothing built yet
    assert L.tc_moments(h) == T.TC_ESTATE
    assert L.tc_walk(h, 0.5) == T.TC_ESTATE
    assert L.tc_forces(h, 1.0, 1e-2, None, None) == T.TC_ESTATE
    assert L.tc_leapfrog(h, 1e-3, fake, fake) == T.TC_ESTATE
    out = (C.c_double * 8)()
    assert L.tc_diag(h, fake, out) == T.TC_ESTATE
    assert L.tc_diag_async(h, fake, fake) == T.TC_ESTATE
    assert L.tc_diag_async(h, fake, None) == T.TC_EINVAL
    assert L.tc_diag_async(h, fake, C.c_void_p((1 << 40) + 4)) == T.TC_EINVAL    # out not 8-byte aligned
    n = C.c_int64()
    assert L.tc_num_cells(h, C.byref(n)) == T.TC_ESTATE
    assert L.tc_get_tests(h, fake) == T.TC_ESTATE
    assert L.tc_get_tests(h, None) == T.TC_EINVAL
    assert L.tc_get_tests(None, fake) == T.TC_EINVAL
    # argument checks come first
    assert L.tc_walk(h, -0.1) == T.TC_EINVAL
    assert L.tc_walk(h, float("nan")) == T.TC_EINVAL
    assert L.tc_walk(h, 1.5) == T.TC_EINVAL
    assert L.tc_forces(h, 1.0, 0.0, None, None) == T.TC_EINVAL
    assert L.tc_forces(h, 1.0, float("inf"), None, None) == T.TC_EINVAL
    assert L.tc_forces(h, float("nan"), 1e-2, None, None) == T.TC_EINVAL
    assert L.tc_leapfrog(h, float("nan"), fake, fake) == T.TC_EINVAL
    # workspace: none set, misaligned, too small
    assert L.tc_build(h, fake, fake, 100, 3, 8, T.TC_F32) == T.TC_EWORKSPACE
    assert L.tc_set_workspace(h, C.c_void_p((1 << 40) + 4), 1 << 20) == T.TC_EINVAL
    assert L.tc_set_workspace(h, fake, 1024) == T.TC_OK
    assert L.tc_build(h, fake, fake, 100, 3, 8, T.TC_F32) == T.TC_EWORKSPACE
    # bad sizes, dims, dtypes, pointers
    assert L.tc_build(h, fake, fake, 0, 3, 8, T.TC_F32) == T.TC_EINVAL
    assert L.tc_build(h, fake, fake, 100, 2, 8, T.TC_F32) == T.TC_EINVAL   # context is 3D
    assert L.tc_build(h, fake, fake, 100, 3, 0, T.TC_F32) == T.TC_EINVAL
    assert L.tc_build(h, fake, fake, 100, 3, 8, 7) == T.TC_EINVAL
    assert L.tc_build(h, None, fake, 100, 3, 8, T.TC_F32) == T.TC_EINVAL
    assert L.tc_build(h, C.c_void_p((1 << 40) + 4), fake, 100, 3, 8, T.TC_F64) == T.TC_EINVAL
    L.tc_destroy(h)
    L.tc_destroy(None)


def test_strerror(L):
    for code in (T.TC_OK, T.TC_EINVAL, T.TC_EWORKSPACE, T.TC_ESTATE, T.TC_EHIP, T.TC_ENONFINITE, 99):
        assert isinstance(L.tc_strerror(code), bytes) and L.tc_strerror(code)


def test_closure_direct_lists_and_modes_check_arguments_first(L):
    """The entry points beyond the core path reject bad arguments and call
    orders on the host, before touching a device."""
    h = _ctx(L)
    h2 = _ctx(L, dim=2)
    fake = C.c_void_p(1 << 40)
    tot = C.c_int64()
    # modes
    assert L.tc_set_multipole(h, 3) == T.TC_EINVAL
    assert L.tc_set_multipole(h2, 2) == T.TC_EINVAL            # quadrupoles are 3D
    assert L.tc_set_multipole(h, 2) == T.TC_OK
    assert L.tc_set_multipole(h, 1) == T.TC_OK
    assert L.tc_set_accumulation(h, 2) == T.TC_EINVAL
    assert L.tc_set_accumulation(h, T.TC_ACC_PLAIN) == T.TC_OK
    assert L.tc_set_split(None, 1) == T.TC_EINVAL
    assert L.tc_set_split(h, 3) == T.TC_EINVAL
    assert L.tc_set_split(h, -1) == T.TC_EINVAL
    for mode in (0, 2, 1):
        assert L.tc_set_split(h, mode) == T.TC_OK
    assert L.tc_set_graph(None, 1) == T.TC_EINVAL
    # direct sum
    assert L.tc_direct(h, fake, 0, 1.0, 1e-2, fake, fake) == T.TC_EINVAL
    assert L.tc_direct(h, None, 10, 1.0, 1e-2, fake, fake) == T.TC_EINVAL
    assert L.tc_direct(h, fake, 10, 1.0, -1.0, fake, fake) == T.TC_EINVAL
    assert L.tc_direct(h, fake, 10, 1.0, 1e-2, fake, fake) == T.TC_ESTATE
    # per-body lists
    assert L.tc_lists_count(h, None, None) == T.TC_EINVAL
    assert L.tc_lists_count(h, C.byref(tot), None) == T.TC_ESTATE
    assert L.tc_lists_forces(h, 1.0, 1e-2, None, 10, None, None) == T.TC_EINVAL
    assert L.tc_lists_forces(h, 1.0, 0.0, fake, 10, None, None) == T.TC_EINVAL
    assert L.tc_lists_forces(h, 1.0, 1e-2, fake, 10, None, None) == T.TC_ESTATE
    # learned closure
    assert L.tc_forces_learned(h, 1.0, 1e-2, 0.8, 0.9, 1.0, None, None) == T.TC_EINVAL   # theta_p >= theta_l
    assert L.tc_forces_learned(h, 1.0, 1e-2, 1.2, 0.5, 1.0, None, None) == T.TC_EINVAL
    assert L.tc_forces_learned(h, 1.0, 1e-2, 0.8, 0.5, -1.0, None, None) == T.TC_EINVAL
    assert L.tc_forces_learned(h2, 1.0, 1e-2, 0.8, 0.5, 1.0, None, None) == T.TC_EINVAL  # 3D only
    assert L.tc_forces_learned(h, 1.0, 1e-2, 0.8, 0.5, 1.0, None, None) == T.TC_ESTATE
    assert L.tc_residuals(h, 0.9, 1e-2, fake, 0, fake, fake, fake, 10, C.byref(tot)) == T.TC_EINVAL
    assert L.tc_residuals(h, 0.9, 1e-2, fake, 10, None, fake, fake, 10, C.byref(tot)) == T.TC_EINVAL
    assert L.tc_residuals(h, 0.9, 1e-2, fake, 10, fake, fake, fake, 10, C.byref(tot)) == T.TC_ESTATE
    assert L.tc_mlp_load(h, fake) == T.TC_ESTATE
    assert L.tc_mlp_get(h, fake) == T.TC_ESTATE
    assert L.tc_mlp_forward(h, fake, 10, None, 11, fake) == T.TC_EINVAL                # nb > nrows
    assert L.tc_mlp_forward(h, fake, 10, None, 5, fake) == T.TC_ESTATE
    assert L.tc_mlp_step(h, fake, fake, 10, None, 5, -1.0, None, None) == T.TC_EINVAL
    assert L.tc_mlp_step(h, fake, fake, 10, None, 70000, 1e-3, None, None) == T.TC_EINVAL  # batch cap
    assert L.tc_mlp_step(h, fake, fake, 10, None, 5, 1e-3, None, None) == T.TC_ESTATE
    assert L.tc_get_learned_counts(h, None, None) == T.TC_ESTATE
    L.tc_destroy(h)
    L.tc_destroy(h2)


def test_size_limits(L):
    # level-order cell indices are packed into 28 bits: the cell bound of
    # n bodies must stay below 2^28
    assert L.tc_workspace_bytes(100_000_000, 3, 16) > 0
    assert L.tc_workspace_bytes(130_000_000, 3, 16) == 0
    assert L.tc_workspace_bytes(2_000_000_001, 3, 256) == 0      # beyond TC_MAX_N


def test_fmm_checks_arguments_first(L):
    h = _ctx(L)
    h2 = _ctx(L, dim=2)
    fake = C.c_void_p(1 << 40)
    sizes = (C.c_int64 * 3)()
    assert L.tc_fmm_buffer_bytes(0, 10, 10, 10) == 0
    assert L.tc_fmm_buffer_bytes(100, 0, 10, 10) == 0
    assert L.tc_fmm_buffer_bytes(100, 10, 1 << 32, 10) == 0
    a = L.tc_fmm_buffer_bytes(100, 10, 10, 10)
    b = L.tc_fmm_buffer_bytes(100, 10, 1000, 10)
    assert 0 < a < b
    assert L.tc_fmm_plan(h, 0.5, None, 1 << 20, 10, 10, 10, sizes) == T.TC_EINVAL
    assert L.tc_fmm_plan(h, 0.5, C.c_void_p((1 << 40) + 8), 1 << 20, 10, 10, 10, sizes) == T.TC_EINVAL
    assert L.tc_fmm_plan(h, -0.5, fake, 1 << 20, 10, 10, 10, sizes) == T.TC_EINVAL
    assert L.tc_fmm_plan(h, float("nan"), fake, 1 << 20, 10, 10, 10, sizes) == T.TC_EINVAL
    assert L.tc_fmm_plan(h, 0.5, fake, 1 << 20, 10, 10, 10, None) == T.TC_EINVAL
    assert L.tc_fmm_plan(h2, 0.5, fake, 1 << 20, 10, 10, 10, sizes) == T.TC_EINVAL   # 3D only
    assert L.tc_fmm_plan(h, 0.5, fake, 1 << 20, 10, 10, 10, sizes) == T.TC_ESTATE    # no moments yet
    assert L.tc_fmm_forces(h, 1.0, 0.0, None, None) == T.TC_EINVAL
    assert L.tc_fmm_forces(h, 1.0, 1e-2, C.c_void_p((1 << 40) + 2), None) == T.TC_EINVAL
    assert L.tc_fmm_forces(h, 1.0, 1e-2, None, None) == T.TC_ESTATE                  # no plan
    assert L.tc_fmm_get_pairs(h, None, None) == T.TC_ESTATE
    L.tc_destroy(h)
    L.tc_destroy(h2)


def test_closure_mode_and_stage_timing_check_arguments_first(L):
    h = _ctx(L)
    fake = C.c_void_p(1 << 40)
    dbl = C.c_double
    assert L.tc_set_closure(None, dbl(0.8), dbl(0.5), dbl(1e-3)) == T.TC_EINVAL
    assert L.tc_set_closure(h, dbl(1.2), dbl(0.5), dbl(1e-3)) == T.TC_EINVAL     # theta_l > 1
    assert L.tc_set_closure(h, dbl(0.5), dbl(0.5), dbl(1e-3)) == T.TC_EINVAL     # theta_p not below theta_l
    assert L.tc_set_closure(h, dbl(0.8), dbl(-0.1), dbl(1e-3)) == T.TC_EINVAL
    assert L.tc_set_closure(h, dbl(0.8), dbl(0.5), dbl(-1.0)) == T.TC_EINVAL
    assert L.tc_set_closure(h, dbl(0.8), dbl(0.5), dbl(float("nan"))) == T.TC_EINVAL
    assert L.tc_set_closure(h, dbl(0.8), dbl(0.5), dbl(float("inf"))) == T.TC_OK
    # the learned walk in a step still needs a force evaluation first
    assert L.tc_leapfrog(h, dbl(1e-3), fake, fake) == T.TC_ESTATE
    assert L.tc_set_closure(h, dbl(0.0), dbl(0.0), dbl(0.0)) == T.TC_OK          # off
    h2 = _ctx(L, dim=2)
    assert L.tc_set_closure(h2, dbl(0.8), dbl(0.5), dbl(1e-3)) == T.TC_EINVAL    # 3D only
    assert L.tc_set_closure(h2, dbl(0.0), dbl(0.0), dbl(0.0)) == T.TC_OK
    ms = (C.c_double * len(T.STAGES))()
    cnt = (C.c_int64 * len(T.STAGES))()
    assert L.tc_set_stage_timing(None, 1) == T.TC_EINVAL
    assert L.tc_set_stage_timing(h, 1) == T.TC_OK
    assert L.tc_get_stage_timing(h, None, cnt) == T.TC_EINVAL
    assert L.tc_get_stage_timing(h, ms, cnt) == T.TC_OK
    assert list(cnt) == [0] * len(T.STAGES)
    assert L.tc_set_stage_timing(h, 0) == T.TC_OK
    L.tc_destroy(h)
    L.tc_destroy(h2)


def test_noalloc_entry_checks_arguments_first(L):
    h = _ctx(L)
    fake = C.c_void_p(1 << 40)
    f = L.tc_forces_noalloc
    dbl = C.c_double
    assert f(None, fake, fake, 1000, 16, T.TC_F32, dbl(0.5), dbl(1.0), dbl(1e-2), None, None) == T.TC_EINVAL
    assert f(h, None, fake, 1000, 16, T.TC_F32, dbl(0.5), dbl(1.0), dbl(1e-2), None, None) == T.TC_EINVAL
    assert f(h, fake, fake, 0, 16, T.TC_F32, dbl(0.5), dbl(1.0), dbl(1e-2), None, None) == T.TC_EINVAL
    assert f(h, fake, fake, 1000, 16, 7, dbl(0.5), dbl(1.0), dbl(1e-2), None, None) == T.TC_EINVAL
    assert f(h, fake, fake, 1000, 16, T.TC_F32, dbl(1.5), dbl(1.0), dbl(1e-2), None, None) == T.TC_EINVAL
    assert f(h, fake, fake, 1000, 16, T.TC_F32, dbl(0.5), dbl(1.0), dbl(0.0), None, None) == T.TC_EINVAL
    assert f(h, fake, fake, 1000, 16, T.TC_F32, dbl(0.5), dbl(1.0), dbl(1e-2), C.c_void_p((1 << 40) + 2),
             None) == T.TC_EINVAL
    # a system whose workspace exceeds the scratch is refused before any device call
    big = 1 << 20
    assert L.tc_workspace_bytes(big, 3, 16) > T.NOALLOC_SCRATCH_BYTES
    assert f(h, fake, fake, big, 16, T.TC_F32, dbl(0.5), dbl(1.0), dbl(1e-2), None, None) == T.TC_EWORKSPACE
    L.tc_destroy(h)
