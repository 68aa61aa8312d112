"""Python binding of libtc (include/tc.h): argument marshalling only.

Every step of the treecode runs in the HIP kernels of ``libtc.so``; PyTorch
provides device memory (tensors) and the stream.  If the library has not
been built this module raises on first use: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tc.h")

TC_OK, TC_EINVAL, TC_EWORKSPACE, TC_ESTATE, TC_EHIP, TC_ENONFINITE = 0, -1, -2, -3, -4, -5
TC_ACC_COMPENSATED, TC_ACC_PLAIN = 0, 1
TC_F32, TC_F64 = 0, 1
GROUP = 64
CLUSTER = 1024
MLP_NPARAM = 5059
NOALLOC_SCRATCH_BYTES = 64 << 20     # TC_NOALLOC_SCRATCH_BYTES
# tc_stage order
STAGES = ("kick_drift", "bbox", "keys", "sort", "gather", "topology", "levels", "groups", "moments", "radii",
          "forces", "kick", "diag")

_LIB = None


class TcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tc error {code}: {msg}")
        self.code = code


def lib():
    """Load libtc.so (built by ``__graft_entry__.build()``)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    P, i32, i64, dbl, sz = C.c_void_p, C.c_int, C.c_int64, C.c_double, C.c_size_t
    sig = {
        "tc_create": (i32, [C.POINTER(C.c_void_p), i32, P]),
        "tc_destroy": (None, [P]),
        "tc_workspace_bytes": (sz, [i64, i32, i32]),
        "tc_set_workspace": (i32, [P, P, sz]),
        "tc_build": (i32, [P, P, P, i64, i32, i32, i32]),
        "tc_moments": (i32, [P]),
        "tc_walk": (i32, [P, dbl]),
        "tc_forces": (i32, [P, dbl, dbl, P, P]),
        "tc_leapfrog": (i32, [P, dbl, P, P]),
        "tc_diag": (i32, [P, P, P]),
        "tc_diag_async": (i32, [P, P, P]),
        "tc_status": (i32, [P]),
        "tc_strerror": (C.c_char_p, [i32]),
        "tc_num_cells": (i32, [P, C.POINTER(C.c_int64)]),
        "tc_get_root": (i32, [P, P, P]),
        "tc_get_keys": (i32, [P, P, P]),
        "tc_get_cells": (i32, [P] * 12),
        "tc_get_counts": (i32, [P, P, P]),
        "tc_get_tests": (i32, [P, P]),
        "tc_num_groups": (i32, [P, C.POINTER(C.c_int64)]),
        "tc_get_groups": (i32, [P, P, P]),
        "tc_set_timing": (i32, [P, i32]),
        "tc_get_timing": (i32, [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "tc_forces_learned": (i32, [P, dbl, dbl, dbl, dbl, dbl, P, P]),
        "tc_get_learned_counts": (i32, [P, P, P]),
        "tc_set_closure": (i32, [P, dbl, dbl, dbl]),
        "tc_forces_noalloc": (i32, [P, P, P, i64, i32, i32, dbl, dbl, dbl, P, P]),
        "tc_set_stage_timing": (i32, [P, i32]),
        "tc_get_stage_timing": (i32, [P, P, P]),
        "tc_residuals": (i32, [P, dbl, dbl, P, i32, P, P, P, i64, C.POINTER(C.c_int64)]),
        "tc_mlp_load": (i32, [P, P]),
        "tc_mlp_get": (i32, [P, P]),
        "tc_mlp_forward": (i32, [P, P, i64, P, i64, P]),
        "tc_mlp_step": (i32, [P, P, P, i64, P, i64, dbl, C.POINTER(C.c_float), P]),
        "tc_direct": (i32, [P, P, i32, dbl, dbl, P, P]),
        "tc_set_graph": (i32, [P, i32]),
        "tc_set_accumulation": (i32, [P, i32]),
        "tc_set_multipole": (i32, [P, i32]),
        "tc_set_split": (i32, [P, i32]),
        "tc_lists_count": (i32, [P, C.POINTER(C.c_int64), P]),
        "tc_lists_forces": (i32, [P, dbl, dbl, P, i64, P, P]),
        "tc_fmm_buffer_bytes": (C.c_size_t, [i64, i64, i64, i64]),
        "tc_fmm_plan": (i32, [P, dbl, P, C.c_size_t, i64, i64, i64, P]),
        "tc_fmm_forces": (i32, [P, dbl, dbl, P, P]),
        "tc_fmm_get_pairs": (i32, [P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def header_functions() -> list[str]:
    """Names of the functions declared in include/tc.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z_]+)\s*\(", text)))


def _check(rc: int):
    if rc != TC_OK:
        raise TcError(rc, lib().tc_strerror(rc).decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def workspace_bytes(n: int, dim: int, leaf_cap: int) -> int:
    return int(lib().tc_workspace_bytes(n, dim, leaf_cap))


class Treecode:
    """One treecode context bound to a stream (default: torch's current).

    ``build(pos, mass)`` -> ``moments()`` -> ``walk(theta)`` ->
    ``forces(G, eps)`` -> ``leapfrog(dt, pos, vel)``, mirroring the C calls.
    The workspace is a torch uint8 tensor grown on demand.
    """

    def __init__(self, dim: int, leaf_cap: int = 16, stream: torch.cuda.Stream | None = None):
        self.dim = dim
        self.leaf_cap = leaf_cap
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(lib().tc_create(C.byref(h), dim, C.c_void_p(self.stream.cuda_stream)))
        self._h = h
        self._ws = None
        self._ws_bytes = 0
        self._keep = ()
        self.n = 0
        self.dtype = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            _LIB.tc_destroy(h)
            self._h = None

    # -- plumbing ----------------------------------------------------------
    def _ensure_ws(self, n: int):
        need = workspace_bytes(n, self.dim, self.leaf_cap)
        if need == 0:
            raise TcError(TC_EINVAL, f"unsupported n={n}, dim={self.dim}, leaf_cap={self.leaf_cap}")
        if need > self._ws_bytes:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.stream.device)
            self._ws_bytes = need
            _check(lib().tc_set_workspace(self._h, _ptr(self._ws), need))

    def _dtype_code(self, t: torch.Tensor) -> int:
        if t.dtype == torch.float32:
            return TC_F32
        if t.dtype == torch.float64:
            return TC_F64
        raise TypeError(f"positions must be float32 or float64, got {t.dtype}")

    @staticmethod
    def _dev(t, name):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous CUDA tensor")

    # -- the calls -----------------------------------------------------------
    def build(self, pos: torch.Tensor, mass: torch.Tensor):
        self._dev(pos, "pos")
        self._dev(mass, "mass")
        if pos.dim() != 2 or pos.shape[1] != self.dim or mass.shape != (pos.shape[0],):
            raise ValueError("pos must be [n][dim] and mass [n]")
        if mass.dtype != pos.dtype:
            raise TypeError("pos and mass must share a dtype")
        n = pos.shape[0]
        self._ensure_ws(n)
        self._keep = (pos, mass)      # the library keeps the mass pointer
        self.dtype = pos.dtype
        _check(lib().tc_build(self._h, _ptr(pos), _ptr(mass), n, self.dim, self.leaf_cap,
                              self._dtype_code(pos)))
        self.n = n

    def moments(self):
        _check(lib().tc_moments(self._h))

    def walk(self, theta: float):
        _check(lib().tc_walk(self._h, float(theta)))

    def forces(self, G: float = 1.0, eps: float = 1e-2, acc=None, pot=None, want_pot=True):
        if acc is None:
            acc = torch.empty((self.n, self.dim), dtype=torch.float32, device=self.stream.device)
        if pot is None and want_pot:
            pot = torch.empty(self.n, dtype=torch.float32, device=self.stream.device)
        for t, nm in ((acc, "acc"), (pot, "pot")):
            if t is not None:
                self._dev(t, nm)
                if t.dtype != torch.float32:
                    raise TypeError(f"{nm} must be float32")
        _check(lib().tc_forces(self._h, float(G), float(eps), _ptr(acc), _ptr(pot)))
        return acc, pot

    def leapfrog(self, dt: float, pos: torch.Tensor, vel: torch.Tensor):
        self._dev(pos, "pos")
        self._dev(vel, "vel")
        if pos.dtype != self.dtype or vel.dtype != self.dtype or pos.shape != vel.shape:
            raise TypeError("pos and vel must match the build dtype and shape")
        self._keep = (pos, self._keep[1])
        _check(lib().tc_leapfrog(self._h, float(dt), _ptr(pos), _ptr(vel)))

    def diag(self, vel: torch.Tensor) -> np.ndarray:
        self._dev(vel, "vel")
        out = np.zeros(8)
        _check(lib().tc_diag(self._h, _ptr(vel), out.ctypes.data_as(C.c_void_p)))
        return out

    def diag_async(self, vel: torch.Tensor, out: torch.Tensor) -> None:
        """Enqueue the diagnostics into `out` (8 float64 on the device), no wait."""
        self._dev(vel, "vel")
        self._dev(out, "out")
        if out.dtype != torch.float64 or out.numel() != 8 or not out.is_contiguous():
            raise TypeError("out must be 8 contiguous float64 values on the device")
        _check(lib().tc_diag_async(self._h, _ptr(vel), _ptr(out)))

    def status(self) -> int:
        return int(lib().tc_status(self._h))

    # -- inspection ----------------------------------------------------------
    def num_cells(self) -> int:
        c = C.c_int64()
        _check(lib().tc_num_cells(self._h, C.byref(c)))
        return int(c.value)

    def root(self):
        lo = np.zeros(self.dim)
        size = np.zeros(1)
        _check(lib().tc_get_root(self._h, lo.ctypes.data_as(C.c_void_p), size.ctypes.data_as(C.c_void_p)))
        return lo, float(size[0])

    def keys(self):
        dev = self.stream.device
        k = torch.empty(self.n, dtype=torch.int64, device=dev)
        p = torch.empty(self.n, dtype=torch.int32, device=dev)
        _check(lib().tc_get_keys(self._h, _ptr(k), _ptr(p)))
        return k, p

    def cells(self, moments: bool = True) -> dict:
        Cn = self.num_cells()
        dev = self.stream.device
        i32 = lambda: torch.empty(Cn, dtype=torch.int32, device=dev)
        out = {"level": i32(), "prefix": torch.empty(Cn, dtype=torch.int64, device=dev),
               "begin": i32(), "count": i32(), "parent": i32(), "skip": i32(), "nch": i32(),
               "leaf": i32()}
        if moments:
            out["M"] = torch.empty(Cn, dtype=torch.float64, device=dev)
            out["com"] = torch.empty((Cn, self.dim), dtype=torch.float64, device=dev)
            out["Q"] = torch.empty((Cn, 6), dtype=torch.float64, device=dev)
        o = out
        _check(lib().tc_get_cells(self._h, _ptr(o["level"]), _ptr(o["prefix"]), _ptr(o["begin"]),
                                  _ptr(o["count"]), _ptr(o["parent"]), _ptr(o["skip"]),
                                  _ptr(o["nch"]), _ptr(o["leaf"]), _ptr(o.get("M")),
                                  _ptr(o.get("com")), _ptr(o.get("Q"))))
        return out

    def num_groups(self) -> int:
        c = C.c_int64()
        _check(lib().tc_num_groups(self._h, C.byref(c)))
        return int(c.value)

    def groups(self):
        """First sorted body and size of every walk group (int32 tensors)."""
        G = self.num_groups()
        dev = self.stream.device
        gb = torch.empty(G, dtype=torch.int32, device=dev)
        gc = torch.empty(G, dtype=torch.int32, device=dev)
        _check(lib().tc_get_groups(self._h, _ptr(gb), _ptr(gc)))
        return gb, gc

    def counts(self):
        G = self.num_groups()
        dev = self.stream.device
        m2p = torch.empty(G, dtype=torch.int64, device=dev)
        p2p = torch.empty(G, dtype=torch.int64, device=dev)
        _check(lib().tc_get_counts(self._h, _ptr(m2p), _ptr(p2p)))
        return m2p, p2p

    def tests(self):
        """Cells tested by each group's walk in the last force evaluation."""
        t = torch.empty(self.num_groups(), dtype=torch.int64, device=self.stream.device)
        _check(lib().tc_get_tests(self._h, _ptr(t)))
        return t

    def interactions(self) -> int:
        """Body-entry interactions of the last force evaluation (self
        included): sum over groups of list length x bodies in the group."""
        m2p, p2p = self.counts()
        _, gc = self.groups()
        per = (m2p + p2p).cpu().numpy()
        return int((per * gc.cpu().numpy().astype(np.int64)).sum())

    # -- learned closure -------------------------------------------------
    def residuals(self, theta: float, eps: float, targets: torch.Tensor, cap: int | None = None):
        """Training pairs for the given original body indices (int32 CUDA
        tensor): (feat [P][10], y [P][3], cell [P]) as CUDA tensors."""
        self._dev(targets, "targets")
        if targets.dtype != torch.int32:
            raise TypeError("targets must be int32")
        dev = self.stream.device
        total = C.c_int64()
        if cap is None:
            _check(lib().tc_residuals(self._h, float(theta), float(eps), _ptr(targets), len(targets),
                                      None, None, None, 0, C.byref(total)))
            cap = int(total.value)
        feat = torch.empty((max(cap, 1), 10), dtype=torch.float32, device=dev)
        y = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=dev)
        cell = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        _check(lib().tc_residuals(self._h, float(theta), float(eps), _ptr(targets), len(targets),
                                  _ptr(feat), _ptr(y), _ptr(cell), cap, C.byref(total)))
        k = min(cap, int(total.value))
        return feat[:k], y[:k], cell[:k]

    def forces_learned(self, theta_l: float, theta_p: float, tau: float, G: float = 1.0, eps: float = 1e-2,
                       acc=None, pot=None, want_pot=True):
        """Forces with the learned closure (network from mlp_load)."""
        if acc is None:
            acc = torch.empty((self.n, self.dim), dtype=torch.float32, device=self.stream.device)
        if pot is None and want_pot:
            pot = torch.empty(self.n, dtype=torch.float32, device=self.stream.device)
        for t, nm in ((acc, "acc"), (pot, "pot")):
            if t is not None:
                self._dev(t, nm)
                if t.dtype != torch.float32:
                    raise TypeError(f"{nm} must be float32")
        _check(lib().tc_forces_learned(self._h, float(G), float(eps), float(theta_l), float(theta_p),
                                       float(tau), _ptr(acc), _ptr(pot)))
        return acc, pot

    def set_closure(self, theta_l: float | None, theta_p: float = 0.5, tau: float = float("inf")):
        """Learned walk (theta_l, theta_p, tau) in leapfrog steps; None (or 0)
        switches back to the plain walk."""
        _check(lib().tc_set_closure(self._h, float(theta_l or 0.0), float(theta_p), float(tau)))

    def learned_counts(self):
        """Per walk group: (learned cells kept, learned cells that fell back)."""
        G = self.num_groups()
        dev = self.stream.device
        kept = torch.empty(G, dtype=torch.int64, device=dev)
        fell = torch.empty(G, dtype=torch.int64, device=dev)
        _check(lib().tc_get_learned_counts(self._h, _ptr(kept), _ptr(fell)))
        return kept, fell

    def mlp_load(self, params: torch.Tensor):
        self._dev(params, "params")
        if params.dtype != torch.float32 or params.numel() != MLP_NPARAM:
            raise TypeError("params must be float32 with 5059 entries")
        self._mlp_params = params
        _check(lib().tc_mlp_load(self._h, _ptr(params)))

    def mlp_get(self) -> torch.Tensor:
        out = torch.empty(MLP_NPARAM, dtype=torch.float32, device=self.stream.device)
        _check(lib().tc_mlp_get(self._h, _ptr(out)))
        return out

    def _batch(self, feat, y, idx):
        self._dev(feat, "feat")
        if feat.dtype != torch.float32 or feat.dim() != 2 or feat.shape[1] != 10:
            raise TypeError("feat must be float32 [rows][10]")
        if y is not None:
            self._dev(y, "y")
            if y.dtype != torch.float32 or tuple(y.shape) != (feat.shape[0], 3):
                raise TypeError("y must be float32 [rows][3] with the rows of feat")
        if idx is not None:
            self._dev(idx, "idx")
            if idx.dtype != torch.int32 or idx.dim() != 1:
                raise TypeError("idx must be a 1-D int32 tensor")
        return feat.shape[0] if idx is None else idx.shape[0]

    def mlp_forward(self, feat: torch.Tensor, idx: torch.Tensor | None = None) -> torch.Tensor:
        nb = self._batch(feat, None, idx)
        out = torch.empty((nb, 3), dtype=torch.float32, device=self.stream.device)
        _check(lib().tc_mlp_forward(self._h, _ptr(feat), feat.shape[0], _ptr(idx), nb, _ptr(out)))
        return out

    def mlp_step(self, feat, y, idx=None, lr=1e-3, want_loss=True, grad=None):
        nb = self._batch(feat, y, idx)
        loss = C.c_float(0.0)
        _check(lib().tc_mlp_step(self._h, _ptr(feat), _ptr(y), feat.shape[0], _ptr(idx), nb, float(lr),
                                 C.byref(loss) if want_loss else None, _ptr(grad)))
        return float(loss.value) if want_loss else None

    # -- reference sums --------------------------------------------------
    def direct(self, targets: torch.Tensor, G: float = 1.0, eps: float = 1e-2):
        """FP64 direct sum for the given original body indices (int32 CUDA
        tensor): (acc [nt][3], pot [nt]) FP64 CUDA tensors."""
        self._dev(targets, "targets")
        if targets.dtype != torch.int32 or targets.dim() != 1:
            raise TypeError("targets must be a 1-D int32 tensor")
        dev = self.stream.device
        acc = torch.empty((len(targets), 3), dtype=torch.float64, device=dev)
        pot = torch.empty(len(targets), dtype=torch.float64, device=dev)
        _check(lib().tc_direct(self._h, _ptr(targets), len(targets), float(G), float(eps), _ptr(acc), _ptr(pot)))
        return acc, pot

    def lists_count(self, want_counts: bool = False):
        """Per-body walks (count pass): total list entries and, optionally,
        the per-body counts (u32 CUDA tensor, bodies in key order)."""
        tot = C.c_int64()
        cnt = torch.empty(self.n, dtype=torch.int32, device=self.stream.device) if want_counts else None
        _check(lib().tc_lists_count(self._h, C.byref(tot), _ptr(cnt)))
        return int(tot.value), cnt

    def lists_forces(self, G: float = 1.0, eps: float = 1e-2, lists=None, want_pot=True):
        """Per-body lists written to `lists` (u32/int32 CUDA tensor of at
        least the counted total; allocated if None) and summed."""
        dev = self.stream.device
        if lists is None:
            total, _ = self.lists_count()
            lists = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
        self._dev(lists, "lists")
        acc = torch.empty((self.n, self.dim), dtype=torch.float32, device=dev)
        pot = torch.empty(self.n, dtype=torch.float32, device=dev) if want_pot else None
        _check(lib().tc_lists_forces(self._h, float(G), float(eps), _ptr(lists), lists.numel(), _ptr(acc), _ptr(pot)))
        return acc, pot, lists

    def fmm_plan(self, theta: float):
        """Dual tree traversal of the fast multipole method at theta into a
        device buffer this object owns (grown, and the plan retried, while a
        capacity is short).  Returns (widest level, M2L pairs, P2P pairs)."""
        ncells = self.num_cells()
        caps = list(getattr(self, "_fmm_caps", None) or (max(64, 8 * ncells), max(64, 64 * ncells),
                                                        max(64, 16 * ncells)))
        sizes = np.zeros(3, dtype=np.int64)
        while True:
            need = int(lib().tc_fmm_buffer_bytes(ncells, *caps))
            if need == 0:
                raise TcError(TC_EINVAL, f"FMM capacities {caps} out of range")
            buf = getattr(self, "_fmm_buf", None)
            if buf is None or buf.numel() < need:
                self._fmm_buf = None
                buf = self._fmm_buf = torch.empty(need, dtype=torch.uint8, device=self.stream.device)
            rc = lib().tc_fmm_plan(self._h, float(theta), _ptr(buf), buf.numel(), *caps,
                                   sizes.ctypes.data_as(C.c_void_p))
            if rc != TC_EWORKSPACE:
                _check(rc)
                break
            grown = [max(c, int(1.25 * z) + 64) if z > c else c for c, z in zip(caps, sizes)]
            caps = grown if grown != caps else [2 * c for c in caps]
        self._fmm_caps = tuple(caps)
        return tuple(int(x) for x in sizes)

    def fmm_forces(self, G: float = 1.0, eps: float = 1e-2, want_pot: bool = True):
        """(acc [n][3], pot [n] or None) of the current FMM plan."""
        dev = self.stream.device
        acc = torch.empty((self.n, 3), dtype=torch.float32, device=dev)
        pot = torch.empty(self.n, dtype=torch.float32, device=dev) if want_pot else None
        _check(lib().tc_fmm_forces(self._h, float(G), float(eps), _ptr(acc), _ptr(pot)))
        return acc, pot

    def fmm_pairs(self, sizes):
        """The current plan's (m2l [k][2], p2p [k][2]) int32 pairs of
        (target, source) pre-order cell indices, grouped by target; sizes as
        returned by fmm_plan."""
        dev = self.stream.device
        m2l = torch.empty((max(sizes[1], 1), 2), dtype=torch.int32, device=dev)
        p2p = torch.empty((max(sizes[2], 1), 2), dtype=torch.int32, device=dev)
        _check(lib().tc_fmm_get_pairs(self._h, _ptr(m2l), _ptr(p2p)))
        return m2l[:sizes[1]], p2p[:sizes[2]]

    def set_split(self, mode):
        """How a group's walk is spread over waves: 1 or True (default) a
        block of 4 waves shares each group's walk for n <= 163840; 2 split
        walks for n <= 12288 in 3D and n <= 24576 in 2D, else as 1; 0 or
        False one wave per group at any n."""
        mode = int(mode)
        _check(lib().tc_set_split(self._h, mode))

    def set_multipole(self, order: int):
        """1: monopole cells (default); 2: add quadrupole terms (3D)."""
        _check(lib().tc_set_multipole(self._h, int(order)))

    def set_accumulation(self, compensated: bool):
        """Compensated chunk sums (default) or one plain running FP32 sum."""
        _check(lib().tc_set_accumulation(self._h, TC_ACC_COMPENSATED if compensated else TC_ACC_PLAIN))

    def set_graph(self, on: bool):
        """Replay the pre-force part of leapfrog steps as a HIP graph (default off)."""
        _check(lib().tc_set_graph(self._h, int(bool(on))))

    def set_timing(self, on: bool):
        _check(lib().tc_set_timing(self._h, int(bool(on))))

    def set_stage_timing(self, on: bool):
        """Events around every stage of the following calls (see stage_timing)."""
        _check(lib().tc_set_stage_timing(self._h, int(bool(on))))

    def stage_timing(self) -> dict:
        """{stage name: (total ms, occurrences)} since set_stage_timing(True)."""
        ms = np.zeros(len(STAGES))
        cnt = np.zeros(len(STAGES), np.int64)
        _check(lib().tc_get_stage_timing(self._h, ms.ctypes.data_as(C.c_void_p), cnt.ctypes.data_as(C.c_void_p)))
        return {name: (float(ms[k]), int(cnt[k])) for k, name in enumerate(STAGES)}

    def timing(self):
        ms, k = C.c_double(), C.c_int64()
        _check(lib().tc_get_timing(self._h, C.byref(ms), C.byref(k)))
        return float(ms.value), int(k.value)
