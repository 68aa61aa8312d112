"""FP64 CPU oracle for the treecode hot path: TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1211_2293_amd``) and never imports it; the only module it shares with
that side is the seeded input generator ``workloads`` (random draws only: the
network's initial parameters come from there).

Contents
--------
* ``liboracle.so`` (``oracle.c``): the FP64 direct sum and the FP64 treecode
  (root cube, Morton digits, recursive subdivision, moments, opening
  criterion, walk, forces) of §3.1 of the paper.
* numpy references written from the same section: a direct sum for small N,
  a naive geometric subdivision (no keys) used to pin the key-based tree,
  leapfrog (kick-drift-kick) and FP64 diagnostics.
* ``mlp``: the learned-closure reference (FP64 MLP with BF16 emulation).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    """Load liboracle.so, building it first if it is missing."""
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        P = C.c_void_p
        i64, i32, dbl = C.c_int64, C.c_int, C.c_double
        L.orc_direct.argtypes = [i64, i32, P, P, dbl, dbl, i64, P, P, P]
        L.orc_direct.restype = None
        L.orc_tree_build.argtypes = [i64, i32, P, P, i32]
        L.orc_tree_build.restype = P
        L.orc_tree_free.argtypes = [P]
        L.orc_tree_free.restype = None
        L.orc_tree_ncells.argtypes = [P]
        L.orc_tree_ncells.restype = i64
        L.orc_tree_root.argtypes = [P, P, P]
        L.orc_tree_root.restype = None
        L.orc_tree_bodies.argtypes = [P, P, P, P]
        L.orc_tree_bodies.restype = None
        L.orc_tree_cells.argtypes = [P] * 12
        L.orc_tree_cells.restype = None
        L.orc_mac_radii.argtypes = [P, dbl, P]
        L.orc_mac_radii.restype = None
        L.orc_walk_counts.argtypes = [P, dbl, i32, P, P]
        L.orc_walk_counts.restype = None
        L.orc_walk_items.argtypes = [P, dbl, i32, i64, P, i64]
        L.orc_walk_items.restype = i64
        L.orc_tree_forces.argtypes = [P, dbl, i32, dbl, dbl, i64, P, P, P]
        L.orc_tree_forces.restype = None
        L.orc_groups.argtypes = [P, i32, i64, P, P]
        L.orc_groups.restype = i64
        L.orc_walk_counts_ranges.argtypes = [P, dbl, i64, P, P, P, P]
        L.orc_walk_counts_ranges.restype = None
        L.orc_walk_tests_ranges.argtypes = [P, dbl, i64, P, P, P]
        L.orc_walk_tests_ranges.restype = None
        L.orc_tree_forces_ranges.argtypes = [P, dbl, dbl, dbl, i64, P, P, i32, P, P]
        L.orc_tree_forces_ranges.restype = None
        L.orc_residuals.argtypes = [P, dbl, dbl, i64, P, i64, P, P, P, P, P]
        L.orc_residuals.restype = i64
        L.orc_sorted_positions.argtypes = [P, i64, P, P]
        L.orc_sorted_positions.restype = None
        L.orc_walk_items_range.argtypes = [P, dbl, i64, i64, P, i64]
        L.orc_walk_items_range.restype = i64
        L.orc_set_num_threads.argtypes = [i32]
        L.orc_set_num_threads.restype = None
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = i32
        L.orc_fmm_pairs.argtypes = [P, dbl, P, i64, P, i64, P, P]
        L.orc_fmm_pairs.restype = i32
        L.orc_fmm_forces.argtypes = [P, dbl, dbl, dbl, P, P]
        L.orc_fmm_forces.restype = i32
        L.orc_fmm_m2l.argtypes = [dbl, P, P, dbl, P]
        L.orc_fmm_m2l.restype = None
        L.orc_fmm_l2l.argtypes = [P, P, P]
        L.orc_fmm_l2l.restype = None
        L.orc_fmm_l2p.argtypes = [P, P, dbl, P, P]
        L.orc_fmm_l2p.restype = None
        _LIB = L
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(k: int) -> None:
    lib().orc_set_num_threads(int(k))


# --------------------------------------------------------------------------
# Direct sum (§3.1 force law with Plummer softening), FP64.
# --------------------------------------------------------------------------
def direct(pos, mass, G=1.0, eps=1e-3, targets=None):
    """FP64 direct sum for the given original-order target indices (all if
    None).  Returns (acc [nt][dim], pot [nt])."""
    pos, mass = _f64(pos), _f64(mass)
    n, dim = pos.shape
    if targets is None:
        nt, tp = n, None
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tp = len(targets), targets
    acc = np.zeros((nt, dim))
    pot = np.zeros(nt)
    lib().orc_direct(n, dim, _p(pos), _p(mass), G, eps, nt, _p(tp), _p(acc), _p(pot))
    return acc, pot


def direct_numpy(pos, mass, G=1.0, eps=1e-3):
    """The same definition as ``direct`` with numpy broadcasting (N <= ~2000):
    an independent second implementation used to pin the C one."""
    pos, mass = _f64(pos), _f64(mass)
    d = pos[None, :, :] - pos[:, None, :]          # d[i, j] = x_j - x_i
    r2 = (d * d).sum(-1) + eps * eps
    np.fill_diagonal(r2, 1.0)                      # self term removed below
    inv = 1.0 / np.sqrt(r2)
    np.fill_diagonal(inv, 0.0)
    w = mass[None, :] * inv
    acc = G * ((w * inv * inv)[:, :, None] * d).sum(1)
    pot = -G * w.sum(1)
    return acc, pot


# --------------------------------------------------------------------------
# Treecode (§3.1), FP64.
# --------------------------------------------------------------------------
class Tree:
    """FP64 treecode tree over positions ``pos`` [n][dim] and masses."""

    def __init__(self, pos, mass, leaf_cap):
        self.pos, self.mass = _f64(pos), _f64(mass)
        self.n, self.dim = self.pos.shape
        self.leaf_cap = leaf_cap
        self.L = 21 if self.dim == 3 else 31
        h = lib().orc_tree_build(self.n, self.dim, _p(self.pos), _p(self.mass), leaf_cap)
        if not h:
            raise ValueError("bad arguments to orc_tree_build")
        self._h = C.c_void_p(h)
        self.ncells = int(lib().orc_tree_ncells(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            _LIB.orc_tree_free(h)
            self._h = None

    def root(self):
        lo = np.zeros(self.dim)
        size = np.zeros(1)
        lib().orc_tree_root(self._h, _p(lo), _p(size))
        return lo, float(size[0])

    def bodies(self):
        ko = np.zeros(self.n, np.uint64)
        ks = np.zeros(self.n, np.uint64)
        pm = np.zeros(self.n, np.uint32)
        lib().orc_tree_bodies(self._h, _p(ko), _p(ks), _p(pm))
        return {"key_orig": ko, "key": ks, "perm": pm}

    def cells(self):
        Cn, d = self.ncells, self.dim
        out = {
            "level": np.zeros(Cn, np.int32), "prefix": np.zeros(Cn, np.uint64),
            "begin": np.zeros(Cn, np.int64), "count": np.zeros(Cn, np.int64),
            "parent": np.zeros(Cn, np.int32), "skip": np.zeros(Cn, np.int32),
            "nch": np.zeros(Cn, np.int32), "leaf": np.zeros(Cn, np.int32),
            "M": np.zeros(Cn), "com": np.zeros((Cn, d)), "Q": np.zeros((Cn, 6)),
        }
        o = out
        lib().orc_tree_cells(self._h, _p(o["level"]), _p(o["prefix"]), _p(o["begin"]),
                             _p(o["count"]), _p(o["parent"]), _p(o["skip"]), _p(o["nch"]),
                             _p(o["leaf"]), _p(o["M"]), _p(o["com"]), _p(o["Q"]))
        return out

    def mac_radii(self, theta):
        r = np.zeros(self.ncells)
        lib().orc_mac_radii(self._h, float(theta), _p(r))
        return r

    def walk_counts(self, theta, gs=64):
        G = (self.n + gs - 1) // gs
        m2p = np.zeros(G, np.int64)
        p2p = np.zeros(G, np.int64)
        lib().orc_walk_counts(self._h, float(theta), gs, _p(m2p), _p(p2p))
        return m2p, p2p

    def walk_items(self, theta, g, gs=64):
        """Terminal items of group g in walk order: c >= 0 accepted cell,
        -1-c opened leaf c."""
        cap = 1 << 16
        while True:
            buf = np.zeros(cap, np.int32)
            k = int(lib().orc_walk_items(self._h, float(theta), gs, int(g), _p(buf), cap))
            if k <= cap:
                return buf[:k]
            cap = k

    def groups(self, gs=64, cluster=1024):
        """Groups of at most gs consecutive sorted bodies that never straddle
        a cluster cell (a maximal cell of at most `cluster` bodies, or a
        deeper leaf): returns (first body, size) arrays."""
        ng = int(lib().orc_groups(self._h, gs, cluster, None, None))
        gb = np.zeros(ng, np.int64)
        gc = np.zeros(ng, np.int64)
        lib().orc_groups(self._h, gs, cluster, _p(gb), _p(gc))
        return gb, gc

    def walk_counts_groups(self, theta, gbeg, gcnt):
        gbeg = np.ascontiguousarray(gbeg, np.int64)
        gcnt = np.ascontiguousarray(gcnt, np.int64)
        m2p = np.zeros(len(gbeg), np.int64)
        p2p = np.zeros(len(gbeg), np.int64)
        lib().orc_walk_counts_ranges(self._h, float(theta), len(gbeg), _p(gbeg), _p(gcnt),
                                     _p(m2p), _p(p2p))
        return m2p, p2p

    def walk_tests_groups(self, theta, gbeg, gcnt):
        """Cells whose opening test runs in each group's walk (the root and
        every child of an opened cell): a measure of the walk's work."""
        gbeg = np.ascontiguousarray(gbeg, np.int64)
        gcnt = np.ascontiguousarray(gcnt, np.int64)
        tests = np.zeros(len(gbeg), np.int64)
        lib().orc_walk_tests_ranges(self._h, float(theta), len(gbeg), _p(gbeg), _p(gcnt), _p(tests))
        return tests

    def forces_groups(self, theta, gbeg, gcnt, G=1.0, eps=1e-3, acc=None, pot=None, order=1):
        """Treecode forces of the bodies of the given groups, original
        order; bodies outside them keep the values in acc/pot (zeros by
        default).  order=2 adds every accepted cell's quadrupole term (3D)."""
        gbeg = np.ascontiguousarray(gbeg, np.int64)
        gcnt = np.ascontiguousarray(gcnt, np.int64)
        if acc is None:
            acc = np.zeros((self.n, self.dim))
        if pot is None:
            pot = np.zeros(self.n)
        lib().orc_tree_forces_ranges(self._h, float(theta), G, eps, len(gbeg), _p(gbeg), _p(gcnt), int(order),
                                     _p(acc), _p(pot))
        return acc, pot

    def walk_forces(self, theta, G=1.0, eps=1e-3, gs=64, cluster=1024, order=1):
        """Treecode forces with the walk groups of the GPU path: runs of at
        most gs consecutive sorted bodies inside cluster cells of at most
        `cluster` bodies."""
        gb, gc = self.groups(gs, cluster)
        return self.forces_groups(theta, gb, gc, G=G, eps=eps, order=order)

    def walk_items_range(self, theta, b, e):
        cap = 1 << 16
        while True:
            buf = np.zeros(cap, np.int32)
            k = int(lib().orc_walk_items_range(self._h, float(theta), int(b), int(e), _p(buf), cap))
            if k <= cap:
                return buf[:k]
            cap = k

    def sorted_positions(self, orig):
        orig = np.ascontiguousarray(orig, np.int64)
        pos = np.zeros(len(orig), np.int64)
        lib().orc_sorted_positions(self._h, len(orig), _p(orig), _p(pos))
        return pos

    def residuals(self, theta, eps, targets):
        """Training pairs of the learned closure for the given original
        body indices: dict with feat [P][10] (FP32), y [P][3] (FP64), target
        (index into targets), cell (pre-order index), count per target."""
        tpos = self.sorted_positions(targets)
        nt = len(tpos)
        cnt = np.zeros(nt, np.int64)
        total = int(lib().orc_residuals(self._h, float(theta), float(eps), nt, _p(tpos), 0, None,
                                        None, None, None, _p(cnt)))
        feat = np.zeros((total, 10), np.float32)
        y = np.zeros((total, 3))
        tg = np.zeros(total, np.int64)
        cl = np.zeros(total, np.int32)
        lib().orc_residuals(self._h, float(theta), float(eps), nt, _p(tpos), total, _p(feat), _p(y),
                            _p(tg), _p(cl), _p(cnt))
        return {"feat": feat, "y": y, "target": tg, "cell": cl, "count": cnt}

    def forces(self, theta, G=1.0, eps=1e-3, gs=64, groups=None):
        """FP64 treecode accelerations and potentials in original order.
        With ``groups`` only those groups' bodies are computed (others 0)."""
        acc = np.zeros((self.n, self.dim))
        pot = np.zeros(self.n)
        if groups is None:
            lib().orc_tree_forces(self._h, float(theta), gs, G, eps, 0, None, _p(acc), _p(pot))
        else:
            gsel = np.ascontiguousarray(groups, dtype=np.int64)
            lib().orc_tree_forces(self._h, float(theta), gs, G, eps, len(gsel), _p(gsel),
                                  _p(acc), _p(pot))
        return acc, pot


# --------------------------------------------------------------------------
# Fast multipole method (3D): the Cartesian expansions to order 3 and the
# dual tree traversal described in oracle.c.
# --------------------------------------------------------------------------
def fmm_m2l(M, Q6, R, eps):
    """Local expansion (40 full-tensor coefficients: Lam_0, Lam_1[3],
    Lam_2[3][3], Lam_3[3][3][3]) of a source of mass M and traceless
    quadrupole Q6 at offset R = centre - source."""
    lam = np.zeros(40)
    lib().orc_fmm_m2l(float(M), _p(_f64(Q6)), _p(_f64(R)), float(eps), _p(lam))
    return lam


def fmm_l2l(lam, t):
    """The expansion lam moved to a centre t further on."""
    out = np.zeros(40)
    lib().orc_fmm_l2l(_p(_f64(lam)), _p(_f64(t)), _p(out))
    return out


def fmm_l2p(lam, dl, G=1.0):
    """(acc[3], pot) of the expansion at offset dl from its centre."""
    acc = np.zeros(3)
    pot = np.zeros(1)
    lib().orc_fmm_l2p(_p(_f64(lam)), _p(_f64(dl)), float(G), _p(acc), _p(pot))
    return acc, float(pot[0])


def fmm_pairs(tree: "Tree", theta):
    """(m2l [k][2], p2p [k][2]) (target, source) pre-order cell ids of the
    dual tree traversal, in traversal order."""
    L = lib()
    nm, npp = np.zeros(1, np.int64), np.zeros(1, np.int64)
    if L.orc_fmm_pairs(tree._h, float(theta), None, 0, None, 0, _p(nm), _p(npp)) != 0:
        raise ValueError("the FMM is 3D only")
    m2l = np.zeros((int(nm[0]), 2), np.int32)
    p2p = np.zeros((int(npp[0]), 2), np.int32)
    L.orc_fmm_pairs(tree._h, float(theta), _p(m2l), len(m2l), _p(p2p), len(p2p), _p(nm), _p(npp))
    return m2l, p2p


def fmm_forces(tree: "Tree", theta, G=1.0, eps=1e-3):
    """FMM acceleration [n][3] and potential [n] of every body (original order)."""
    acc = np.zeros((tree.n, 3))
    pot = np.zeros(tree.n)
    if lib().orc_fmm_forces(tree._h, float(theta), float(G), float(eps), _p(acc), _p(pot)) != 0:
        raise ValueError("the FMM is 3D only")
    return acc, pot


def group_bodies(tree: Tree, groups, gs=64):
    """Original indices of the bodies of the given groups (sorted order)."""
    perm = tree.bodies()["perm"]
    idx = [np.arange(g * gs, min((g + 1) * gs, tree.n)) for g in groups]
    return perm[np.concatenate(idx)].astype(np.int64)


# --------------------------------------------------------------------------
# Naive geometric subdivision (§3.1: divide the space into 4 or 8 subspaces
# until a subspace holds at most the threshold), with no keys and no sort.
# --------------------------------------------------------------------------
def geometric_tree(pos, leaf_cap, lo, size, L):
    """Cells as (level, frozenset of original body indices), in depth-first
    order with subspaces visited in the order x-high-bit first.  Each
    subspace is split at the midpoint of the cube: a body goes to the upper
    half along an axis iff its offset from the cube's low corner, scaled to
    2^L units, is at least the midpoint.  Pure Python: small N only."""
    pos = _f64(pos)
    n, dim = pos.shape
    scale = 2.0 ** L / size
    t = (pos - np.asarray(lo)[None, :]) * scale      # offset in 2^L units
    out = []

    def rec(level, origin, members):
        out.append((level, frozenset(members)))
        if len(members) <= leaf_cap or level == L:
            return
        half = 2.0 ** (L - level - 1)
        kids = {}
        for b in members:
            code = 0
            sub = []
            for a in range(dim):
                mid = origin[a] + half
                # a body on the far face of the root cube (offset 2^L) is
                # above every midpoint, so it lands in the last subspace
                up = t[b, a] >= mid
                code = (code << 1) | int(up)
                sub.append(origin[a] + half if up else origin[a])
            kids.setdefault(code, (tuple(sub), []))[1].append(b)
        for code in sorted(kids):
            org, mem = kids[code]
            rec(level + 1, org, mem)

    rec(0, tuple(0.0 for _ in range(dim)), list(range(n)))
    return out


# --------------------------------------------------------------------------
# Leapfrog kick-drift-kick and FP64 diagnostics.
# --------------------------------------------------------------------------
def kdk(pos, vel, acc0, dt, force):
    """One kick-drift-kick step: v+ = v + dt/2 a(x); x' = x + dt v+;
    v' = v+ + dt/2 a(x').  ``force(x)`` returns the accelerations.  Returns
    (x', v', a(x'))."""
    vh = vel + 0.5 * dt * acc0
    x1 = pos + dt * vh
    a1 = force(x1)
    v1 = vh + 0.5 * dt * a1
    return x1, v1, a1


def diagnostics(mass, vel, acc, pot):
    """FP64 E_kin, E_pot, momentum and sum m a: E_kin = 1/2 sum m v^2,
    E_pot = 1/2 sum m phi.  Returns 8 numbers: E_kin, E_pot, P[3], F[3]
    (2D fills the z components with 0)."""
    mass, vel, acc, pot = _f64(mass), _f64(vel), _f64(acc), _f64(pot)
    out = np.zeros(8)
    out[0] = 0.5 * np.sum(mass * np.sum(vel * vel, axis=1))
    out[1] = 0.5 * np.sum(mass * pot)
    d = vel.shape[1]
    out[2:2 + d] = (mass[:, None] * vel).sum(0)
    out[5:5 + d] = (mass[:, None] * acc).sum(0)
    return out


def rel_l2(a, ref):
    """Relative L2 error sqrt(sum |a - ref|^2 / sum |ref|^2)."""
    a, ref = np.asarray(a, np.float64), np.asarray(ref, np.float64)
    return float(np.sqrt(((a - ref) ** 2).sum() / (ref ** 2).sum()))
