"""Seeded synthetic inputs for the treecode path.

This module only draws random numbers: it holds none of the method's
arithmetic and imports neither the GPU library nor the oracle, so both can be
fed from it.  Every generator works in FP64 with
``numpy.random.default_rng(seed)`` and rounds to the working dtype (FP32
unless a workload keeps FP64 state); the rounded values are the ground truth
handed to both sides.

The paper states its data-set sizes (10,000 / 50,000 / 100,000 bodies) but
not their distribution (§4.1); the workloads below follow the configurations
this project is measured on, scaled down by ``n`` for tests.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    pos: np.ndarray          # [n][dim]
    vel: np.ndarray          # [n][dim]
    mass: np.ndarray         # [n]
    G: float = 1.0
    eps: float = 1e-2
    theta: float = 0.5
    leaf_cap: int = 16
    dt: float = 1e-3
    steps: int = 10
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.pos.shape[0]

    @property
    def dim(self) -> int:
        return self.pos.shape[1]


def _isotropic(rng, n):
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def plummer(rng, n, a=1.0, M=1.0, G=1.0, rmax_over_a=10.0):
    """Plummer sphere of n bodies, scale a, total mass M: radii by inverting
    the cumulative mass profile, r = a (U^(-2/3) - 1)^(-1/2), redrawn beyond
    rmax; speeds by the rejection method of Aarseth, Henon & Wielen (1974),
    v = q sqrt(2) (1 + r^2)^(-1/4) in G = M = a = 1 units.  Returns positions
    and velocities in FP64, centred on the origin."""
    r = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        u = rng.uniform(0.0, 1.0, todo.size)
        u = np.maximum(u, 1e-300)
        rr = 1.0 / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        ok = rr <= rmax_over_a
        r[todo[ok]] = rr[ok]
        todo = todo[~ok]
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x1 = rng.uniform(0.0, 1.0, todo.size)
        x2 = rng.uniform(0.0, 1.0, todo.size)
        ok = 0.1 * x2 < x1 * x1 * (1.0 - x1 * x1) ** 3.5
        q[todo[ok]] = x1[ok]
        todo = todo[~ok]
    v = q * np.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    pos = _isotropic(rng, n) * r[:, None] * a
    vel = _isotropic(rng, n) * v[:, None] * np.sqrt(G * M / a)
    return pos, vel


def uniform_cube(n=4096, seed=1):
    """3D uniform in [0,1)^3, equal masses 1/N, at rest; FP64 state;
    G = 1, eps = 1e-3, theta = 0.5, leaf_cap = 8, dt = 1e-3, one step."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, (n, 3))
    return Workload("uniform-cube", pos, np.zeros((n, 3)), np.full(n, 1.0 / n),
                    eps=1e-3, theta=0.5, leaf_cap=8, dt=1e-3, steps=1)


def gaussian_disk(n=262_144, seed=2):
    """2D Gaussian disk, sigma = 1, equal masses 1/N, at rest; FP32;
    eps = 1e-2, theta = 0.5, leaf_cap = 16, dt = 1e-3, 10 steps."""
    rng = np.random.default_rng(seed)
    pos = rng.normal(0.0, 1.0, (n, 2))
    return Workload("gaussian-disk-2d", pos.astype(np.float32), np.zeros((n, 2), np.float32),
                    np.full(n, 1.0 / n, np.float32), eps=1e-2, theta=0.5, leaf_cap=16,
                    dt=1e-3, steps=10)


def plummer_sphere(n=1_048_576, seed=3):
    """3D Plummer sphere, a = 1, M = 1, equal masses, virial velocities;
    FP32; eps = 1e-2, theta = 0.5, leaf_cap = 16, dt = 1e-3, 10 steps."""
    rng = np.random.default_rng(seed)
    pos, vel = plummer(rng, n)
    return Workload("plummer-3d", pos.astype(np.float32), vel.astype(np.float32),
                    np.full(n, 1.0 / n, np.float32), eps=1e-2, theta=0.5, leaf_cap=16,
                    dt=1e-3, steps=10)


def two_plummer(n=4_194_304, seed=4):
    """Two Plummer spheres (a = 1, masses 1 and 0.3, body counts in that
    ratio, equal body masses 1.3/N), centres 10 apart on x with the centre
    of mass at the origin, each moving at 0.5 toward the other; FP32;
    eps = 1e-2, theta in {0.3, 0.5, 0.7}."""
    rng = np.random.default_rng(seed)
    n1 = int(round(n / 1.3))
    n2 = n - n1
    p1, v1 = plummer(rng, n1, M=1.0)
    p2, v2 = plummer(rng, n2, M=0.3)
    p1[:, 0] -= 10.0 * 0.3 / 1.3
    p2[:, 0] += 10.0 * 1.0 / 1.3
    v1[:, 0] += 0.5
    v2[:, 0] -= 0.5
    pos = np.concatenate([p1, p2])
    vel = np.concatenate([v1, v2])
    mass = np.full(n, 1.3 / n)
    return Workload("two-plummer", pos.astype(np.float32), vel.astype(np.float32),
                    mass.astype(np.float32), eps=1e-2, theta=0.5, leaf_cap=16,
                    extra={"thetas": [0.3, 0.5, 0.7], "n1": n1, "n2": n2})


def clustered(n=16_777_216, seed=5, nclusters=32):
    """32 Plummer subclusters with scale radii 10^U(-2,-1), centres uniform
    in [0,10)^3, Pareto(2.35) body masses (x_m = 1) normalised to a total of
    1; each subcluster is truncated at 10 scale radii and carries virial
    velocities for its own mass, no bulk motion; FP32; eps = 1e-3,
    dt = 5e-4, 100 steps."""
    rng = np.random.default_rng(seed)
    per = np.full(nclusters, n // nclusters)
    per[: n - per.sum()] += 1
    m = (1.0 - rng.uniform(0.0, 1.0, n)) ** (-1.0 / 2.35)
    m /= m.sum()
    radii = 10.0 ** rng.uniform(-2.0, -1.0, nclusters)
    centres = rng.uniform(0.0, 10.0, (nclusters, 3))
    pos = np.empty((n, 3))
    vel = np.empty((n, 3))
    o = 0
    for k in range(nclusters):
        nk = int(per[k])
        Mk = float(m[o:o + nk].sum())
        p, v = plummer(rng, nk, a=float(radii[k]), M=Mk)
        pos[o:o + nk] = p + centres[k]
        vel[o:o + nk] = v
        o += nk
    return Workload("clustered-32", pos.astype(np.float32), vel.astype(np.float32),
                    m.astype(np.float32), eps=1e-3, theta=0.7, leaf_cap=16, dt=5e-4,
                    steps=100, extra={"radii": radii, "centres": centres})


def sample_indices(n, count=8192, seed=104):
    """Seeded sample of body indices (without replacement) for error checks."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(count, n), replace=False)).astype(np.int64)


# closure network shapes in the library's canonical parameter order
MLP_SHAPES = [(10, 64), (64,), (64, 64), (64,), (64, 3), (3,)]


def mlp_params(seed=0):
    """Seeded initial network parameters, FP32, canonical order (W1 [10][64],
    b1, W2 [64][64], b2, W3 [64][3], b3): weights uniform in +-1/sqrt(fan_in),
    biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            bound = 1.0 / np.sqrt(shape[0])
            parts.append(rng.uniform(-bound, bound, shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def batch_order(npairs, steps, batch, seed=0):
    """Seeded sample order for minibatch training: concatenated random
    permutations of range(npairs), at least steps * batch entries, int32."""
    rng = np.random.default_rng(seed)
    reps = (steps * batch) // max(npairs, 1) + 1
    return np.concatenate([rng.permutation(npairs) for _ in range(reps)]).astype(np.int32)


def training_draws(npairs, epochs=40, batch=4096, init_seed=0, order_seed=0):
    """The random draws of one training run: the initial parameters
    (mlp_params(init_seed)) and a minibatch order long enough for
    max(1, epochs * npairs // batch) steps of `batch` samples."""
    steps = max(1, epochs * int(npairs) // batch)
    return mlp_params(init_seed), batch_order(npairs, steps, batch, order_seed)


BY_NAME = {
    "uniform-cube": uniform_cube,
    "gaussian-disk-2d": gaussian_disk,
    "plummer-3d": plummer_sphere,
    "two-plummer": two_plummer,
    "clustered-32": clustered,
}
