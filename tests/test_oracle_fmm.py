"""Pins of the oracle's fast multipole method against what the mathematics
fixes: closed forms of the expansions, their order of convergence, the
exactness of moving a local expansion, the direct sum at theta = 0, and the
partition of every body's sources by the dual tree traversal."""
import numpy as np
import pytest

import oracle
import workloads


def test_m2l_two_body_quadrupole_closed_form():
    # two masses m at +-a on z: the potential on the axis at distance R is
    # m/(R-a) + m/(R+a) = (2m/R)(1 + a^2/R^2 + ...); the expansion to the
    # quadrupole keeps the first two terms, and its z-gradient is their
    # derivative
    m, a, R = 0.7, 0.3, 5.0
    Q6 = np.array([-2 * m * a * a, -2 * m * a * a, 4 * m * a * a, 0.0, 0.0, 0.0])
    lam = oracle.fmm_m2l(2 * m, Q6, np.array([0.0, 0.0, R]), 0.0)
    assert lam[0] == pytest.approx((2 * m / R) * (1 + a * a / R**2), rel=1e-14)
    assert lam[3] == pytest.approx(-(2 * m / R**2) * (1 + 3 * a * a / R**2), rel=1e-14)
    assert lam[1] == 0.0 and lam[2] == 0.0
    # the same pair off the axis: the truncated expansion agrees with the
    # exact potential to O((a/R)^4)
    Rv = np.array([3.0, 2.0, 4.0])
    lam = oracle.fmm_m2l(2 * m, Q6, Rv, 0.0)
    exact = m / np.linalg.norm(Rv - [0, 0, a]) + m / np.linalg.norm(Rv + [0, 0, a])
    r = np.linalg.norm(Rv)
    assert abs(lam[0] - exact) / exact < 3 * (a / r) ** 4


def test_m2l_point_source_exact_at_centre():
    # with no quadrupole the coefficients at the centre are the softened
    # potential and field of a point mass
    src, M, eps = np.array([3.0, -1.0, 2.0]), 1.3, 0.05
    lam = oracle.fmm_m2l(M, np.zeros(6), -src, eps)
    d = src
    s = (d @ d + eps * eps) ** -0.5
    acc, pot = oracle.fmm_l2p(lam, np.zeros(3), G=2.0)
    np.testing.assert_allclose(acc, 2.0 * M * d * s**3, rtol=1e-14)
    assert pot == pytest.approx(-2.0 * M * s, rel=1e-14)


def test_l2p_order_of_convergence():
    # a third-order local expansion: potential error O(h^4), field O(h^3);
    # halving the offset divides them by 16 and 8 (a wrong or missing term
    # of any order would lower the ratio)
    src, M, eps = np.array([3.0, -1.0, 2.0]), 1.3, 0.05
    lam = oracle.fmm_m2l(M, np.zeros(6), -src, eps)
    u = np.array([0.3, 0.5, -0.4])
    u /= np.linalg.norm(u)
    ea, ep = [], []
    for h in [0.2, 0.1, 0.05]:
        d = src - h * u
        s = (d @ d + eps * eps) ** -0.5
        acc, pot = oracle.fmm_l2p(lam, h * u)
        ea.append(np.linalg.norm(acc - M * d * s**3))
        ep.append(abs(pot + M * s))
    assert 7.6 < ea[0] / ea[1] < 8.4 and 7.8 < ea[1] / ea[2] < 8.2
    assert 14.5 < ep[0] / ep[1] < 16.5 and 15.0 < ep[1] / ep[2] < 16.5


def test_l2l_is_exact():
    # a local expansion is a cubic polynomial; moving its centre re-expands
    # the same polynomial, so both evaluate alike everywhere
    rng = np.random.default_rng(7)
    lam = np.zeros(40)
    for _ in range(3):
        lam += oracle.fmm_m2l(rng.uniform(0.5, 2), rng.normal(size=6) * [1, 1, 0, 1, 1, 1] * 0.1,
                              rng.normal(size=3) * 4 + 8, 0.01)
    t = np.array([0.2, -0.1, 0.15])
    moved = oracle.fmm_l2l(lam, t)
    for x in rng.normal(size=(5, 3)) * 0.3:
        a1, p1 = oracle.fmm_l2p(lam, x)
        a2, p2 = oracle.fmm_l2p(moved, x - t)
        np.testing.assert_allclose(a2, a1, rtol=1e-12, atol=1e-15)
        assert p2 == pytest.approx(p1, rel=1e-13)


def test_theta_zero_is_the_direct_sum():
    w = workloads.plummer_sphere(n=3000, seed=11)
    t = oracle.Tree(w.pos, w.mass, 16)
    m2l, p2p = oracle.fmm_pairs(t, 0.0)
    assert len(m2l) == 0
    acc, pot = oracle.fmm_forces(t, 0.0, G=1.5, eps=w.eps)
    ad, pd = oracle.direct(w.pos, w.mass, G=1.5, eps=w.eps)
    assert oracle.rel_l2(acc, ad) < 1e-13 and oracle.rel_l2(pot, pd) < 1e-13


def _ancestors(parent, c):
    out = [c]
    while parent[out[-1]] >= 0:
        out.append(parent[out[-1]])
    return out


@pytest.mark.parametrize("theta", [0.4, 0.8])
def test_traversal_partitions_every_bodys_sources(theta):
    # for every leaf, the sources reached through M2L at the leaf or any
    # ancestor plus its direct partners are all bodies, each exactly once
    w = workloads.plummer_sphere(n=2000, seed=12)
    t = oracle.Tree(w.pos, w.mass, 8)
    cl = t.cells()
    begin, count, parent, leaf = cl["begin"], cl["count"], cl["parent"], cl["leaf"]
    m2l, p2p = oracle.fmm_pairs(t, theta)
    assert len(m2l) > 0
    by_target_m = {}
    for a, b in m2l:
        by_target_m.setdefault(int(a), []).append(int(b))
    by_target_p = {}
    for a, b in p2p:
        assert leaf[a] and leaf[b]
        by_target_p.setdefault(int(a), []).append(int(b))
    for c in np.flatnonzero(leaf):
        hits = np.zeros(t.n, np.int64)
        for anc in _ancestors(parent, int(c)):
            for b in by_target_m.get(anc, []):
                hits[begin[b]:begin[b] + count[b]] += 1
        for b in by_target_p.get(int(c), []):
            hits[begin[b]:begin[b] + count[b]] += 1
        assert (hits == 1).all(), (c, np.unique(hits))


def test_fmm_error_falls_with_theta():
    # statistical sanity, not a pin: smaller theta, smaller error
    w = workloads.plummer_sphere(n=4096, seed=13)
    t = oracle.Tree(w.pos, w.mass, 16)
    ad, _ = oracle.direct(w.pos, w.mass, eps=w.eps)
    errs = [oracle.rel_l2(oracle.fmm_forces(t, th, eps=w.eps)[0], ad) for th in (0.3, 0.5, 0.8)]
    assert errs[0] < errs[1] < errs[2] < 3e-2
