"""Pins of the FP64 direct sum (the exact softened result of the force law of
§3.1) against closed forms, Newton's third law and a second, independent
numpy implementation."""
import json
import math
import os

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def golden(golden_dir):
    with open(os.path.join(golden_dir, "closed_forms.json")) as f:
        return json.load(f)


def test_two_body_softened_closed_form(golden):
    c = golden["two_body_softened"]
    acc, pot = oracle.direct(np.array(c["pos"], float), np.array(c["mass"]), G=c["G"],
                             eps=math.sqrt(c["eps2"]))
    np.testing.assert_allclose(acc, np.array(c["acc"]), rtol=1e-14, atol=1e-17)
    np.testing.assert_allclose(pot, np.array(c["pot"]), rtol=1e-14)


def test_two_body_scales_with_G_and_mass():
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    a1, p1 = oracle.direct(pos, np.array([1.0, 1.0]), G=1.0, eps=0.0)
    a2, p2 = oracle.direct(pos, np.array([1.0, 3.0]), G=2.0, eps=0.0)
    # body 0 feels G m1 / r^2 toward +x; body 1 feels G m0 / r^2 toward -x
    assert a1[0, 0] == 1.0 and a1[1, 0] == -1.0
    assert a2[0, 0] == 6.0 and a2[1, 0] == -2.0
    assert p2[0] == -6.0 and p2[1] == -2.0


def test_equilateral_triangle(golden):
    c = golden["equilateral_triangle"]
    s = c["side"]
    R = s / math.sqrt(3.0)
    ang = np.array([90.0, 210.0, 330.0]) * math.pi / 180.0
    pos = np.stack([R * np.cos(ang), R * np.sin(ang), np.zeros(3)], axis=1)
    acc, pot = oracle.direct(pos, np.ones(3), G=1.0, eps=0.0)
    for i in range(3):
        mag = np.linalg.norm(acc[i])
        assert abs(mag - c["acc_magnitude"]) < 1e-14
        # points at the centroid (the origin)
        cosang = -np.dot(acc[i], pos[i]) / (mag * np.linalg.norm(pos[i]))
        assert abs(cosang - 1.0) < 1e-14
    np.testing.assert_allclose(pot, c["pot"], rtol=1e-14)


def test_cube_vertices(golden):
    c = golden["cube_vertices"]
    pos = np.array([[x, y, z] for x in (-1.0, 1.0) for y in (-1.0, 1.0) for z in (-1.0, 1.0)])
    acc, pot = oracle.direct(pos, np.ones(8), G=1.0, eps=0.0)
    # every vertex: each component points inward with the same magnitude
    np.testing.assert_allclose(acc * np.sign(pos), c["acc_per_axis"], rtol=1e-14)
    np.testing.assert_allclose(pot, c["pot"], rtol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_newton_third_law(dim):
    rng = np.random.default_rng(11)
    n = 700
    pos = rng.normal(size=(n, dim))
    mass = rng.uniform(0.5, 2.0, n)
    acc, _ = oracle.direct(pos, mass, G=1.0, eps=1e-2)
    total = (mass[:, None] * acc).sum(0)
    scale = np.abs(mass[:, None] * acc).sum()
    assert np.all(np.abs(total) <= 1e-14 * scale)


@pytest.mark.parametrize("dim,eps", [(2, 1e-2), (3, 1e-3), (3, 0.0)])
def test_direct_matches_numpy(dim, eps):
    rng = np.random.default_rng(12)
    n = 500
    pos = rng.uniform(size=(n, dim))
    mass = rng.uniform(0.1, 1.0, n)
    a, p = oracle.direct(pos, mass, G=1.3, eps=eps)
    b, q = oracle.direct_numpy(pos, mass, G=1.3, eps=eps)
    assert oracle.rel_l2(a, b) < 1e-13
    assert oracle.rel_l2(p, q) < 1e-13


def test_direct_targets_subset():
    rng = np.random.default_rng(13)
    pos = rng.uniform(size=(300, 3))
    mass = rng.uniform(0.1, 1.0, 300)
    a, p = oracle.direct(pos, mass, eps=1e-3)
    t = np.array([5, 0, 299, 17])
    b, q = oracle.direct(pos, mass, eps=1e-3, targets=t)
    np.testing.assert_array_equal(a[t], b)
    np.testing.assert_array_equal(p[t], q)
