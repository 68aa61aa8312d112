"""Pins of the oracle's time step (each body updates position and velocity
from the computed forces, §3.1; kick-drift-kick leapfrog) and of its FP64
diagnostics, against time reversibility, Kepler's two-body orbit and closed
forms."""
import math

import numpy as np

import oracle


def _direct_force(mass, eps=0.0):
    return lambda x: oracle.direct(x, mass, G=1.0, eps=eps)[0]


def test_time_reversibility():
    rng = np.random.default_rng(31)
    n = 64
    x = rng.normal(0, 1, (n, 3))
    v = rng.normal(0, 0.3, (n, 3))
    m = np.full(n, 1.0 / n)
    f = _direct_force(m, eps=0.05)
    a = f(x)
    x1, v1, a1 = x, v, a
    for _ in range(10):
        x1, v1, a1 = oracle.kdk(x1, v1, a1, 1e-3, f)
    for _ in range(10):
        x1, v1, a1 = oracle.kdk(x1, v1, a1, -1e-3, f)
    assert np.abs(x1 - x).max() < 1e-13
    assert np.abs(v1 - v).max() < 1e-13


def test_circular_orbit_energy_and_period():
    # two equal masses m = 0.5 on a circular orbit of separation 1, G = 1:
    # relative speed sqrt(G M / r) = 1, period 2 pi sqrt(r^3 / (G M)) = 2 pi
    m = np.array([0.5, 0.5])
    x = np.array([[-0.5, 0.0, 0.0], [0.5, 0.0, 0.0]])
    v = np.array([[0.0, -0.5, 0.0], [0.0, 0.5, 0.0]])
    f = _direct_force(m)
    a = f(x)
    acc0, pot0 = oracle.direct(x, m, eps=0.0)
    e0 = oracle.diagnostics(m, v, acc0, pot0)
    # closed form: E_kin = 2 * 1/2 * 0.5 * 0.25 = 0.125, E_pot = -G m m / r = -0.25
    assert abs(e0[0] - 0.125) < 1e-15 and abs(e0[1] + 0.25) < 1e-15
    for dt, tol in ((2 * math.pi / 2000, 2e-5), (2 * math.pi / 4000, 5e-6)):
        x1, v1, a1 = x.copy(), v.copy(), a.copy()
        emax = 0.0
        for _ in range(int(round(2 * math.pi / dt))):
            x1, v1, a1 = oracle.kdk(x1, v1, a1, dt, f)
            acc, pot = oracle.direct(x1, m, eps=0.0)
            d = oracle.diagnostics(m, v1, acc, pot)
            emax = max(emax, abs((d[0] + d[1]) - (e0[0] + e0[1])))
        assert emax < tol                       # second order in dt
        assert np.abs(x1 - x).max() < 50 * tol  # back where it started
    # total momentum of the symmetric start is zero and stays zero
    assert np.abs(oracle.diagnostics(m, v1, a1, pot)[2:5]).max() < 1e-15


def test_diagnostics_closed_form_two_body():
    m = np.array([2.0, 3.0])
    x = np.array([[0.0, 0.0], [0.0, 2.0]])
    v = np.array([[1.0, 0.0], [0.0, -1.0]])
    acc, pot = oracle.direct(x, m, eps=0.0)
    d = oracle.diagnostics(m, v, acc, pot)
    assert d[0] == 0.5 * (2.0 * 1.0 + 3.0 * 1.0)
    assert d[1] == -2.0 * 3.0 / 2.0
    np.testing.assert_array_equal(d[2:5], [2.0, -3.0, 0.0])
    np.testing.assert_allclose(d[5:8], [0.0, 0.0, 0.0], atol=1e-15)
