"""Pins of the oracle's model functions against what the paper fixes.

- The velocity set is the cube-symmetric 15-velocity set of Sec. 2, Eq. (vv).
- The equilibrium of Eqs. (eq)/(e18) must satisfy the five moment
  constraints (e1)-(e5) exactly (up to rounding), for any state and any
  admissible constants: a dropped term, a wrong sign or a wrong group
  coefficient breaks at least one of them.
- Moment recovery is the inverse of the equilibrium on (rho, u, T).
- minmod of Sec. 3 is the median of (X, Y, 0).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")
TRIPLES = json.load(open(GOLDEN))["parameter_triples"]["triples"]


def test_velocity_set_is_the_papers():
    c1, c2, eta0 = 8.0, 24.0, 8.0
    v, eta = oracle.velocities(c1, c2, eta0)
    k = c2 / math.sqrt(3.0)
    expect = {(0.0, 0.0, 0.0)}
    for a in range(3):
        for s in (1.0, -1.0):
            e = [0.0, 0.0, 0.0]
            e[a] = s * c1
            expect.add(tuple(e))
    for sx, sy, sz in itertools.product((1.0, -1.0), repeat=3):
        expect.add((sx * k, sy * k, sz * k))
    got = {tuple(float(x) for x in row) for row in v}
    assert got == expect
    assert eta[0] == eta0 and np.all(eta[1:] == 0.0)
    # documented order: rest, +x,-x,+y,-y,+z,-z, then diagonals with bit a of
    # (i-7) giving the sign of axis a (clear -> +)
    assert np.array_equal(v[1], [c1, 0, 0]) and np.array_equal(v[2], [-c1, 0, 0])
    assert np.array_equal(v[5], [0, 0, c1]) and np.array_equal(v[6], [0, 0, -c1])
    for d in range(8):
        for a in range(3):
            assert v[7 + d][a] == (-k if (d >> a) & 1 else k)


@pytest.mark.parametrize("triple", TRIPLES)
@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0, 1.2])
def test_equilibrium_satisfies_moment_constraints(triple, gamma):
    c1, c2, eta0 = triple
    b = 2.0 / (gamma - 1.0)
    v, eta = oracle.velocities(c1, c2, eta0)
    rng = np.random.default_rng(hash((tuple(triple), gamma)) % 2 ** 32)
    for _ in range(20):
        rho = rng.uniform(0.05, 200.0)
        u = rng.uniform(-1.2, 1.2, size=3) * c1
        T = math.exp(rng.uniform(math.log(0.05), math.log(100.0)))
        f = oracle.equilibrium(c1, c2, eta0, gamma, rho, *u, T)
        P = rho * T
        usq = float(u @ u)
        e2 = (v * v).sum(axis=1) + eta * eta
        vn = np.sqrt((v * v).sum(axis=1))
        af = np.abs(f)
        tol = 1e-13  # rounding of 15-term sums, scaled by the sum of |terms|
        # (e1) mass
        assert abs(f.sum() - rho) <= tol * af.sum()
        # (e2) momentum
        np.testing.assert_allclose(f @ v, rho * u, rtol=0, atol=tol * (af @ vn))
        # (e3) energy
        assert abs(f @ e2 - rho * (b * T + usq)) <= tol * (af @ e2)
        # (e4) momentum flux
        Pi = np.einsum("i,ia,ib->ab", f, v, v)
        np.testing.assert_allclose(Pi, P * np.eye(3) + rho * np.outer(u, u), rtol=0,
                                   atol=tol * (af @ (vn * vn)))
        # (e5) energy flux
        q = np.einsum("i,i,ia->a", f, e2, v)
        np.testing.assert_allclose(q, rho * ((b + 2.0) * T + usq) * u, rtol=0,
                                   atol=tol * (af @ (e2 * vn)))


@pytest.mark.parametrize("triple", TRIPLES)
def test_moments_invert_equilibrium(triple):
    c1, c2, eta0 = triple
    rng = np.random.default_rng(7)
    for _ in range(20):
        rho = rng.uniform(0.1, 10.0)
        u = rng.uniform(-1.0, 1.0, size=3) * c1
        T = rng.uniform(0.1, 50.0)
        f = oracle.equilibrium(c1, c2, eta0, 1.4, rho, *u, T)
        q = oracle.moments_of(c1, c2, eta0, 1.4, f)
        assert abs(q[0] - rho) <= 1e-13 * rho * c2
        np.testing.assert_allclose(q[1:4], u, rtol=0, atol=1e-12 * c2)
        # T carries the cancellation E/rho - u^2: bound relative to c2^2/b
        assert abs(q[4] - T) <= 1e-12 * (c2 * c2 + u @ u)


def test_equilibrium_rest_state_and_symmetry():
    """At u = 0 every group is isotropic: all six axis populations are equal
    and all eight diagonal ones are equal; rest population (b-3) rho T/eta0^2."""
    c1, c2, eta0, gamma = 8.0, 24.0, 8.0, 1.4
    b = 2.0 / (gamma - 1.0)
    f = oracle.equilibrium(c1, c2, eta0, gamma, 1.3, 0.0, 0.0, 0.0, 2.1)
    assert np.ptp(f[1:7]) == 0.0 and np.ptp(f[7:]) == 0.0
    assert f[0] == pytest.approx((b - 3.0) * 1.3 * 2.1 / eta0 ** 2, rel=1e-15)


def _minmod_reference(x, y):
    """Same sign: the argument of smaller magnitude; otherwise zero."""
    if x > 0 and y > 0:
        return min(x, y)
    if x < 0 and y < 0:
        return max(x, y)
    return 0.0


def test_minmod_is_median_with_zero():
    vals = [0.0, -0.0, 1.0, -1.0, 0.5, -0.5, 2.0, -2.0, 1e-300, -1e-300, 3.25, -7.5, 1e300]
    for x in vals:
        for y in vals:
            got = oracle.minmod(x, y)
            assert got == _minmod_reference(x, y)
            assert got == float(np.median([x, y, 0.0]))
    rng = np.random.default_rng(3)
    for x, y in rng.normal(size=(2000, 2)):
        assert oracle.minmod(x, y) == _minmod_reference(x, y)
