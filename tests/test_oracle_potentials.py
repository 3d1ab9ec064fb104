"""Pins the oracle's two potentials (Sec. 2.1) to closed forms and to -grad(phi).

The golden values in tests/golden/closed_forms.json are derived by hand from the
definitions; none of them comes from code in this repository.
"""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def test_lj_minimum_and_zero_crossing(orc):
    g = GOLDEN["lj_minimum"]
    e, fr = orc.lj(g["r"] ** 2)
    assert e == pytest.approx(g["energy"], abs=1e-14)
    assert abs(fr) < 1e-12
    g = GOLDEN["lj_zero_crossing"]
    e, fr = orc.lj(g["r"] ** 2)
    assert e == pytest.approx(g["energy"], abs=1e-15)
    # fr * r is the radial force (F_j = fr * d, |d| = r)
    assert fr * g["r"] == pytest.approx(g["radial_force"], rel=1e-15)


def test_lj_scaling_with_eps_sigma(orc):
    # phi2(r; eps, sigma) = eps * phi2(r / sigma; 1, 1): the minimum moves to 2^(1/6) sigma
    sigma, eps = 1.7, 0.3
    rmin = 2.0 ** (1.0 / 6.0) * sigma
    e, fr = orc.lj(rmin ** 2, eps, sigma)
    assert e == pytest.approx(-eps, rel=1e-14)
    assert abs(fr) < 1e-13


@pytest.mark.parametrize("r", [0.95, 1.1, 1.5, 2.2, 2.49])
def test_lj_force_is_minus_derivative(orc, r):
    h = 1e-6
    ep, _ = orc.lj((r + h) ** 2)
    em, _ = orc.lj((r - h) ** 2)
    _, fr = orc.lj(r * r)
    assert fr * r == pytest.approx(-(ep - em) / (2 * h), rel=1e-7)


def _equilateral(side):
    return (np.array([side, 0.0, 0.0]), np.array([0.5 * side, 0.5 * math.sqrt(3.0) * side, 0.0]))


def test_atm_equilateral(orc):
    g = GOLDEN["atm_equilateral"]
    s, nu = g["side"], g["nu"]
    u, w = _equilateral(s)
    assert orc.atm_energy(u, w, nu) == pytest.approx(g["energy_coeff"] * nu / s ** 9, rel=1e-14)
    f = orc.atm_forces(u, w, nu)
    pos = np.array([[0.0, 0.0, 0.0], u, w])
    centroid = pos.mean(axis=0)
    for a in range(3):
        out = pos[a] - centroid
        out /= np.linalg.norm(out)
        mag = np.linalg.norm(f[a])
        assert mag == pytest.approx(g["force_coeff"] * nu / s ** 10, rel=1e-13)
        assert np.dot(f[a], out) == pytest.approx(mag, rel=1e-13)  # radial, outward


def test_atm_collinear(orc):
    g = GOLDEN["atm_collinear"]
    d, nu = g["spacing"], g["nu"]
    u = np.array([d, 0.0, 0.0])
    w = np.array([2 * d, 0.0, 0.0])
    assert orc.atm_energy(u, w, nu) == pytest.approx(g["energy_coeff"] * nu / d ** 9, rel=1e-14)


def test_atm_right_angle(orc):
    g = GOLDEN["atm_right_angle"]
    l1, l2 = g["legs"]
    u = np.array([l1, 0.0, 0.0])
    w = np.array([0.0, l2, 0.0])
    assert orc.atm_energy(u, w, g["nu"]) == pytest.approx(g["energy"], rel=1e-14)
    # the right angle may sit at any vertex: put it at j instead of i
    u2 = np.array([l1, 0.0, 0.0])
    w2 = np.array([l1, l2, 0.0])
    assert orc.atm_energy(u2, w2, g["nu"]) == pytest.approx(g["energy"], rel=1e-14)


def test_atm_energy_symmetric_under_relabelling(orc):
    rng = np.random.default_rng(7)
    for _ in range(20):
        p = rng.normal(size=(3, 3))
        base = orc.atm_energy(p[1] - p[0], p[2] - p[0])
        for perm in [(1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0), (2, 0, 1)]:
            q = p[list(perm)]
            assert orc.atm_energy(q[1] - q[0], q[2] - q[0]) == pytest.approx(base, rel=1e-12)


def test_atm_forces_are_minus_gradient(orc):
    """Central differences of the cosine-form energy pin the (a, b, c) force algebra."""
    rng = np.random.default_rng(11)
    h = 1e-6
    for _ in range(25):
        p = rng.uniform(-1.2, 1.2, size=(3, 3))
        f = orc.atm_forces(p[1] - p[0], p[2] - p[0], 0.5)
        num = np.zeros((3, 3))
        for a in range(3):
            for c in range(3):
                pp = p.copy(); pp[a, c] += h
                pm = p.copy(); pm[a, c] -= h
                ep = orc.atm_energy(pp[1] - pp[0], pp[2] - pp[0], 0.5)
                em = orc.atm_energy(pm[1] - pm[0], pm[2] - pm[0], 0.5)
                num[a, c] = -(ep - em) / (2 * h)
        scale = np.abs(f).max()
        assert np.abs(f - num).max() <= 1e-6 * scale
        # Newton's third law across the triplet (Sec. 2.2): the three forces cancel
        assert np.abs(f.sum(axis=0)).max() <= 1e-13 * scale


def test_atm_euler_virial(orc):
    """phi3 is homogeneous of degree -9 in the positions: sum_a x_a . F_a = 9 phi3."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        p = rng.uniform(-1.5, 1.5, size=(3, 3))
        f = orc.atm_forces(p[1] - p[0], p[2] - p[0], 0.2)
        e = orc.atm_energy(p[1] - p[0], p[2] - p[0], 0.2)
        w = sum(np.dot(p[a], f[a]) for a in range(3))
        assert w == pytest.approx(9.0 * e, rel=1e-10, abs=1e-14)
