"""Pins of the oracle's average-density measure (orc_density).

The measure is the SPH density of Eq. 6 with the poly6 kernel and the
particle itself included, over neighbour sets found at the positions it is
given; the paper's evaluation (Section 7, Fig. 9) averages it over all
particles.  Each test checks the oracle against something other than
itself: integer shell sums on an exact lattice, and an O(n^2) brute force
whose kernel constant comes from quadrature rather than from the closed
form.  CPU only.
"""
import math

import numpy as np
import pytest

import oracle
import scenes


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)


def _exact_lattice(n1, s=1.0 / 16.0, pad=4):
    """Unjittered n1^3 lattice with binary-exact spacing s, h = 2 s and
    mass rho0 s^3 in a padded box: every distance and h^2 are exact."""
    h = 2.0 * s
    origin = np.array([pad * h] * 3)
    x = scenes.lattice(n1, n1, n1, origin, spacing=s)
    hi = origin + n1 * s + pad * h
    sc = scenes.Scene(name="exact", x0=x, v0=np.zeros_like(x), lo=(0, 0, 0), hi=hi, h=h,
                      rho0=1000.0, mass=1000.0 * s ** 3, eps=12.0, gravity=(0, 0, 0),
                      n_min=1, n_max=1)
    return sc, x


def test_exact_lattice_shell_sums():
    """With h = 2 s and m = rho0 s^3, rho_i / rho0 = 315 S_i / (32768 pi),
    where S_i = sum over the lattice offsets k = r^2/s^2 < 4 present around
    i (the particle itself included) of (4 - k)^3.  Counting the offsets by
    hand:
      interior  1 + 6 + 12 + 8 points: 64 + 162 + 96 + 8 = 330
      face      1 + 5 +  8 + 4 points: 64 + 135 + 64 + 4 = 267
      edge      1 + 4 +  5 + 2 points: 64 + 108 + 40 + 2 = 214
      corner    1 + 3 +  3 + 1 points: 64 +  81 + 24 + 1 = 170
    (points at r = 2 s = h are outside the strict support)."""
    n1 = 6
    sc, x = _exact_lattice(n1)
    rho = oracle.density(sc, x) / float(sc.rho0)
    idx = np.arange(n1 ** 3)
    ijk = np.stack([idx % n1, (idx // n1) % n1, idx // (n1 * n1)], axis=1)
    faces = np.sum((ijk == 0) | (ijk == n1 - 1), axis=1)  # outer faces a particle touches
    shell = {0: 330, 1: 267, 2: 214, 3: 170}
    for nf, S in shell.items():
        want = 315.0 * S / (32768.0 * math.pi)
        got = rho[faces == nf]
        assert got.size > 0
        assert np.allclose(got, want, rtol=1e-13, atol=0), (nf, got.min(), got.max(), want)
    assert abs(315.0 * 330 / (32768.0 * math.pi) - 1.009775166894685) < 1e-14


def _poly6_constant_by_quadrature(h):
    """K with integral over the ball of K (h^2 - r^2)^3 equal to one, by
    Gauss-Legendre (exact for this degree-8 radial integrand)."""
    t, w = np.polynomial.legendre.leggauss(8)
    r = 0.5 * h * (t + 1.0)
    return 1.0 / (0.5 * h * np.sum(w * 4.0 * math.pi * r * r * (h * h - r * r) ** 3))


def _brute_force_density(x, h, mass):
    K = _poly6_constant_by_quadrature(h)
    d2 = np.sum((x[:, None, :] - x[None, :, :]) ** 2, axis=2)
    w = np.where(d2 < h * h, (h * h - d2) ** 3, 0.0)  # j = i contributes h^6
    return mass * K * w.sum(axis=1)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (40, 2), (300, 3), (700, 4)])
def test_random_clouds_equal_brute_force(n, seed):
    """Random clouds with exact duplicates, clustered pairs across cell
    faces and pairs planted just inside and just outside r = h: the grid
    search with its strict radius test equals the all-pairs sum."""
    sc = scenes.random_cloud(n, seed=seed, extent=0.45, n_min=1, n_max=2)
    x = sc.x0.astype(np.float64)
    if n >= 40:
        rng = np.random.default_rng(seed + 100)
        h = float(sc.h)
        a = x[rng.choice(n, size=8, replace=False)]
        u = rng.normal(size=(8, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        r = h * np.array([0.999, 0.9999, 1.001, 0.5, 0.25, 0.01, 0.99, 0.75])
        b = np.clip(a + r[:, None] * u, sc.lo + 1e-3, sc.hi - 1e-3)
        x = np.concatenate([x, b])
        sc = scenes.Scene(name="cloud+pairs", x0=x, v0=np.zeros_like(x), lo=sc.lo, hi=sc.hi,
                          n_min=1, n_max=2)
    rho = oracle.density(sc, x)
    ref = _brute_force_density(x, float(sc.h), float(sc.mass))
    assert np.allclose(rho, ref, rtol=1e-12, atol=0)
    assert np.all(rho >= float(sc.mass) * _poly6_constant_by_quadrature(float(sc.h)) * float(sc.h) ** 6 * (1 - 1e-12))


def test_density_at_moved_positions_uses_those_positions():
    """After three steps of a small dam break the measure, evaluated at the
    new positions, equals the brute force at those positions (neighbour
    sets found afresh, not carried from a step)."""
    sc = scenes.block(9, 7, 8, seed=5, n_min=2, n_max=4, levels="random", vel_sigma=0.3)
    x, _ = oracle.run(sc, steps=3)
    rho = oracle.density(sc, x)
    ref = _brute_force_density(x, float(sc.h), float(sc.mass))
    assert np.allclose(rho, ref, rtol=1e-12, atol=0)
    # and differs from the density at the start (the positions moved)
    assert np.abs(oracle.density(sc, sc.x0.astype(np.float64)) - rho).max() > 1e-3 * float(sc.rho0)


def test_empty_and_single_particle():
    sc = scenes.Scene(name="empty", x0=np.zeros((0, 3)), v0=np.zeros((0, 3)), lo=(0, 0, 0),
                      hi=(1, 1, 1), n_min=1, n_max=1)
    assert oracle.density(sc, np.zeros((0, 3))).shape == (0,)
    x = np.array([[0.5, 0.5, 0.5]])
    sc = scenes.Scene(name="one", x0=x, v0=np.zeros_like(x), lo=(0, 0, 0), hi=(1, 1, 1),
                      n_min=1, n_max=1)
    h, m = float(sc.h), float(sc.mass)
    # alone: m W(0) = m 315 / (64 pi h^3)
    assert math.isclose(oracle.density(sc, x)[0], m * 315.0 / (64.0 * math.pi * h ** 3), rel_tol=1e-14)
