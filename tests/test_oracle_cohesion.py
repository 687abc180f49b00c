"""Pins of the oracle's force-based cohesion option (CPU).

The option is named beside the unilateral density constraint at the end of
Section 7's setup, by reference to the works cited there; the oracle takes
the cohesion kernel C(r) of Akinci et al. (2013) as the force's profile.
The pins check it against what that definition fixes without retyping it:
values the two polynomial branches must share, closed forms at r = h/2 and
r -> 0, the sign change, a pair's closed-form motion through a whole step,
Newton's third law, that the sets come from x* but the forces from x, and
that gamma = 0 is the plain step bit for bit.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import pytest

import oracle
import scenes

H = 0.1


def test_spline_values_fixed_by_its_definition():
    h = H
    # r = h/2: both branches give 32/(pi h^9) * h^6/64 = 1/(2 pi h^3)
    peak = 1.0 / (2.0 * math.pi * h ** 3)
    assert oracle.cohesion_spline(0.5 * h, h) == pytest.approx(peak, rel=1e-12)
    lo = oracle.cohesion_spline(0.5 * h * (1 - 1e-9), h)
    hi = oracle.cohesion_spline(0.5 * h * (1 + 1e-9), h)
    assert lo == pytest.approx(peak, rel=1e-6) and hi == pytest.approx(peak, rel=1e-6)
    # (h - r)^3 r^3 is largest at r = h/2, so C is largest there
    for r in (0.3 * h, 0.45 * h, 0.55 * h, 0.8 * h):
        assert oracle.cohesion_spline(r, h) < peak
    # r -> 0: 32/(pi h^9) * (-h^6/64) = -1/(2 pi h^3) (repulsion at short range)
    assert oracle.cohesion_spline(1e-9 * h, h) == pytest.approx(-peak, rel=1e-6)
    # support ends at h; r = 0 has no direction and gives nothing
    assert oracle.cohesion_spline(h, h) == 0.0
    assert oracle.cohesion_spline(1.01 * h, h) == 0.0
    assert oracle.cohesion_spline(0.0, h) == 0.0


def test_spline_changes_sign_once_inside_half_h():
    # 2 (h - r)^3 r^3 = h^6/64 has one root in (0, h/2): C < 0 below it,
    # C > 0 from it to h
    h = H
    r = np.linspace(1e-6 * h, h * (1 - 1e-9), 20001)
    c = np.array([oracle.cohesion_spline(t, h) for t in r])
    s = np.sign(c)
    flips = np.flatnonzero(s[1:] != s[:-1])
    assert flips.size == 1
    r0 = r[flips[0]]
    assert 0.0 < r0 < 0.5 * h
    # at the root, u = r/h solves 2 (1 - u)^3 u^3 = 1/64: check by bisection
    f = lambda u: 2.0 * (1 - u) ** 3 * u ** 3 - 1.0 / 64.0
    a, b = 1e-9, 0.5
    for _ in range(200):
        m = 0.5 * (a + b)
        a, b = (m, b) if f(a) * f(m) > 0 else (a, m)
    assert r0 / h == pytest.approx(a, abs=1e-4)


def _pair_scene(r, gamma, v=(0.0, 0.0, 0.0)):
    # two particles on the x axis in a box far larger than h: no wall acts
    c = np.array([0.8, 0.8, 0.8])
    x = np.stack([c - [0.5 * r, 0, 0], c + [0.5 * r, 0, 0]]).astype(np.float32)
    vel = np.stack([v, [0.0, 0.0, 0.0]]).astype(np.float32)
    sc = scenes.Scene(name="pair", x0=x, v0=vel, lo=(0, 0, 0), hi=(1.6, 1.6, 1.6),
                      n_min=1, n_max=1, gravity=np.zeros(3, np.float32))
    # the unilateral constraint leaves a pair below rest density alone, so
    # only the cohesion moves it
    return dataclasses.replace(sc, unilateral=True, cohesion=float(gamma))


@pytest.mark.parametrize("r_over_h,gamma", [(0.8, 0.3), (0.55, 2.0), (0.2, 1.0)])
def test_pair_moves_by_the_closed_form(r_over_h, gamma):
    sc = _pair_scene(r_over_h * H, gamma)
    x0 = sc.x0.astype(np.float64)
    x1, v1, info = oracle.apbf_step(sc, sc.x0, sc.v0, trace=True)
    assert list(info["nbr_count"]) == [1, 1]
    assert np.all(info["lambda_iter"] == 0.0)
    r = float(np.linalg.norm(x0[1] - x0[0]))
    m, dt = float(sc.mass), float(sc.dt)
    # a_0 = -gamma m C(r) (x_0 - x_1)/r, a_1 = -a_0; x' = x + dt^2 a
    c = oracle.cohesion_spline(r, float(sc.h))
    a0 = -gamma * m * c * (x0[0] - x0[1]) / r
    assert np.allclose(x1[0] - x0[0], dt * dt * a0, rtol=1e-12, atol=1e-18)
    assert np.allclose(x1[1] - x0[1], -dt * dt * a0, rtol=1e-12, atol=1e-18)
    assert np.allclose(v1[0], dt * a0, rtol=1e-9, atol=1e-15)
    # attraction beyond the sign change, repulsion inside it
    gap = np.linalg.norm(x1[1] - x1[0]) - r
    assert (gap < 0) == (c > 0)


def test_shift_is_clamped_into_the_box():
    # a pair inside the repulsive range with one particle on the wall x = 0:
    # the shift pushes it outward, and the box clamp (Fig. 7's wall contact)
    # holds it on the wall while its partner moves by the closed form
    r = 0.2 * H
    x = np.array([[0.0, 0.5, 0.5], [r, 0.5, 0.5]], np.float32)
    sc = scenes.Scene(name="wallpair", x0=x, v0=np.zeros_like(x), lo=(0, 0, 0), hi=(1, 1, 1),
                      n_min=1, n_max=1, gravity=np.zeros(3, np.float32))
    sc = dataclasses.replace(sc, unilateral=True, cohesion=1.0)
    x1, _, _ = oracle.apbf_step(sc, sc.x0, sc.v0)
    c = oracle.cohesion_spline(float(x[1, 0]), float(sc.h))
    assert c < 0
    push = float(sc.dt) ** 2 * 1.0 * float(sc.mass) * abs(c)
    assert x1[0, 0] == 0.0
    assert x1[1, 0] == pytest.approx(float(x[1, 0]) + push, rel=1e-12)
    assert np.array_equal(x1[:, 1:], x[:, 1:].astype(np.float64))
    # with the bilateral constraint the solve sees the clamped shift: the
    # same step without cohesion, from a velocity that predicts exactly the
    # clamped shifted positions, gives the same result
    sc2 = dataclasses.replace(sc, unilateral=False)
    y1, _, info = oracle.apbf_step(sc2, sc2.x0, sc2.v0, trace=True)
    assert np.any(info["lambda_iter"] != 0.0)
    pre = x.astype(np.float64)
    target = pre.copy()
    target[0, 0] = 0.0
    target[1, 0] += push
    v_eq = (target - pre) / float(sc.dt)
    z1, _, _ = oracle.apbf_step(dataclasses.replace(sc2, cohesion=0.0), pre, v_eq)
    assert np.allclose(y1, z1, rtol=0, atol=1e-12)


def test_newtons_third_law_on_a_cloud():
    sc = scenes.random_cloud(300, seed=7, extent=0.6, dup_frac=0.02, vel_sigma=0.3)
    sc = dataclasses.replace(sc, cohesion=0.7)
    _, _, info = oracle.apbf_step(sc, sc.x0, sc.v0, trace=True)
    a = oracle.cohesion_accel(sc, sc.x0, info["nbr_off"], info["nbr_ids"])
    assert np.abs(a).max() > 0
    assert np.allclose(a.sum(axis=0), 0.0, atol=1e-9 * np.abs(a).max() * len(a))


def test_sets_from_the_prediction_forces_from_the_start_positions():
    # a moving cloud well inside its box, below rest density everywhere:
    # the unilateral solve leaves every particle alone, and x* differs from
    # x by dt v, so a force evaluated at x* (or over sets found at x) would
    # differ
    rng = np.random.default_rng(11)
    x = rng.uniform(0.15, 0.85, size=(200, 3)).astype(np.float32)
    v = rng.normal(0.0, 0.8, size=x.shape).astype(np.float32)
    sc = scenes.Scene(name="cloud", x0=x, v0=v, lo=(0, 0, 0), hi=(1, 1, 1), n_min=1, n_max=1,
                      gravity=np.zeros(3, np.float32))
    sc = dataclasses.replace(sc, unilateral=True, cohesion=0.5)
    x0 = sc.x0.astype(np.float64)
    x1, _, info = oracle.apbf_step(sc, sc.x0, sc.v0, trace=True)
    assert np.all(info["lambda_iter"] == 0.0)
    pre = info["xs_iter"][0]           # x* before the cohesion shift
    n = sc.n
    # brute-force sets at x* (strict radius test), ascending IDs
    d2 = ((pre[:, None, :] - pre[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.inf)
    nb = [np.flatnonzero(d2[i] < float(sc.h) ** 2) for i in range(n)]
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(b) for b in nb])
    ids = np.concatenate(nb).astype(np.int32)
    assert np.array_equal(off, info["nbr_off"]) and np.array_equal(ids, info["nbr_ids"])
    assert off[-1] > n  # the cloud has pairs
    a_x = oracle.cohesion_accel(sc, x0, off, ids)
    a_xs = oracle.cohesion_accel(sc, pre, off, ids)
    assert np.abs(a_x - a_xs).max() > 1e-3 * np.abs(a_x).max()
    dt = float(sc.dt)
    assert np.allclose(x1, pre + dt * dt * a_x, rtol=0, atol=1e-15)


def test_zero_gamma_is_the_plain_step_bit_for_bit():
    sc = scenes.block(6, 5, 7, seed=3, vel_sigma=0.3, n_min=2, n_max=4, levels="random")
    x_a, v_a, _ = oracle.apbf_step(sc, sc.x0, sc.v0)
    x_b, v_b, _ = oracle.apbf_step(dataclasses.replace(sc, cohesion=0.0), sc.x0, sc.v0)
    assert np.array_equal(x_a, x_b) and np.array_equal(v_a, v_b)
    x_c, _, _ = oracle.apbf_step(dataclasses.replace(sc, cohesion=0.4), sc.x0, sc.v0)
    assert not np.array_equal(x_a, x_c)


@pytest.mark.parametrize("gamma", [-1.0, float("nan"), float("inf")])
def test_invalid_gamma_is_rejected(gamma):
    sc = dataclasses.replace(scenes.block(3, 3, 3, seed=1), cohesion=gamma)
    with pytest.raises(ValueError):
        oracle.apbf_step(sc, sc.x0, sc.v0)
