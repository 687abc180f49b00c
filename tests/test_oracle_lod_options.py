"""Pins of the oracle's level options of Section 4.1 and of the unilateral
density constraint.

Several cameras: levels on a line between two cameras, computed by hand
(the particle takes the higher of the two cameras' levels).  Automatic
range: the nearest particle iterates n_max times and the farthest n_min,
doubling every distance (positions scaled by 2 about the camera) changes no
level, a range of zero width gives n_max, and with the visible-surface model
the particles seen get n_max.  Unilateral constraint: a dilute pair is left
to fall freely (its constraint is inactive), and in the first iteration the
unilateral lambda is exactly min(bilateral lambda, 0).
"""
import dataclasses

import numpy as np
import pytest

import oracle
import scenes


def _line_scene(xs, **kw):
    x = np.stack([np.asarray(xs, np.float64), np.zeros(len(xs)), np.zeros(len(xs))], -1)
    base = dict(name="line", x0=x.astype(np.float32), v0=np.zeros((len(xs), 3), np.float32),
                lo=(-5, -5, -5), hi=(5, 5, 5), n_min=1, n_max=4, lod_mode=scenes.LOD_DTC)
    base.update(kw)
    return scenes.Scene(**base)


def test_two_cameras_take_the_higher_level():
    # camera A at x = -0.5 and B at x = 1.5, both with range [0.5, 1.5];
    # t = d - 0.5, level = 4 - floor(4 t), clamped to [1, 4]
    xs = [0.0, 0.3, 0.5, 0.7, 1.0]
    sc = _line_scene(xs, camera=(-0.5, 0, 0), d_near=0.5, d_far=1.5,
                     extra_cameras=(((1.5, 0, 0), (0.5, 1.5)),))
    lv = oracle.levels(sc, sc.x0.astype(np.float64))
    # x=0: A 4, B 1 | 0.3: A 3, B 2 | 0.5: 2, 2 | 0.7: A 2, B 3 | 1.0: A 1, B 4
    assert list(lv) == [4, 3, 2, 3, 4]
    one = dataclasses.replace(sc, extra_cameras=())
    assert list(oracle.levels(one, one.x0.astype(np.float64))) == [4, 3, 2, 2, 1]


def test_far_extra_camera_changes_nothing():
    sc = scenes.tank_1m()
    sub = dataclasses.replace(sc, x0=sc.x0[::97].copy(), v0=sc.v0[::97].copy())
    far = dataclasses.replace(sub, extra_cameras=(((100.0, 100.0, 100.0), (1.0, 2.0)),))
    a = oracle.levels(sub, sub.x0.astype(np.float64))
    b = oracle.levels(far, far.x0.astype(np.float64))
    assert np.array_equal(a, b)


def test_automatic_range_ends_and_scale_invariance():
    rng = np.random.default_rng(4)
    x = rng.uniform(-1.0, 1.0, size=(500, 3)) + np.array([0.0, 0.0, 3.0])
    sc = scenes.Scene(name="cloud", x0=x.astype(np.float32), v0=np.zeros((500, 3), np.float32),
                      lo=(-10, -10, -10), hi=(10, 10, 10), n_min=2, n_max=7,
                      lod_mode=scenes.LOD_DTC, camera=(0, 0, 0), d_near=100.0, d_far=200.0,
                      auto_range=True)
    lv = oracle.levels(sc, sc.x0.astype(np.float64))
    d = np.linalg.norm(sc.x0.astype(np.float64), axis=1)
    assert lv[np.argmin(d)] == 7 and lv[np.argmax(d)] == 2
    assert len(set(lv.tolist())) == 6
    # scaling every position by 2 about the camera scales every float32
    # distance by 2 exactly: the same levels
    sc2 = dataclasses.replace(sc, x0=(2 * sc.x0).astype(np.float32))
    assert np.array_equal(oracle.levels(sc2, sc2.x0.astype(np.float64)), lv)
    # the given range is not used: with the fixed range [100, 200] all would be n_max
    fixed = dataclasses.replace(sc, auto_range=False)
    assert np.all(oracle.levels(fixed, fixed.x0.astype(np.float64)) == 7)


def test_automatic_range_of_zero_width():
    sc = _line_scene([0.25], camera=(0, 0, 0), auto_range=True)
    assert list(oracle.levels(sc, sc.x0.astype(np.float64))) == [4]


def test_automatic_range_with_the_visible_surface():
    # a slab seen head-on: the front layer is seen (distance 0, n_max), the
    # back layer is the deepest (n_min)
    s = scenes.SPACING
    i, j, k = np.meshgrid(np.arange(10), np.arange(10), np.arange(6), indexing="ij")
    x = np.stack([(i - 4.5) * s, (j - 4.5) * s, 20.0 + k * s], -1).reshape(-1, 3)
    sc = scenes.Scene(name="slab", x0=x.astype(np.float32), v0=np.zeros_like(x, np.float32),
                      lo=(-50, -50, -50), hi=(50, 50, 50), n_min=1, n_max=6,
                      lod_mode=scenes.LOD_DTVS, camera=(0, 0, 0), forward=(0, 0, 1), up=(0, 1, 0),
                      focal=600.0, image=(64, 64), splat=0.025, d_near=5.0, d_far=6.0,
                      auto_range=True)
    lv = oracle.levels(sc, sc.x0.astype(np.float64))
    kk = k.reshape(-1)
    assert np.all(lv[kk == 0] == 6) and np.all(lv[kk == 5] == 1)


def test_unilateral_pair_falls_freely():
    # two particles 0.9 h apart: far below rest density, so the unilateral
    # constraint is inactive and the step is a free fall
    x = np.array([[0.0, 0.0, 0.0], [0.09, 0.0, 0.0]])
    base = scenes.Scene(name="pair", x0=x.astype(np.float32), v0=np.zeros((2, 3), np.float32),
                        lo=(-1, -1, -1), hi=(1, 1, 1), n_min=3, n_max=3)
    uni = dataclasses.replace(base, unilateral=True)
    x0, v0 = base.x0.astype(np.float64), base.v0.astype(np.float64)
    g, dt = base.gravity.astype(np.float64), float(base.dt)
    xu, vu, _ = oracle.apbf_step(uni, x0, v0)
    np.testing.assert_allclose(xu, x0 + dt * dt * g, rtol=0, atol=1e-15)
    np.testing.assert_allclose(vu, np.broadcast_to(dt * g, vu.shape), rtol=0, atol=1e-12)
    xb, _, _ = oracle.apbf_step(base, x0, v0)
    assert xb[1, 0] - xb[0, 0] < 0.09 - 1e-4  # the bilateral constraint pulls them together


def test_unilateral_lambda_is_the_compressive_part():
    sc = scenes.block(9, 8, 7, seed=2, n_min=2, n_max=5, levels="random", vel_sigma=0.5)
    uni = dataclasses.replace(sc, unilateral=True)
    x0, v0 = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    _, _, ib = oracle.apbf_step(sc, x0, v0, trace=True)
    _, _, iu = oracle.apbf_step(uni, x0, v0, trace=True)
    lb, lu = ib["lambda_iter"][0], iu["lambda_iter"][0]
    assert (lb > 0).any() and (lb < 0).any()
    assert np.array_equal(lu, np.minimum(lb, 0.0))
    assert np.all(iu["lambda_iter"] <= 0.0)


def test_level_guard_band_marks_the_bin_edges():
    # levels 1..4 over [0.5, 1.5]: u = 4 (d - 0.5) changes level at d = 0.75,
    # 1.0 and 1.25 (exact binary values); the clamped ends change nothing
    xs = [0.5, 0.6, 0.75, 0.9, 1.0, 1.1, 1.25, 1.4, 1.5]
    sc = _line_scene(xs, camera=(0, 0, 0), d_near=0.5, d_far=1.5)
    lv, near = oracle.levels(sc, sc.x0.astype(np.float64), guard=True)
    assert list(lv) == [4, 4, 3, 3, 2, 2, 1, 1, 1]
    assert list(near) == [False, False, True, False, True, False, True, False, False]


def test_float32_levels_differ_only_inside_the_guard_band():
    # the same map evaluated in float32 (one rounding per operation) on the
    # 1M tank's initial positions: any particle whose float32 level differs
    # from the FP64 one lies inside the guard band, and the band is narrow
    sc = scenes.tank_1m()
    x = sc.x0[::7].astype(np.float64)
    sub = dataclasses.replace(sc, x0=sc.x0[::7].copy(), v0=sc.v0[::7].copy())
    lv, near = oracle.levels(sub, x, guard=True)
    f = np.float32
    q = sub.x0 - np.asarray(sc.camera, f)
    d = np.sqrt(((q[:, 0] * q[:, 0]) + (q[:, 1] * q[:, 1])) + (q[:, 2] * q[:, 2]))
    t = np.clip((d - f(sc.d_near)) / (f(sc.d_far) - f(sc.d_near)), f(0), f(1))
    lv32 = np.clip(sc.n_max - np.floor(t * f(sc.n_max - sc.n_min + 1)).astype(np.int64),
                   sc.n_min, sc.n_max)
    assert np.all((lv32 == lv) | near)
    assert near.mean() < 1e-3
