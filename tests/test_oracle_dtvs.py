"""Pins of the oracle's distance-to-the-visible-surface levels (Section 4.1).

The particles seen by the camera are the surface; a particle's level comes
from its distance to the surface along its pixel's ray, mapped linearly
onto n_max .. n_min like the distance-to-camera model.  These pins fix the
model by geometry that does not depend on the splatting code: a lone
particle is visible, a particle straight behind another is as far from the
surface as from that particle, the layers of a slab seen head-on are one
spacing apart, and particles behind the camera or outside the image take
the lowest level.
"""
import dataclasses

import numpy as np

import oracle
import scenes


def _scene(x, n_min=1, n_max=8, **kw):
    x = np.asarray(x, np.float32).reshape(-1, 3)
    sc = scenes.Scene(name="dtvs", x0=x, v0=np.zeros_like(x), lo=(-50, -50, -50), hi=(50, 50, 50),
                      n_min=n_min, n_max=n_max, dims=(1, 1, 1))
    base = dict(camera=np.zeros(3, np.float32), forward=(0, 0, 1), up=(0, 1, 0), focal=200.0,
                image=(64, 64), splat=0.025, d_near=0.0, d_far=0.4, lod_mode=scenes.LOD_DTVS)
    base.update(kw)
    return dataclasses.replace(sc, **base)


def test_lone_particle_is_visible():
    sc = _scene([[0.01, -0.02, 1.0]])
    assert oracle.levels(sc, sc.x0.astype(np.float64))[0] == sc.n_max


def test_particle_behind_another_on_the_same_ray():
    # d = 0.15 of d_far = 0.4 over 8 levels: t = 0.375, level 8 - floor(3.0) = 5
    sc = _scene([[0.0, 0.0, 1.0], [0.0, 0.0, 1.15]])
    lv = oracle.levels(sc, sc.x0.astype(np.float64))
    assert lv[0] == 8 and lv[1] == 8 - int(np.floor(0.15 / 0.4 * 8))


def test_slab_layers_seen_head_on():
    # 8 layers of a 10 x 10 lattice, spacing s, 20 m in front of the camera;
    # with d_near = -s/2 and d_far = 7.5 s, layer k maps to t = (k + 0.5) / 8,
    # i.e. level 8 - k for any distance within half a spacing of k s
    s = scenes.SPACING
    i, j, k = np.meshgrid(np.arange(10), np.arange(10), np.arange(8), indexing="ij")
    x = np.stack([(i - 4.5) * s, (j - 4.5) * s, 20.0 + k * s], -1).reshape(-1, 3)
    sc = _scene(x, focal=600.0, image=(64, 64), d_near=-s / 2, d_far=7.5 * s)
    lv = oracle.levels(sc, sc.x0.astype(np.float64))
    assert np.array_equal(lv, 8 - k.reshape(-1))


def test_behind_the_camera_and_outside_the_image():
    sc = _scene([[0.0, 0.0, -1.0], [5.0, 0.0, 1.0], [0.0, 0.0, 0.01], [0.0, 0.0, 1.0]])
    lv = oracle.levels(sc, sc.x0.astype(np.float64))
    # behind; far outside the 64-pixel image (u = 32 + 1000); closer than the
    # splat radius; visible
    assert list(lv) == [1, 1, 1, 8]


def test_splat_footprint_hides_a_particle_only_within_its_radius():
    # focal 200, splat 0.025 at depth 1: a footprint of ceil(5) = 5 pixels;
    # 1 pixel is 0.005 at depth 1
    near = [0.0, 0.0, 1.0]
    hidden = [0.02 * 1.2, 0.0, 1.2]    # 4 pixels to the side, within the footprint
    seen = [0.04 * 1.2, 0.0, 1.2]      # 8 pixels to the side, outside it
    sc = _scene([near, hidden, seen])
    lv = oracle.levels(sc, sc.x0.astype(np.float64))
    d_hidden = np.linalg.norm(hidden) - 1.0
    assert lv[0] == 8 and lv[2] == 8
    assert lv[1] == 8 - int(np.floor(np.float32(d_hidden) / np.float32(0.4) * 8))
    assert lv[1] < 8


def test_step_uses_the_visible_surface_levels():
    # a dam-break block seen from the side: the face towards the camera
    # iterates n_max times, the far side n_min times
    sc = scenes.block(12, 8, 10, seed=3, n_min=2, n_max=7)
    lo = sc.x0.min(axis=0).astype(np.float64)
    hi = sc.x0.max(axis=0).astype(np.float64)
    mid = (lo + hi) / 2
    sc = scenes.with_dtvs(sc, camera=(mid[0], mid[1], lo[2] - 3.0), target=mid, d_far=0.4)
    lv = oracle.levels(sc, sc.x0.astype(np.float64))
    z = sc.x0[:, 2]
    assert np.all(lv[z == z.min()] == 7)
    assert np.all(lv[z == z.max()] == 2)
    x1, _, info = oracle.apbf_step(sc, sc.x0, sc.v0, trace=True)
    assert np.array_equal(info["levels"], lv)


def test_distance_is_along_the_ray_not_the_view_axis():
    # two particles on one ray 30 degrees off the view axis, 0.17 apart: the
    # distance to the surface is 0.17 (level 8 - floor(3.4) = 5), not its
    # projection on the axis, 0.147 (which would give level 6)
    ray = np.array([np.sin(np.pi / 6), 0.0, np.cos(np.pi / 6)])
    sc = _scene([1.0 * ray, 1.17 * ray], focal=50.0)
    lv = oracle.levels(sc, sc.x0.astype(np.float64))
    assert list(lv) == [8, 5]
