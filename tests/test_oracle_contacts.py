"""Pins of the oracle's obstacle contacts and pre-stabilisation (Section 4.3,
Fig. 6; the contact lines of Fig. 7; signed-distance obstacles, Section 6).

The projections are pinned by geometry computed independently of the oracle:
the point they return lies on the obstacle's surface (its implicit equation),
and its distance to the input point matches a brute-force minimum over a dense
sampling of the surface.  The step-level pins use single particles without
neighbours, where a step reduces to prediction, contact handling and the
velocity update: a particle predicted inside an obstacle ends on its surface;
pre-stabilisation moves x and x* together, so the particle keeps the
velocity v + dt g (Fig. 6's point), while a particle outside the
pre-stabilised set gains the push-out as velocity; only particles with
N_i < S are pre-stabilised.  Invariants close it: obstacles far away change
nothing bit for bit, and after every step of a multi-dam-break run no
particle lies inside the cone (deeper than rounding).
"""
import dataclasses

import numpy as np
import pytest

import oracle
import scenes

SPHERE, CONE, BOX = scenes.OB_SPHERE, scenes.OB_CONE, scenes.OB_BOX


def _sphere_surface(c, R, m=600):
    th = np.linspace(0, np.pi, m)
    ph = np.linspace(0, 2 * np.pi, 2 * m, endpoint=False)
    T, P = np.meshgrid(th, ph, indexing="ij")
    pts = np.stack([np.sin(T) * np.cos(P), np.cos(T), np.sin(T) * np.sin(P)], -1).reshape(-1, 3)
    return np.asarray(c) + R * pts, np.pi * R / m


def _box_surface(c, e, step=0.0025):
    faces = []
    for ax in range(3):
        o1, o2 = [a for a in range(3) if a != ax]
        u = np.arange(-e[o1], e[o1] + step / 2, step)
        w = np.arange(-e[o2], e[o2] + step / 2, step)
        U, W = np.meshgrid(u, w, indexing="ij")
        for sgn in (-1.0, 1.0):
            f = np.zeros(U.shape + (3,))
            f[..., ax] = sgn * e[ax]
            f[..., o1] = U
            f[..., o2] = W
            faces.append(f.reshape(-1, 3))
    return np.asarray(c) + np.concatenate(faces), step


def _cone_surface(c, R, H, step=0.004):
    # the slant, from the apex down to twice the base radius (the cone
    # stands on the floor: its slant continues below the base circle)
    pts = []
    L = np.hypot(R, H)
    for s in np.arange(0.0, 2 * L + step / 2, step):
        r = R * s / L
        y = H * (1 - s / L)
        k = max(1, int(np.ceil(2 * np.pi * r / step)))
        ph = np.arange(k) * 2 * np.pi / k
        pts.append(np.stack([r * np.cos(ph), np.full(k, y), r * np.sin(ph)], -1))
    return np.asarray(c) + np.concatenate(pts), step


def _on_surface(kind, c, a, y, tol=1e-12):
    d = np.asarray(y) - np.asarray(c)
    if kind == SPHERE:
        return abs(np.linalg.norm(d) - a[0]) <= tol
    if kind == BOX:
        q = np.abs(d) - np.asarray(a)
        return abs(q.max()) <= tol and np.all(q <= tol)
    rho = np.hypot(d[0], d[2])
    return abs(rho / a[0] + d[1] / a[1] - 1.0) <= tol and d[1] <= a[1] + tol


def _inside(kind, c, a, x):
    d = np.asarray(x) - np.asarray(c)
    if kind == SPHERE:
        return np.linalg.norm(d) < a[0]
    if kind == BOX:
        return bool(np.all(np.abs(d) < np.asarray(a)))
    return np.hypot(d[0], d[2]) / a[0] + d[1] / a[1] < 1.0


@pytest.mark.parametrize("kind,c,a,maker", [
    (SPHERE, (0.1, -0.2, 0.3), (0.5, 0.0, 0.0), lambda c, a: _sphere_surface(c, a[0])),
    (BOX, (0.0, 0.1, -0.1), (0.3, 0.2, 0.4), lambda c, a: _box_surface(c, a)),
    (CONE, (0.2, 0.0, -0.3), (0.5, 0.8, 0.0), lambda c, a: _cone_surface(c, a[0], a[1])),
])
def test_projection_is_the_closest_surface_point(kind, c, a, maker):
    surf, step = maker(c, a)
    rng = np.random.default_rng(kind)
    # points drawn around the obstacle; about half fall inside
    if kind == CONE:
        lo = np.asarray(c) - (1.3 * a[0], 0.3 * a[1], 1.3 * a[0])
        hi = np.asarray(c) + (1.3 * a[0], a[1], 1.3 * a[0])
    else:
        ext = np.array(a if kind == BOX else (a[0],) * 3)
        lo, hi = np.asarray(c) - 1.1 * ext, np.asarray(c) + 1.1 * ext
    seen_inside = 0
    for _ in range(300):
        x = rng.uniform(lo, hi)
        y = oracle.obstacle_project(kind, c, a, x)
        assert (y is not None) == _inside(kind, c, a, x)
        if y is None:
            continue
        seen_inside += 1
        dmin = np.sqrt(((surf - x) ** 2).sum(axis=1)).min()
        assert _on_surface(kind, c, a, y, tol=1e-9)
        dist = np.linalg.norm(y - x)
        # no sample of the surface is nearer than the projection, and the
        # projection is not nearer than the surface can be
        assert dist <= dmin + 1e-12
        assert dist >= dmin - step
        if seen_inside == 40:
            break
    assert seen_inside == 40


def test_points_outside_are_not_moved():
    for kind, c, a, x in [(SPHERE, (0, 0, 0), (1, 0, 0), (0.6, 0.8, 0.001)),
                          (SPHERE, (0, 0, 0), (0.5, 0, 0), (0.0, 0.0, 0.6)),
                          (BOX, (0, 0, 0), (1, 2, 3), (1.0001, 0.0, 0.0)),
                          (CONE, (0, 0, 0), (1, 2, 0), (0.51, 1.0, 0.0)),
                          (CONE, (0, 0, 0), (1, 2, 0), (1.11, -0.2, 0.0)),
                          (CONE, (0, 0, 0), (1, 2, 0), (0.0, 2.001, 0.0))]:
        assert oracle.obstacle_project(kind, c, a, x) is None
    # below the base circle the slant continues: a point there is inside
    y = oracle.obstacle_project(CONE, (0, 0, 0), (1, 2, 0), (1.05, -0.2, 0.0))
    assert y is not None and y[0] > 1.05


def test_degenerate_projections():
    # centre of a sphere: straight up; on the cone axis: in the +x plane
    y = oracle.obstacle_project(SPHERE, (1, 2, 3), (0.5, 0, 0), (1, 2, 3))
    np.testing.assert_allclose(y, [1, 2.5, 3], rtol=0, atol=1e-15)
    y = oracle.obstacle_project(CONE, (0, 0, 0), (1, 2, 0), (0.0, 1.5, 0.0))
    assert y[0] > 0 and y[2] == 0 and _on_surface(CONE, (0, 0, 0), (1, 2, 0), y, 1e-12)
    # box: least penetration through +z
    y = oracle.obstacle_project(BOX, (0, 0, 0), (1, 1, 1), (0.2, -0.3, 0.9))
    np.testing.assert_allclose(y, [0.2, -0.3, 1.0], rtol=0, atol=0)


def test_contact_finding_margins():
    h = 0.1
    # sphere: grown radius 1.1; box: half extents + h per axis; cone: the
    # slant moved out by h (distance to the slant line below h)
    assert oracle.contact_found(SPHERE, (0, 0, 0), (1, 0, 0), (1.09, 0, 0), h)
    assert not oracle.contact_found(SPHERE, (0, 0, 0), (1, 0, 0), (1.11, 0, 0), h)
    assert oracle.contact_found(BOX, (0, 0, 0), (1, 1, 1), (1.09, 1.09, 1.09), h)
    assert not oracle.contact_found(BOX, (0, 0, 0), (1, 1, 1), (1.09, 1.11, 0), h)
    n = np.array([2.0, 1.0]) / np.sqrt(5.0)  # outward normal of the slant (rho, y)
    on = np.array([0.5, 1.0])                 # a point of the slant line
    for s, found in ((0.09, True), (0.11, False)):
        rho, y = on + s * n
        assert oracle.contact_found(CONE, (0, 0, 0), (1, 2, 0), (0.6 * rho, y, 0.8 * rho), h) == found


def _single(x, v, obstacles, stab_iters=0, stab_s=1, levels=(1,), n_max=None):
    x = np.asarray(x, np.float32).reshape(-1, 3)
    v = np.asarray(v, np.float32).reshape(-1, 3)
    lv = np.asarray(levels, np.uint8)
    nm = int(lv.max()) if n_max is None else n_max
    return scenes.Scene(name="contact", x0=x, v0=v, lo=(-2, -2, -2), hi=(2, 2, 2),
                        n_min=1, n_max=nm, lod_mode=scenes.LOD_EXPLICIT, levels=lv,
                        obstacles=obstacles, stab_iters=stab_iters, stab_s=stab_s)


def test_particle_predicted_inside_a_sphere_ends_on_its_surface():
    c, R = np.array([0.0, 0.0, 0.0]), 0.5
    sc = _single([0.05, 0.52, 0.0], [0.0, -3.0, 0.0], ((SPHERE, c, (R, 0, 0)),))
    x, v = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    x1, v1, info = oracle.apbf_step(sc, x, v, trace=True)
    xs = x[0] + sc.dt * (v[0] + sc.dt * sc.gravity.astype(np.float64))
    assert np.linalg.norm(xs - c) < R  # predicted inside
    assert info["contacts"][0] == 1
    # on the surface, on the ray from the centre through x*
    assert abs(np.linalg.norm(x1[0] - c) - R) < 1e-12
    u = (xs - c) / np.linalg.norm(xs - c)
    np.testing.assert_allclose(x1[0], c + R * u, rtol=0, atol=1e-12)
    np.testing.assert_allclose(v1[0], (x1[0] - x[0]) / sc.dt, rtol=1e-12)


@pytest.mark.parametrize("kind,c,a", [(SPHERE, (0.0, 0.0, 0.0), (0.5, 0.0, 0.0)),
                                      (BOX, (0.0, 0.0, 0.0), (0.4, 0.5, 0.3)),
                                      (CONE, (0.0, 0.0, 0.0), (0.6, 0.55, 0.0))])
def test_prestabilisation_keeps_the_velocity(kind, c, a):
    # Fig. 6: a low-level particle predicted inside an obstacle is moved out
    # with its current position, so the step adds no velocity; without
    # pre-stabilisation the push-out becomes velocity
    x, v = [0.05, 0.53, 0.02], [0.0, -3.0, 0.0]
    with_stab = _single(x, v, ((kind, c, a),), stab_iters=1, stab_s=2, levels=(1,), n_max=2)
    no_stab = dataclasses.replace(with_stab, stab_s=1)
    g = with_stab.gravity.astype(np.float64)
    x0, v0 = with_stab.x0.astype(np.float64), with_stab.v0.astype(np.float64)
    xa, va, _ = oracle.apbf_step(with_stab, x0, v0)
    xb, vb, _ = oracle.apbf_step(no_stab, x0, v0)
    vpred = v0[0] + with_stab.dt * g
    xs = x0[0] + with_stab.dt * vpred
    (_, c32, a32), = with_stab.obstacles  # the float32 values the step uses
    y = oracle.obstacle_project(kind, c32, a32, xs)
    assert y is not None
    np.testing.assert_allclose(xa[0], y, rtol=0, atol=1e-12)
    np.testing.assert_allclose(xb[0], y, rtol=0, atol=1e-12)
    np.testing.assert_allclose(va[0], vpred, rtol=0, atol=1e-9)
    np.testing.assert_allclose(vb[0], (y - x0[0]) / with_stab.dt, rtol=1e-12)
    assert np.linalg.norm(vb[0] - vpred) > 1.0


def test_only_particles_below_the_set_are_prestabilised():
    # three lone particles falling into three spheres, levels 1, 2, 3, S = 2:
    # only the level-1 particle is pre-stabilised (N_i < S)
    cs = (-1.2, 0.0, 1.2)
    obst = tuple((SPHERE, (c, 0.0, 0.0), (0.5, 0, 0)) for c in cs)
    sc = _single([[c, 0.52, 0.0] for c in cs], [[0, -3.0, 0]] * 3, obst,
                 stab_iters=2, stab_s=2, levels=(1, 2, 3))
    x0, v0 = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    x1, v1, info = oracle.apbf_step(sc, x0, v0, trace=True)
    assert list(info["contacts"]) == [1, 2, 4]
    vpred = v0 + sc.dt * sc.gravity.astype(np.float64)
    np.testing.assert_allclose(v1[0], vpred[0], rtol=0, atol=1e-9)
    for i in (1, 2):  # pushed out by the solver's contact response
        assert v1[i, 1] > vpred[i, 1] + 1.0
    for i, c in enumerate(cs):
        assert abs(np.linalg.norm(x1[i] - (c, 0, 0)) - 0.5) < 1e-12


def test_far_obstacles_change_nothing():
    sc = scenes.block(8, 6, 7, seed=2, n_min=2, n_max=5, levels="random", vel_sigma=0.3)
    far = dataclasses.replace(sc, obstacles=((SPHERE, (5.0, 5.0, 5.0), (0.5, 0, 0)),
                                             (CONE, (-3.0, 0.0, 0.0), (0.4, 0.5, 0))),
                              stab_iters=2, stab_s=4)
    x0, v0 = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    xa, va, _ = oracle.apbf_step(sc, x0, v0)
    xb, vb, info = oracle.apbf_step(far, x0, v0, trace=True)
    assert not info["contacts"].any()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)


def test_no_particle_inside_the_cone_after_any_step():
    sc = scenes.multi_dam_break(a=7, ny=9, box=(1.4, 0.9, 1.4), cone=(0.3, 0.45), n_min=2,
                                n_max=5, stab_iters=1, stab_s=4)
    # aim the blocks at the cone
    v = np.zeros_like(sc.x0)
    mid = np.array([0.7, 0.0, 0.7])
    d = mid - sc.x0.astype(np.float64)
    d[:, 1] = 0.0
    v[:] = 1.5 * d / np.linalg.norm(d, axis=1, keepdims=True)
    sc = dataclasses.replace(sc, v0=v)
    (kind, c, a), = sc.obstacles
    x, v = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    touched = 0
    for _ in range(25):
        x, v, info = oracle.apbf_step(sc, x, v, trace=True)
        touched = max(touched, int(info["contacts"].astype(bool).sum()))
        for xi in x:  # outside, or on the surface up to rounding
            y = oracle.obstacle_project(kind, c, a, xi)
            assert y is None or np.linalg.norm(y - xi) < 1e-12
    assert touched > 100
