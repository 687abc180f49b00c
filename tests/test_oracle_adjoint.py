"""Pins of the oracle's reverse mode (fixed-structure step and rollout).

The reverse mode holds each step's levels, neighbour sets and wall contacts
fixed, so the function it differentiates is the oracle's own
``apbf_step_fixed`` (the step of Fig. 7 with Eqs. 4-7 and the gating of
Eqs. 9-11, replayed with a given structure).  The pins compare it with
things fixed independently of the reverse-mode code: central finite
differences of the forward oracle (element by element on a tiny scene,
along random directions on larger ones), the closed forms of a ballistic
and of a wall-clamped particle, and the Jacobian of the spiky gradient by
finite differences.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import scenes


def _structure(sc, x, v):
    _, _, info = oracle.apbf_step(sc, x, v, trace=True)
    return info["levels"], info["nbr_off"], info["nbr_ids"]


def _loss(sc, x, v, frozen, a, b):
    x1, v1 = oracle.rollout_fixed(sc, x, v, frozen)
    return float(np.sum(a * x1) + np.sum(b * v1))


def _clamped_scene(seed=11, nx=4, ny=3, nz=3):
    """A jittered block with random levels whose bottom layer and one side
    move into the walls fast enough for the prediction clamp to act, and
    which sits against the walls so the iteration clamps act too."""
    sc = scenes.block(nx, ny, nz, seed=seed, levels="random", n_min=1, n_max=4, vel_sigma=0.3)
    v = sc.v0.copy()
    x = sc.x0
    v[x[:, 1] < 0.05, 1] -= 4.0
    v[x[:, 0] < 0.05, 0] -= 4.0
    return dataclasses.replace(sc, v0=v)


def test_spiky_hessian_matches_finite_differences():
    h = scenes.H
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = rng.normal(size=3)
        d *= rng.uniform(0.05, 0.95) * h / np.linalg.norm(d)
        H = oracle.spiky_hess(d, h)
        e = 1e-7 * h
        fd = np.zeros((3, 3))
        for c in range(3):
            dp, dm = d.copy(), d.copy()
            dp[c] += e
            dm[c] -= e
            fd[:, c] = (oracle.spiky_grad(dp, h) - oracle.spiky_grad(dm, h)) / (2 * e)
        np.testing.assert_allclose(H, fd, rtol=1e-6, atol=1e-6 * np.abs(H).max())
        np.testing.assert_allclose(H, H.T, rtol=0, atol=1e-12 * np.abs(H).max())
    assert not oracle.spiky_hess(np.array([h, 0.0, 0.0]), h).any()
    assert not oracle.spiky_hess(np.zeros(3), h).any()


def test_ballistic_particle_closed_form():
    # one particle far from the walls: x' = x + dt v + dt^2 g, v' = v + dt g
    sc = scenes.block(1, 1, 1, box=(np.zeros(3), np.full(3, 1.0)), origin=(0.5, 0.5, 0.5),
                      jitter=0.0)
    x, v = sc.x0.astype(np.float64), np.array([[0.1, -0.2, 0.3]])
    frozen = [_structure(sc, x, v)]
    a, b = np.array([[0.3, -1.2, 0.7]]), np.array([[2.0, 0.5, -0.4]])
    gx, gv = oracle.rollout_vjp(sc, x, v, frozen, a, b)
    np.testing.assert_allclose(gx, a, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(gv, sc.dt * a + b, rtol=1e-13, atol=1e-13)


def test_wall_clamped_particle_closed_form():
    # falling onto the floor: y' = lo_y whatever x_y, v_y, so only v' = (lo - y)/dt
    # carries a y-gradient, to x_y, of -b_y / dt; x and z are ballistic
    sc = scenes.block(1, 1, 1, box=(np.zeros(3), np.full(3, 1.0)), origin=(0.5, 0.5, 0.5),
                      jitter=0.0)
    x = np.array([[0.5, 0.01, 0.5]])
    v = np.array([[0.1, -3.0, 0.0]])
    frozen = [_structure(sc, x, v)]
    x1, _ = oracle.rollout_fixed(sc, x, v, frozen)
    assert x1[0, 1] == sc.lo[1]
    a, b = np.array([[0.3, -1.2, 0.7]]), np.array([[2.0, 0.5, -0.4]])
    gx, gv = oracle.rollout_vjp(sc, x, v, frozen, a, b)
    np.testing.assert_allclose(gx[0], [a[0, 0], -b[0, 1] / sc.dt, a[0, 2]], rtol=1e-13)
    np.testing.assert_allclose(gv[0], [sc.dt * a[0, 0] + b[0, 0], 0.0, sc.dt * a[0, 2] + b[0, 2]],
                               rtol=1e-13)


def test_step_vjp_every_element_matches_finite_differences():
    # brute force on a tiny scene: every one of the 6n input adjoints
    sc = _clamped_scene(seed=3, nx=2, ny=2, nz=2)
    x, v = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    frozen = [_structure(sc, x, v)]
    lv, off, ids = frozen[0]
    assert len(set(lv.tolist())) > 1 and len(ids) > 0
    rng = np.random.default_rng(1)
    a, b = rng.normal(size=x.shape), rng.normal(size=x.shape)
    gx, gv = oracle.rollout_vjp(sc, x, v, frozen, a, b)
    e = 1e-7
    for arr, g in ((x, gx), (v, gv)):
        fd = np.zeros_like(g)
        for i in range(arr.shape[0]):
            for c in range(3):
                keep = arr[i, c]
                arr[i, c] = keep + e
                lp = _loss(sc, x, v, frozen, a, b)
                arr[i, c] = keep - e
                lm = _loss(sc, x, v, frozen, a, b)
                arr[i, c] = keep
                fd[i, c] = (lp - lm) / (2 * e)
        scale = np.abs(g).max()
        np.testing.assert_allclose(g, fd, rtol=0, atol=2e-6 * scale)


@pytest.mark.parametrize("steps", [1, 3])
def test_vjp_directional_finite_differences(steps):
    # larger scene with random levels and wall contacts, along random directions
    sc = _clamped_scene(seed=5 + steps)
    x, v = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    _, _, frozen = oracle.rollout_structure(sc, x, v, steps)
    # the scene exercises the clamps and the gating
    x1, _ = oracle.rollout_fixed(sc, x, v, frozen)
    assert np.any(x1 == sc.lo) and len(set(frozen[0][0].tolist())) > 1
    rng = np.random.default_rng(steps)
    a, b = rng.normal(size=x.shape), rng.normal(size=x.shape)
    gx, gv = oracle.rollout_vjp(sc, x, v, frozen, a, b)

    def central(e, dx, dv):
        lp = _loss(sc, x + e * dx, v + e * dv, frozen, a, b)
        lm = _loss(sc, x - e * dx, v - e * dv, frozen, a, b)
        return (lp - lm) / (2 * e)

    e = 1e-7
    for _ in range(4):
        dx, dv = rng.normal(size=x.shape), rng.normal(size=x.shape)
        # Richardson step removes the e^2 term of the central difference (the
        # several-step map is strongly curved)
        fd = (4.0 * central(e / 2, dx, dv) - central(e, dx, dv)) / 3.0
        an = float(np.sum(gx * dx) + np.sum(gv * dv))
        assert abs(an - fd) <= 1e-6 * max(abs(fd), np.linalg.norm(gx) + np.linalg.norm(gv)), (an, fd)


def test_vjp_is_linear_in_the_output_adjoint():
    sc = _clamped_scene(seed=9)
    x, v = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    frozen = [_structure(sc, x, v)]
    rng = np.random.default_rng(2)
    a1, b1, a2, b2 = (rng.normal(size=x.shape) for _ in range(4))
    g1 = oracle.rollout_vjp(sc, x, v, frozen, a1, b1)
    g2 = oracle.rollout_vjp(sc, x, v, frozen, a2, b2)
    g12 = oracle.rollout_vjp(sc, x, v, frozen, 2 * a1 - a2, 2 * b1 - b2)
    for u, w, s in zip(g1, g2, g12):
        np.testing.assert_allclose(s, 2 * u - w, rtol=1e-12, atol=1e-12 * np.abs(s).max())


def test_translation_invariance_of_the_adjoint():
    # far from the walls the step commutes with translation, so the x-adjoints
    # of a translation-invariant loss (sum of velocities) sum to zero per axis
    sc = scenes.block(3, 3, 3, seed=4, levels="random", box=(np.zeros(3), np.full(3, 2.0)),
                      origin=(0.8, 0.8, 0.8), vel_sigma=0.1)
    x, v = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    frozen = [_structure(sc, x, v)]
    rng = np.random.default_rng(3)
    b = rng.normal(size=x.shape)
    gx, _ = oracle.rollout_vjp(sc, x, v, frozen, np.zeros_like(x), b)
    assert np.abs(gx).max() > 1.0
    np.testing.assert_allclose(gx.sum(axis=0), 0.0, atol=1e-9 * np.abs(gx).max() * len(gx))
