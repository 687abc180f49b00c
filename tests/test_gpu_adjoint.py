"""GPU parity of the reverse mode (pbf_rollout_forward / pbf_rollout_backward).

The library's adjoint (gathers over each particle's neighbour list, FP32) is
compared element by element with the oracle's FP64 reverse mode (pair
scatters), itself pinned against finite differences on the CPU.  Both hold
each step's levels, neighbour sets and wall contacts fixed; the tests check
that the two sides ran on the same structure.

Tolerance: max |g_gpu - g_oracle| <= tol * max |g_oracle| per output (x
and v adjoints separately).  The adjoint is a product of per-iteration
Jacobians evaluated at the FP32 forward trajectory.  After one step, a
random one-ulp change of the float32 input moves the oracle's own FP64
adjoint by 1e-5 to 3e-5 (max-norm, relative); tol = ADJ_REL = 1e-4 is about
4x that.  Over several steps the same one-ulp change moves it by 1e-3 to
1e-1: particles resting on a wall flip their clamp mask, and isolated
free-surface particles take corrections that amplify input changes.  The
multi-step tests therefore measure that spread (tests/parity.py) and take
4x it.
"""
import dataclasses

import numpy as np
import pytest
import torch  # noqa: F401  (first import can be slow; keep it out of test timeouts)

import oracle
import scenes
from parity import adjoint_spread, check_levels, neighbour_mismatch, pos_tol, ref_csr

pytestmark = pytest.mark.gpu

ADJ_REL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    oracle.build(force=False)
    from paper_1608_04721_amd import _lib
    _lib.load()


def _sim(sc, **kw):
    from paper_1608_04721_amd import Sim
    return Sim(sc, **kw)


def _wall_block(seed=21, nx=11, ny=9, nz=7, n_max=4):
    """Jittered block with random levels whose bottom layer and x = 0 face
    move into the walls, so both clamps act."""
    sc = scenes.block(nx, ny, nz, seed=seed, levels="random", n_min=1, n_max=n_max, vel_sigma=0.3)
    v = sc.v0.copy()
    v[sc.x0[:, 1] < 0.05, 1] -= 4.0
    v[sc.x0[:, 0] < 0.05, 0] -= 4.0
    return dataclasses.replace(sc, v0=v.astype(np.float32))


def _cotangents(n, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(n, 3)).astype(np.float32),
            rng.normal(size=(n, 3)).astype(np.float32))


def _compare(g, ref, what, rel=ADJ_REL):
    scale = float(np.abs(ref).max())
    err = float(np.abs(g.astype(np.float64) - ref).max())
    print(f"{what}: max err {err:.3e}, scale {scale:.3e}, ratio {err / max(scale, 1e-30):.2e}")
    assert np.all(np.isfinite(g)), f"{what}: non-finite adjoint"
    assert err <= rel * scale, f"{what}: {err:.3e} > {rel:.0e} * {scale:.3e}"
    return err / max(scale, 1e-30)


def _dtc_block():
    sc = scenes.block(10, 8, 9, seed=7, vel_sigma=0.2, n_min=2, n_max=6).with_lod(scenes.LOD_DTC)
    cam = np.array([0.0, 0.2, -0.5], np.float32)
    d = np.linalg.norm(sc.x0.astype(np.float64) - cam, axis=1)
    sc.camera, sc.d_near, sc.d_far = cam, np.float32(d.min()), np.float32(d.max())
    return sc


CASES = {
    "walls_random_levels": _wall_block,
    "dam_break_4k": scenes.dam_break_4k,
    "dtc_levels": _dtc_block,
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_step_adjoint_matches_oracle(case):
    sc = CASES[case]()
    x0, v0 = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    sim = _sim(sc)
    sim.rollout_forward(1, 1)
    # same structure on both sides: the GPU's levels (checked against the
    # oracle's FP64 levels, either level at a bin edge) for both
    lv = sim.debug_levels().astype(np.int32)
    check_levels(sc, x0, lv)
    x1, v1, info = oracle.apbf_step(sc, x0, v0, trace=True, mode=scenes.LOD_EXPLICIT, levels=lv)
    frozen = [(info["levels"], info["nbr_off"], info["nbr_ids"])]
    assert neighbour_mismatch(sc, sim.debug_neighbours(), ref_csr(info), info["xs_iter"][0]) == 0
    assert np.abs(sim.positions() - x1).max() <= pos_tol(sc)
    a, b = _cotangents(sc.n, 1)
    gx, gv = sim.rollout_backward(a, b)
    rx, rv = oracle.rollout_vjp(sc, x0, v0, frozen, a.astype(np.float64), b.astype(np.float64))
    _compare(gx, rx, f"{case} dL/dx0")
    _compare(gv, rv, f"{case} dL/dv0")


def test_rollout_adjoint_away_from_walls():
    # a slowly moving block in mid-air with random levels: no contact acts;
    # the free surface alone makes several steps ill-conditioned (isolated
    # surface particles take large corrections), so the bar is measured too
    sc = scenes.block(9, 8, 7, seed=6, levels="random", n_min=1, n_max=5, vel_sigma=0.1,
                      box=(np.zeros(3), np.full(3, 2.0)), origin=(0.6, 0.6, 0.6))
    a, b = _cotangents(sc.n, 2)
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    (xT, frozen, rx, rv), spread = adjoint_spread(sc, 3, lambda _: (a64, b64))
    assert not np.any(xT == sc.lo) and not np.any(xT == sc.hi)
    tol = max(ADJ_REL, 4 * spread)
    sim = _sim(sc)
    sim.rollout_forward(3, 2)
    assert np.abs(sim.positions() - xT).max() <= 3 * pos_tol(sc)
    gx, gv = sim.rollout_backward(a, b)
    print(f"one-ulp spread of the oracle adjoint: {spread:.2e}")
    _compare(gx, rx, "3 steps, no walls, dL/dx0", rel=tol)
    _compare(gv, rv, "3 steps, no walls, dL/dv0", rel=tol)


def test_rollout_adjoint_through_walls():
    sc = _wall_block(seed=5, nx=9, ny=8, nz=7)
    a, b = _cotangents(sc.n, 2)
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    (xT, frozen, rx, rv), spread = adjoint_spread(sc, 4, lambda _: (a64, b64))
    tol = max(ADJ_REL, 4 * spread)
    sim = _sim(sc)
    sim.rollout_forward(4, 2)
    assert np.abs(sim.positions() - xT).max() <= 4 * pos_tol(sc)
    gx, gv = sim.rollout_backward(a, b)
    print(f"one-ulp spread of the oracle adjoint: {spread:.2e}")
    _compare(gx, rx, "4 steps, walls, dL/dx0", rel=tol)
    _compare(gv, rv, "4 steps, walls, dL/dv0", rel=tol)


def test_checkpoint_interval_does_not_change_the_gradient():
    sc = _wall_block(seed=8, nx=7, ny=6, nz=5)
    a, b = _cotangents(sc.n, 3)
    out = []
    for every in (1, 2, 3, 5, 9):
        sim = _sim(sc)
        sim.rollout_forward(5, every)
        out.append(sim.rollout_backward(a, b))
    for gx, gv in out[1:]:
        assert np.array_equal(gx, out[0][0]) and np.array_equal(gv, out[0][1])


def test_backward_keeps_the_final_state_and_repeats():
    sc = _wall_block(seed=9, nx=6, ny=6, nz=6)
    a, b = _cotangents(sc.n, 4)
    sim = _sim(sc)
    sim.rollout_forward(3, 2)
    xT, vT = sim.positions(), sim.velocities()
    g1 = sim.rollout_backward(a, b)
    assert np.array_equal(sim.positions(), xT) and np.array_equal(sim.velocities(), vT)
    g2 = sim.rollout_backward(a, b)
    assert np.array_equal(g1[0], g2[0]) and np.array_equal(g1[1], g2[1])
    # continuing after the reverse pass equals never having run it, and the
    # recomputed steps do not count in the running totals
    ref = _sim(sc)
    ref.step(3)
    sim.step(2)
    ref.step(2)
    assert np.array_equal(sim.positions(), ref.positions())
    assert np.array_equal(sim.velocities(), ref.velocities())
    s, r = sim.stats(), ref.stats()
    assert s["total_steps"] == r["total_steps"] == 5
    assert s["total_particle_iterations"] == r["total_particle_iterations"]


def test_backward_needs_a_fresh_rollout():
    from paper_1608_04721_amd import PbfError
    sc = _wall_block(seed=10, nx=4, ny=4, nz=4)
    a, b = _cotangents(sc.n, 5)
    sim = _sim(sc)
    with pytest.raises(PbfError) as e:
        sim.rollout_backward(a, b)
    assert e.value.status == -1
    sim.rollout_forward(2, 1)
    sim.step(1)
    with pytest.raises(PbfError):
        sim.rollout_backward(a, b)
    sim.rollout_forward(2, 1)
    x, v, _ = sim.get_state()
    sim.set_state(x, v)
    with pytest.raises(PbfError):
        sim.rollout_backward(a, b)
    with pytest.raises(PbfError):
        sim.rollout_forward(0, 1)
    with pytest.raises(PbfError):
        sim.rollout_forward(2, 0)


def test_batched_adjoint_equals_each_scene_alone():
    scs = [_wall_block(seed=11, nx=5, ny=4, nz=6),
           dataclasses.replace(scenes.block(7, 5, 4, seed=12, vel_sigma=0.4, n_min=2, n_max=5,
                                            levels="random"), dt=scenes.DT_DEEP),
           scenes.block(3, 9, 3, seed=13, n_min=3, n_max=3)]
    cot = [_cotangents(s.n, 20 + i) for i, s in enumerate(scs)]
    sim = _sim(scs)
    sim.rollout_forward(3, 2)
    gx, gv = sim.rollout_backward(np.concatenate([c[0] for c in cot]),
                                  np.concatenate([c[1] for c in cot]))
    off = sim.offsets
    for i, s in enumerate(scs):
        one = _sim(s)
        one.rollout_forward(3, 2)
        ox, ov = one.rollout_backward(*cot[i])
        assert np.array_equal(gx[off[i]:off[i + 1]], ox)
        assert np.array_equal(gv[off[i]:off[i + 1]], ov)


def test_device_buffers_and_autograd_match_host_path():
    import torch
    from paper_1608_04721_amd import rollout
    sc = _wall_block(seed=14, nx=6, ny=5, nz=5)
    a, b = _cotangents(sc.n, 6)
    sim = _sim(sc)
    sim.rollout_forward(2, 1)
    hx, hv = sim.rollout_backward(a, b)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    ox = torch.empty_like(da)
    ov = torch.empty_like(db)
    sim.rollout_backward(da, db, ox, ov)
    assert np.array_equal(ox.cpu().numpy(), hx) and np.array_equal(ov.cpu().numpy(), hv)
    # torch.autograd.Function over the same rollout
    sim2 = _sim(sc)
    x0 = torch.from_numpy(sc.x0.astype(np.float32)).cuda().requires_grad_(True)
    v0 = torch.from_numpy(sc.v0.astype(np.float32)).cuda().requires_grad_(True)
    xT, vT = rollout(sim2, x0, v0, 2, 1)
    assert np.array_equal(xT.detach().cpu().numpy(), sim.positions())
    loss = (xT * da).sum() + (vT * db).sum()
    loss.backward()
    assert np.array_equal(x0.grad.cpu().numpy(), hx)
    assert np.array_equal(v0.grad.cpu().numpy(), hv)


def test_training_rollout_velocity_gradient():
    """The differentiable-rollout workload (32,768 particles, N = 6, dt =
    1/120, loss = mean squared distance of the final positions to a seeded
    target cloud, gradient with respect to the initial velocities, one
    checkpoint segment), over the 3 steps after which the oracle's own
    gradient still moves by only ~1e-3 under one-ulp input changes (by 5
    steps the block's collapse onto the floor moves it by 10-100%): the GPU
    gradient against the oracle's reverse mode element by element, and its
    directional derivatives along 16 seeded directions against FP64 central
    differences of the oracle (eps = 1e-6)."""
    sc = scenes.rollout_32k()
    steps = 3
    n = sc.n
    x0, v0 = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    tgt = sc.target.astype(np.float64)

    def cot(xT):
        return (2.0 / n) * (xT - tgt), np.zeros((n, 3))

    (xT, frozen, _, rv), spread = adjoint_spread(sc, steps, cot)
    tol = max(ADJ_REL, 4 * spread)
    sim = _sim(sc)
    sim.rollout_forward(steps, 5)
    xg = sim.positions().astype(np.float64)
    assert np.abs(xg - xT).max() <= steps * pos_tol(sc)
    _, gv = sim.rollout_backward(((2.0 / n) * (xg - tgt)).astype(np.float32),
                                 np.zeros((n, 3), np.float32))
    print(f"one-ulp spread of the oracle adjoint: {spread:.2e}")
    _compare(gv, rv, "rollout_32k dL/dv0", rel=tol)

    def loss(v):
        x1, _ = oracle.rollout_fixed(sc, x0, v, frozen)
        return float(np.mean(np.sum((x1 - tgt) ** 2, axis=1)))

    rng = np.random.default_rng(16)
    e = 1e-6
    worst = 0.0
    for _ in range(16):
        u = rng.normal(size=(n, 3))
        fd = (loss(v0 + e * u) - loss(v0 - e * u)) / (2 * e)
        an = float(np.sum(gv.astype(np.float64) * u))
        # sum_i g_i . u_i with unit-variance u has the size of |g|
        err = abs(an - fd) / np.linalg.norm(rv)
        worst = max(worst, err)
        assert err <= tol, (an, fd)
    print(f"directional derivatives: worst error {worst:.2e} of |g|")


def test_rollout_32k_stated_checkpointing():
    """The stated reverse-mode configuration: 32,768 particles, N = 6, 20
    steps with a checkpoint every 5 steps, so four segments are recomputed
    from their checkpoints during the reverse pass.  The recomputed steps
    are bit-identical to the recorded ones (ties of the counting sort are
    broken by particle ID), so the gradient must equal, bit for bit, that of
    one segment recorded whole; 10 steps every 5 against every step, and
    every 3 (segments of uneven length), likewise.  (Against the oracle the
    20-step gradient is not comparable element by element: a one-ulp change
    of the input moves the oracle's own gradient by O(1) after 5 steps, and
    the 3-step comparison is test_training_rollout_velocity_gradient.)"""
    sc = scenes.rollout_32k()
    n = sc.n
    tgt = sc.target.astype(np.float64)

    def grad(steps, every):
        sim = _sim(sc)
        sim.rollout_forward(steps, every)
        xg = sim.positions().astype(np.float64)
        g = ((2.0 / n) * (xg - tgt)).astype(np.float32)
        gx, gv = sim.rollout_backward(g, np.zeros((n, 3), np.float32))
        sim.close()
        return gx, gv

    a, b = grad(20, 5), grad(20, 20)
    assert np.all(np.isfinite(a[0])) and np.all(np.isfinite(a[1]))
    assert float(np.abs(a[1]).max()) > 0.0
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    c, d, e = grad(10, 5), grad(10, 1), grad(10, 3)
    for o in (d, e):
        assert np.array_equal(c[0], o[0]) and np.array_equal(c[1], o[1])
