"""GPU parity of one batch whose scenes combine every scene option at once:
distance-to-the-visible-surface levels (Section 4.1) with a cone obstacle,
pre-stabilisation (Section 4.3) and cohesion; distance-to-camera levels with
an automatic range, a second camera, the unilateral constraint and a sphere;
a plain dam break; explicit random levels with cohesion and a box obstacle.

One step of such a context runs the depth splat, the range pass, the
cohesion pass, the contact pass and the contact variant of the update pass,
each scene taking only its own options.  Each scene of the batch must equal
its own context bit for bit, graph replays must equal direct launches, and
five steps of the batch are compared with the oracle scene by scene from the
GPU's own state (levels checked first, then taken from the GPU; contact sets
bit-exact outside the guard band of the grown obstacle surfaces).
"""
import dataclasses

import numpy as np
import pytest
import torch  # noqa: F401  (first import can be slow; keep it out of test timeouts)

import oracle
import scenes
from parity import check_levels, pos_tol
from test_gpu_contacts import _near_bound

pytestmark = pytest.mark.gpu

SPHERE, CONE, BOX = scenes.OB_SPHERE, scenes.OB_CONE, scenes.OB_BOX


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


def _scenes():
    # four small dam breaks aimed at a cone, seen from the side (visible surface)
    md = scenes.multi_dam_break(a=6, ny=7, box=(1.2, 0.8, 1.2), cone=(0.3, 0.4), n_min=2, n_max=5,
                                stab_iters=1, stab_s=4)
    (_, c, _), = md.obstacles
    d = np.asarray(c, np.float64) - md.x0.astype(np.float64)
    d[:, 1] = 0.0
    v = 3.0 * d / np.linalg.norm(d, axis=1, keepdims=True)
    md = dataclasses.replace(md, v0=v.astype(np.float32))
    lo, hi = md.x0.min(axis=0).astype(np.float64), md.x0.max(axis=0).astype(np.float64)
    mid = (lo + hi) / 2
    a = dataclasses.replace(scenes.with_dtvs(md, camera=(mid[0] + 0.3, mid[1] + 0.8, lo[2] - 3.0),
                                             target=mid, d_far=0.4), cohesion=0.6)
    # distance to two cameras with an automatic range, unilateral, a sphere
    b = dataclasses.replace(scenes.block(10, 8, 9, seed=11, n_min=2, n_max=6, vel_sigma=0.3),
                            lod_mode=scenes.LOD_DTC, camera=(-1.0, 0.8, -1.0), d_near=1.0,
                            d_far=2.5, auto_range=True, extra_cameras=(((1.6, 0.2, 1.4), (0.5, 2.0)),),
                            unilateral=True, obstacles=((SPHERE, (0.25, 0.15, 0.22), (0.12, 0, 0)),),
                            stab_iters=2, stab_s=4)
    c = scenes.dam_break_4k()
    # explicit random levels, cohesion and a box
    d = dataclasses.replace(scenes.block(8, 7, 6, seed=12, n_min=1, n_max=4, levels="random",
                                         vel_sigma=0.3),
                            cohesion=0.4, obstacles=((BOX, (0.3, 0.1, 0.15), (0.06, 0.06, 0.06)),),
                            stab_iters=1, stab_s=3)
    return [a, b, c, d]


def test_each_scene_equals_its_own_context():
    scs = _scenes()
    with _sim(scs) as batch, _sim(scs) as graphed:
        graphed.set_graph(True)
        for _ in range(5):
            batch.step(1)
            graphed.step(1)
            assert np.array_equal(batch.positions(), graphed.positions())
        xb, lb, mb = batch.positions(), batch.debug_levels(), batch.debug_contacts()
        vb = batch.velocities()
        off = batch.offsets
    # every option is in use and reaches some particles
    assert len(set(lb[off[0]:off[1]].tolist())) >= 3
    assert mb[off[0]:off[1]].any() and mb[off[1]:off[2]].any() and mb[off[3]:off[4]].any()
    assert not mb[off[2]:off[3]].any()
    for i, sc in enumerate(scs):
        with _sim(sc) as one:
            one.step(5)
            s = slice(off[i], off[i + 1])
            assert np.array_equal(one.positions(), xb[s]), f"scene {i} positions"
            assert np.array_equal(one.velocities(), vb[s]), f"scene {i} velocities"
            assert np.array_equal(one.debug_levels(), lb[s]), f"scene {i} levels"
            assert np.array_equal(one.debug_contacts(), mb[s]), f"scene {i} contacts"


def test_batch_steps_match_oracle_scene_by_scene():
    scs = _scenes()
    with _sim(scs) as sim:
        sim.set_graph(True)
        off = sim.offsets
        x, v = sim.positions(), sim.velocities()
        touched = np.zeros(len(scs), np.int64)
        for step in range(5):
            sim.step(1)
            lv, mask = sim.debug_levels().astype(np.int32), sim.debug_contacts()
            xg = sim.positions().astype(np.float64)
            vg = sim.velocities().astype(np.float64)
            for i, sc in enumerate(scs):
                s = slice(off[i], off[i + 1])
                check_levels(sc, x[s], lv[s])
                x_ref, v_ref, info = oracle.apbf_step(sc, x[s].astype(np.float64),
                                                      v[s].astype(np.float64), trace=True,
                                                      mode=scenes.LOD_EXPLICIT, levels=lv[s])
                tol = pos_tol(sc)
                err = float(np.abs(xg[s] - x_ref).max())
                print(f"step {step} scene {i}: max position error {err:.2e} (bound {tol:.1e}), "
                      f"contacts {int(info['contacts'].astype(bool).sum())}")
                assert err <= tol, f"step {step} scene {i}: {err:.3e} > {tol:.1e}"
                assert np.abs(vg[s] - v_ref).max() <= tol / float(sc.dt)
                bad = (mask[s] != info["contacts"])
                if sc.obstacles:
                    bad &= ~_near_bound(sc, info["xs_iter"][0])
                assert not bad.any(), f"step {step} scene {i}: {int(bad.sum())} contact sets differ"
                touched[i] = max(touched[i], int(info["contacts"].astype(bool).sum()))
            x, v = sim.positions(), sim.velocities()
    assert touched[0] > 0 and touched[1] > 0 and touched[3] > 0 and touched[2] == 0
