"""GPU parity of the force-based cohesion option against the FP64 oracle.

The cohesion pass adds dt^2 a_i (clamped into the box) to the prediction,
with a_i evaluated at the start-of-step positions over the neighbour lists
found at the predicted positions.  Each test checks one step against the
oracle at the plain bound (1e-5 of the largest box extent), and that the
cohesion moved the result by far more than that bound.
"""
import dataclasses

import numpy as np
import pytest
import torch  # noqa: F401  (first import can be slow; keep it out of test timeouts)

import oracle
import scenes
from parity import (check_levels, compare_keys, neighbour_mismatch, pos_tol, ref_csr,
                    ulp_sensitivity)

pytestmark = pytest.mark.gpu


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


def _one_step(sc, graph=False, tol=None, **kw):
    x_ref, v_ref, info = oracle.apbf_step(sc, sc.x0, sc.v0, trace=True)
    with _sim(sc, **kw) as sim:
        sim.set_graph(graph)
        sim.step(1)
        x = sim.positions().astype(np.float64)
        v = sim.velocities().astype(np.float64)
        bad, _ = compare_keys(sc, sim.debug_keys(), info["keys"], info["xs_iter"][0])
        assert bad == 0
        assert np.array_equal(sim.debug_levels().astype(np.int32), info["levels"])
        nb = neighbour_mismatch(sc, sim.debug_neighbours(), ref_csr(info), info["xs_iter"][0])
        assert nb == 0
        st = sim.stats()
    tol = pos_tol(sc) if tol is None else tol
    err = float(np.abs(x - x_ref).max())
    assert err <= tol, f"positions: {err:.3e} > {tol:.1e}"
    assert float(np.abs(v - v_ref).max()) <= tol / float(sc.dt)
    return x, x_ref, err, st


def _effect(sc):
    x0, _, _ = oracle.apbf_step(dataclasses.replace(sc, cohesion=0.0), sc.x0, sc.v0)
    x1, _, _ = oracle.apbf_step(sc, sc.x0, sc.v0)
    return float(np.abs(x1 - x0).max())


@pytest.mark.parametrize("gamma", [0.2, 1.0])
def test_moving_block_one_step(gamma):
    sc = scenes.block(13, 9, 11, seed=5, n_min=2, n_max=5, levels="random", vel_sigma=0.4)
    sc = dataclasses.replace(sc, cohesion=gamma)
    _, _, err, _ = _one_step(sc)
    eff = _effect(sc)
    print(f"gamma={gamma}: max position error {err:.2e}, cohesion moved positions by {eff:.2e}")
    assert eff > 20 * pos_tol(sc)


def test_block_on_the_walls_graph_replay():
    # a block in the corner of its box: the shift is clamped on three walls
    sc = scenes.block(10, 10, 10, seed=6, n_min=3, n_max=3, vel_sigma=0.3,
                      box=(np.zeros(3), np.full(3, 0.5)))
    sc = dataclasses.replace(sc, cohesion=2.0, unilateral=True)
    _, _, err, _ = _one_step(sc, graph=True)
    print(f"walls: max position error {err:.2e}")


def test_stage_overflow_path():
    # 16 particles per cell: tile stages exceed LDS and take the HBM path
    sc = scenes.random_cloud(16000, seed=41, extent=1.0, n_min=1, n_max=2, dup_frac=0.0)
    sc = dataclasses.replace(sc, cohesion=0.3)
    _, _, err, st = _one_step(sc, max_neighbours=1000)
    print(f"overflow: max position error {err:.2e}, tiles staged from HBM {st['tiles_unstaged']}")
    assert st["tiles_unstaged"] > 0


def test_random_cloud_with_duplicates():
    # coincident particles give no cohesion force; sparse clouds are
    # ill-conditioned, so the bound is 4x the oracle's own one-ulp spread
    sc = scenes.random_cloud(900, seed=8, extent=0.45, n_min=1, n_max=3, dup_frac=0.05)
    sc = dataclasses.replace(sc, cohesion=0.5)
    tol = max(pos_tol(sc), 4.0 * ulp_sensitivity(sc)[0])
    _, _, err, _ = _one_step(sc, tol=tol)
    print(f"cloud: max position error {err:.2e} (tolerance {tol:.1e})")


def test_batch_mixed_cohesion_equals_serial_and_oracle():
    scs = [dataclasses.replace(scenes.block(7, 5, 6, seed=1, n_min=2, n_max=4, levels="random",
                                            vel_sigma=0.2), cohesion=0.8),
           scenes.block(9, 8, 7, seed=2, n_min=3, n_max=6, levels="random", vel_sigma=0.5),
           dataclasses.replace(scenes.block(6, 6, 6, seed=3, n_min=1, n_max=3, vel_sigma=0.3),
                               cohesion=0.1)]
    with _sim(scs) as batch:
        batch.step(3)
        xb = [batch.scene_positions(i) for i in range(len(scs))]
    for i, sc in enumerate(scs):
        with _sim(sc) as one:
            one.step(3)
            assert np.array_equal(one.positions(), xb[i]), f"scene {i} differs from serial"
    with _sim(scs) as batch:
        batch.set_graph(True)
        batch.step(1)
        for i, sc in enumerate(scs):
            x_ref, _, _ = oracle.apbf_step(sc, sc.x0, sc.v0)
            assert np.abs(batch.scene_positions(i) - x_ref).max() <= pos_tol(sc), i


def test_tank_1m_one_step():
    sc = dataclasses.replace(scenes.tank_1m(), cohesion=0.2)
    x_ref, v_ref, info = oracle.apbf_step(sc, sc.x0, sc.v0, trace=True)
    rng = np.random.default_rng(1)
    sample = rng.choice(sc.n, size=3000, replace=False)
    with _sim(sc) as sim:
        sim.set_graph(True)
        sim.step(1)
        x = sim.positions().astype(np.float64)
        lv = sim.debug_levels().astype(np.int32)
        check_levels(sc, sc.x0, lv)
        nb = neighbour_mismatch(sc, sim.debug_neighbours(), ref_csr(info), info["xs_iter"][0],
                                ids=sample)
        assert nb == 0
    if not np.array_equal(lv, info["levels"]):  # a particle at a bin edge: same levels both sides
        x_ref, v_ref, _ = oracle.apbf_step(sc, sc.x0, sc.v0, mode=scenes.LOD_EXPLICIT, levels=lv)
    err = float(np.abs(x - x_ref).max())
    print(f"tank with cohesion: max position error {err:.2e}")
    assert err <= pos_tol(sc)


def test_setting_and_removing_cohesion():
    from paper_1608_04721_amd import PbfError
    sc = scenes.block(8, 7, 6, seed=9, n_min=2, n_max=4, levels="random", vel_sigma=0.3)
    with _sim(sc) as a, _sim(dataclasses.replace(sc, cohesion=0.6)) as b:
        a.set_graph(True)
        b.set_graph(True)
        for bad in (-0.1, float("nan"), float("inf")):
            with pytest.raises(PbfError):
                b.set_cohesion(bad)
        with pytest.raises(PbfError):
            b.set_cohesion(0.5, scene=1)
        with pytest.raises(PbfError):  # the reverse mode does not differentiate it
            b.rollout_forward(2, 1)
        b.step(1)
        a.step(1)
        assert not np.array_equal(a.positions(), b.positions())
        b.set_cohesion(0.0)  # removed: both contexts take the same steps again
        a.set_cohesion(0.0)
        xa, va, _ = a.get_state()
        b.set_state(xa, va)
        a.step(2)
        b.step(2)
        assert np.array_equal(a.positions(), b.positions())
