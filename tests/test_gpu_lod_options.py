"""GPU parity of the level options of Section 4.1 (several cameras, automatic
distance range) and of the unilateral density constraint.

Levels are integers chosen by floating point: the GPU decides them in
float32, the oracle in FP64 and reports the particles within its guard band
of a bin edge.  They are compared against the oracle evaluated at the GPU's
own positions, equal away from the edges and either level at an edge (the
hand-computed cases sit on exactly representable values and match bit for
bit); steps are compared like the other parity tests, with the oracle
taking the GPU's levels.
"""
import dataclasses

import numpy as np
import pytest
import torch  # noqa: F401  (first import can be slow; keep it out of test timeouts)

import oracle
import scenes
from parity import check_levels, pos_tol

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


def _block(**kw):
    sc = scenes.block(14, 10, 12, seed=5, n_min=2, n_max=7, vel_sigma=0.3)
    base = dict(lod_mode=scenes.LOD_DTC, camera=(-1.0, 0.8, -1.0), d_near=1.0, d_far=2.5)
    base.update(kw)
    return dataclasses.replace(sc, **base)


def test_two_cameras_on_a_line():
    xs = [0.0, 0.3, 0.5, 0.7, 1.0]
    x = np.stack([np.asarray(xs), np.zeros(5), np.zeros(5)], -1).astype(np.float32)
    sc = scenes.Scene(name="line", x0=x, v0=np.zeros_like(x), lo=(-5, -5, -5), hi=(5, 5, 5),
                      n_min=1, n_max=4, lod_mode=scenes.LOD_DTC, camera=(-0.5, 0, 0),
                      d_near=0.5, d_far=1.5, extra_cameras=(((1.5, 0, 0), (0.5, 1.5)),),
                      gravity=(0, 0, 0))
    with _sim(sc) as sim:
        sim.step(1)
        assert list(sim.debug_levels()) == [4, 3, 2, 3, 4]


@pytest.mark.parametrize("case", ["cameras", "auto", "cameras_auto"])
def test_dtc_options_match_oracle_every_step(case):
    kw = {}
    if case in ("cameras", "cameras_auto"):
        kw["extra_cameras"] = (((1.6, 0.2, 1.4), (0.5, 2.0)), ((0.3, 2.5, 0.3), (1.5, 3.0)))
    if case in ("auto", "cameras_auto"):
        kw["auto_range"] = True
    sc = _block(**kw)
    with _sim(sc) as sim:
        sim.set_graph(True)
        x = sc.x0.astype(np.float64)
        v = sc.v0.astype(np.float64)
        for _ in range(4):
            sim.step(1)
            lv = sim.debug_levels().astype(np.int32)
            check_levels(sc, x, lv)
            x_ref, v_ref, info = oracle.apbf_step(sc, x, v, trace=True, mode=scenes.LOD_EXPLICIT,
                                                  levels=lv)
            xg, vg = sim.positions(), sim.velocities()
            assert np.abs(xg - x_ref).max() <= pos_tol(sc)
            x, v = xg.astype(np.float64), vg.astype(np.float64)
        lv = info["levels"]
    assert len(set(lv.tolist())) >= 3


def test_dtvs_automatic_range():
    sc = scenes.block(14, 10, 12, seed=5, n_min=2, n_max=7, vel_sigma=0.2)
    lo = sc.x0.min(axis=0).astype(np.float64)
    hi = sc.x0.max(axis=0).astype(np.float64)
    mid = (lo + hi) / 2
    sc = scenes.with_dtvs(sc, camera=(mid[0] + 0.3, mid[1] + 0.8, lo[2] - 3.0), target=mid, d_far=0.4)
    sc = dataclasses.replace(sc, auto_range=True)
    with _sim(sc) as sim:
        for _ in range(3):
            x = sim.positions().astype(np.float64)
            sim.step(1)
            lv = sim.debug_levels().astype(np.int32)
            check_levels(sc, x, lv)
    assert len(set(lv.tolist())) >= 4


def test_full_size_tank_with_cameras_and_automatic_range():
    tank = scenes.tank_1m()
    sc = dataclasses.replace(tank, auto_range=True,
                             extra_cameras=(((-3.2, 6.4, 3.2), (0.0, 1.0)),))
    with _sim(sc) as sim:
        sim.set_graph(True)
        sim.step(1)
        lv = sim.debug_levels().astype(np.int32)
    at_edge = check_levels(sc, sc.x0, lv)
    print("tank levels", np.bincount(lv, minlength=11)[5:], f"({at_edge} at a bin edge)")


def test_unilateral_steps_match_oracle():
    sc = dataclasses.replace(
        scenes.block(12, 9, 10, seed=7, n_min=2, n_max=6, levels="random", vel_sigma=0.5),
        unilateral=True)
    with _sim(sc) as sim:
        x = sc.x0.astype(np.float64)
        v = sc.v0.astype(np.float64)
        for _ in range(3):
            x_ref, v_ref, info = oracle.apbf_step(sc, x, v, trace=True)
            sim.step(1)
            xg, vg = sim.positions(), sim.velocities()
            assert np.abs(xg - x_ref).max() <= pos_tol(sc)
            assert np.abs(vg - v_ref).max() <= pos_tol(sc) / float(sc.dt)
            assert np.all(sim.debug_lambda() <= 0.0)
            x, v = xg.astype(np.float64), vg.astype(np.float64)
    # the bilateral run differs (surface particles are pulled inwards)
    with _sim(dataclasses.replace(sc, unilateral=False)) as b, _sim(sc) as u:
        b.step(3)
        u.step(3)
        assert np.abs(b.positions() - u.positions()).max() > 1e-4


def test_batch_mixes_options():
    a = _block(auto_range=True, extra_cameras=(((1.6, 0.2, 1.4), (0.5, 2.0)),))
    b = scenes.dam_break_4k()
    c = dataclasses.replace(scenes.block(8, 7, 6, seed=8, n_min=1, n_max=5, levels="random"),
                            unilateral=True)
    d = _block(auto_range=True)
    scs = [a, b, c, d]
    with _sim(scs) as sim:
        sim.step(3)
        xb, lb = sim.positions(), sim.debug_levels()
        off = sim.offsets
    for i, sc in enumerate(scs):
        with _sim(sc) as one:
            one.step(3)
            assert np.array_equal(one.positions(), xb[off[i]:off[i + 1]])
            assert np.array_equal(one.debug_levels(), lb[off[i]:off[i + 1]])


def test_invalid_options_rejected():
    from paper_1608_04721_amd import PBF_LOD_DTC, PBF_LOD_DTVS, PbfError
    sc = scenes.dam_break_4k()
    with _sim(sc) as sim:
        good = dict(camera=(0.0, 1.0, -1.0), d_near=0.5, d_far=2.0)
        sim.set_lod(PBF_LOD_DTC, **good, auto_range=True)
        cam = ((0.0, 0.0, 0.0), (0.5, 1.0))
        for kw in (dict(extra_cameras=(cam,) * 4),
                   dict(extra_cameras=(((0.0, 0.0, 0.0), (1.0, 1.0)),)),
                   dict(extra_cameras=(((np.inf, 0.0, 0.0), (0.5, 1.0)),)),
                   dict(d_near=2.0, d_far=1.0)):
            with pytest.raises(PbfError) as e:
                sim.set_lod(PBF_LOD_DTC, **{**good, **kw})
            assert e.value.status == -1
        with pytest.raises(PbfError):
            sim.set_lod(PBF_LOD_DTVS, camera=(0.0, 0.5, -2.0), forward=(0, 0, 1), up=(0, 1, 0),
                        focal=100.0, image=(64, 64), splat=0.025, d_near=0.0, d_far=1.0,
                        extra_cameras=(cam,))
        sim.step(1)
    with _sim(dataclasses.replace(sc, unilateral=True)) as sim:
        with pytest.raises(PbfError) as e:
            sim.rollout_forward(2, 1)
        assert e.value.status == -1
