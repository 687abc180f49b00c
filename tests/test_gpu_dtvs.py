"""GPU parity of the distance-to-the-visible-surface levels (Section 4.1).

The depth image is a rasterisation whose pixels, splat radii and minima
are decided in float32 in a fixed order on both sides (projection, splat
radius, distance, depth minimum); the linear map of the resulting distance
onto the levels is FP64 in the oracle, so the levels must match it except
for particles within its guard band of a bin edge, where either level is
accepted.  The step that uses them is then checked like any other step,
with the oracle taking the GPU's levels.
"""
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


def _side_view(sc, dist=3.0, d_far=0.4):
    lo = sc.x0.min(axis=0).astype(np.float64)
    hi = sc.x0.max(axis=0).astype(np.float64)
    mid = (lo + hi) / 2
    return scenes.with_dtvs(sc, camera=(mid[0] + 0.3, mid[1] + 0.8, lo[2] - dist), target=mid,
                            d_far=d_far)


def test_levels_match_oracle_and_step():
    sc = _side_view(scenes.block(14, 10, 12, seed=5, n_min=2, n_max=7, vel_sigma=0.2))
    lv_ref = oracle.levels(sc, sc.x0.astype(np.float64))
    assert len(set(lv_ref.tolist())) >= 4  # the scene spans the level range
    with _sim(sc) as sim:
        sim.step(1)
        lv = sim.debug_levels().astype(np.int32)
        check_levels(sc, sc.x0, lv)
        x_ref, v_ref, info = oracle.apbf_step(sc, sc.x0, sc.v0, trace=True,
                                              mode=scenes.LOD_EXPLICIT, levels=lv)
        x = sim.positions().astype(np.float64)
        assert np.abs(x - x_ref).max() <= pos_tol(sc)
        # levels of the next step, from the GPU's own positions
        sim.step(1)
        check_levels(sc, x, sim.debug_levels())


def test_full_size_tank_levels():
    tank = scenes.tank_1m()
    sc = scenes.with_dtvs(tank, camera=tank.camera, target=(3.2, 1.6, 3.2), d_far=1.0)
    with _sim(sc) as sim:
        sim.set_graph(True)
        sim.step(1)
        lv = sim.debug_levels().astype(np.int32)
    at_edge = check_levels(sc, sc.x0, lv)
    print("tank levels", np.bincount(lv, minlength=11)[5:], f"({at_edge} at a bin edge)")


def test_wide_splats_and_moving_tank():
    # splats of up to 16 pixels: every workgroup's box exceeds the LDS tile
    # and each particle writes its square to the image directly
    blk = scenes.block(14, 10, 12, seed=9, n_min=2, n_max=7, vel_sigma=0.3)
    lo = blk.x0.min(axis=0).astype(np.float64)
    hi = blk.x0.max(axis=0).astype(np.float64)
    mid = (lo + hi) / 2
    sc = scenes.with_dtvs(blk, camera=(mid[0] + 0.1, mid[1] + 0.3, lo[2] - 0.8), target=mid,
                          focal=500.0, d_far=0.4)
    with _sim(sc) as sim:
        for _ in range(3):
            x = sim.positions().astype(np.float64)
            sim.step(1)
            check_levels(sc, x, sim.debug_levels())
    # the full tank after some motion: workgroups straddling the end of a
    # cell row take the direct path, the others the LDS tile
    tank = scenes.tank_1m()
    sc = scenes.with_dtvs(tank, camera=tank.camera, target=(3.2, 1.6, 3.2), d_far=4.0)
    with _sim(sc) as sim:
        sim.set_graph(True)
        sim.step(8)
        x = sim.positions().astype(np.float64)
        sim.step(1)
        lv = sim.debug_levels().astype(np.int32)
    check_levels(sc, x, lv)


def test_batch_mixes_level_sources():
    a = _side_view(scenes.block(9, 7, 8, seed=6, n_min=1, n_max=6, vel_sigma=0.2))
    b = scenes.dam_break_4k().with_lod(scenes.LOD_DTC, n_min=2, n_max=5)
    b.camera, b.d_near, b.d_far = np.array([0.4, 1.0, -0.8], np.float32), np.float32(0.5), np.float32(2.0)
    c = _side_view(scenes.block(6, 9, 7, seed=7, n_min=3, n_max=8, vel_sigma=0.3), dist=2.0)
    scs = [a, b, c]
    with _sim(scs) as sim:
        sim.step(2)
        xb, lb = sim.positions(), sim.debug_levels()
        off = sim.offsets
    for i, sc in enumerate(scs):
        with _sim(sc) as one:
            one.step(2)
            assert np.array_equal(one.positions(), xb[off[i]:off[i + 1]])
            assert np.array_equal(one.debug_levels(), lb[off[i]:off[i + 1]])


def test_graph_replay_equals_direct_launch():
    sc = _side_view(scenes.block(10, 8, 9, seed=8, n_min=2, n_max=6, vel_sigma=0.3))
    with _sim(sc) as a, _sim(sc) as b:
        b.set_graph(True)
        for _ in range(4):
            a.step(1)
            b.step(1)
            assert np.array_equal(a.positions(), b.positions())
            assert np.array_equal(a.debug_levels(), b.debug_levels())


def test_invalid_descriptors_are_rejected():
    from paper_1608_04721_amd import PBF_LOD_DTVS, PbfError
    sc = scenes.dam_break_4k()
    good = dict(camera=(0.0, 0.5, -2.0), forward=(0.0, 0.0, 1.0), up=(0.0, 1.0, 0.0), focal=100.0,
                image=(64, 64), splat=0.025, d_near=0.0, d_far=1.0)
    with _sim(sc) as sim:
        sim.set_lod(PBF_LOD_DTVS, **good)
        for bad in (dict(focal=0.0), dict(image=(0, 64)), dict(image=(64, 9000)), dict(splat=-1.0),
                    dict(camera=(np.nan, 0.0, 0.0)), dict(d_far=0.0)):
            with pytest.raises(PbfError) as e:
                sim.set_lod(PBF_LOD_DTVS, **{**good, **bad})
            assert e.value.status == -1
        sim.step(1)  # still usable with the last valid descriptor
