"""Error paths forced from the host: non-finite state and allocation
failures under a device-memory bound.  Every kernel still runs on valid
data; the failures are decided on the host before or instead of a launch.
A failed call must leave the context as it was: the tests step it
afterwards and compare, bit for bit, with a context that never failed.
"""
import numpy as np
import pytest
import torch  # noqa: F401  (first import can be slow; keep it out of test timeouts)

import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    from paper_1608_04721_amd import _lib
    _lib.load()


@pytest.fixture()
def lib():
    from paper_1608_04721_amd import _lib
    L = _lib.load()
    yield L
    L.pbf_set_memory_limit(0)


def _sim(sc, **kw):
    from paper_1608_04721_amd import Sim
    return Sim(sc, **kw)


def _scene():
    return scenes.block(12, 10, 9, seed=14, n_min=2, n_max=6, levels="random", vel_sigma=0.3)


def _steps(sim, k):
    out = []
    for _ in range(k):
        sim.step(1)
        out.append(sim.positions())
    return out


def test_set_state_nonfinite_rejected_and_state_kept():
    from paper_1608_04721_amd import PbfError
    from paper_1608_04721_amd._lib import PBF_ERR_NONFINITE
    sc = _scene()
    with _sim(sc) as ref:
        ref.step(2)
        want = _steps(ref, 2)
    with _sim(sc) as sim:
        sim.step(2)
        x, v, step = sim.get_state()
        for arr, val in ((x, np.nan), (v, np.inf)):
            bad_x, bad_v = x.copy(), v.copy()
            (bad_x if arr is x else bad_v)[5, 1] = val
            with pytest.raises(PbfError) as e:
                sim.set_state(bad_x, bad_v, step)
            assert e.value.status == PBF_ERR_NONFINITE
        assert sim.get_state()[2] == step
        got = _steps(sim, 2)
    for a, b in zip(want, got):
        assert np.array_equal(a, b)


def test_create_out_of_memory_returns_no_context(lib):
    import ctypes
    from paper_1608_04721_amd import make_params
    from paper_1608_04721_amd._lib import PBF_ERR_OUT_OF_MEMORY
    sc = _scene()
    held = lib.pbf_device_bytes()
    p = make_params(sc)
    x = np.ascontiguousarray(sc.x0, np.float32)
    v = np.ascontiguousarray(sc.v0, np.float32)
    with _sim(sc):
        need = lib.pbf_device_bytes() - held  # what one context of this scene holds
    assert lib.pbf_device_bytes() == held and need > 4096
    for budget in (1, 4096, need // 2, need - 1):
        lib.pbf_set_memory_limit(held + budget)
        ctx = ctypes.c_void_p()
        st = lib.pbf_create(ctypes.byref(p), x.ctypes.data, v.ctypes.data, 0, None, ctypes.byref(ctx))
        assert st == PBF_ERR_OUT_OF_MEMORY, budget
        assert not ctx.value
        assert lib.pbf_device_bytes() == held  # what it did allocate was freed
    lib.pbf_set_memory_limit(0)
    with _sim(sc) as sim:
        assert lib.pbf_device_bytes() > held
        sim.step(1)
    assert lib.pbf_device_bytes() == held


@pytest.mark.parametrize("graph", [False, True])
def test_set_lod_out_of_memory_leaves_scene_table(lib, graph):
    """A visible-surface level source needs a depth image; when it cannot be
    allocated the call fails and the context keeps its old level source,
    depth layout and captured steps."""
    from paper_1608_04721_amd import PbfError
    from paper_1608_04721_amd._lib import PBF_ERR_OUT_OF_MEMORY
    sc = _scene()
    mid = sc.x0.mean(axis=0).astype(np.float64)
    dv = scenes.with_dtvs(sc, camera=(mid[0], mid[1] + 0.5, -2.0), target=mid, d_far=0.4,
                          image=(2048, 2048))
    with _sim(sc) as ref:
        ref.set_graph(graph)
        ref.step(2)
        want = _steps(ref, 3)
        lv_want = ref.debug_levels()
    with _sim(sc) as sim:
        sim.set_graph(graph)
        sim.step(2)
        held = lib.pbf_device_bytes()
        lib.pbf_set_memory_limit(held + 1024)  # far less than a 2048^2 image
        with pytest.raises(PbfError) as e:
            sim.set_lod(scenes.LOD_DTVS, camera=dv.camera, d_near=float(dv.d_near),
                        d_far=float(dv.d_far), forward=dv.forward, up=dv.up, focal=float(dv.focal),
                        image=tuple(int(a) for a in dv.image), splat=float(dv.splat))
        assert e.value.status == PBF_ERR_OUT_OF_MEMORY
        assert lib.pbf_device_bytes() == held
        lib.pbf_set_memory_limit(0)
        got = _steps(sim, 3)
        assert np.array_equal(sim.debug_levels(), lv_want)
        sim.sync()
    for a, b in zip(want, got):
        assert np.array_equal(a, b)


def test_density_and_rollout_out_of_memory_then_succeed(lib):
    """The density measure's and the rollout's buffers are allocated on first
    use; under the bound both calls fail with nothing held, and succeed once
    it is lifted, with the same results as a context that never failed."""
    from paper_1608_04721_amd import PbfError
    from paper_1608_04721_amd._lib import PBF_ERR_OUT_OF_MEMORY
    sc = _scene()
    with _sim(sc) as ref:
        ref.step(2)
        d_want = ref.density(per_particle=True)
        ref.rollout_forward(3, 2)
        x_want = ref.positions()
    with _sim(sc) as sim:
        sim.step(2)
        held = lib.pbf_device_bytes()
        lib.pbf_set_memory_limit(held + 4096)
        with pytest.raises(PbfError) as e:
            sim.density(per_particle=True)
        assert e.value.status == PBF_ERR_OUT_OF_MEMORY
        assert lib.pbf_device_bytes() == held
        with pytest.raises(PbfError) as e:
            sim.rollout_forward(3, 2)
        assert e.value.status == PBF_ERR_OUT_OF_MEMORY
        assert lib.pbf_device_bytes() == held
        lib.pbf_set_memory_limit(0)
        d_got = sim.density(per_particle=True)
        assert d_got[0] == d_want[0] and d_got[1] == d_want[1]
        assert np.array_equal(d_got[2], d_want[2])
        sim.rollout_forward(3, 2)
        assert np.array_equal(sim.positions(), x_want)
