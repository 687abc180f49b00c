"""Debug poisoning of the step's float buffers (pbf_debug_poison).

With poisoning on, every step first fills the buffers it writes before it
reads them (predicted positions, both x* buffers with their lambda lanes,
the free halves of the position and velocity buffers) with quiet NaNs.  A
step that reads only what it wrote gives the same bits as without; a stray
read would turn into NaN results or PBF_ERR_NONFINITE at the next sync.
Each case here runs with and without poisoning from the same state and
requires bit-identical positions and velocities: direct and graph launches,
the LDS and the HBM stage paths, a batch with every scene option, and the
recomputing reverse pass of a checkpointed rollout.
"""
import numpy as np
import pytest
import torch  # noqa: F401  (first import can be slow; keep it out of test timeouts)

import oracle
import scenes
from test_gpu_batch_options import _scenes as _all_option_scenes

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


def _run(sc, steps, poison, graph, **kw):
    with _sim(sc, **kw) as sim:
        sim.set_graph(graph)
        if poison:
            sim.debug_poison(True)
        sim.step(steps)
        sim.sync()
        return sim.positions(), sim.velocities()


CASES = {
    "block_direct": (lambda: scenes.block(13, 9, 11, seed=5, n_min=2, n_max=6, levels="random",
                                          vel_sigma=0.4), 4, False, {}),
    "tank_1m_graph": (scenes.tank_1m, 3, True, {}),
    "hbm_stage_path": (lambda: scenes.random_cloud(16000, seed=41, extent=1.0, n_min=1, n_max=2,
                                                   dup_frac=0.0), 2, False, {"max_neighbours": 1000}),
    "all_options_batch": (_all_option_scenes, 5, True, {}),
}


@pytest.mark.parametrize("name", list(CASES))
def test_poisoned_steps_are_bit_identical(name):
    make, steps, graph, kw = CASES[name]
    sc = make()
    x0, v0 = _run(sc, steps, False, graph, **kw)
    x1, v1 = _run(sc, steps, True, graph, **kw)
    assert np.isfinite(x1).all() and np.isfinite(v1).all()
    assert np.array_equal(x0, x1), f"{name}: positions differ under poisoning"
    assert np.array_equal(v0, v1), f"{name}: velocities differ under poisoning"


def test_switching_poisoning_mid_run():
    sc = scenes.dam_break_4k()
    with _sim(sc) as a, _sim(sc) as b:
        a.set_graph(True)
        b.set_graph(True)
        a.step(2)
        b.debug_poison(True)
        b.step(2)
        b.debug_poison(False)
        a.step(2)
        b.step(2)
        assert np.array_equal(a.positions(), b.positions())
        from paper_1608_04721_amd import PbfError
        with pytest.raises(PbfError):
            b._check(b._lib.pbf_debug_poison(b._ctx, 2), "pbf_debug_poison")


def test_rollout_gradients_unchanged_by_poisoning():
    sc = scenes.block(8, 7, 6, seed=3, n_min=2, n_max=4, levels="random", vel_sigma=0.3)
    rng = np.random.default_rng(7)
    gx = rng.normal(size=(sc.n, 3)).astype(np.float32)
    gv = rng.normal(size=(sc.n, 3)).astype(np.float32)
    out = []
    for poison in (False, True):
        with _sim(sc) as sim:
            if poison:
                sim.debug_poison(True)
            sim.rollout_forward(6, 2)
            xf = sim.positions()
            dx, dv = sim.rollout_backward(gx, gv)
            out.append((xf, np.array(dx), np.array(dv)))
    for a, b in zip(out[0], out[1]):
        assert np.isfinite(b).all()
        assert np.array_equal(a, b)
