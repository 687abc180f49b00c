"""pbf_density_noalloc, the entry point for callers that cannot allocate
device memory: its results equal pbf_density's bit for bit (same kernels,
same summation order), on two calls in a row with the second context
smaller than the first, with host and device outputs; it allocates nothing
(the library's device-byte count is unchanged by it); and a context whose
work space exceeds the fixed array is refused before anything is enqueued.
"""
import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    from paper_1608_04721_amd import _lib
    _lib.load()


def _check_against_density(sc, steps):
    from paper_1608_04721_amd import Sim, _lib
    lib = _lib.load()
    with Sim(sc) as sim:
        sim.step(steps)
        sim.sync()
        held = lib.pbf_device_bytes()
        rho_h = np.full(sim.n, np.nan, np.float32)
        m0, x0 = sim.density_noalloc(rho_h)
        assert lib.pbf_device_bytes() == held, "the no-allocation entry point allocated"
        rho_d = torch.full((sim.n,), float("nan"), dtype=torch.float32, device="cuda")
        m1, x1 = sim.density_noalloc(rho_d)
        torch.cuda.synchronize()
        m2, x2 = sim.density_noalloc(None)
        assert lib.pbf_device_bytes() == held
        mr, xr, rho_r = sim.density(per_particle=True)
    n = sum(s.n for s in sc) if isinstance(sc, list) else sc.n
    print(f"n={n}: mean {m0:.9f} max {x0:.9f} (pbf_density {mr:.9f} {xr:.9f})", flush=True)
    assert (m0, x0) == (mr, xr) == (m1, x1) == (m2, x2)
    assert np.array_equal(rho_h, rho_r)
    assert np.array_equal(rho_d.cpu().numpy(), rho_r)


def test_noalloc_equals_density_two_calls_second_smaller():
    big = scenes.block(30, 24, 28, seed=11, n_min=2, n_max=6, levels="random", vel_sigma=0.3)
    small = scenes.block(9, 7, 8, seed=12, n_min=1, n_max=3, levels="random", vel_sigma=0.5)
    assert small.n < big.n
    _check_against_density(big, 3)
    _check_against_density(small, 2)


def test_noalloc_batch_of_scenes():
    scs = [scenes.block(7, 6, 5, seed=4, n_min=1, n_max=4, levels="random", vel_sigma=0.3),
           scenes.dam_break_4k()]
    _check_against_density(scs, 2)


def test_noalloc_refuses_a_context_beyond_the_array():
    from paper_1608_04721_amd import PbfError, Sim, _lib
    sc = scenes.block(40, 40, 40, seed=5)  # 64,000 particles
    # 1,000 neighbour codes per particle: 64,000 * (2 * 1,000 + 36) B > 64 MiB
    with Sim(sc, max_neighbours=1000) as sim:
        sim.step(1)
        sim.sync()
        with pytest.raises(PbfError) as ei:
            sim.density_noalloc()
        assert ei.value.status == _lib.PBF_ERR_INVALID_ARG
        # the context is usable afterwards, and the measure still works
        sim.step(1)
        sim.density()


def test_noalloc_needs_a_step():
    from paper_1608_04721_amd import PbfError, Sim
    with Sim(scenes.dam_break_4k()) as sim:
        with pytest.raises(PbfError):
            sim.density_noalloc()
