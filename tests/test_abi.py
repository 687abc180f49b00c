"""The C-ABI library loads, exports every symbol that include/pbf.h
declares, and rejects bad arguments on the host before touching a GPU."""
import ctypes
import re
import subprocess
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "pbf.h"


def _header_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pbf_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1608_04721_amd import _lib
    if not _lib.LIB_PATH.exists():
        pytest.fail("libpbf.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_and_binding_agree():
    from paper_1608_04721_amd import _lib
    assert _header_functions() == sorted(_lib.SIGNATURES)


def test_library_exports_every_declared_symbol(lib):
    from paper_1608_04721_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", str(_lib.LIB_PATH)],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pbf_\w+)", out))
    missing = [f for f in _header_functions() if f not in exported]
    assert not missing, missing
    for f in _header_functions():
        assert getattr(lib, f) is not None


def test_host_only_queries(lib):
    from paper_1608_04721_amd import kernel_names
    names = kernel_names()
    assert len(names) == lib.pbf_kernel_count()
    assert {"lambda", "update", "neighbours", "lod_predict"} <= set(names)
    assert lib.pbf_kernel_name(-1) is None and lib.pbf_kernel_name(len(names)) is None
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.pbf_status_string(s)
    assert lib.pbf_last_error(None) == b"null context"


def _params(**kw):
    from paper_1608_04721_amd import _lib
    p = _lib.PbfParams()
    p.n, p.n_min, p.n_max = 8, 1, 4
    for d in range(3):
        p.box_lo[d], p.box_hi[d] = 0.0, 1.0
    p.h, p.rho0, p.mass, p.eps, p.dt = 0.1, 1000.0, 0.125, 12.0, 1.0 / 60.0
    p.gravity[1] = -9.81
    for k, v in kw.items():
        if k in ("box_lo", "box_hi", "grid_dims", "gravity"):
            for d in range(3):
                getattr(p, k)[d] = v[d]
        else:
            setattr(p, k, v)
    return p


@pytest.mark.parametrize("bad", [
    dict(n=-1), dict(n_min=0), dict(n_min=5, n_max=4), dict(n_max=33), dict(h=0.0),
    dict(h=float("nan")), dict(rho0=-1.0), dict(mass=0.0), dict(eps=-1.0), dict(dt=0.0),
    dict(box_hi=(1.0, -1.0, 1.0)), dict(grid_dims=(4, -1, 4)), dict(flags=2),
    dict(max_neighbours=-3), dict(gravity=(0.0, float("inf"), 0.0)),
])
def test_invalid_params_rejected_on_host(lib, bad):
    """Argument checks return PBF_ERR_INVALID_ARG before any HIP call, so
    they are safe to exercise without a GPU."""
    from paper_1608_04721_amd import _lib
    p = _params(**bad)
    x = np.zeros(3 * max(p.n, 0), np.float32)
    ctx = ctypes.c_void_p()
    st = lib.pbf_create(ctypes.byref(p), x.ctypes.data, x.ctypes.data, 0, None, ctypes.byref(ctx))
    assert st == _lib.PBF_ERR_INVALID_ARG
    assert not ctx.value


def test_null_arguments_rejected(lib):
    from paper_1608_04721_amd import _lib
    p = _params()
    ctx = ctypes.c_void_p()
    assert lib.pbf_create(None, None, None, 0, None, ctypes.byref(ctx)) == _lib.PBF_ERR_INVALID_ARG
    assert lib.pbf_create(ctypes.byref(p), None, None, 0, None, ctypes.byref(ctx)) == _lib.PBF_ERR_INVALID_ARG
    assert lib.pbf_create(ctypes.byref(p), None, None, 0, None, None) == _lib.PBF_ERR_INVALID_ARG
    assert lib.pbf_batch_create(0, ctypes.byref(p), None, None, 0, None, ctypes.byref(ctx)) == _lib.PBF_ERR_INVALID_ARG
    assert lib.pbf_step(None, 1) == _lib.PBF_ERR_INVALID_ARG
    assert lib.pbf_sync(None) == _lib.PBF_ERR_INVALID_ARG
    assert lib.pbf_read_positions(None, None, 0) == _lib.PBF_ERR_INVALID_ARG
    assert lib.pbf_set_graph(None, 1) == _lib.PBF_ERR_INVALID_ARG
    assert lib.pbf_density(None, None, None, 0) == _lib.PBF_ERR_INVALID_ARG
    assert lib.pbf_density_noalloc(None, None, None, 0) == _lib.PBF_ERR_INVALID_ARG
    assert lib.pbf_batch_set_cohesion(None, 0, 1.0) == _lib.PBF_ERR_INVALID_ARG
    lib.pbf_destroy(None)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1608_04721_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", tmp_path / "missing.so")
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


@pytest.mark.parametrize("where,bad", [("x0", np.nan), ("x0", np.inf), ("v0", -np.inf),
                                       ("v0", np.nan)])
def test_nonfinite_inputs_rejected_on_host(lib, where, bad):
    """pbf_create checks host inputs for NaN/Inf before any HIP call and
    returns PBF_ERR_NONFINITE without a context."""
    from paper_1608_04721_amd import _lib
    p = _params()
    x = np.full(3 * p.n, 0.5, np.float32)
    v = np.zeros(3 * p.n, np.float32)
    (x if where == "x0" else v)[7] = bad
    ctx = ctypes.c_void_p()
    st = lib.pbf_create(ctypes.byref(p), x.ctypes.data, v.ctypes.data, 0, None, ctypes.byref(ctx))
    assert st == _lib.PBF_ERR_NONFINITE
    assert not ctx.value
    # a batch with the bad value in its second scene is rejected the same way
    pp = (_lib.PbfParams * 2)(_params(), _params())
    x2 = np.concatenate([np.full(3 * p.n, 0.5, np.float32), x])
    v2 = np.concatenate([np.zeros(3 * p.n, np.float32), v])
    st = lib.pbf_batch_create(2, pp, x2.ctypes.data, v2.ctypes.data, 0, None, ctypes.byref(ctx))
    assert st == _lib.PBF_ERR_NONFINITE
    assert not ctx.value


def test_memory_limit_arguments(lib):
    """The device-memory bound is host state: a negative bound is rejected,
    and with no context alive the library holds no device memory."""
    from paper_1608_04721_amd import _lib
    assert lib.pbf_set_memory_limit(-1) == _lib.PBF_ERR_INVALID_ARG
    assert lib.pbf_set_memory_limit(1 << 20) == _lib.PBF_OK
    assert lib.pbf_set_memory_limit(0) == _lib.PBF_OK
    assert lib.pbf_device_bytes() == 0
