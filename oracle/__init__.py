"""FP64 CPU oracle of the adaptive PBF step (ctypes wrapper of oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
never does.  It shares no code with the HIP path; both read their inputs
from the ``scenes`` generator only.

See oracle.c for the equations followed and the readings taken where the
paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB_PATH = _HERE / "liboracle.so"

ORC_OK, ORC_ERR_ARG, ORC_ERR_MEM = 0, -1, -3


def build(force: bool = True) -> Path:
    """Compile oracle.c with gcc (OpenMP, strict FP: no contraction)."""
    if force or not _LIB_PATH.exists() or _LIB_PATH.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB_PATH.with_suffix(".so.tmp")
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", str(_SRC), "-o", str(tmp), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_min", ctypes.c_int32), ("n_max", ctypes.c_int32),
                ("dims", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("h", ctypes.c_double), ("rho0", ctypes.c_double),
                ("mass", ctypes.c_double), ("eps", ctypes.c_double), ("dt", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("unilateral", ctypes.c_int32),
                ("cohesion", ctypes.c_double)]


class Lod(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("levels", ctypes.POINTER(ctypes.c_int32)),
                ("camera", ctypes.c_double * 3), ("d_near", ctypes.c_double),
                ("d_far", ctypes.c_double), ("forward", ctypes.c_double * 3),
                ("up", ctypes.c_double * 3), ("focal", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("splat", ctypes.c_double), ("n_extra", ctypes.c_int32),
                ("extra_camera", (ctypes.c_double * 3) * 3),
                ("extra_range", (ctypes.c_double * 2) * 3), ("auto_range", ctypes.c_int32)]


class Trace(ctypes.Structure):
    _fields_ = [("levels", ctypes.POINTER(ctypes.c_int32)),
                ("keys", ctypes.POINTER(ctypes.c_uint32)),
                ("perm", ctypes.POINTER(ctypes.c_int32)),
                ("nbr_count", ctypes.POINTER(ctypes.c_int32)),
                ("nbr_ids", ctypes.POINTER(ctypes.c_int32)),
                ("nbr_cap", ctypes.c_int64), ("nbr_total", ctypes.c_int64),
                ("xs_iter", ctypes.POINTER(ctypes.c_double)),
                ("lambda_iter", ctypes.POINTER(ctypes.c_double)),
                ("contacts", ctypes.POINTER(ctypes.c_uint8))]


MAX_OBSTACLES = 4


class Obstacle(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("c", ctypes.c_double * 3), ("a", ctypes.c_double * 3)]


class Contacts(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("ob", Obstacle * MAX_OBSTACLES),
                ("stab_iters", ctypes.c_int32), ("stab_s", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)  # rebuilds when oracle.c is newer than the library
        L = ctypes.CDLL(str(_LIB_PATH))
        L.orc_poly6.restype = ctypes.c_double
        L.orc_poly6.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_spiky_grad.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_double)]
        L.orc_apbf_step.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Lod),
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Trace)]
        L.orc_apbf_step_contacts.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Lod),
                                             ctypes.POINTER(Contacts), ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.POINTER(Trace)]
        L.orc_obstacle_project.argtypes = [ctypes.POINTER(Obstacle), ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]
        L.orc_contact_found.argtypes = [ctypes.POINTER(Obstacle), ctypes.POINTER(ctypes.c_double),
                                        ctypes.c_double]
        L.orc_pbf_step.argtypes = [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_void_p]
        L.orc_density.argtypes = [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p]
        L.orc_apbf_step_fixed.argtypes = [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_apbf_step_fixed_vjp.argtypes = [ctypes.POINTER(Params), ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_spiky_hess.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_double)]
        L.orc_levels.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Lod), ctypes.c_void_p,
                                 ctypes.c_void_p]
        L.orc_levels_guarded.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Lod), ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]
        L.orc_cell_keys.argtypes = [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p]
        L.orc_counting_sort.argtypes = [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]
        L.orc_cohesion_spline.restype = ctypes.c_double
        L.orc_cohesion_spline.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_cohesion_accel.argtypes = [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]
        L.orc_set_threads.argtypes = [ctypes.c_int32]
        L.orc_get_threads.restype = ctypes.c_int32
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def poly6(r2: float, h: float) -> float:
    return float(lib().orc_poly6(float(r2), float(h)))


def cohesion_spline(r: float, h: float) -> float:
    """The cohesion kernel C(r) of the force-based cohesion option."""
    return float(lib().orc_cohesion_spline(float(r), float(h)))


def cohesion_accel(scene, x, off, ids) -> np.ndarray:
    """Cohesion accelerations at positions x (n x 3) over the neighbour
    sets given as CSR (off[n+1], ids in particle-ID order)."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    p = params(scene, n=x.shape[0])
    off = np.ascontiguousarray(off, np.int64)
    ids = np.ascontiguousarray(ids, np.int32)
    a = np.zeros_like(x)
    rc = lib().orc_cohesion_accel(ctypes.byref(p), x.ctypes.data, off.ctypes.data,
                                  ids.ctypes.data if ids.size else None, a.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_cohesion_accel failed ({rc})")
    return a


def spiky_grad(d, h: float) -> np.ndarray:
    d = np.ascontiguousarray(d, np.float64).reshape(3)
    out = np.zeros(3, np.float64)
    lib().orc_spiky_grad(_ptr(d, ctypes.c_double), float(h), _ptr(out, ctypes.c_double))
    return out


def params(scene, n=None, n_min=None, n_max=None) -> Params:
    """Widen a scene's float32 parameters to the oracle's float64 struct."""
    p = Params()
    p.n = scene.n if n is None else int(n)
    p.n_min = scene.n_min if n_min is None else int(n_min)
    p.n_max = scene.n_max if n_max is None else int(n_max)
    for d in range(3):
        p.dims[d] = int(scene.dims[d])
        p.lo[d] = float(scene.lo[d])
        p.hi[d] = float(scene.hi[d])
        p.g[d] = float(scene.gravity[d])
    p.h, p.rho0, p.mass = float(scene.h), float(scene.rho0), float(scene.mass)
    p.eps, p.dt = float(scene.eps), float(scene.dt)
    p.unilateral = int(bool(getattr(scene, "unilateral", False)))
    p.cohesion = float(getattr(scene, "cohesion", 0.0))
    return p


class _LodHolder:
    def __init__(self, scene, mode=None, levels=None):
        self.lod = Lod()
        self.lod.mode = scene.lod_mode if mode is None else int(mode)
        lv = scene.levels if levels is None else levels
        self.levels = None
        if self.lod.mode == 1:
            self.levels = np.ascontiguousarray(lv, np.int32)
            self.lod.levels = _ptr(self.levels, ctypes.c_int32)
        for d in range(3):
            self.lod.camera[d] = float(scene.camera[d])
            self.lod.forward[d] = float(getattr(scene, "forward", (0, 0, 1))[d])
            self.lod.up[d] = float(getattr(scene, "up", (0, 1, 0))[d])
        self.lod.d_near, self.lod.d_far = float(scene.d_near), float(scene.d_far)
        self.lod.focal = float(getattr(scene, "focal", 1.0))
        w, h = getattr(scene, "image", (1, 1))
        self.lod.width, self.lod.height = int(w), int(h)
        self.lod.splat = float(getattr(scene, "splat", 0.0))
        extra = getattr(scene, "extra_cameras", ())
        self.lod.n_extra = len(extra)
        for k, (cam, (dn, df)) in enumerate(extra):
            for d in range(3):
                self.lod.extra_camera[k][d] = float(cam[d])
            self.lod.extra_range[k][0], self.lod.extra_range[k][1] = float(dn), float(df)
        self.lod.auto_range = int(bool(getattr(scene, "auto_range", False)))


def _obstacle(kind, centre, a) -> Obstacle:
    o = Obstacle()
    o.kind = int(kind)
    for d in range(3):
        o.c[d] = float(centre[d])
        o.a[d] = float(a[d])
    return o


def contacts(scene):
    """The scene's obstacles and pre-stabilisation settings, or None."""
    obs = getattr(scene, "obstacles", ())
    if not obs and not getattr(scene, "stab_iters", 0):
        return None
    oc = Contacts()
    oc.count = len(obs)
    for k, (kind, centre, a) in enumerate(obs):
        oc.ob[k] = _obstacle(kind, centre, a)
    oc.stab_iters = int(scene.stab_iters)
    oc.stab_s = int(scene.stab_s)
    return oc


def obstacle_project(kind, centre, a, x):
    """Closest surface point of a solid obstacle to x if x is inside it,
    else None (float64)."""
    o = _obstacle(kind, centre, a)
    x = np.ascontiguousarray(x, np.float64).reshape(3)
    y = np.zeros(3, np.float64)
    inside = lib().orc_obstacle_project(ctypes.byref(o), _ptr(x, ctypes.c_double),
                                        _ptr(y, ctypes.c_double))
    return y if inside else None


def contact_found(kind, centre, a, x, margin) -> bool:
    o = _obstacle(kind, centre, a)
    x = np.ascontiguousarray(x, np.float64).reshape(3)
    return bool(lib().orc_contact_found(ctypes.byref(o), _ptr(x, ctypes.c_double), float(margin)))


def levels(scene, x, guard: bool = False):
    """Levels N_i (Eq. 8) at positions x, in FP64.  guard=True also returns a
    bool array marking the particles within the guard band of a bin edge,
    where a lower-precision evaluation may give the neighbouring level."""
    p = params(scene)
    hold = _LodHolder(scene)
    x = np.ascontiguousarray(x, np.float64)
    out = np.zeros(scene.n, np.int32)
    near = np.zeros(max(scene.n, 1), np.uint8)
    rc = lib().orc_levels_guarded(ctypes.byref(p), ctypes.byref(hold.lod), x.ctypes.data,
                                  out.ctypes.data, near.ctypes.data)
    if rc != ORC_OK:
        raise ValueError(f"orc_levels failed ({rc})")
    return (out, near[:scene.n].astype(bool)) if guard else out


def apbf_step(scene, x, v, trace=False, mode=None, levels=None, n_min=None, n_max=None):
    """Advance float64 (n, 3) arrays x, v by one APBF step (copies are made).

    Returns (x, v, info); with trace=True info holds levels, keys, perm,
    neighbour CSR (count, ids), x* before/after every iteration and lambda
    after every lambda pass."""
    p = params(scene, n_min=n_min, n_max=n_max)
    hold = _LodHolder(scene, mode, levels)
    oc = contacts(scene)
    ocp = ctypes.byref(oc) if oc is not None else None
    x = np.array(x, np.float64, order="C").reshape(-1, 3)
    v = np.array(v, np.float64, order="C").reshape(-1, 3)
    n, K = p.n, p.n_max
    info = {}
    tr = None
    if trace:
        info = {
            "levels": np.zeros(n, np.int32), "keys": np.zeros(n, np.uint32),
            "perm": np.zeros(n, np.int32), "nbr_count": np.zeros(n, np.int32),
            "xs_iter": np.zeros((K + 1, n, 3), np.float64),
            "lambda_iter": np.zeros((K, n), np.float64),
            "contacts": np.zeros(n, np.uint8),
        }
        tr = Trace()
        tr.levels = _ptr(info["levels"], ctypes.c_int32)
        tr.keys = _ptr(info["keys"], ctypes.c_uint32)
        tr.perm = _ptr(info["perm"], ctypes.c_int32)
        tr.nbr_count = _ptr(info["nbr_count"], ctypes.c_int32)
        tr.xs_iter = _ptr(info["xs_iter"], ctypes.c_double)
        tr.lambda_iter = _ptr(info["lambda_iter"], ctypes.c_double)
        tr.contacts = _ptr(info["contacts"], ctypes.c_uint8)
        # first call sizes the neighbour list, second call fills it
        x0, v0 = x.copy(), v.copy()
        tr.nbr_cap = 0
        rc = lib().orc_apbf_step_contacts(ctypes.byref(p), ctypes.byref(hold.lod), ocp,
                                          x0.ctypes.data, v0.ctypes.data, ctypes.byref(tr))
        if rc != ORC_OK:
            raise ValueError(f"orc_apbf_step failed ({rc})")
        ids = np.zeros(max(int(tr.nbr_total), 1), np.int32)
        info["nbr_ids"] = ids[: int(tr.nbr_total)]
        tr.nbr_ids = _ptr(ids, ctypes.c_int32)
        tr.nbr_cap = ids.size
    rc = lib().orc_apbf_step_contacts(ctypes.byref(p), ctypes.byref(hold.lod), ocp, x.ctypes.data,
                                      v.ctypes.data, ctypes.byref(tr) if tr is not None else None)
    if rc != ORC_OK:
        raise ValueError(f"orc_apbf_step failed ({rc})")
    if trace:
        off = np.zeros(n + 1, np.int64)
        np.cumsum(info["nbr_count"], out=off[1:])
        info["nbr_off"] = off
    return x, v, info


def pbf_step(scene, x, v, iters):
    """Plain PBF step with a fixed iteration count (separate loop, no gating)."""
    p = params(scene)
    x = np.array(x, np.float64, order="C").reshape(-1, 3)
    v = np.array(v, np.float64, order="C").reshape(-1, 3)
    rc = lib().orc_pbf_step(ctypes.byref(p), int(iters), x.ctypes.data, v.ctypes.data)
    if rc != ORC_OK:
        raise ValueError(f"orc_pbf_step failed ({rc})")
    return x, v


def density(scene, x) -> np.ndarray:
    p = params(scene)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    rho = np.zeros(p.n, np.float64)
    rc = lib().orc_density(ctypes.byref(p), x.ctypes.data, rho.ctypes.data)
    if rc != ORC_OK:
        raise ValueError(f"orc_density failed ({rc})")
    return rho


def cell_keys(scene, xs) -> np.ndarray:
    p = params(scene, n=len(xs))
    xs = np.ascontiguousarray(xs, np.float64).reshape(-1, 3)
    out = np.zeros(p.n, np.uint32)
    lib().orc_cell_keys(ctypes.byref(p), xs.ctypes.data, out.ctypes.data)
    return out


def counting_sort(scene, keys) -> np.ndarray:
    keys = np.ascontiguousarray(keys, np.uint32)
    p = params(scene, n=keys.size)
    G = int(np.prod(scene.dims.astype(np.int64)))
    perm = np.zeros(keys.size, np.int32)
    start = np.zeros(G + 1, np.int64)
    rc = lib().orc_counting_sort(ctypes.byref(p), keys.ctypes.data, perm.ctypes.data,
                                 start.ctypes.data)
    if rc != ORC_OK:
        raise ValueError("orc_counting_sort failed")
    return perm


def run(scene, steps=None, x=None, v=None, mode=None, levels=None):
    """Run the oracle for a number of steps from the scene's initial state."""
    x = scene.x0.astype(np.float64) if x is None else x
    v = scene.v0.astype(np.float64) if v is None else v
    for _ in range(scene.steps if steps is None else steps):
        x, v, _ = apbf_step(scene, x, v, mode=mode, levels=levels)
    return x, v


def apbf_step_fixed(scene, x, v, levels, nbr_off, nbr_ids):
    """One step with the given levels and neighbour sets (CSR by particle ID)
    held fixed; returns float64 (x, v)."""
    p = params(scene)
    x = np.array(x, np.float64, order="C").reshape(-1, 3)
    v = np.array(v, np.float64, order="C").reshape(-1, 3)
    lv = np.ascontiguousarray(levels, np.int32)
    off = np.ascontiguousarray(nbr_off, np.int64)
    ids = np.ascontiguousarray(nbr_ids, np.int32)
    if ids.size == 0:
        ids = np.zeros(1, np.int32)
    rc = lib().orc_apbf_step_fixed(ctypes.byref(p), lv.ctypes.data, off.ctypes.data,
                                   ids.ctypes.data, x.ctypes.data, v.ctypes.data)
    if rc != ORC_OK:
        raise ValueError(f"orc_apbf_step_fixed failed ({rc})")
    return x, v


def spiky_hess(d, h: float) -> np.ndarray:
    """3x3 Jacobian of spiky_grad with respect to p_i at d = p_i - p_j."""
    d = np.ascontiguousarray(d, np.float64)
    out = np.zeros(9, np.float64)
    lib().orc_spiky_hess(_ptr(d, ctypes.c_double), float(h), _ptr(out, ctypes.c_double))
    return out.reshape(3, 3)


def apbf_step_fixed_vjp(scene, x, v, levels, nbr_off, nbr_ids, gx, gv):
    """Reverse mode of apbf_step_fixed at (x, v): the adjoints (gx, gv) of
    the step's outputs (x', v') in, those of (x, v) out (float64, by ID)."""
    p = params(scene)
    x = np.ascontiguousarray(np.asarray(x, np.float64).reshape(-1, 3))
    v = np.ascontiguousarray(np.asarray(v, np.float64).reshape(-1, 3))
    gx = np.array(gx, np.float64, order="C").reshape(-1, 3)
    gv = np.array(gv, np.float64, order="C").reshape(-1, 3)
    lv = np.ascontiguousarray(levels, np.int32)
    off = np.ascontiguousarray(nbr_off, np.int64)
    ids = np.ascontiguousarray(nbr_ids, np.int32)
    if ids.size == 0:
        ids = np.zeros(1, np.int32)
    rc = lib().orc_apbf_step_fixed_vjp(ctypes.byref(p), lv.ctypes.data, off.ctypes.data,
                                       ids.ctypes.data, x.ctypes.data, v.ctypes.data,
                                       gx.ctypes.data, gv.ctypes.data)
    if rc != ORC_OK:
        raise ValueError(f"orc_apbf_step_fixed_vjp failed ({rc})")
    return gx, gv


def rollout_vjp(scene, x, v, frozen, gx, gv):
    """Reverse mode of rollout_fixed from (x, v): replays the steps keeping
    every step's input state, then applies the step adjoints last to first."""
    states = []
    x = np.asarray(x, np.float64)
    v = np.asarray(v, np.float64)
    for lv, off, ids in frozen:
        states.append((x, v))
        x, v = apbf_step_fixed(scene, x, v, lv, off, ids)
    for (xs, vs), (lv, off, ids) in zip(reversed(states), reversed(frozen)):
        gx, gv = apbf_step_fixed_vjp(scene, xs, vs, lv, off, ids, gx, gv)
    return gx, gv


def rollout_structure(scene, x, v, steps):
    """Run `steps` steps and record each step's levels and neighbour sets
    (the discrete structure an adjoint holds fixed); returns the final
    float64 state and the list of (levels, off, ids)."""
    x = np.asarray(x, np.float64)
    v = np.asarray(v, np.float64)
    frozen = []
    for _ in range(steps):
        x1, v1, info = apbf_step(scene, x, v, trace=True)
        frozen.append((info["levels"], info["nbr_off"], info["nbr_ids"]))
        x, v = x1, v1
    return x, v, frozen


def rollout_fixed(scene, x, v, frozen):
    """Replay a rollout with recorded structure (see rollout_structure)."""
    for lv, off, ids in frozen:
        x, v = apbf_step_fixed(scene, x, v, lv, off, ids)
    return x, v
