"""Adaptive position-based fluids on one MI355X: Python binding of libpbf.

``Sim`` wraps one context of the C ABI (one or many scenes advanced
together).  Everything here is argument marshalling; each step of the
solver runs in the library's HIP kernels.  PyTorch is used only when the
caller hands over device tensors or a stream.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (PBF_FLAG_UNILATERAL, PBF_LOD_DTC, PBF_LOD_DTVS,  # noqa: F401
                   PBF_LOD_EXPLICIT, PBF_LOD_UNIFORM, PBF_MAX_CAMERAS,
                   PBF_MAX_ITERS, PBF_MAX_OBSTACLES, PBF_OBSTACLE_BOX, PBF_OBSTACLE_CONE,
                   PBF_OBSTACLE_SPHERE, PbfContactDesc, PbfLodDesc, PbfParams, PbfStepStats)

__all__ = ["Sim", "PbfError", "make_params", "PBF_LOD_UNIFORM", "PBF_LOD_EXPLICIT",
           "PBF_LOD_DTC", "PBF_LOD_DTVS", "PBF_OBSTACLE_SPHERE", "PBF_OBSTACLE_CONE",
           "PBF_OBSTACLE_BOX", "kernel_names", "rollout"]


class PbfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def make_params(src, max_neighbours: int = 0) -> PbfParams:
    """pbf_params from any object with the scene attributes (n, n_min, n_max,
    dims, lo, hi, h, rho0, mass, eps, dt, gravity, and optionally
    unilateral)."""
    p = PbfParams()
    p.n = int(src.n)
    p.n_min, p.n_max = int(src.n_min), int(src.n_max)
    dims = getattr(src, "dims", None)
    for d in range(3):
        p.grid_dims[d] = int(dims[d]) if dims is not None else 0
        p.box_lo[d] = float(src.lo[d])
        p.box_hi[d] = float(src.hi[d])
        p.gravity[d] = float(src.gravity[d])
    p.h, p.rho0, p.mass = float(src.h), float(src.rho0), float(src.mass)
    p.eps, p.dt = float(src.eps), float(src.dt)
    p.max_neighbours = int(max_neighbours)
    p.flags = PBF_FLAG_UNILATERAL if getattr(src, "unilateral", False) else 0
    return p


def kernel_names():
    L = _lib.load()
    return [L.pbf_kernel_name(k).decode() for k in range(L.pbf_kernel_count())]


def _is_tensor(a):
    return type(a).__module__.startswith("torch")


class Sim:
    """A libpbf context over one or more scenes.

    scenes: a scene object or a sequence of them (attributes as in
    make_params plus x0, v0 and optionally lod_mode, levels, camera, d_near,
    d_far).  x0/v0 may instead be given explicitly as float32 arrays (host)
    or torch CUDA tensors (device), scenes concatenated.
    """

    def __init__(self, scenes, x0=None, v0=None, stream=None, max_neighbours: int = 0,
                 apply_lod: bool = True):
        self._lib = _lib.load()
        self._ctx = ctypes.c_void_p()
        seq = list(scenes) if isinstance(scenes, (list, tuple)) else [scenes]
        self.n_scenes = len(seq)
        self.counts = [int(s.n) for s in seq]
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)]).astype(np.int64)
        self.n = int(self.offsets[-1])
        params = (PbfParams * len(seq))(*[make_params(s, max_neighbours) for s in seq])
        on_dev = 0
        keep = []
        if x0 is None:
            x0 = np.concatenate([_f32(s.x0).reshape(-1) for s in seq]) if self.n else np.zeros(0, np.float32)
            v0 = np.concatenate([_f32(s.v0).reshape(-1) for s in seq]) if self.n else np.zeros(0, np.float32)
        if _is_tensor(x0):
            on_dev = 1 if x0.is_cuda else 0
            x0 = x0.contiguous()
            v0 = v0.contiguous()
            keep = [x0, v0]
            xp, vp = (x0.data_ptr(), v0.data_ptr()) if on_dev else (x0.numpy(), v0.numpy())
            if not on_dev:
                keep = [_f32(xp), _f32(vp)]
                xp, vp = keep[0].ctypes.data, keep[1].ctypes.data
        else:
            keep = [_f32(x0).reshape(-1), _f32(v0).reshape(-1)]
            xp, vp = keep[0].ctypes.data, keep[1].ctypes.data
        sp = None
        if stream is not None:
            sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        st = self._lib.pbf_batch_create(len(seq), params, xp, vp, on_dev, sp,
                                        ctypes.byref(self._ctx))
        if st != 0:
            raise PbfError(st, "pbf_batch_create failed: "
                           + self._lib.pbf_status_string(st).decode())
        self.scenes = seq
        if apply_lod:
            for i, s in enumerate(seq):
                mode = getattr(s, "lod_mode", PBF_LOD_UNIFORM)
                if mode != PBF_LOD_UNIFORM:
                    self.set_lod(mode, levels=getattr(s, "levels", None),
                                 camera=getattr(s, "camera", None),
                                 d_near=getattr(s, "d_near", 0.0), d_far=getattr(s, "d_far", 1.0),
                                 scene=i, forward=getattr(s, "forward", (0.0, 0.0, 1.0)),
                                 up=getattr(s, "up", (0.0, 1.0, 0.0)),
                                 focal=getattr(s, "focal", 1.0), image=getattr(s, "image", (1, 1)),
                                 splat=getattr(s, "splat", 0.0),
                                 extra_cameras=getattr(s, "extra_cameras", ()),
                                 auto_range=getattr(s, "auto_range", False))
                if getattr(s, "obstacles", ()) or getattr(s, "stab_iters", 0):
                    self.set_obstacles(s.obstacles, stab_iters=getattr(s, "stab_iters", 0),
                                       stab_set=getattr(s, "stab_s", 1), scene=i)
                if getattr(s, "cohesion", 0.0):
                    self.set_cohesion(s.cohesion, scene=i)

    # ------------------------------------------------------------ helpers
    def _check(self, st, what):
        if st != 0:
            msg = self._lib.pbf_last_error(self._ctx).decode()
            raise PbfError(st, f"{what}: {msg}")

    def close(self):
        if self._ctx:
            self._lib.pbf_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------ core
    def set_lod(self, mode, levels=None, camera=None, d_near=0.0, d_far=1.0, scene=0,
                forward=(0.0, 0.0, 1.0), up=(0.0, 1.0, 0.0), focal=1.0, image=(1, 1), splat=0.0,
                extra_cameras=(), auto_range=False):
        """Level source of one scene (PBF_LOD_*).  extra_cameras: further DTC
        cameras as (camera, (d_near, d_far)) pairs; auto_range: ranges found
        every step from the particles."""
        d = PbfLodDesc()
        d.mode = int(mode)
        if len(extra_cameras) > PBF_MAX_CAMERAS - 1:
            raise PbfError(-1, f"at most {PBF_MAX_CAMERAS - 1} further cameras")
        d.n_extra_cameras = len(extra_cameras)
        for k, (cam, (dn, df)) in enumerate(extra_cameras):
            for a in range(3):
                d.extra_camera[k][a] = float(cam[a])
            d.extra_range[k][0], d.extra_range[k][1] = float(dn), float(df)
        d.auto_range = int(bool(auto_range))
        for a in range(3):
            d.forward[a] = float(forward[a])
            d.up[a] = float(up[a])
        d.focal, d.splat = float(focal), float(splat)
        d.width, d.height = int(image[0]), int(image[1])
        keep = None
        if mode == PBF_LOD_EXPLICIT:
            if _is_tensor(levels) and levels.is_cuda:
                keep = levels.contiguous()
                d.levels = keep.data_ptr()
                d.levels_on_device = 1
            else:
                keep = np.ascontiguousarray(np.asarray(levels), dtype=np.uint8)
                d.levels = keep.ctypes.data
        if camera is not None:
            for a in range(3):
                d.camera[a] = float(camera[a])
        d.d_near, d.d_far = float(d_near), float(d_far)
        self._check(self._lib.pbf_batch_set_lod(self._ctx, int(scene), ctypes.byref(d)),
                    "pbf_batch_set_lod")
        del keep

    def set_obstacles(self, obstacles=(), stab_iters: int = 0, stab_set: int = 1, scene: int = 0):
        """Solid obstacles ((kind, centre, a) tuples, PBF_OBSTACLE_*) and
        pre-stabilisation of the particles with N_i < stab_set."""
        d = PbfContactDesc()
        d.count = len(obstacles)
        if d.count > PBF_MAX_OBSTACLES:
            raise PbfError(-1, f"at most {PBF_MAX_OBSTACLES} obstacles")
        for k, (kind, centre, a) in enumerate(obstacles):
            d.obstacles[k].kind = int(kind)
            for j in range(3):
                d.obstacles[k].centre[j] = float(centre[j])
                d.obstacles[k].a[j] = float(a[j])
        d.stab_iters, d.stab_set = int(stab_iters), int(stab_set)
        self._check(self._lib.pbf_batch_set_obstacles(self._ctx, int(scene), ctypes.byref(d)),
                    "pbf_batch_set_obstacles")

    def set_cohesion(self, gamma: float, scene: int = 0):
        """Force-based cohesion coefficient of one scene (0 removes it)."""
        self._check(self._lib.pbf_batch_set_cohesion(self._ctx, int(scene), float(gamma)),
                    "pbf_batch_set_cohesion")

    def step(self, n_steps: int = 1):
        self._check(self._lib.pbf_step(self._ctx, int(n_steps)), "pbf_step")

    def sync(self):
        self._check(self._lib.pbf_sync(self._ctx), "pbf_sync")

    def positions(self, out=None) -> np.ndarray:
        """(n, 3) float32 positions in ID order; ``out`` may be a CUDA tensor."""
        return self._read(self._lib.pbf_read_positions, out, "pbf_read_positions")

    def velocities(self, out=None) -> np.ndarray:
        return self._read(self._lib.pbf_read_velocities, out, "pbf_read_velocities")

    def _read(self, fn, out, what):
        if out is not None and _is_tensor(out) and out.is_cuda:
            self._check(fn(self._ctx, out.data_ptr(), 1), what)
            return out
        buf = np.empty(3 * self.n, np.float32)
        self._check(fn(self._ctx, buf.ctypes.data, 0), what)
        return buf.reshape(-1, 3)

    def scene_positions(self, scene: int) -> np.ndarray:
        buf = np.empty(3 * self.counts[scene], np.float32)
        self._check(self._lib.pbf_batch_read_positions(self._ctx, int(scene), buf.ctypes.data, 0),
                    "pbf_batch_read_positions")
        return buf.reshape(-1, 3)

    # ------------------------------------------------------------ control
    def set_graph(self, enable: bool):
        self._check(self._lib.pbf_set_graph(self._ctx, int(bool(enable))), "pbf_set_graph")

    def set_block_size(self, kernel, threads: int):
        if isinstance(kernel, str):
            kernel = kernel_names().index(kernel)
        self._check(self._lib.pbf_set_block_size(self._ctx, int(kernel), int(threads)),
                    "pbf_set_block_size")

    def profile_enable(self, enable: bool = True):
        self._check(self._lib.pbf_profile_enable(self._ctx, int(bool(enable))), "pbf_profile_enable")

    def profile_read(self) -> dict:
        k = self._lib.pbf_kernel_count()
        ms = np.zeros(k, np.float64)
        cnt = np.zeros(k, np.int64)
        self._check(self._lib.pbf_profile_read(self._ctx, ms.ctypes.data, cnt.ctypes.data, k),
                    "pbf_profile_read")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(kernel_names())}

    # ------------------------------------------------------------ debug/state
    def stats(self) -> dict:
        s = PbfStepStats()
        self._check(self._lib.pbf_stats(self._ctx, ctypes.byref(s)), "pbf_stats")
        return {"n_iters": s.n_iters, "active": list(s.active[: s.n_iters]),
                "particle_iterations": s.particle_iterations,
                "neighbour_pairs": s.neighbour_pairs, "max_neighbours": s.max_neighbours,
                "total_particle_iterations": s.total_particle_iterations,
                "total_steps": s.total_steps, "max_stage": s.max_stage,
                "tiles_unstaged": s.tiles_unstaged}

    def debug_keys(self) -> np.ndarray:
        out = np.empty(self.n, np.uint32)
        self._check(self._lib.pbf_debug_keys(self._ctx, out.ctypes.data), "pbf_debug_keys")
        return out

    def debug_permutation(self) -> np.ndarray:
        out = np.empty(self.n, np.int32)
        self._check(self._lib.pbf_debug_permutation(self._ctx, out.ctypes.data),
                    "pbf_debug_permutation")
        return out

    def debug_neighbour_counts(self) -> np.ndarray:
        """|N_i| of the last step, ID order."""
        counts = np.empty(self.n, np.int32)
        total = ctypes.c_int64(0)
        self._check(self._lib.pbf_debug_neighbours(self._ctx, counts.ctypes.data, None, 0,
                                                   ctypes.byref(total)), "pbf_debug_neighbours")
        return counts

    def debug_neighbours(self):
        """(counts[n], ids concatenated, offsets[n+1]) with ascending IDs."""
        counts = np.empty(self.n, np.int32)
        total = ctypes.c_int64(0)
        self._check(self._lib.pbf_debug_neighbours(self._ctx, counts.ctypes.data, None, 0,
                                                   ctypes.byref(total)), "pbf_debug_neighbours")
        ids = np.empty(max(total.value, 1), np.int32)
        self._check(self._lib.pbf_debug_neighbours(self._ctx, counts.ctypes.data, ids.ctypes.data,
                                                   ids.size, ctypes.byref(total)),
                    "pbf_debug_neighbours")
        off = np.zeros(self.n + 1, np.int64)
        np.cumsum(counts, out=off[1:])
        return counts, ids[: total.value], off

    def debug_lambda(self) -> np.ndarray:
        out = np.empty(self.n, np.float32)
        self._check(self._lib.pbf_debug_lambda(self._ctx, out.ctypes.data), "pbf_debug_lambda")
        return out

    def debug_contacts(self) -> np.ndarray:
        out = np.zeros(self.n, np.uint8)
        self._check(self._lib.pbf_debug_contacts(self._ctx, out.ctypes.data), "pbf_debug_contacts")
        return out

    def debug_poison(self, enable: bool = True):
        """Fill the float buffers each step writes before reading them with
        NaNs first (a debug check; results are unchanged when it passes)."""
        self._check(self._lib.pbf_debug_poison(self._ctx, int(bool(enable))), "pbf_debug_poison")

    def debug_levels(self) -> np.ndarray:
        out = np.empty(self.n, np.uint8)
        self._check(self._lib.pbf_debug_levels(self._ctx, out.ctypes.data), "pbf_debug_levels")
        return out

    def get_state(self):
        x = np.empty(3 * self.n, np.float32)
        v = np.empty(3 * self.n, np.float32)
        step = ctypes.c_int64(0)
        self._check(self._lib.pbf_get_state(self._ctx, x.ctypes.data, v.ctypes.data,
                                            ctypes.byref(step)), "pbf_get_state")
        return x.reshape(-1, 3), v.reshape(-1, 3), step.value

    def set_state(self, x, v, step: int = 0):
        x = _f32(x).reshape(-1)
        v = _f32(v).reshape(-1)
        self._check(self._lib.pbf_set_state(self._ctx, x.ctypes.data, v.ctypes.data, int(step)),
                    "pbf_set_state")

    def density(self, per_particle: bool = False):
        """Average density after the last step: (mean, max) of rho_i / rho0
        over all particles, plus the per-particle values in ID order if
        per_particle."""
        out = (ctypes.c_double * 2)()
        rho = np.empty(self.n, np.float32) if per_particle else None
        self._check(self._lib.pbf_density(self._ctx, out,
                                          rho.ctypes.data if per_particle else None, 0),
                    "pbf_density")
        return (out[0], out[1], rho) if per_particle else (out[0], out[1])

    def density_noalloc(self, rho_out=None):
        """The same measure through pbf_density_noalloc, which allocates no
        device memory (its work space is a fixed per-GPU array).  rho_out:
        None, a float32 host array or a CUDA tensor of n values, filled in
        ID order.  Returns (mean, max)."""
        out = (ctypes.c_double * 2)()
        ptr, on_dev = None, 0
        if rho_out is not None:
            if isinstance(rho_out, np.ndarray):
                assert rho_out.dtype == np.float32 and rho_out.size == self.n
                ptr = rho_out.ctypes.data
            else:
                assert rho_out.is_cuda and rho_out.numel() == self.n and rho_out.is_contiguous()
                ptr, on_dev = rho_out.data_ptr(), 1
        self._check(self._lib.pbf_density_noalloc(self._ctx, out, ptr, on_dev),
                    "pbf_density_noalloc")
        return out[0], out[1]

    # ------------------------------------------------ differentiable rollout
    def rollout_forward(self, n_steps: int, ckpt_every: int = 1):
        """Advance n_steps steps, checkpointing every ckpt_every steps for a
        later rollout_backward."""
        self._check(self._lib.pbf_rollout_forward(self._ctx, int(n_steps), int(ckpt_every)),
                    "pbf_rollout_forward")

    def rollout_backward(self, dl_dx, dl_dv, out_x=None, out_v=None):
        """Adjoints of the rollout's initial (x, v) from those of its final
        state (ID order, (n, 3)).  Host arrays give host arrays; CUDA tensors
        (with CUDA tensors out_x, out_v to fill) stay on the device."""
        if _is_tensor(dl_dx) and dl_dx.is_cuda:
            gx, gv = dl_dx.contiguous(), dl_dv.contiguous()
            if out_x is None or out_v is None:
                raise ValueError("device adjoints need device out_x and out_v")
            self._check(self._lib.pbf_rollout_backward(self._ctx, gx.data_ptr(), gv.data_ptr(),
                                                       out_x.data_ptr(), out_v.data_ptr(), 1),
                        "pbf_rollout_backward")
            return out_x, out_v
        gx, gv = _f32(dl_dx).reshape(-1), _f32(dl_dv).reshape(-1)
        ox = np.empty(3 * self.n, np.float32)
        ov = np.empty(3 * self.n, np.float32)
        self._check(self._lib.pbf_rollout_backward(self._ctx, gx.ctypes.data, gv.ctypes.data,
                                                   ox.ctypes.data, ov.ctypes.data, 0),
                    "pbf_rollout_backward")
        return ox.reshape(-1, 3), ov.reshape(-1, 3)


def rollout(sim: Sim, x0, v0, n_steps: int, ckpt_every: int = 1):
    """Differentiable rollout for PyTorch: sets sim's state to the CUDA
    tensors (x0, v0) ((n, 3) float32, ID order), advances n_steps steps and
    returns the final (x, v) as new tensors; backward() calls the library's
    reverse mode (levels, neighbour sets and wall contacts of every step held
    fixed)."""
    import torch

    class _Rollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, v):
            xc, vc = x.detach(), v.detach()
            sim.set_state(xc.cpu().numpy(), vc.cpu().numpy())  # host entry point
            sim.rollout_forward(n_steps, ckpt_every)
            xo = torch.empty((sim.n, 3), device=x.device, dtype=torch.float32)
            vo = torch.empty_like(xo)
            sim.positions(out=xo)
            sim.velocities(out=vo)
            sim.sync()  # the copies ran on the library's stream
            return xo, vo

        @staticmethod
        def backward(ctx, gx, gv):
            gx = torch.zeros((sim.n, 3), device="cuda", dtype=torch.float32) if gx is None else gx
            gv = torch.zeros((sim.n, 3), device="cuda", dtype=torch.float32) if gv is None else gv
            ox = torch.empty((sim.n, 3), device=gx.device, dtype=torch.float32)
            ov = torch.empty_like(ox)
            torch.cuda.current_stream().synchronize()
            sim.rollout_backward(gx.float(), gv.float(), ox, ov)
            return ox, ov

    return _Rollout.apply(x0, v0)
