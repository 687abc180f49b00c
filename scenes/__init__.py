"""Seeded synthetic scene generators.

This module only builds inputs: particle lattices, jitter, initial
velocities, box extents, solver parameters, camera placement and targets.
It holds none of the solver's arithmetic, and it is the one piece shared by
the FP64 oracle and the HIP path.  Every random draw uses
``numpy.random.default_rng(seed)`` in float64 and is rounded to float32,
so both sides consume identical float32 arrays.

The paper's scenes (dam break, double dam break, multi dam break) give
particle counts and iteration ranges but no box, smoothing length or mass,
so the workloads here are stand-ins of the same kind and scale: dam-break
blocks in a corner of a box and a large tank, on a lattice of spacing
``s = 0.05`` with ``h = 2 s``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

F32 = np.float32

#: lattice spacing, smoothing length, rest density and time step
SPACING = 0.05
H = 0.1
RHO0 = 1000.0
DT = 1.0 / 60.0
#: two steps per 60 Hz frame, as in the paper's evaluation: columns deeper than
#: ~32 lattice layers are not held up by 5-10 Jacobi iterations at dt = 1/60
#: (a confined 64-layer column collapses to 60x rest density within 40 steps
#: in the FP64 oracle) but are at dt = 1/120
DT_DEEP = 1.0 / 120.0
GRAVITY = (0.0, -9.81, 0.0)
#: constraint relaxation added to the denominator of lambda: about the value of
#: that denominator on the rest lattice (1194.86 for h = 2 s), which halves each
#: Newton step; at eps <= 100 the Jacobi iteration grows in the bulk instead of
#: converging (measured growth 1.3-1.8x per iteration)
EPS = 1200.0
JITTER = 1e-3

LOD_UNIFORM = 0
LOD_EXPLICIT = 1
LOD_DTC = 2
LOD_DTVS = 3

#: solid obstacle kinds: (kind, centre, a) with a = (radius, 0, 0) for a
#: sphere, (base radius, height, 0) for a cone standing on its base disc
#: (centre = centre of the base, apex up), half extents for a box
OB_SPHERE = 1
OB_CONE = 2
OB_BOX = 3


@dataclasses.dataclass
class Scene:
    """One fluid scene: float32 arrays plus solver parameters.

    ``x0``/``v0`` are (n, 3) float32 arrays in particle-ID order.
    ``dims`` is the uniform-grid resolution (cells of edge ``h`` from ``lo``).
    ``lod_mode`` selects uniform levels (every particle iterates ``n_max``
    times), explicit per-ID ``levels``, or distance-to-camera levels from
    ``camera``/``d_near``/``d_far``.
    """

    name: str
    x0: np.ndarray
    v0: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    h: float = F32(H)
    rho0: float = F32(RHO0)
    mass: float = F32(RHO0 * SPACING ** 3)
    eps: float = F32(EPS)
    dt: float = F32(DT)
    gravity: np.ndarray = dataclasses.field(
        default_factory=lambda: np.array(GRAVITY, dtype=F32))
    n_min: int = 1
    n_max: int = 1
    dims: np.ndarray = None
    lod_mode: int = LOD_UNIFORM
    levels: Optional[np.ndarray] = None
    camera: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros(3, dtype=F32))
    d_near: float = F32(0.0)
    d_far: float = F32(1.0)
    # distance to the visible surface: camera frame, focal length (pixels),
    # image size (pixels) and splat radius of a particle
    forward: np.ndarray = dataclasses.field(
        default_factory=lambda: np.array([0.0, 0.0, 1.0], dtype=F32))
    up: np.ndarray = dataclasses.field(
        default_factory=lambda: np.array([0.0, 1.0, 0.0], dtype=F32))
    focal: float = F32(256.0)
    image: tuple = (256, 256)
    splat: float = F32(SPACING / 2)
    steps: int = 1
    target: Optional[np.ndarray] = None
    # solid obstacles ((kind, centre, a) tuples, float32 values) and
    # pre-stabilisation: stab_iters iterations for the particles with
    # level < stab_s
    obstacles: tuple = ()
    stab_iters: int = 0
    stab_s: int = 1
    # distance-to-camera levels from further cameras ((camera, (d_near,
    # d_far)) pairs; the particle takes the highest level), ranges found
    # automatically every step, and the unilateral density constraint
    extra_cameras: tuple = ()
    auto_range: bool = False
    unilateral: bool = False
    # coefficient gamma of the force-based cohesion (0: none)
    cohesion: float = 0.0

    def __post_init__(self):
        self.x0 = np.ascontiguousarray(self.x0, dtype=F32).reshape(-1, 3)
        self.v0 = np.ascontiguousarray(self.v0, dtype=F32).reshape(-1, 3)
        self.lo = np.asarray(self.lo, dtype=F32).reshape(3)
        self.hi = np.asarray(self.hi, dtype=F32).reshape(3)
        self.gravity = np.asarray(self.gravity, dtype=F32).reshape(3)
        self.camera = np.asarray(self.camera, dtype=F32).reshape(3)
        self.h, self.rho0, self.mass = F32(self.h), F32(self.rho0), F32(self.mass)
        self.eps, self.dt = F32(self.eps), F32(self.dt)
        self.d_near, self.d_far = F32(self.d_near), F32(self.d_far)
        self.forward = np.asarray(self.forward, dtype=F32).reshape(3)
        self.up = np.asarray(self.up, dtype=F32).reshape(3)
        self.focal, self.splat = F32(self.focal), F32(self.splat)
        self.image = (int(self.image[0]), int(self.image[1]))
        if self.dims is None:
            self.dims = grid_dims(self.lo, self.hi, self.h)
        self.dims = np.asarray(self.dims, dtype=np.int32).reshape(3)
        if self.levels is not None:
            self.levels = np.ascontiguousarray(self.levels, dtype=np.uint8)
        self.obstacles = tuple((int(k), tuple(F32(v) for v in c), tuple(F32(v) for v in a))
                               for k, c, a in self.obstacles)
        self.extra_cameras = tuple((tuple(F32(v) for v in cam), (F32(r[0]), F32(r[1])))
                                   for cam, r in self.extra_cameras)

    @property
    def n(self) -> int:
        return int(self.x0.shape[0])

    def with_lod(self, mode, levels=None, n_min=None, n_max=None) -> "Scene":
        s = dataclasses.replace(self)
        s.lod_mode = mode
        if levels is not None:
            s.levels = np.ascontiguousarray(levels, dtype=np.uint8)
        if n_min is not None:
            s.n_min = int(n_min)
        if n_max is not None:
            s.n_max = int(n_max)
        return s


def look_at(camera, target, up=(0.0, 1.0, 0.0)):
    """Unit forward and up vectors (float32) of a camera at `camera` looking
    at `target`, with `up` made orthogonal to the view direction."""
    c = np.asarray(camera, np.float64)
    f = np.asarray(target, np.float64) - c
    f /= np.linalg.norm(f)
    u = np.asarray(up, np.float64)
    u = u - np.dot(u, f) * f
    u /= np.linalg.norm(u)
    return f.astype(F32), u.astype(F32)


def with_dtvs(sc: "Scene", camera, target, d_near=0.0, d_far=None, focal=None, image=None,
              splat=None) -> "Scene":
    """The scene with distance-to-the-visible-surface levels seen from
    `camera` looking at `target`.  Defaults: 2.5 pixels per spacing at the
    nearest particle (splats of about 1.25 pixels' radius, so the visible
    surface is closed), an image just covering the particles, d_far = 20
    spacings, splat radius = half a spacing."""
    f, u = look_at(camera, target)
    x = sc.x0.astype(np.float64) - np.asarray(camera, np.float64)
    z = x @ f.astype(np.float64)
    r = np.cross(f.astype(np.float64), u.astype(np.float64))
    if focal is None:
        focal = 2.5 * z.min() / SPACING
    if image is None:
        ang = np.max(np.abs(np.stack([x @ r, x @ u.astype(np.float64)], 1)) / z[:, None])
        side = int(np.ceil(2 * focal * ang)) + 8
        image = (side, side)
    d_far = 20 * SPACING if d_far is None else d_far
    splat = SPACING / 2 if splat is None else splat
    return dataclasses.replace(sc, lod_mode=LOD_DTVS, camera=np.asarray(camera, F32), forward=f,
                               up=u, focal=F32(focal), image=tuple(image), splat=F32(splat),
                               d_near=F32(d_near), d_far=F32(d_far))


def grid_dims(lo, hi, h) -> np.ndarray:
    """Cells per axis: ceil(extent / h), at least 1.

    The float32 box and h are widened to float64; a relative slack of 1e-9
    keeps an extent that is a whole number of cells from gaining a cell.
    """
    ext = np.asarray(hi, np.float64) - np.asarray(lo, np.float64)
    q = ext / np.float64(h)
    d = np.ceil(q * (1.0 - 1e-9)).astype(np.int64)
    return np.maximum(d, 1).astype(np.int32)


def lattice(nx, ny, nz, origin, spacing=SPACING, count=None) -> np.ndarray:
    """Points origin + spacing/2 + spacing*(i, j, k), x fastest, y, then z.

    ``count`` truncates the point list (a partial last layer in z-major
    order); the result is float64.
    """
    i = np.arange(nx)
    j = np.arange(ny)
    k = np.arange(nz)
    zz, yy, xx = np.meshgrid(k, j, i, indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1).astype(np.float64)
    pts = np.asarray(origin, np.float64) + spacing * (pts + 0.5)
    if count is not None:
        pts = pts[:count]
    return pts


def _jitter(rng, pts, amp=JITTER):
    return pts + rng.uniform(-amp, amp, size=pts.shape)


def _camera_range(x0: np.ndarray, cam) -> tuple:
    """Distance range of the t = 0 particles to the camera (user-set range)."""
    d = np.linalg.norm(x0.astype(np.float64) - np.asarray(cam, np.float64), axis=1)
    if d.size == 0:
        return F32(0.0), F32(1.0)
    return F32(d.min()), F32(d.max())


def dam_break_4k(seed: int = 1) -> Scene:
    """4,096 particles (16^3 lattice, spacing 0.05, jitter U(-1e-3, 1e-3)) in
    a 1.6^3 box, v = 0, plain PBF with N = 4, 10 steps."""
    rng = np.random.default_rng(seed)
    x = _jitter(rng, lattice(16, 16, 16, (0.0, 0.0, 0.0)))
    return Scene(name="dam_break_4k", x0=x, v0=np.zeros_like(x),
                 lo=(0, 0, 0), hi=(1.6, 1.6, 1.6), n_min=4, n_max=4,
                 lod_mode=LOD_UNIFORM, steps=10)


def dam_break_262k(seed: int = 2) -> Scene:
    """262,144 particles (64^3 block) in the corner of a 2:1:1 tank
    12.8 x 6.4 x 6.4, v = 0, plain PBF with N = 10, dt = 1/120, 100 steps."""
    rng = np.random.default_rng(seed)
    x = _jitter(rng, lattice(64, 64, 64, (0.0, 0.0, 0.0)))
    return Scene(name="dam_break_262k", x0=x, v0=np.zeros_like(x),
                 lo=(0, 0, 0), hi=(12.8, 6.4, 6.4), n_min=10, n_max=10,
                 lod_mode=LOD_UNIFORM, steps=100, dt=DT_DEEP)


def tank_1m(seed: int = 3) -> Scene:
    """1,048,576 particles (128 x 64 x 128 lattice filling the lower half of
    a 6.4^3 box), velocities N(0, 0.1^2) per component, distance-to-camera
    levels N_i in {5..10} (near -> 10), camera at (3.2, 6.4, -3.2), dt = 1/120,
    100 steps.
    """
    rng = np.random.default_rng(seed)
    x = _jitter(rng, lattice(128, 64, 128, (0.0, 0.0, 0.0)))
    v = rng.normal(0.0, 0.1, size=x.shape)
    cam = (3.2, 6.4, -3.2)
    x32 = x.astype(F32)
    dn, df = _camera_range(x32, cam)
    return Scene(name="tank_1m", x0=x32, v0=v, lo=(0, 0, 0), hi=(6.4, 6.4, 6.4),
                 n_min=5, n_max=10, lod_mode=LOD_DTC, camera=cam,
                 d_near=dn, d_far=df, steps=100, dt=DT_DEEP)


def dam_break_batch(seed: int = 4, n_scenes: int = 64,
                    n_lo: int = 4096, n_hi: int = 131072) -> list:
    """Independent dam-break scenes with log-uniform particle counts in
    [n_lo, n_hi] and per-scene iteration ranges 3 <= Nmin <= Nmax <= 10.

    Each block is a x ny x a lattice points (a = ceil(n^(1/3)),
    ny = ceil(n / a^2)), the last layer truncated to n points; the box is
    twice the block extent per axis; the camera sits above the far side.
    """
    rng = np.random.default_rng(seed)
    pairs = [(a, b) for a in range(3, 11) for b in range(a, 11)]
    out = []
    for s in range(n_scenes):
        n = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        a = int(math.ceil(n ** (1.0 / 3.0) - 1e-9))
        ny = int(math.ceil(n / (a * a)))
        pts = lattice(a, ny, a, (0.0, 0.0, 0.0))
        # order y-slowest so that truncating to n points leaves a partial
        # top layer (the last y-layer), as a settled block would have
        order = np.lexsort((pts[:, 0], pts[:, 2], pts[:, 1]))
        pts = pts[order][:n]
        x = _jitter(rng, pts)
        ext = np.array([a, ny, a], np.float64) * SPACING
        hi = 2.0 * ext
        nmin, nmax = pairs[int(rng.integers(len(pairs)))]
        cam = (hi[0] / 2.0, hi[1], -hi[2] / 2.0)
        x32 = x.astype(F32)
        dn, df = _camera_range(x32, cam)
        out.append(Scene(name=f"batch{s:02d}", x0=x32, v0=np.zeros_like(x32),
                         lo=(0, 0, 0), hi=hi, n_min=nmin, n_max=nmax,
                         lod_mode=LOD_DTC, camera=cam, d_near=dn, d_far=df,
                         steps=100, dt=DT_DEEP))
    return out


def multi_dam_break(seed: int = 6, a: int = 35, ny: int = 46, box=(6.4, 3.2, 6.4),
                    cone=(1.5, 2.0), n_min: int = 4, n_max: int = 8, stab_iters: int = 1,
                    stab_s: int = 6, steps: int = 100) -> Scene:
    """Four dam-break blocks of a x ny x a lattice points in the corners of a
    box, around a solid cone standing on the floor at the box centre (base
    radius, height = ``cone``): the multi-dam-break scene of Section 7.3
    (4 x 56,350 = 225,400 particles at the defaults).  Distance-to-camera
    levels N_i in {n_min..n_max}, camera above the front edge; particles
    with N_i < stab_s get stab_iters pre-stabilisation iterations; dt =
    1/120, v = 0.
    """
    rng = np.random.default_rng(seed)
    X, Y, Z = (float(v) for v in box)
    w = a * SPACING
    blocks = [lattice(a, ny, a, (ox, 0.0, oz)) for oz in (0.0, Z - w) for ox in (0.0, X - w)]
    x = _jitter(rng, np.concatenate(blocks))
    cam = (X / 2.0, 2.0 * Y, -Z / 2.0)
    x32 = x.astype(F32)
    dn, df = _camera_range(x32, cam)
    obst = ((OB_CONE, (X / 2.0, 0.0, Z / 2.0), (cone[0], cone[1], 0.0)),)
    return Scene(name="multi_dam_break", x0=x32, v0=np.zeros_like(x32), lo=(0, 0, 0),
                 hi=box, n_min=n_min, n_max=n_max, lod_mode=LOD_DTC, camera=cam,
                 d_near=dn, d_far=df, steps=steps, dt=DT_DEEP, obstacles=obst,
                 stab_iters=stab_iters, stab_s=stab_s)


def rollout_32k(seed: int = 5) -> Scene:
    """32,768 particles (32^3 lattice) in a 3.2^3 box, v0 = 0, N = 6,
    dt = 1/120, 20 steps, with a target cloud x0 + N(0, 0.05^2) paired by
    particle ID."""
    rng = np.random.default_rng(seed)
    x = _jitter(rng, lattice(32, 32, 32, (0.0, 0.0, 0.0)))
    x32 = x.astype(F32)
    tgt = (x32.astype(np.float64) + rng.normal(0.0, 0.05, size=x.shape)).astype(F32)
    return Scene(name="rollout_32k", x0=x32, v0=np.zeros_like(x32),
                 lo=(0, 0, 0), hi=(3.2, 3.2, 3.2), n_min=6, n_max=6,
                 lod_mode=LOD_UNIFORM, steps=20, target=tgt, dt=DT_DEEP)


def block(nx, ny, nz, seed=0, box=None, origin=(0.0, 0.0, 0.0), vel_sigma=0.0,
          n_min=1, n_max=4, levels="uniform", jitter=JITTER) -> Scene:
    """Small dam-break block of nx x ny x nz lattice points (ragged sizes are
    fine) for parity tests.  ``levels`` is "uniform", "random" (explicit
    U{n_min..n_max} per particle) or an array."""
    rng = np.random.default_rng(seed)
    x = lattice(nx, ny, nz, origin)
    if jitter:
        x = _jitter(rng, x, jitter)
    v = rng.normal(0.0, vel_sigma, size=x.shape) if vel_sigma else np.zeros_like(x)
    if box is None:
        ext = np.array([nx, ny, nz], np.float64) * SPACING
        box = (np.zeros(3), 2.0 * ext + np.asarray(origin))
    lo, hi = box
    sc = Scene(name=f"block{nx}x{ny}x{nz}", x0=x, v0=v, lo=lo, hi=hi,
               n_min=n_min, n_max=n_max, lod_mode=LOD_UNIFORM)
    if isinstance(levels, str):
        if levels == "random":
            lv = rng.integers(n_min, n_max + 1, size=sc.n)
            sc = sc.with_lod(LOD_EXPLICIT, levels=lv)
    else:
        sc = sc.with_lod(LOD_EXPLICIT, levels=np.asarray(levels))
    return sc


def random_cloud(n, seed=0, extent=0.5, n_min=1, n_max=4, dup_frac=0.05,
                 vel_sigma=0.5) -> Scene:
    """Random points in a small box with a fraction of exact duplicates
    (coincident pairs) and random explicit levels: an irregular edge case."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, extent, size=(n, 3))
    ndup = int(dup_frac * n)
    if ndup and n > 1:
        src = rng.integers(0, n, size=ndup)
        dst = rng.integers(0, n, size=ndup)
        x[dst] = x[src]
    v = rng.normal(0.0, vel_sigma, size=x.shape)
    lv = rng.integers(n_min, n_max + 1, size=n)
    sc = Scene(name=f"cloud{n}", x0=x, v0=v, lo=(0, 0, 0),
               hi=(extent, extent, extent), n_min=n_min, n_max=n_max)
    return sc.with_lod(LOD_EXPLICIT, levels=lv)


CONFIGS = {
    "dam_break_4k": dam_break_4k,
    "dam_break_262k": dam_break_262k,
    "tank_1m": tank_1m,
    "rollout_32k": rollout_32k,
}
