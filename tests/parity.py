"""Comparison helpers for GPU-vs-oracle parity (test infrastructure).

Tolerances:
  positions  max |x_gpu - x_oracle| <= 1e-5 * (largest box extent);
  velocities the same bound divided by dt (v = (x* - x)/dt);
  keys       bit-exact for particles whose predicted position is farther
             than KEY_GUARD (1e-5 * largest extent) from every cell face;
  neighbours bit-exact sets, except pairs whose oracle distance is within
             NBR_GUARD = 1e-4 * h of the radius h;
  permutation bit-exact whenever no key is ambiguous (as above).
FP32 rounding of a coordinate near 6.4 is 4.8e-7, and one step's FP32
arithmetic moves positions by a few ulps, so both guards are >= 10x the
rounding they absorb.
"""
from __future__ import annotations

import numpy as np

import scenes


def extent(sc) -> float:
    return float(np.max(sc.hi.astype(np.float64) - sc.lo.astype(np.float64)))


def pos_tol(sc) -> float:
    return 1e-5 * extent(sc)


def key_ambiguous(sc, xs) -> np.ndarray:
    """Particles whose predicted position lies within the key guard of a
    cell face (either side)."""
    g = 1e-5 * extent(sc)
    q = (xs - sc.lo.astype(np.float64)) / float(sc.h)
    frac = q - np.floor(q)
    d = np.minimum(frac, 1.0 - frac) * float(sc.h)
    return np.any(d <= g, axis=1)


def compare_keys(sc, gpu_keys, ref_keys, xs_ref):
    amb = key_ambiguous(sc, xs_ref)
    bad = (gpu_keys != ref_keys) & ~amb
    return int(bad.sum()), int(amb.sum())


def neighbour_mismatch(sc, gpu, ref, xs_ref, ids=None):
    """Count neighbour-set differences outside the radius guard band.

    gpu/ref: (counts, ids, offsets); ids restricts the check to a sample."""
    h = float(sc.h)
    g = 1e-4 * h
    gc, gi, go = gpu
    rc, ri, ro = ref
    check = range(len(go) - 1) if ids is None else ids
    bad = 0
    for i in check:
        a = gi[go[i]:go[i + 1]]
        b = ri[ro[i]:ro[i + 1]]
        if a.size == b.size and np.array_equal(a, b):
            continue
        diff = np.setxor1d(a, b)
        r = np.linalg.norm(xs_ref[diff] - xs_ref[i], axis=1)
        bad += int(np.sum(np.abs(r - h) > g))
    return bad


def ref_csr(info):
    return info["nbr_count"], info["nbr_ids"], info["nbr_off"]


def ulp_sensitivity(sc, trials=3, seed=0):
    """Largest change of the oracle's one-step positions and final lambdas
    when every input coordinate moves by one float32 ulp (random direction).

    Sparse random clouds hold isolated pairs whose corrections exceed h;
    there one ulp of input moves the exact result by more than 1e-5 of the
    box, so no float32 evaluation can meet that bound.  Tests of such inputs
    take 4x this measured spread as their tolerance."""
    import oracle

    x1, _, i1 = oracle.apbf_step(sc, sc.x0, sc.v0, trace=True)
    lv = i1["levels"]
    lam1 = i1["lambda_iter"][lv - 1, np.arange(sc.n)]
    rng = np.random.default_rng(seed)
    dx = dl = 0.0
    for _ in range(trials):
        d = np.where(rng.random(sc.x0.shape) < 0.5, -np.inf, np.inf).astype(np.float32)
        xp = np.nextafter(sc.x0, d).astype(np.float64)
        x2, _, i2 = oracle.apbf_step(sc, xp, sc.v0, trace=True)
        lam2 = i2["lambda_iter"][lv - 1, np.arange(sc.n)]
        dx = max(dx, float(np.abs(x2 - x1).max()))
        dl = max(dl, float(np.abs(lam2 - lam1).max()))
    return dx, dl


def adjoint_spread(sc, steps, cot_fn, trials=2, seed=0):
    """Largest relative change of the oracle's reverse mode (max-norm, x and
    v adjoints) when every input position moves by one float32 ulp (random
    direction), with the same frozen structure.  cot_fn(x_T) gives the
    output adjoints.  Rollouts through wall contacts are ill-conditioned:
    a particle resting on a wall flips its clamp mask under such a change,
    so multi-step tests take 4x this spread as their tolerance."""
    import oracle

    x0, v0 = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    xT, _, frozen = oracle.rollout_structure(sc, x0, v0, steps)
    rx, rv = oracle.rollout_vjp(sc, x0, v0, frozen, *cot_fn(xT))
    rng = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(trials):
        x32 = x0.astype(np.float32)
        up = np.nextafter(x32, np.float32(np.inf))
        dn = np.nextafter(x32, np.float32(-np.inf))
        xp = np.where(rng.integers(0, 2, size=x0.shape).astype(bool), up, dn).astype(np.float64)
        xTp, _ = oracle.rollout_fixed(sc, xp, v0, frozen)
        px, pv = oracle.rollout_vjp(sc, xp, v0, frozen, *cot_fn(xTp))
        worst = max(worst, np.abs(px - rx).max() / np.abs(rx).max(),
                    np.abs(pv - rv).max() / np.abs(rv).max())
    return (xT, frozen, rx, rv), worst


def check_levels(sc, x, lv_gpu):
    """GPU levels (Eq. 8) against the oracle's FP64 levels at positions x:
    equal for every particle away from a bin edge; within the oracle's guard
    band of an edge (where the float32 evaluation may round to the other
    side) either neighbouring level is accepted.  Returns the number of
    particles whose levels differ (all of them at an edge)."""
    import oracle

    ref, near = oracle.levels(sc, np.asarray(x, np.float64), guard=True)
    lv = np.asarray(lv_gpu).astype(np.int64)
    diff = lv != ref
    away = diff & ~near
    assert not away.any(), f"levels differ away from bin edges at {np.flatnonzero(away)[:10]}"
    assert np.all(np.abs(lv - ref)[diff] <= 1)
    return int(diff.sum())


def ulp_spread_per_particle(sc, x, v, trials=3, seed=0, levels=None):
    """Per-particle conditioning of one oracle step from the state (x, v):
    the largest change of each particle's position and final lambda over
    `trials` runs in which every input coordinate moves by one float32 ulp
    (random direction).

    In a moving fluid a few particles (splash droplets with a handful of
    neighbours) get corrections so large that one ulp of input moves their
    exact result by more than 1e-5 of the box.  Tests of such states keep
    the plain bound for every particle whose spread is below it and give the
    rest 4x their own spread, so one droplet does not loosen the bound for
    the whole fluid."""
    import oracle

    # with `levels`, every run uses those levels (a one-ulp move must not
    # carry a particle across a level's bin edge)
    kw = {} if levels is None else dict(mode=scenes.LOD_EXPLICIT, levels=levels)
    x32 = np.asarray(x, np.float32)
    x1, v1, i1 = oracle.apbf_step(sc, x32, v, trace=True, **kw)
    lv = i1["levels"]
    n = x32.shape[0]
    lam1 = i1["lambda_iter"][lv - 1, np.arange(n)]
    rng = np.random.default_rng(seed)
    dx = np.zeros(n)
    dl = np.zeros(n)
    for _ in range(trials):
        d = np.where(rng.random(x32.shape) < 0.5, -np.inf, np.inf).astype(np.float32)
        xp = np.nextafter(x32, d).astype(np.float64)
        x2, _, i2 = oracle.apbf_step(sc, xp, v, trace=True, **kw)
        lam2 = i2["lambda_iter"][lv - 1, np.arange(n)]
        dx = np.maximum(dx, np.abs(x2 - x1).max(axis=1))
        dl = np.maximum(dl, np.abs(lam2 - lam1))
    return (x1, v1, i1), dx, dl
