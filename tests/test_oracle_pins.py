"""Pins of the FP64 oracle against what the mathematics fixes.

Each test checks the oracle against something other than itself:
quadrature, hand-derived closed forms on lattices, brute force, library
sorts, symmetry and invariance properties, and the reduction of the
adaptive loop to plain PBF (Eqs. 9-11 with every level equal to the
maximum).  They run on the CPU only.
"""
import math

import numpy as np
import pytest

import oracle
import scenes

pytestmark = pytest.mark.filterwarnings("ignore")


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)


def _exact_lattice_scene(nx, ny, nz, s=1.0 / 16.0, pad=4, eps=12.0):
    """Unjittered lattice with a binary-exact spacing s and h = 2 s, zero
    gravity and velocity, mass rho0 s^3, block centred in a padded box."""
    h = 2.0 * s
    origin = np.array([pad * h] * 3)
    x = scenes.lattice(nx, ny, nz, origin, spacing=s)
    hi = origin + np.array([nx, ny, nz]) * s + pad * h
    sc = scenes.Scene(name="exact", x0=x, v0=np.zeros_like(x), lo=(0, 0, 0), hi=hi,
                      h=h, rho0=1000.0, mass=1000.0 * s ** 3, eps=eps,
                      gravity=(0, 0, 0), n_min=1, n_max=1)
    # float32 of these values is exact; keep the float64 lattice for the oracle
    return sc, x


# ---------------------------------------------------------------- kernels
def test_poly6_normalised_by_quadrature():
    """The density kernel integrates to one over its support (Eq. 6 needs a
    normalised W).  Gauss-Legendre with 8 nodes is exact for the degree-8
    radial integrand 4 pi r^2 W(r)."""
    for h in (0.1, 0.37, 1.0):
        t, w = np.polynomial.legendre.leggauss(8)
        r = 0.5 * h * (t + 1.0)
        vals = np.array([oracle.poly6(ri * ri, h) for ri in r])
        integral = 0.5 * h * np.sum(w * 4.0 * math.pi * r * r * vals)
        assert abs(integral - 1.0) < 1e-12
    assert oracle.poly6(0.1 ** 2, 0.1) == 0.0  # compact support, r = h excluded


def test_spiky_gradient_is_gradient_of_normalised_spiky_kernel():
    """Rebuild the radial profile W(r) = int_r^h |grad W| from the oracle's
    gradient, check it integrates to one, has the spiky shape (1 - r/h)^3,
    and that finite differences of it reproduce the gradient vector
    (magnitude and sign: it points from p_j towards ... away from p_j)."""
    h = 0.1
    t3, w3 = np.polynomial.legendre.leggauss(6)

    def mag(r):
        return np.linalg.norm(oracle.spiky_grad([r, 0.0, 0.0], h))

    def profile(r):
        nodes = r + 0.5 * (h - r) * (t3 + 1.0)
        return 0.5 * (h - r) * np.sum(w3 * np.array([mag(q) for q in nodes]))

    tq, wq = np.polynomial.legendre.leggauss(10)
    rr = 0.5 * h * (tq + 1.0)
    vol = 0.5 * h * np.sum(wq * 4.0 * math.pi * rr * rr * np.array([profile(q) for q in rr]))
    assert abs(vol - 1.0) < 1e-10
    w0 = profile(0.0)
    for r in (0.01, 0.05, 0.083):
        assert abs(profile(r) / w0 - (1.0 - r / h) ** 3) < 1e-12
    rng = np.random.default_rng(0)
    for _ in range(20):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        r = rng.uniform(0.05, 0.95) * h
        d = r * u
        g = oracle.spiky_grad(d, h)
        fd = np.zeros(3)
        e = 1e-6
        for a in range(3):
            dp, dm = d.copy(), d.copy()
            dp[a] += e
            dm[a] -= e
            fd[a] = (profile(np.linalg.norm(dp)) - profile(np.linalg.norm(dm))) / (2 * e)
        assert np.allclose(g, fd, rtol=1e-6, atol=1e-6 * np.abs(g).max())
        assert np.dot(g, d) < 0.0  # descends away from the neighbour
    assert np.all(oracle.spiky_grad([0, 0, 0], h) == 0.0)
    assert np.all(oracle.spiky_grad([h, 0, 0], h) == 0.0)


# ------------------------------------------------------- lattice closed forms
SQ2, SQ3 = math.sqrt(2.0), math.sqrt(3.0)


def _shell_constants(s, h, rho0, mass):
    K6 = 315.0 / (64.0 * math.pi * h ** 9)
    Ks = 45.0 / (math.pi * h ** 6)
    return K6, Ks


def test_rest_lattice_density_lambda_and_zero_correction():
    """Deep inside a rest lattice with h = 2 s: 26 neighbours (shells
    r^2/s^2 = 1, 2, 3 with 6, 12, 8 points; r = h is excluded),
    rho/rho0 = 315 * 330 / (32768 pi), S = (m/rho0^2) Ks^2 s^4
    [6 + 12 (2-sqrt2)^4 + 8 (2-sqrt3)^4], lambda = -C/(S + eps), and no
    correction by symmetry."""
    n1 = 8
    sc, x = _exact_lattice_scene(n1, n1, n1)
    s, h = 1.0 / 16.0, 1.0 / 8.0
    rho0, mass, eps = 1000.0, 1000.0 / 16.0 ** 3, 12.0
    _, _, info = oracle.apbf_step(sc, x, np.zeros_like(x), trace=True)
    idx = np.arange(n1 ** 3)
    ii, jj, kk = idx % n1, (idx // n1) % n1, idx // (n1 * n1)
    interior = (np.minimum.reduce([ii, jj, kk]) >= 1) & (np.maximum.reduce([ii, jj, kk]) <= n1 - 2)
    deep = (np.minimum.reduce([ii, jj, kk]) >= 2) & (np.maximum.reduce([ii, jj, kk]) <= n1 - 3)
    assert np.all(info["nbr_count"][interior] == 26)
    ratio = 315.0 * 330.0 / (32768.0 * math.pi)
    assert abs(ratio - 1.009775166894685) < 1e-14
    K6, Ks = _shell_constants(s, h, rho0, mass)
    S = mass / rho0 ** 2 * Ks ** 2 * s ** 4 * (6 + 12 * (2 - SQ2) ** 4 + 8 * (2 - SQ3) ** 4)
    lam = -(ratio - 1.0) / (S + eps)
    got = info["lambda_iter"][0][interior]
    assert np.allclose(got, lam, rtol=1e-12, atol=0)
    moved = info["xs_iter"][1][deep] - info["xs_iter"][0][deep]
    assert np.abs(moved).max() < 1e-15


def test_rest_lattice_constant_matches_unit_lattice():
    """The closed forms above do not depend on the scale s once h = 2 s and
    m = rho0 s^3; at s = 0.05, S_rest = 1194.862..."""
    s, h, rho0 = 0.05, 0.1, 1000.0
    m = rho0 * s ** 3
    Ks = 45.0 / (math.pi * h ** 6)
    S = m / rho0 ** 2 * Ks ** 2 * s ** 4 * (6 + 12 * (2 - SQ2) ** 4 + 8 * (2 - SQ3) ** 4)
    assert abs(S - 1194.8623717657538) < 1e-8
    # self density m W(0) / rho0 = 315 / (512 pi)
    assert abs(m * oracle.poly6(0.0, h) / rho0 - 315.0 / (512.0 * math.pi)) < 1e-14


def test_surface_particle_closed_form():
    """Top-centre particle of a 5 x 3 x 5 lattice: 8 in-plane and 9 lower
    neighbours.  rho = m K6 s^6 * 267, the gradient sum points along -y with
    |sum grad W| = Ks s^2 [1 + 4 (2-sqrt2)^2/sqrt2 + 4 (2-sqrt3)^2/sqrt3],
    lambda follows Eq. 4 with both terms, and the correction pulls the
    particle straight down into the fluid."""
    sc, x = _exact_lattice_scene(5, 3, 5)
    s, h = 1.0 / 16.0, 1.0 / 8.0
    rho0, mass, eps = 1000.0, 1000.0 / 16.0 ** 3, 12.0
    i = 2 + 5 * (2 + 3 * 2)  # (ix, iy, iz) = (2, 2, 2)
    _, _, info = oracle.apbf_step(sc, x, np.zeros_like(x), trace=True)
    assert info["nbr_count"][i] == 17
    K6, Ks = _shell_constants(s, h, rho0, mass)
    rho = mass * K6 * s ** 6 * 267.0
    C = rho / rho0 - 1.0
    gy = -Ks * s ** 2 * (1 + 4 * (2 - SQ2) ** 2 / SQ2 + 4 * (2 - SQ3) ** 2 / SQ3)
    g2 = Ks ** 2 * s ** 4 * (5 + 8 * (2 - SQ2) ** 4 + 4 * (2 - SQ3) ** 4)
    lam = -C / (mass / rho0 ** 2 * (gy * gy + g2) + eps)
    assert abs(info["lambda_iter"][0][i] - lam) < 1e-12 * abs(lam)
    dp = info["xs_iter"][1][i] - info["xs_iter"][0][i]
    assert abs(dp[0]) < 1e-15 and abs(dp[2]) < 1e-15
    assert dp[1] < -1e-6


def test_isolated_pair_closed_form():
    """Two particles alone at distance r < h: equal lambdas
    -C / (2 (m/rho0^2) Ks^2 (h-r)^4 + eps) with C = (m K6/rho0)(h^6 +
    (h^2 - r^2)^3) - 1, and Delta p_1 = (2 lambda / rho0) grad W(d) = -Delta p_2
    (Eq. 7); one iteration, then v = Delta p / dt."""
    rng = np.random.default_rng(3)
    for trial in range(5):
        h = 0.1
        r = rng.uniform(0.1, 0.9) * h
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        c = np.array([0.5, 0.5, 0.5])
        x = np.stack([c + 0.5 * r * u, c - 0.5 * r * u])
        sc = scenes.Scene(name="pair", x0=x, v0=np.zeros_like(x), lo=(0, 0, 0), hi=(1, 1, 1),
                          gravity=(0, 0, 0), n_min=1, n_max=1)
        rho0, mass, eps = float(sc.rho0), float(sc.mass), float(sc.eps)
        dt = float(sc.dt)
        d = x[0] - x[1]
        rr = np.linalg.norm(d)
        K6 = 315.0 / (64.0 * math.pi * h ** 9)
        Ks = 45.0 / (math.pi * h ** 6)
        h64 = float(sc.h)
        K6 = 315.0 / (64.0 * math.pi * h64 ** 9)
        Ks = 45.0 / (math.pi * h64 ** 6)
        C = mass * K6 * (h64 ** 6 + (h64 ** 2 - rr ** 2) ** 3) / rho0 - 1.0
        lam = -C / (2.0 * mass / rho0 ** 2 * Ks ** 2 * (h64 - rr) ** 4 + eps)
        dp1 = 2.0 * lam / rho0 * (-Ks * (h64 - rr) ** 2 / rr) * d
        x1, v1, info = oracle.apbf_step(sc, x, np.zeros_like(x), trace=True)
        assert np.allclose(info["lambda_iter"][0], lam, rtol=1e-12)
        assert np.allclose(x1[0] - x[0], dp1, rtol=1e-10, atol=1e-18)
        assert np.allclose(x1[1] - x[1], -dp1, rtol=1e-10, atol=1e-18)
        assert np.allclose(v1[0], dp1 / dt, rtol=1e-9)
        assert C < 0 and lam > 0  # under-dense pair attracts


# ------------------------------------------------------------ neighbours/sort
def _brute_neighbours(xs, h):
    n = xs.shape[0]
    out = []
    for i in range(n):
        d = xs - xs[i]
        r2 = np.einsum("ij,ij->i", d, d)
        m = r2 < h * h
        m[i] = False
        out.append(np.nonzero(m)[0])
    return out


def _csr_lists(info):
    off, ids = info["nbr_off"], info["nbr_ids"]
    return [ids[off[i]:off[i + 1]] for i in range(len(off) - 1)]


@pytest.mark.parametrize("case", ["dam_break_4k", "cloud256", "cloud33", "cloud1"])
def test_grid_neighbours_equal_brute_force(case):
    if case == "dam_break_4k":
        sc = scenes.dam_break_4k()
    else:
        sc = scenes.random_cloud(int(case[5:]), seed=7, extent=0.35)
    _, _, info = oracle.apbf_step(sc, sc.x0, sc.v0, trace=True)
    xs = info["xs_iter"][0]
    got = _csr_lists(info)
    want = _brute_neighbours(xs, float(sc.h))
    for i in range(sc.n):
        assert np.array_equal(got[i], want[i]), i


def test_keys_and_counting_sort():
    """Cell keys are x-fastest floor((x - lo)/h) with clamping, and the
    counting sort equals a library stable argsort by key (ties by ID)."""
    sc = scenes.random_cloud(500, seed=11, extent=0.7)
    _, _, info = oracle.apbf_step(sc, sc.x0, sc.v0, trace=True)
    xs = info["xs_iter"][0]
    c = np.floor((xs - sc.lo.astype(np.float64)) / float(sc.h)).astype(np.int64)
    c = np.clip(c, 0, sc.dims.astype(np.int64) - 1)
    keys = (c[:, 2] * sc.dims[1] + c[:, 1]) * sc.dims[0] + c[:, 0]
    assert np.array_equal(info["keys"], keys.astype(np.uint32))
    assert np.array_equal(info["perm"], np.argsort(keys, kind="stable").astype(np.int32))
    # particles clamped onto the upper wall land in the last cell, not outside
    assert keys.max() < int(np.prod(sc.dims.astype(np.int64)))


# ---------------------------------------------------- solver-loop properties
def _free_blob(seed=5):
    sc = scenes.block(6, 5, 7, seed=seed, box=((0, 0, 0), (2.0, 2.0, 2.0)),
                      origin=(0.7, 0.7, 0.7), n_min=1, n_max=5)
    sc.gravity = np.zeros(3, np.float32)
    return sc


def test_zero_net_correction_when_all_active():
    """With every particle active and no wall contact, Eq. 7 is antisymmetric
    in (i, j), so sum_i Delta p_i = 0 to round-off."""
    sc = _free_blob()
    _, _, info = oracle.apbf_step(sc, sc.x0, sc.v0, trace=True)
    for k in range(sc.n_max):
        dp = info["xs_iter"][k + 1] - info["xs_iter"][k]
        scale = np.abs(dp).sum()
        assert scale > 0
        assert np.abs(dp.sum(axis=0)).max() < 1e-12 * scale


def test_net_correction_nonzero_in_mixed_activity():
    """When some neighbours are finished, corrections are one-sided and the
    sum no longer cancels: a finished particle must not move."""
    sc = _free_blob()
    rng = np.random.default_rng(1)
    lv = rng.integers(1, sc.n_max + 1, size=sc.n)
    sc = sc.with_lod(scenes.LOD_EXPLICIT, levels=lv)
    _, _, info = oracle.apbf_step(sc, sc.x0, sc.v0, trace=True)
    for k in range(1, sc.n_max):
        dp = info["xs_iter"][k + 1] - info["xs_iter"][k]
        if (lv > k).any() and (lv <= k).any():
            assert np.abs(dp.sum(axis=0)).max() > 1e-9 * np.abs(dp).sum()


def test_gating_invariant():
    """A particle is not corrected in iteration k >= N_i and keeps its last
    lambda (finished set of Eq. 11)."""
    sc = scenes.block(9, 6, 7, seed=2, n_min=2, n_max=6, levels="random", vel_sigma=0.3)
    _, _, info = oracle.apbf_step(sc, sc.x0, sc.v0, trace=True)
    lv = info["levels"]
    assert np.array_equal(lv, sc.levels.astype(np.int32))
    for k in range(sc.n_max):
        fin = lv <= k
        act = ~fin
        assert np.array_equal(info["xs_iter"][k + 1][fin], info["xs_iter"][k][fin])
        if k > 0:
            assert np.array_equal(info["lambda_iter"][k][fin], info["lambda_iter"][k - 1][fin])
        moved = np.any(info["xs_iter"][k + 1][act] != info["xs_iter"][k][act], axis=1)
        assert moved.mean() > 0.5


@pytest.mark.parametrize("nmax", [1, 3, 4])
def test_apbf_with_uniform_levels_is_plain_pbf(nmax):
    """Every N_i = n_max makes every P_l = P_1 (Eqs. 9-11): the adaptive step
    equals the separate plain-PBF routine bit for bit."""
    sc = scenes.dam_break_4k()
    sc.n_min = 1
    sc.n_max = nmax
    x, v = sc.x0.astype(np.float64), sc.v0.astype(np.float64)
    xa, va = x, v
    xp, vp = x, v
    for _ in range(3):
        xa, va, _ = oracle.apbf_step(sc, xa, va, mode=scenes.LOD_UNIFORM)
        xp, vp = oracle.pbf_step(sc, xp, vp, nmax)
    assert np.array_equal(xa, xp) and np.array_equal(va, vp)
    lv = np.full(sc.n, nmax, np.int32)
    xe, ve, _ = oracle.apbf_step(sc, x, v, mode=scenes.LOD_EXPLICIT, levels=lv)
    x1, v1 = oracle.pbf_step(sc, x, v, nmax)
    assert np.array_equal(xe, x1) and np.array_equal(ve, v1)


def test_ballistic_isolated_particle():
    """A particle with no neighbours: v' = v + dt g, x' = x + dt v'."""
    x = np.array([[0.5, 0.9, 0.4]])
    v = np.array([[0.3, -0.2, 0.1]])
    sc = scenes.Scene(name="one", x0=x, v0=v, lo=(0, 0, 0), hi=(1, 1, 1), n_min=3, n_max=3)
    dt, g = float(sc.dt), sc.gravity.astype(np.float64)
    x1, v1, _ = oracle.apbf_step(sc, x, v)
    vw = v + dt * g
    xw = x + dt * vw
    assert np.allclose(x1, xw, rtol=0, atol=1e-15)
    assert np.allclose(v1, vw, rtol=1e-12, atol=1e-12)


def test_wall_clamp():
    """A particle predicted through the floor ends on it and its velocity is
    what moved it there."""
    x = np.array([[0.5, 0.001, 0.5]])
    v = np.array([[0.0, -1.0, 0.0]])
    sc = scenes.Scene(name="floor", x0=x, v0=v, lo=(0, 0, 0), hi=(1, 1, 1), n_min=1, n_max=1)
    x1, v1, _ = oracle.apbf_step(sc, x, v)
    assert x1[0, 1] == 0.0
    assert abs(v1[0, 1] - (-0.001 / float(sc.dt))) < 1e-12


def test_translation_by_whole_cells():
    sc = scenes.block(7, 5, 6, seed=4, n_min=1, n_max=3, levels="random", vel_sigma=0.2)
    x1, v1, _ = oracle.apbf_step(sc, sc.x0, sc.v0)
    shift = np.array([3, 1, 2]) * float(sc.h)
    sh = scenes.Scene(name="shift", x0=sc.x0.astype(np.float64) + shift, v0=sc.v0,
                      lo=sc.lo.astype(np.float64) + shift, hi=sc.hi.astype(np.float64) + shift,
                      n_min=1, n_max=3).with_lod(scenes.LOD_EXPLICIT, levels=sc.levels)
    sh.dims = sc.dims
    # oracle takes float64; pass the exact shifted float64 state
    x2, v2, _ = oracle.apbf_step(sh, sc.x0.astype(np.float64) + shift, sc.v0)
    assert np.allclose(x2 - shift, x1, rtol=0, atol=1e-12)
    assert np.allclose(v2, v1, rtol=0, atol=1e-9)


def test_id_permutation_invariance():
    sc = scenes.block(6, 6, 6, seed=8, n_min=1, n_max=4, levels="random", vel_sigma=0.2)
    x1, v1, _ = oracle.apbf_step(sc, sc.x0, sc.v0)
    rng = np.random.default_rng(2)
    p = rng.permutation(sc.n)
    sp = scenes.Scene(name="perm", x0=sc.x0[p], v0=sc.v0[p], lo=sc.lo, hi=sc.hi, n_min=1,
                      n_max=4).with_lod(scenes.LOD_EXPLICIT, levels=sc.levels[p])
    x2, v2, _ = oracle.apbf_step(sp, sp.x0, sp.v0)
    assert np.allclose(x2, x1[p], rtol=0, atol=1e-12)
    assert np.allclose(v2, v1[p], rtol=0, atol=1e-9)


def test_distance_to_camera_levels():
    """Linear map of camera distance to levels (Section 4.1): at or inside
    d_near -> n_max, at or beyond d_far -> n_min, equal-width bins between."""
    cam = np.array([0.0, 0.0, 0.0])
    dists = np.array([0.5, 1.0, 1.0 + 1e-9, 1.5, 1.999, 2.0, 3.0])
    x = np.stack([dists, np.zeros_like(dists), np.zeros_like(dists)], axis=1)
    sc = scenes.Scene(name="lod", x0=x, v0=np.zeros_like(x), lo=(0, 0, 0), hi=(4, 4, 4),
                      n_min=5, n_max=10, lod_mode=scenes.LOD_DTC, camera=cam,
                      d_near=1.0, d_far=2.0)
    lv = oracle.levels(sc, x)
    # t = 0, 0, ~0, 0.5, ~1, 1, 1  ->  10 - floor(6 t)
    assert list(lv) == [10, 10, 10, 7, 5, 5, 5]


def test_level_validation():
    sc = scenes.block(3, 3, 3, n_min=2, n_max=4, levels=np.full(27, 5))
    with pytest.raises(ValueError):
        oracle.apbf_step(sc, sc.x0, sc.v0)
