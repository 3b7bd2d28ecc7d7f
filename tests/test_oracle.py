"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test is chosen so that a plausible mistake in the oracle (a dropped term,
a wrong sign or index, a transposed operand, an off-by-one in the sample
placement or the voxel lookup) fails at least one of them. None of them calls
the HIP library.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from tests import brute_eq1

BG = (1.0, 1.0, 1.0)


def _one_ray_view(eye, target=(0.0, 0.0, 0.0), up=(0.3, 0.2, 1.0)):
    """A 1x1 image whose only pixel ray is the camera's forward axis."""
    K = np.array([[1.0, 0, 0.5], [0, 1.0, 0.5], [0, 0, 1]])
    return K, synth.look_at(eye, target, up=up)


def _const_scene(k, D, l, sig, uval, bval, **kw):
    sigma = np.full((k, k, k), sig, np.float32)
    u = np.broadcast_to(np.asarray(uval, np.float32).reshape(1, 1, 1, D, 3),
                        (k, k, k, D, 3)).copy()
    beta = np.broadcast_to(np.asarray(bval, np.float32).reshape(1, 1, D), (l, l, D)).copy()
    return oracle.Scene(beta, sigma, u, **kw)


def _tiny_random(seed, k=4, D=3, l=4, density=0.6):
    rng = np.random.default_rng(seed)
    sigma = (rng.uniform(0, 8, (k, k, k)) * (rng.uniform(size=(k, k, k)) < density)).astype(
        np.float32)
    u = rng.uniform(-1, 1, (k, k, k, D, 3)).astype(np.float32)
    beta = rng.dirichlet(np.ones(D), (l, l)).astype(np.float32)
    return sigma, u, beta


# ----------------------------------------------------------------- Eq. 1 brute force

@pytest.mark.parametrize("seed,in_box,eps,dir_linear", [
    (0, False, 0.0, False), (1, True, 0.0, False), (2, False, 0.3, False), (3, True, 0.05, False),
    (4, False, 0.0, True), (5, True, 0.05, True), (6, False, 0.0, True)])
def test_brute_force_eq1(seed, in_box, eps, dir_linear):
    """Literal Eq. 1 in 50 digits (O(N^2) transmittance sums, voxel and direction
    cells found by search, bilinear direction weights from the distances to the
    surrounding cell centres) agrees with the oracle to 1e-12 on a tiny scene."""
    k, D, l, N = 4, 3, 4, 16
    sigma, u, beta = _tiny_random(seed, k, D, l)
    sc = oracle.Scene(beta, sigma, u, pos_linear=False, dir_linear=dir_linear, in_box=in_box,
                      bg=(0.2, 0.5, 0.9))
    # seed 6 looks down at the scene (theta near pi, inside the last theta row's clamp)
    el = -1.3 if seed == 6 else 0.35
    v = synth.orbit_view(2.2, 0.3 + seed, el, 3, 3, 1.0, 3.4, f=2.0)
    res = oracle.render(sc, v.K, v.c2w, 3, 3, v.near, v.far, N, eps, tol=None)
    for q in range(9):
        x, y = q % 3, q // 3
        ref = brute_eq1.render_pixel(sigma, u, beta, k, D, l, v.K, v.c2w, x, y, v.near, v.far,
                                     N, eps, (0.2, 0.5, 0.9), in_box=in_box,
                                     dir_linear=dir_linear)
        np.testing.assert_allclose(res["rgba"][q], [float(r) for r in ref], rtol=0, atol=1e-12)


# ----------------------------------------------------------------- closed forms

@pytest.mark.parametrize("eye,target,chord", [
    ((-4.0, 0.3, -0.2), (0.0, 0.3, -0.2), 2.0),
    ((-3.0, -3.0, -3.0), (0.0, 0.0, 0.0), 2.0 * math.sqrt(3.0)),
    ((-3.0, -3.0, 0.1), (0.0, 0.0, 0.1), 2.0 * math.sqrt(2.0))])
@pytest.mark.parametrize("eps", [0.0, 1e-2])
def test_homogeneous_medium(eye, target, chord, eps):
    """Box filled with constant sigma, u and beta, samples inside the box:
    C = c (1 - exp(-sigma L)) + exp(-sigma L) bg with L the chord length; with
    termination L becomes n delta, n = min(N, floor(ln(1/eps)/(sigma delta)) + 1)."""
    D, N, sig = 2, 64, 3.5
    uval = np.array([[0.3, -0.2, 0.9], [0.5, 0.1, -0.4]], np.float32).astype(np.float64)
    bval = np.array([0.25, 0.75])
    c = bval @ uval
    bg = np.array([0.1, 0.6, 0.35])
    sc = _const_scene(6, D, 4, sig, uval, bval, in_box=True, bg=tuple(bg))
    K, c2w = _one_ray_view(eye, target)
    res = oracle.render(sc, K, c2w, 1, 1, 0.0, 100.0, N, eps, tol=None)
    L = chord
    if eps > 0:
        dl = chord / N
        n = min(N, math.floor(math.log(1 / eps) / (sig * dl)) + 1)
        L = n * dl
    T = math.exp(-sig * L)
    expect = np.concatenate([c * (1 - T) + T * bg, [1 - T]])
    np.testing.assert_allclose(res["rgba"][0], expect, rtol=0, atol=1e-12)


def test_empty_cache_gives_background():
    D = 8
    sc = _const_scene(16, D, 8, 0.0, np.random.default_rng(0).uniform(-1, 1, (D, 3)),
                      np.full(D, 1.0 / D), bg=(0.3, 0.7, 0.9))
    v = synth.orbit_view(3.0, 0.7, 0.4, 9, 7, 2.0, 4.0)
    res = oracle.render(sc, v.K, v.c2w, 7, 9, 2.0, 4.0, 32, 1e-4)
    assert np.all(res["rgba"] == np.array([0.3, 0.7, 0.9, 0.0]))


def test_single_voxel_axis_ray():
    """One occupied voxel, a ray along +x through the middle of its row:
    C = c (1 - exp(-sigma n delta)) + exp(-sigma n delta) bg with n the count of
    sample midpoints inside the voxel's x extent (counted in exact rationals)."""
    k, D = 8, 1
    sigma = np.zeros((k, k, k), np.float32)
    u = np.zeros((k, k, k, D, 3), np.float32)
    vx, vy, vz = 5, 2, 6
    sigma[vz, vy, vx] = 7.0
    u[vz, vy, vx, 0] = [0.9, -0.3, 0.4]
    beta = np.ones((4, 4, D), np.float32)
    sc = oracle.Scene(beta, sigma, u, dir_linear=False, bg=BG)
    h = Fraction(2, k)
    y0 = -1 + (vy + Fraction(3, 10)) * h
    z0 = -1 + (vz + Fraction(7, 10)) * h
    eye = (-3.0, float(y0), float(z0))
    K, c2w = _one_ray_view(eye, (0.0, float(y0), float(z0)))
    near, far, N = Fraction(1), Fraction(5), 100
    res = oracle.render(sc, K, c2w, 1, 1, float(near), float(far), N, 0.0, tol=None)
    delta = (far - near) / N
    a, b = -1 + vx * h, -1 + (vx + 1) * h
    n = sum(1 for i in range(N) if a <= -3 + near + (i + Fraction(1, 2)) * delta < b)
    assert n == 6
    T = math.exp(-7.0 * n * float(delta))
    col = np.array([0.9, -0.3, 0.4], dtype=np.float32).astype(np.float64)
    expect = np.concatenate([col * (1 - T) + T * np.array(BG), [1 - T]])
    np.testing.assert_allclose(res["rgba"][0], expect, rtol=0, atol=1e-12)


def test_nearest_lookup_matches_cell_search():
    k, D = 8, 2
    sigma, u, beta = _tiny_random(5, k, D, 4, density=1.0)
    sc = oracle.Scene(beta, sigma, u, pos_linear=False)
    rng = np.random.default_rng(1)
    pts = rng.uniform(-1.2, 1.2, (500, 3))
    pts[:20] = rng.integers(0, k + 1, (20, 3)) * (2.0 / k) - 1.0  # exactly on faces
    # just below faces (the lower cell) by 1e-6 and 1e-4 voxel
    pts[20:40] = rng.integers(1, k, (20, 3)) * (2.0 / k) - 1.0 - 1e-6 * (2.0 / k)
    pts[40:60] = rng.integers(1, k, (20, 3)) * (2.0 / k) - 1.0 - 1e-4 * (2.0 / k)
    sig, uu = oracle.lookup_pos(sc, pts)
    for p, s, uv in zip(pts, sig, uu):
        cells = [brute_eq1._cell_of(Fraction(float(x)), Fraction(-1), Fraction(1), k)
                 for x in p]
        if any(c is None for c in cells):
            assert s == 0 and np.all(uv == 0)
        else:
            assert s == sigma[cells[2], cells[1], cells[0]]
            assert np.array_equal(uv, u[cells[2], cells[1], cells[0]])


def test_trilinear_reproduces_linear_field():
    """Values at voxel centres sampled from an affine field are reproduced
    exactly by the trilinear lookup at interior points."""
    k, D = 8, 2
    h = 2.0 / k
    c = -1 + (np.arange(k) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    sigma = (2.0 + 0.5 * X - 0.25 * Y + 0.75 * Z).astype(np.float32)
    A = np.random.default_rng(3).uniform(-0.5, 0.5, (D, 3, 4))
    u = (A[..., 0] * X[..., None, None] + A[..., 1] * Y[..., None, None] +
         A[..., 2] * Z[..., None, None] + A[..., 3]).astype(np.float32)
    beta = np.ones((4, 4, D), np.float32)
    sc = oracle.Scene(beta, sigma, u, pos_linear=True)
    pts = np.random.default_rng(4).uniform(-1 + h / 2, 1 - h / 2, (300, 3))
    s, uu = oracle.lookup_pos(sc, pts)
    xs, ys, zs = pts[:, 0], pts[:, 1], pts[:, 2]
    np.testing.assert_allclose(s, 2.0 + 0.5 * xs - 0.25 * ys + 0.75 * zs, atol=2e-6)
    ref = (A[None, ..., 0] * xs[:, None, None] + A[None, ..., 1] * ys[:, None, None]
           + A[None, ..., 2] * zs[:, None, None] + A[None, ..., 3])
    np.testing.assert_allclose(uu, ref, atol=2e-6)  # inputs are float32 samples


def test_bilinear_direction_lookup():
    """A field affine in phi at the cell centres is reproduced away from the
    seam; across the seam the lookup is continuous; a constant field is exact."""
    l, D = 16, 3
    ph_c = (np.arange(l) + 0.5) * 2 * math.pi / l
    coef = np.array([0.2, -0.1, 0.05])
    beta = np.broadcast_to((0.5 + coef[None, :] * ph_c[:, None])[None], (l, l, D)).astype(
        np.float32).copy()
    sc = oracle.Scene(beta, np.zeros((2, 2, 2), np.float32), np.zeros((2, 2, 2, D, 3),
                                                                         np.float32))
    rng = np.random.default_rng(7)
    th = rng.uniform(0.3, 2.8, 200)
    ph = rng.uniform(ph_c[0], ph_c[-1], 200)
    dirs = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
    b = oracle.lookup_dir(sc, dirs)
    np.testing.assert_allclose(b, 0.5 + coef[None, :] * ph[:, None], atol=1e-6)
    e = 1e-7
    a1 = oracle.lookup_dir(sc, [[math.cos(-e), math.sin(-e), 0.0]])
    a2 = oracle.lookup_dir(sc, [[math.cos(e), math.sin(e), 0.0]])
    np.testing.assert_allclose(a1, a2, atol=1e-6)
    np.testing.assert_allclose(a1[0], 0.5 + coef * math.pi, atol=1e-6)  # seam = mean of ends
    const = np.broadcast_to(np.array([0.1, 0.3, 0.6], np.float32), (l, l, D)).copy()
    sc2 = oracle.Scene(const, np.zeros((2, 2, 2), np.float32),
                       np.zeros((2, 2, 2, D, 3), np.float32))
    np.testing.assert_allclose(oracle.lookup_dir(sc2, dirs), np.tile(const[0, 0], (200, 1)),
                               atol=1e-7)


def test_bilinear_direction_lookup_theta_axis():
    """The theta half of the bilinear lookup (readings R4, R5): a field
    bilinear in (theta, phi) at the cell centres, f = a + b theta + c phi +
    e theta phi, is reproduced exactly between the first and last centres
    (both axes and the cross term); above the last theta centre and below the
    first the lookup clamps to the edge row, so it is constant in theta there."""
    l, D = 12, 2
    th_c = (np.arange(l) + 0.5) * math.pi / l
    ph_c = (np.arange(l) + 0.5) * 2 * math.pi / l
    coef = np.array([[0.3, 0.1, -0.05, 0.02], [0.6, -0.08, 0.03, -0.01]])

    def field(th, ph):
        th, ph = np.asarray(th)[..., None], np.asarray(ph)[..., None]
        return coef[:, 0] + coef[:, 1] * th + coef[:, 2] * ph + coef[:, 3] * th * ph

    TH, PH = np.meshgrid(th_c, ph_c, indexing="ij")
    beta = field(TH, PH).astype(np.float32)
    sc = oracle.Scene(beta, np.zeros((2, 2, 2), np.float32),
                      np.zeros((2, 2, 2, D, 3), np.float32))

    def dirs_of(th, ph):
        return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)

    rng = np.random.default_rng(17)
    ph = rng.uniform(ph_c[0], ph_c[-1], 400)
    th = rng.uniform(th_c[0], th_c[-1], 400)
    # float32 storage of beta: about 6e-8 relative
    np.testing.assert_allclose(oracle.lookup_dir(sc, dirs_of(th, ph)), field(th, ph), atol=1e-6)
    th_lo = rng.uniform(1e-3, th_c[0], 100)
    np.testing.assert_allclose(oracle.lookup_dir(sc, dirs_of(th_lo, ph[:100])),
                               field(np.full(100, th_c[0]), ph[:100]), atol=1e-6)
    th_hi = rng.uniform(th_c[-1], math.pi - 1e-3, 100)
    np.testing.assert_allclose(oracle.lookup_dir(sc, dirs_of(th_hi, ph[:100])),
                               field(np.full(100, th_c[-1]), ph[:100]), atol=1e-6)
    # at a theta centre the lookup is that row's phi interpolation, exactly
    j = 5
    b = oracle.lookup_dir(sc, dirs_of(np.full(50, th_c[j]), ph[:50]))
    np.testing.assert_allclose(b, field(np.full(50, th_c[j]), ph[:50]), atol=1e-6)


# ----------------------------------------------------------------- counts behind the byte count

def _counts_scene(k, ob, occupied, sig):
    """k^3 grid, one brick of edge ob set: voxels listed in ``occupied`` get
    density sig (all voxels of the brick when occupied is a brick index)."""
    sigma = np.zeros((k, k, k), np.float32)
    u = np.zeros((k, k, k, 1, 3), np.float32)
    for (x, y, z) in occupied:
        sigma[z, y, x] = sig
        u[z, y, x, 0] = [0.2, 0.4, 0.6]
    beta = np.ones((4, 4, 1), np.float32)
    return oracle.Scene(beta, sigma, u, dir_linear=False, bg=BG, occ_brick=ob)


def test_occupied_sample_count_closed_form():
    """Samples in occupied bricks before the stop (the count behind the
    algorithmic bytes of the render): k = 16, bricks of 4 voxels, an axis ray
    along +x through one occupied brick. Without termination the count is the
    number of sample midpoints inside the brick's x extent (exact rationals),
    whatever the voxel densities inside it; with termination it stops after
    n = min(m, floor(ln(1/eps) / (sigma delta)) + 1) samples of a brick filled
    with sigma, and samples after the stop are not counted."""
    k, ob = 16, 4
    h = Fraction(2, k)
    y0 = -1 + (5 + Fraction(3, 10)) * h   # voxel row y = 5 (brick 1)
    z0 = -1 + (13 + Fraction(6, 10)) * h  # z = 13 (brick 3)
    K, c2w = _one_ray_view((-3.0, float(y0), float(z0)), (0.0, float(y0), float(z0)),
                           up=(0.0, 0.0, 1.0))
    near, far, N = Fraction(1), Fraction(5), 100
    delta = (far - near) / N
    xs = [-3 + near + (i + Fraction(1, 2)) * delta for i in range(N)]
    a, b = -1 + 8 * h, -1 + 12 * h        # brick bx = 2: voxels 8..11
    m = sum(1 for x in xs if a <= x < b)
    in_box = sum(1 for x in xs if -1 <= x <= 1)
    one = sum(1 for x in xs if -1 + 9 * h <= x < -1 + 10 * h)
    assert (m, in_box, one) == (12, 50, 3)
    # one voxel of the brick has density: every sample in the brick counts
    sc = _counts_scene(k, ob, [(9, 5, 13)], 7.0)
    c = oracle.render(sc, K, c2w, 1, 1, float(near), float(far), N, 0.0, tol=None)["counts"]
    assert (c["rays"], c["hit"], c["samples"], c["occ_samples"], c["nonzero_samples"]) == \
        (1, 1, in_box, m, one)
    # the whole brick filled with sigma = 40: sigma delta = 1.6, eps = 1e-2
    sig, eps = 40.0, 1e-2
    brick = [(x, y, z) for x in range(8, 12) for y in range(4, 8) for z in range(12, 16)]
    sc = _counts_scene(k, ob, brick, sig)
    c = oracle.render(sc, K, c2w, 1, 1, float(near), float(far), N, eps, tol=None)["counts"]
    n = min(m, math.floor(math.log(1 / eps) / (sig * float(delta))) + 1)
    assert n == 3
    first = sum(1 for x in xs if -1 <= x < a)  # in-box samples before the brick
    assert (c["occ_samples"], c["nonzero_samples"], c["samples"]) == (n, n, first + n)
    # a stop point inside the band of reading R8 (optical depth 4.8 against
    # ln(1/eps) = 4.7995): the oracle also evaluates the sample after it, as
    # an admissible variant, but the counts stop with the primary result
    eps_b = math.exp(-4.7995)
    res = oracle.render(sc, K, c2w, 1, 1, float(near), float(far), N, eps_b,
                        tol=oracle.DEFAULT_TOL)
    assert res["ncand"][0] >= 2  # (the direction lookup of this axis ray is on cell borders too)
    assert res["counts"]["occ_samples"] == min(m, math.floor(4.7995 / (sig * float(delta))) + 1)
    # no occupancy grid given: nothing is counted as occupied
    sc = oracle.Scene(np.ones((4, 4, 1), np.float32), sc.sigma, sc.u, dir_linear=False)
    c = oracle.render(sc, K, c2w, 1, 1, float(near), float(far), N, eps, tol=None)["counts"]
    assert c["occ_samples"] == 0


def test_hit_ray_count_closed_form():
    """Rays whose interval is non-empty: a camera on the -x axis looking at
    the box face-on sees the box as its front face (distance 2, half-width 1),
    so a pixel's ray hits exactly when |x + 1/2 - cx| < f/2 and
    |y + 1/2 - cy| < f/2 (no pixel lies on the silhouette with f = 12.5). In
    NEAR_FAR mode every ray has the interval [near, far]."""
    W = H = 21
    f, cx = 12.5, 10.5
    K = np.array([[f, 0, cx], [0, f, cx], [0, 0, 1.0]])
    c2w = synth.look_at((-3.0, 0.0, 0.0), (0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0))
    n_axis = sum(1 for x in range(W) if abs(x + 0.5 - cx) < f / 2)
    assert n_axis == 13
    sc = _const_scene(8, 1, 4, 2.0, [[0.1, 0.2, 0.3]], [1.0], in_box=True)
    c = oracle.render(sc, K, c2w, H, W, 0.5, 10.0, 8, 0.0, tol=None)["counts"]
    assert (c["rays"], c["hit"]) == (W * H, n_axis ** 2)
    sc = _const_scene(8, 1, 4, 2.0, [[0.1, 0.2, 0.3]], [1.0], in_box=False)
    c = oracle.render(sc, K, c2w, H, W, 0.5, 10.0, 8, 0.0, tol=None)["counts"]
    assert (c["rays"], c["hit"]) == (W * H, W * H)


def test_threaded_bands_equal_single_thread():
    """The oracle split into row bands over several threads (the all-core CPU
    baseline) gives bitwise the single-threaded results and the same counts."""
    sig, u, beta, _ = synth.scene_arrays(synth.SceneSpec(k=32, D=4, l=8, n_ellipsoids=5,
                                                         seed=12))
    sc = oracle.Scene(beta, sig, u, in_box=True, occ_brick=8)
    v = synth.orbit_view(3.0, 0.9, 0.3, 23, 19, 2.0, 4.0)
    one = oracle.render(sc, v.K, v.c2w, 19, 23, 2.0, 4.0, 48, 1e-4)
    pix = np.sort(np.random.default_rng(2).choice(19 * 23, 200, replace=False))
    one_p = oracle.render(sc, v.K, v.c2w, 19, 23, 2.0, 4.0, 48, 1e-4, pix=pix)
    for threads in (2, 5, 8):
        many = oracle.render(sc, v.K, v.c2w, 19, 23, 2.0, 4.0, 48, 1e-4, threads=threads)
        for key in ("rgba", "cand", "ncand", "flags"):
            assert np.array_equal(one[key], many[key]), key
        assert one["counts"] == many["counts"]
        many_p = oracle.render(sc, v.K, v.c2w, 19, 23, 2.0, 4.0, 48, 1e-4, pix=pix,
                               threads=threads)
        assert np.array_equal(one_p["rgba"], many_p["rgba"])
        assert one_p["counts"] == many_p["counts"]
    assert one["counts"]["occ_samples"] > 0


# ----------------------------------------------------------------- rays and intervals

def test_pixel_rays_follow_opencv_axes():
    W, H, f = 9, 7, 10.8
    v = synth.orbit_view(3.0, 0.0, 0.0, W, H, 2.0, 4.0, f=f)
    o, d = oracle.pixel_ray(v.K, v.c2w, H, W, (W - 1) / 2, (H - 1) / 2)
    np.testing.assert_allclose(o, [3.0, 0.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(d, [-1.0, 0.0, 0.0], atol=1e-15)  # through the look-at point
    _, dc = oracle.pixel_ray(v.K, v.c2w, H, W, 0, 0)
    ang = math.atan(math.hypot(W / 2 - 0.5, H / 2 - 0.5) / f)
    assert abs(math.acos(-dc[0]) - ang) < 1e-12
    # seen from +x looking at the origin with +z up, image right is world +y
    assert dc[1] < 0 and dc[2] > 0  # top-left pixel: left and up
    _, dr = oracle.pixel_ray(v.K, v.c2w, H, W, W - 1, (H - 1) / 2)
    assert dr[1] > 0 and abs(dr[2]) < 1e-15


def test_box_clip_chords():
    sc = _const_scene(2, 1, 2, 1.0, [[0, 0, 0]], [1.0], in_box=True)
    hit, t0, t1 = oracle.interval(sc, (-3, 0.2, 0.1), (1, 0, 0), 0.0, 10.0)
    assert hit and abs(t0 - 2) < 1e-15 and abs(t1 - 4) < 1e-15
    dd = np.ones(3) / math.sqrt(3)
    hit, t0, t1 = oracle.interval(sc, -2 * dd * math.sqrt(3), dd, 0.0, 10.0)
    assert hit and abs((t1 - t0) - 2 * math.sqrt(3)) < 1e-12
    hit, *_ = oracle.interval(sc, (-3, 1.5, 0.0), (1, 0, 0), 0.0, 10.0)  # parallel, outside
    assert not hit
    hit, t0, t1 = oracle.interval(sc, (-3, 0.0, 0.0), (1, 0, 0), 2.5, 3.0)  # near/far inside
    assert hit and (t0, t1) == (2.5, 3.0)


# ----------------------------------------------------------------- compositing

def test_textbook_compositor_d1():
    """D = 1 and beta = 1 reduce Eq. 5 to c = u; the result equals the classic
    product-form compositor w_i = alpha_i prod_{j<i} (1 - alpha_j) over the
    oracle's own samples."""
    sig, u, beta = synth.scene_arrays(synth.SceneSpec(k=32, D=1, l=4, n_ellipsoids=10,
                                                      seed=3))[:3]
    beta[:] = 1.0
    sc = oracle.Scene(beta, sig, u, bg=(0.25, 0.5, 0.75))
    v = synth.orbit_view(3.0, 0.4, 0.3, 16, 16, 2.0, 4.0)
    res = oracle.render(sc, v.K, v.c2w, 16, 16, 2.0, 4.0, 48, 0.0, tol=None)
    checked = 0
    for pidx in range(256):
        x, y = pidx % 16, pidx // 16
        t, s, rgb, dl = oracle.trace(sc, v.K, v.c2w, 16, 16, 2.0, 4.0, 48, x, y)
        a = 1.0 - np.exp(-s * dl)
        w = a * np.concatenate([[1.0], np.cumprod(1.0 - a)[:-1]])
        C = (w[:, None] * rgb).sum(0) + (1 - w.sum()) * np.array([0.25, 0.5, 0.75])
        np.testing.assert_allclose(res["rgba"][pidx], np.concatenate([C, [w.sum()]]),
                                   atol=1e-12)
        checked += s.max() > 0
    assert checked >= 30


def test_one_hot_beta_selects_component():
    sig, u, beta = synth.scene_arrays(synth.SceneSpec(k=24, D=4, l=8, n_ellipsoids=3,
                                                      seed=4))[:3]
    v = synth.orbit_view(3.0, 1.0, 0.2, 12, 12, 2.0, 4.0)
    for j in range(4):
        onehot = np.zeros_like(beta)
        onehot[..., j] = 1.0
        a = oracle.render(oracle.Scene(onehot, sig, u), v.K, v.c2w, 12, 12, 2, 4, 40, 1e-3,
                          tol=None)
        b = oracle.render(oracle.Scene(np.ones((8, 8, 1), np.float32), sig,
                                       u[..., j:j + 1, :].copy()), v.K, v.c2w, 12, 12, 2, 4,
                          40, 1e-3, tol=None)
        np.testing.assert_array_equal(a["rgba"], b["rgba"])


def test_linearity_in_radiance():
    sig, u, beta = synth.scene_arrays(synth.SceneSpec(k=24, D=3, l=8, n_ellipsoids=4,
                                                      seed=5))[:3]
    # radiance on a 2^-10 grid so that the mixture below is exact in float32
    u = (np.round(u * 1024) / 1024).astype(np.float32)
    u2 = (np.round(np.random.default_rng(9).uniform(-1, 1, u.shape) * 1024) / 1024).astype(
        np.float32)
    v = synth.orbit_view(3.0, 2.0, -0.3, 10, 10, 2.0, 4.0)

    def r(uu):
        return oracle.render(oracle.Scene(beta, sig, uu, bg=(0, 0, 0)), v.K, v.c2w, 10, 10,
                             2, 4, 40, 1e-3, tol=None)["rgba"]

    a, b = 0.5, -0.25
    mix = (np.float64(a) * u + np.float64(b) * u2)
    assert np.array_equal(mix.astype(np.float32).astype(np.float64), mix)  # exact inputs
    lhs = r(mix.astype(np.float32))
    rhs = a * r(u) + b * r(u2)
    np.testing.assert_allclose(lhs[:, :3], rhs[:, :3], atol=1e-12)
    np.testing.assert_allclose(lhs[:, 3], r(u)[:, 3], atol=0)


def test_weights_and_convexity():
    sig, u, beta, _ = synth.scene_arrays(synth.SceneSpec(k=32, D=4, l=8, n_ellipsoids=5,
                                                         seed=6))
    bg = np.array([0.9, -0.2, 0.4])
    sc = oracle.Scene(beta, sig, u, bg=tuple(bg))
    v = synth.orbit_view(3.0, 0.1, 0.5, 14, 14, 2.0, 4.0)
    res = oracle.render(sc, v.K, v.c2w, 14, 14, 2, 4, 40, 1e-4, tol=None)
    A = res["rgba"][:, 3]
    assert np.all((A >= 0) & (A <= 1))
    for pidx in range(0, 196, 3):
        _, s, rgb, _ = oracle.trace(sc, v.K, v.c2w, 14, 14, 2, 4, 40, pidx % 14, pidx // 14)
        used = np.concatenate([rgb[s > 0], bg[None]])
        lo, hi = used.min(0), used.max(0)
        c = res["rgba"][pidx, :3]
        assert np.all(c >= lo - 1e-12) and np.all(c <= hi + 1e-12)


def test_termination_error_bound():
    sig, u, beta, _ = synth.scene_arrays(synth.SceneSpec(k=32, D=4, l=8, n_ellipsoids=6,
                                                         seed=7))
    sc = oracle.Scene(beta, sig, u, bg=BG)
    v = synth.orbit_view(3.0, 0.7, 0.4, 20, 20, 2.0, 4.0)
    full = oracle.render(sc, v.K, v.c2w, 20, 20, 2, 4, 64, 0.0, tol=None)["rgba"]
    for eps in (1e-1, 1e-2, 1e-4):
        cut = oracle.render(sc, v.K, v.c2w, 20, 20, 2, 4, 64, eps, tol=None)["rgba"]
        # |c| <= 1 (u in [-1,1], beta convex) and bg = 1, so |c - bg| <= 2
        assert np.abs(cut - full)[:, :3].max() <= 2 * eps + 1e-12
        assert np.abs(cut - full)[:, 3].max() <= eps + 1e-12


def test_segment_split_over_operator():
    """Compositing [near, mid) and [mid, far) separately and joining them with
    the over operator equals compositing [near, far)."""
    sig, u, beta, _ = synth.scene_arrays(synth.SceneSpec(k=32, D=4, l=8, n_ellipsoids=5,
                                                         seed=8))
    sc = oracle.Scene(beta, sig, u, bg=(0.0, 0.0, 0.0))
    v = synth.orbit_view(3.0, 1.3, 0.2, 12, 12, 2.0, 4.0)
    N, m = 64, 24
    mid = 2.0 + m * (2.0 / N)
    full = oracle.render(sc, v.K, v.c2w, 12, 12, 2.0, 4.0, N, 0.0, tol=None)["rgba"]
    a = oracle.render(sc, v.K, v.c2w, 12, 12, 2.0, mid, m, 0.0, tol=None)["rgba"]
    b = oracle.render(sc, v.K, v.c2w, 12, 12, mid, 4.0, N - m, 0.0, tol=None)["rgba"]
    np.testing.assert_allclose(full[:, :3], a[:, :3] + (1 - a[:, 3:]) * b[:, :3], atol=1e-12)
    np.testing.assert_allclose(1 - full[:, 3], (1 - a[:, 3]) * (1 - b[:, 3]), atol=1e-12)


def test_brick_sparse_source_equals_dense():
    spec = synth.SceneSpec(k=32, D=4, l=8, n_ellipsoids=5, seed=9)
    sig, u, beta, p = synth.scene_arrays(spec)
    slot, ss, su = synth.brick_sparse(p, 8)
    v = synth.orbit_view(3.0, 0.5, 0.3, 16, 16, 2.0, 4.0)
    dense = oracle.render(oracle.Scene(beta, sig, u, occ_brick=8), v.K, v.c2w, 16, 16, 2, 4,
                          48, 1e-4)
    sparse = oracle.render(oracle.Scene(beta, k=32, sparse=(8, slot, ss, su), occ_brick=8),
                           v.K, v.c2w, 16, 16, 2, 4, 48, 1e-4)
    assert np.array_equal(dense["rgba"], sparse["rgba"])
    assert dense["counts"] == sparse["counts"]
    assert dense["counts"]["occ_samples"] >= dense["counts"]["nonzero_samples"] > 0


def test_cell_boundary_ambiguity_and_face_ties():
    """A sample exactly on a voxel face takes the upper cell (reading R6,
    R6b) with no alternative; a sample 2e-4 voxel below a face lies in the lower
    cell but within the band of reading R13, so both voxels are admissible and
    the oracle enumerates the variants."""
    k, D = 4, 1
    sigma = np.zeros((k, k, k), np.float32)
    u = np.zeros((k, k, k, D, 3), np.float32)
    sigma[1, 1, 1] = 5.0
    sigma[1, 1, 2] = 9.0
    u[1, 1, 1, 0] = [1, 0, 0]
    u[1, 1, 2, 0] = [0, 1, 0]
    beta = np.ones((3, 3, 1), np.float32)  # l = 3: the ray is not on a direction-cell border
    sc = oracle.Scene(beta, sigma, u, dir_linear=False, bg=(0, 0, 0))
    # rays along +y through the voxel row y = 1, z = 1 (two samples in it)
    K, c2w = _one_ray_view((0.0, -3.0, -0.25), (0.0, 0.0, -0.25), up=(0.0, 0.0, 1.0))
    res = oracle.render(sc, K, c2w, 1, 1, 2.0, 4.0, 8, 0.0)
    assert res["ncand"][0] == 1  # x exactly on the face between voxels 1 and 2
    assert res["rgba"][0, 0] == 0 and res["rgba"][0, 1] > 0  # upper cell: voxel 2
    xb = -(2.0 / k) * 2e-4  # just below that face
    K, c2w = _one_ray_view((xb, -3.0, -0.25), (xb, 0.0, -0.25), up=(0.0, 0.0, 1.0))
    res = oracle.render(sc, K, c2w, 1, 1, 2.0, 4.0, 8, 0.0)
    assert res["ncand"][0] == 4 and res["flags"][0] & oracle.AMBIG
    first, last = res["cand"][0, 0], res["cand"][0, 3]
    assert first[0] > 0 and first[1] == 0   # primary: both samples in the lower cell
    assert last[0] == 0 and last[1] > 0     # both in the upper cell
    np.testing.assert_array_equal(res["rgba"][0], first)
    xf = -(2.0 / k) * 2e-3  # outside the band: one result
    K, c2w = _one_ray_view((xf, -3.0, -0.25), (xf, 0.0, -0.25), up=(0.0, 0.0, 1.0))
    assert oracle.render(sc, K, c2w, 1, 1, 2.0, 4.0, 8, 0.0)["ncand"][0] == 1


def test_commensurate_lattice_has_no_face_ties():
    """With k/N = 4 voxels per sample (paper-scale ratio, here k=64, N=16 inside
    the box) rays crossing the box between opposite faces put every sample on
    a voxel face; such samples take the upper cell (readings R6, R6b) and are
    not ambiguous, so no pixel overflows the enumeration."""
    spec = synth.paper_scene_spec(k=64)
    p = synth.draw(spec)
    slot, ss, su = synth.brick_sparse(p, 8)
    beta = synth.beta_table(p)
    sc = oracle.Scene(beta, k=64, sparse=(8, slot, ss, su), in_box=True)
    v = synth.paper_orbit(4, W=64, H=64)[0]
    a = oracle.render(sc, v.K, v.c2w, 64, 64, v.near, v.far, 16, 1e-4)
    assert a["counts"]["unchecked_pixels"] == 0
    assert a["counts"]["ambiguous_pixels"] < 0.02 * 64 * 64
    # the lattice is real: a ray through the x faces has every sample on a face
    o, d = oracle.pixel_ray(v.K, v.c2w, 64, 64, 32, 32)
    hit, t0, t1 = oracle.interval(sc, o, d, 0.0, 100.0)
    g = (o[0] + (t0 + (np.arange(16) + 0.5) * (t1 - t0) / 16) * d[0] + 1.0) * 32
    assert hit and np.abs(g - np.round(g)).max() < 1e-9


# ---------------------------------------------------------------- voxel traversal (N = 0)

@pytest.mark.parametrize("k", [5, 6, 16])
@pytest.mark.parametrize("eye, target, chord", [
    ((3.0, 0.0, 0.0), (0.0, 0.0, 0.0), 2.0),
    ((3.0, 3.0, 0.0), (0.0, 0.0, 0.0), 2.0 * math.sqrt(2.0)),
    ((3.0, 3.0, 3.0), (0.0, 0.0, 0.0), 2.0 * math.sqrt(3.0)),
])
def test_voxel_traversal_homogeneous_exact(k, eye, target, chord):
    """Every voxel visited with its own length: in a homogeneous box the pieces
    sum to the chord exactly, so C = c (1 - exp(-sigma L)) + exp(-sigma L) bg
    holds at any resolution (no quadrature error), in NEAR_FAR mode too (the
    traversal stays inside the box)."""
    D, sig = 2, 3.5
    uval = np.array([[0.3, -0.2, 0.9], [0.5, 0.1, -0.4]], np.float32).astype(np.float64)
    bval = np.array([0.25, 0.75])
    c = bval @ uval
    bg = np.array([0.1, 0.6, 0.35])
    K, c2w = _one_ray_view(eye, target)
    T = math.exp(-sig * chord)
    expect = np.concatenate([c * (1 - T) + T * bg, [1 - T]])
    for in_box in (True, False):
        sc = _const_scene(k, D, 4, sig, uval, bval, in_box=in_box, bg=tuple(bg))
        res = oracle.render(sc, K, c2w, 1, 1, 0.0, 100.0, 0, 0.0, tol=None)
        np.testing.assert_allclose(res["rgba"][0], expect, rtol=0, atol=1e-12)


def test_voxel_traversal_termination_on_an_axis_ray():
    """Axis ray (along -x) through a homogeneous box of k voxels: the pieces
    are the k cells between the voxel faces, each one voxel long; the stop
    rule (stop before a piece once the optical depth exceeds ln(1/eps)) keeps
    the first n pieces, L their total length, and
    C = c (1 - exp(-sigma L)) + exp(-sigma L) bg."""
    k, D, sig, eps = 20, 1, 9.0, 1e-2
    h = 2.0 / k
    sc = _const_scene(k, D, 4, sig, [[0.2, 0.5, -0.7]], [1.0], bg=BG)
    K, c2w = _one_ray_view((3.0, 0.013, -0.021), (0.0, 0.013, -0.021))
    res = oracle.render(sc, K, c2w, 1, 1, 0.0, 100.0, 0, eps, tol=None)
    pieces = [h] * k
    L, lim = 0.0, math.log(1 / eps)
    for p in pieces:
        if sig * L > lim:
            break
        L += p
    assert L < 2.0 - 1e-9
    T = math.exp(-sig * L)
    col = np.array([0.2, 0.5, -0.7], np.float32).astype(np.float64)
    expect = np.concatenate([col * (1 - T) + T * np.array(BG), [1 - T]])
    np.testing.assert_allclose(res["rgba"][0], expect, rtol=0, atol=1e-12)


def _slab_length(o, d, lo, hi):
    """Length of the ray o + t d (t >= 0) inside the axis-aligned box [lo, hi]."""
    t0, t1 = 0.0, np.inf
    for a in range(3):
        if d[a] == 0.0:
            if not lo[a] <= o[a] <= hi[a]:
                return 0.0
            continue
        ta, tb = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return max(0.0, t1 - t0)


def test_voxel_traversal_single_voxel_slab_length():
    """One occupied interior voxel, rays in many directions: the piece inside
    the voxel has the length of the ray clipped to the voxel's cell, so
    C = c (1 - exp(-sigma l)) + exp(-sigma l) bg with l from a slab test."""
    k, D = 6, 1
    vx, vy, vz = 2, 3, 3
    sigma = np.zeros((k, k, k), np.float32)
    u = np.zeros((k, k, k, D, 3), np.float32)
    sigma[vz, vy, vx] = 11.0
    u[vz, vy, vx, 0] = [0.9, -0.3, 0.4]
    beta = np.ones((4, 4, D), np.float32)
    sc = oracle.Scene(beta, sigma, u, dir_linear=False, bg=BG)
    h = 2.0 / k
    lo = np.array([-1 + vx * h, -1 + vy * h, -1 + vz * h])
    centre = lo + h / 2
    col = np.array([0.9, -0.3, 0.4], np.float32).astype(np.float64)
    rng = np.random.default_rng(4)
    hits = 0
    for _ in range(200):
        eye = rng.normal(size=3)
        eye = eye / np.linalg.norm(eye) * 3.0
        target = centre + rng.uniform(-0.8, 0.8, 3) * h
        K, c2w = _one_ray_view(eye, target, up=tuple(rng.normal(size=3)))
        o, d = oracle.pixel_ray(K, c2w, 1, 1, 0, 0)
        res = oracle.render(sc, K, c2w, 1, 1, 0.0, 100.0, 0, 0.0, tol=None)
        ell = _slab_length(o, d, lo, lo + h)
        hits += ell > 0
        T = math.exp(-11.0 * ell)
        expect = np.concatenate([col * (1 - T) + T * np.array(BG), [1 - T]])
        np.testing.assert_allclose(res["rgba"][0], expect, rtol=0, atol=1e-12)
    assert hits > 50


def test_voxel_traversal_is_the_limit_of_fixed_samples():
    """With nearest lookups the field is constant on each piece, so the
    midpoint rule with N samples converges to the traversal as N grows: the
    error shrinks about fourfold from N = 4096 to 16384 and stays small."""
    sig, u, beta = _tiny_random(7, k=6, D=2)
    sc = oracle.Scene(beta, sig, u, in_box=True, bg=BG)
    v = synth.orbit_view(3.2, 0.4, 0.35, 8, 8, 0.0, 100.0, f=6.0)
    ref = oracle.render(sc, v.K, v.c2w, 8, 8, 0.0, 100.0, 0, 0.0, tol=None)["rgba"]
    errs = [np.abs(oracle.render(sc, v.K, v.c2w, 8, 8, 0.0, 100.0, N, 0.0, tol=None)["rgba"]
                   - ref).max() for N in (4096, 16384)]
    assert errs[1] < 5e-3 and errs[1] < errs[0] / 2.5


def test_voxel_traversal_termination_bound_and_trilinear_rejected():
    """|C(eps) - C(0)| <= eps max|c - bg| for the traversal too; trilinear
    lookups have no piecewise-constant reading and are rejected."""
    sig, u, beta = _tiny_random(8, k=6, D=2)
    sc = oracle.Scene(beta, sig, u, in_box=True, bg=BG)
    v = synth.orbit_view(3.2, 1.4, -0.3, 8, 8, 0.0, 100.0, f=6.0)
    eps = 2e-2
    a = oracle.render(sc, v.K, v.c2w, 8, 8, 0.0, 100.0, 0, eps, tol=None)["rgba"]
    b = oracle.render(sc, v.K, v.c2w, 8, 8, 0.0, 100.0, 0, 0.0, tol=None)["rgba"]
    cmax = np.abs(u).sum(axis=-2).max() + 1.0
    assert np.abs(a - b).max() <= eps * cmax
    assert np.abs(a - b).max() > 0.0
    sl = oracle.Scene(beta, sig, u, in_box=True, bg=BG, pos_linear=True)
    with pytest.raises(ValueError):
        oracle.render(sl, v.K, v.c2w, 8, 8, 0.0, 100.0, 0, 0.0)


# ---------------------------------------------------------------- enclosure of unchecked pixels

def test_enclosure_contains_every_enumerated_variant():
    """A pixel with more ambiguous lookups than are enumerated is checked
    against interval bounds of all its admissible results. With a wide
    ambiguity band (0.02 voxel on a k = 8 grid), a stop band and nearest
    direction cells, the pixels that five enumerated choices cover exactly
    become unenumerated with one choice; every result of the full enumeration
    lies inside their bounds."""
    sigma, u, beta = _tiny_random(21, k=8, D=2, l=4, density=0.8)
    sc = oracle.Scene(beta, sigma, u, dir_linear=False, in_box=True, bg=(0.2, 0.6, 0.9))
    v = synth.orbit_view(2.6, 0.45, 0.3, 14, 12, 0.0, 10.0, f=9.0)
    full = oracle.render(sc, v.K, v.c2w, 12, 14, 0.0, 10.0, 24, 0.05, tol=(0.02, 0.05, 0.05, 5))
    part = oracle.render(sc, v.K, v.c2w, 12, 14, 0.0, 10.0, 24, 0.05, tol=(0.02, 0.05, 0.05, 1))
    enumerated = (full["flags"] & oracle.UNCHECKED) == 0
    bounded = ((part["flags"] & oracle.UNCHECKED) != 0) & enumerated
    assert bounded.sum() >= 40
    lo, hi = part["env"][:, 0], part["env"][:, 1]
    for q in np.nonzero(bounded)[0]:
        cands = full["cand"][q, :full["ncand"][q]]
        assert len(cands) > 2
        assert np.all(cands >= lo[q] - 1e-12) and np.all(cands <= hi[q] + 1e-12), q
    # the bounds are those of the variants, not the trivial colour range
    width = (hi - lo)[bounded].max(axis=1)
    assert np.median(width) < 0.2
    # enumerated pixels: the enclosure is the hull of their results
    for q in np.nonzero(~((part["flags"] & oracle.UNCHECKED) != 0))[0][:20]:
        c = part["cand"][q, :part["ncand"][q]]
        assert np.array_equal(part["env"][q, 0], c.min(0)) and \
            np.array_equal(part["env"][q, 1], c.max(0))


def test_enclosure_is_exact_without_variation():
    """Every candidate voxel and direction cell of a homogeneous box holds the
    same values, so the interval bounds of a pixel forced out of the
    enumeration collapse onto the closed form of the homogeneous medium; with
    termination, a stop point in the band widens them to both stops, one
    sample's worth of optical depth apart."""
    D, N, sig = 2, 64, 3.5
    uval = np.array([[0.3, -0.2, 0.9], [0.5, 0.1, -0.4]], np.float32).astype(np.float64)
    bval = np.array([0.25, 0.75])
    c = bval @ uval
    bg = np.array([0.1, 0.6, 0.35])
    sc = _const_scene(6, D, 4, sig, uval, bval, in_box=True, bg=tuple(bg), dir_linear=False)
    # a ray along +x with phi = 0: on the direction cache's seam, an ambiguous cell
    K, c2w = _one_ray_view((-4.0, 0.31, -0.17), (0.0, 0.31, -0.17), up=(0.0, 0.0, 1.0))
    r = oracle.render(sc, K, c2w, 1, 1, 0.0, 100.0, N, 0.0, tol=(1e-3, 1e-5, 1e-3, -1))
    assert r["flags"][0] & oracle.UNCHECKED
    T = math.exp(-sig * 2.0)
    expect = np.concatenate([c * (1 - T) + T * bg, [1 - T]])
    np.testing.assert_allclose(r["env"][0, 0], expect, atol=1e-12)
    np.testing.assert_allclose(r["env"][0, 1], expect, atol=1e-12)
    # termination with the stop point inside the band
    dl = 2.0 / N
    n = 12                                    # sigma dl n = 2.1875 crosses the limit
    lim = sig * dl * (n - 0.5) + 0.01          # between samples n - 1 and n
    eps = math.exp(-lim)
    r = oracle.render(sc, K, c2w, 1, 1, 0.0, 100.0, N, eps, tol=(1e-3, 1e-5, 0.2, -1))
    lo, hi = r["env"][0]
    for m in (n, n + 1):                      # stop after n or n + 1 samples
        Tm = math.exp(-sig * dl * m)
        e = np.concatenate([c * (1 - Tm) + Tm * bg, [1 - Tm]])
        assert np.all(e >= lo - 1e-12) and np.all(e <= hi + 1e-12), m
    assert (hi - lo).max() < 0.2
