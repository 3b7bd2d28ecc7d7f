"""Properties of the HIP render path that hold exactly or in closed form."""
import math

import numpy as np
import pytest

import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16", "fp8"])
@pytest.mark.parametrize("pos_linear", [False, True])
def test_empty_cache_is_background_bitwise(storage, pos_linear):
    k, D, l = 16, 4, 8
    sig = np.zeros((k, k, k), np.float32)
    u = np.random.default_rng(0).uniform(-1, 1, (k, k, k, D, 3)).astype(np.float32)
    beta = np.full((l, l, D), 1.0 / D, np.float32)
    bg = (0.3, 0.7, 0.9)
    for brick in (0, 4):
        cache = G.make_cache(sig, u, beta, storage=storage, pos_linear=pos_linear, brick=brick,
                             bg=bg)
        out = G.render_gpu(cache, synth.orbit_view(3.0, 0.7, 0.4, 37, 29, 2.0, 4.0), 64, 1e-4)
        expect = np.array(bg + (0.0,), np.float32).astype(np.float64)
        assert np.array_equal(out, np.broadcast_to(expect, out.shape))


@pytest.mark.parametrize("storage", ["f32", "fp8"])
@pytest.mark.parametrize("pos_linear", [False, True])
def test_occupancy_skipping_is_exact(storage, pos_linear):
    """Rendering with the brick bitgrid equals rendering without it, bitwise."""
    sig, u, beta = G.config1_scene()
    v = G.config1_view()
    outs = [G.render_gpu(G.make_cache(sig, u, beta, storage=storage, pos_linear=pos_linear,
                                      brick=b), v, 128, 1e-4) for b in (0, 4, 8, 16)]
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_deterministic():
    sig, u, beta = G.config1_scene()
    v = G.config1_view()
    cache = G.make_cache(sig, u, beta, storage="f16")
    a = G.render_gpu(cache, v, 128, 1e-4)
    b = G.render_gpu(cache, v, 128, 1e-4)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("eps", [0.0, 1e-2])
def test_homogeneous_medium_closed_form(eps):
    """Box filled with constant sigma, u, beta; samples in the box: every pixel
    is c (1 - exp(-sigma L)) + exp(-sigma L) bg with L its chord through the box
    (or n delta with termination)."""
    import oracle
    k, D, l, N, s = 8, 2, 4, 64, 3.5
    uval = np.array([[0.3, -0.2, 0.9], [0.5, 0.1, -0.4]], np.float32)
    bval = np.array([0.25, 0.75], np.float32)
    sig = np.full((k, k, k), s, np.float32)
    u = np.broadcast_to(uval, (k, k, k, D, 3)).copy()
    beta = np.broadcast_to(bval, (l, l, D)).copy()
    bg = np.array([0.1, 0.6, 0.35])
    cache = G.make_cache(sig, u, beta, in_box=True, bg=tuple(bg))
    v = synth.orbit_view(3.5, 0.3, 0.2, 24, 24, 0.0, 100.0, f=20.0)
    out = G.render_gpu(cache, v, N, eps)
    c = bval.astype(np.float64) @ uval.astype(np.float64)
    sc = oracle.Scene(beta, sig, u, in_box=True)
    for p in range(24 * 24):
        o, d = oracle.pixel_ray(v.K, v.c2w, 24, 24, p % 24, p // 24)
        hit, t0, t1 = oracle.interval(sc, o, d, 0.0, 100.0)
        if not hit:
            assert np.array_equal(out[p], np.concatenate([bg, [0.0]]).astype(np.float32))
            continue
        L = t1 - t0
        if eps > 0:
            dl = L / N
            L = min(N, math.floor(math.log(1 / eps) / (s * dl)) + 1) * dl
        T = math.exp(-s * L)
        expect = np.concatenate([c * (1 - T) + T * bg, [1 - T]])
        # FP32 slab clipping: grazing chords carry ~1e-5 relative error in t
        np.testing.assert_allclose(out[p], expect, atol=1e-4)


def test_linearity_in_radiance():
    """With bg = 0: render(a u + b u') = a render(u) + b render(u') up to FP32."""
    sig, u, beta = G.config1_scene()
    v = G.config1_view()
    u2 = np.random.default_rng(5).uniform(-1, 1, u.shape).astype(np.float32)
    r = lambda uu: G.render_gpu(G.make_cache(sig, uu, beta, bg=(0, 0, 0)), v, 128, 1e-4)
    mix = (0.5 * u.astype(np.float64) - 0.25 * u2).astype(np.float32)
    lhs, a, b = r(mix), r(u), r(u2)
    np.testing.assert_allclose(lhs[:, :3], 0.5 * a[:, :3] - 0.25 * b[:, :3], atol=2e-6)
    assert np.array_equal(lhs[:, 3], a[:, 3])


def test_skip_distance_is_chessboard_distance():
    """The skip distance equals scipy's chessboard distance transform of the
    occupancy, capped at 63 (library routine): over the bitgrid's bricks, or
    for bitgrids finer than 8^3 over 8^3 bricks holding any set bit."""
    from scipy import ndimage
    sig, u, beta = G.config1_scene()
    for brick, lin in ((8, False), (4, True), (2, False), (16, False)):
        cache = G.make_cache(sig, u, beta, pos_linear=lin, brick=brick)
        occ = cache.occupancy()
        dist = cache.skip_distance()
        assert occ.any() and not occ.all()
        f = max(1, 8 // brick)
        n = occ.shape[0] // f
        occ_d = occ.reshape(n, f, n, f, n, f).any(axis=(1, 3, 5))
        ref = np.minimum(ndimage.distance_transform_cdt(~occ_d, metric="chessboard"), 63)
        assert np.array_equal(dist, ref), brick
    assert G.make_cache(sig, u, beta, brick=0).skip_distance().size == 0


@pytest.mark.parametrize("storage", ["f32", "fp8"])
def test_distance_skipping_is_exact_paper_like(storage):
    """A k=256 scene of the paper-scale generator (sparse, thin shells), samples
    in the box: renders with skipping over 4-, 8- and 16-voxel bricks equal the
    render without an occupancy grid, bitwise, on orbit views."""
    import paper_2103_10380_amd as fn
    import torch
    spec = synth.paper_scene_spec(k=256)
    p = synth.draw(spec)
    beta = synth.beta_table(p)
    caches = []
    for brick in (0, 4, 8, 16):
        desc = fn.make_desc(spec.k, spec.D, spec.l, storage=storage, brick=brick,
                            sample_mode=fn.IN_BOX)
        c = fn.Cache.create_empty(desc, beta)
        for phase in ("scan", "upload") if storage == "fp8" else ("upload",):
            for z0 in range(0, spec.k, 32):
                sg = synth.density(p, z0, 32, "cuda")
                uu = synth.radiance(p, z0, 32, "cuda")
                (c.scan_slab if phase == "scan" else c.upload_slab)(z0, sg, uu)
        c.finalize()
        caches.append(c)
    for v in synth.paper_orbit(5, W=160, H=144):
        outs = [G.render_gpu(c, v, 192, 1e-4) for c in caches]
        assert (outs[0][:, 3] > 0).mean() > 0.05
        for o in outs[1:]:
            assert np.array_equal(outs[0], o)
    torch.cuda.synchronize()
