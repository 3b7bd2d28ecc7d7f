"""The refill schedule (the wave-level ray queue: retired lanes refilled from
a per-wave pool of set-up rays in LDS) and the wide kernel (more records in
flight per lane) against one tile per wave: every ray is computed by one lane
with the same arithmetic, so images are bitwise equal, for every storage
format, dense and brick-sparse caches, both lookups, both sample modes, single
views and batches of uneven views."""
import numpy as np
import pytest

import oracle
import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _restore_schedule():
    import paper_2103_10380_amd as fn
    yield
    fn.set_schedule("auto")


def _both(fn_render):
    """The render under the tile schedule and under the refill schedule; the
    wide kernel's and the split rays' renders (split applies to single views
    of dense caches with nearest lookups; other launches asked for it run
    wide) are checked against the tile one here too."""
    import torch
    import paper_2103_10380_amd as fn
    out = {}
    for sch in ("tiles", "refill", "wide", "split"):
        fn.set_schedule(sch)
        out[sch] = fn_render()
        torch.cuda.synchronize()
    a = out["tiles"]
    for other in ("wide", "split"):
        w = out[other]
        for x, y in (zip(a, w) if isinstance(a, list) else [(a, w)]):
            assert torch.equal(x, y), other
    return a, out["refill"]


@pytest.mark.parametrize("storage,sparse,pos_linear,in_box", [
    ("f32", False, False, False), ("f16", False, False, True), ("bf16", False, False, False),
    ("fp8", False, False, True), ("f32", True, False, True), ("fp8", True, False, False),
    ("f16", False, True, True), ("f32", False, True, False)])
def test_refill_equals_tiles_bitwise(storage, sparse, pos_linear, in_box):
    import torch
    import paper_2103_10380_amd as fn
    sig, u, beta = G.config1_scene()
    cache = G.make_cache(sig, u, beta, storage=storage, pos_linear=pos_linear, in_box=in_box,
                         sparse=sparse)
    v = G.config1_view()
    a, b = _both(lambda: fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, 128, 1e-4))
    assert torch.equal(a, b)
    assert (a[..., 3] > 0).float().mean().item() > 0.05
    views = synth.random_views(9, 7, [(64, 64), (37, 29), (200, 120), (8, 8), (1, 3)],
                               (3.0, 5.0), (-1.0, 1.0), 0.0 if in_box else 2.0,
                               100.0 if in_box else 4.5)
    a, b = _both(lambda: fn.render_batch(cache, views, 96, 1e-3))
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    cache.destroy()


def test_refill_paper_like_scene_and_no_grid():
    """A k=256 scene of the paper-scale generator in the box (long empty runs,
    distance-field jumps, thin shells) with 8^3 bricks (a 4 KiB bitgrid, held
    in LDS by the tile kernel), 2^3 bricks (256 KiB, too large for LDS: every
    kernel reads it from memory) and no occupancy grid: refill and wide equal
    tiles bitwise, and the three grid settings give the same images."""
    import torch
    import paper_2103_10380_amd as fn
    spec = synth.paper_scene_spec(k=256)
    p = synth.draw(spec)
    beta = synth.beta_table(p)
    caches = []
    for brick in (8, 2, 0):
        desc = fn.make_desc(spec.k, spec.D, spec.l, storage="f32", brick=brick,
                            sample_mode=fn.IN_BOX)
        c = fn.Cache.create_empty(desc, beta)
        for z0 in range(0, spec.k, 32):
            c.upload_slab(z0, synth.density(p, z0, 32, "cuda"), synth.radiance(p, z0, 32, "cuda"))
        c.finalize()
        caches.append(c)
    views = synth.paper_orbit(6, W=200, H=168)
    outs = []
    for c in caches:
        a, b = _both(lambda: fn.render_batch(c, views, 192, 1e-4))
        for x, y in zip(a, b):
            assert torch.equal(x, y)
        outs.append(a)
    for other in outs[1:]:
        for x, y in zip(outs[0], other):
            assert torch.equal(x, y)
    assert np.mean([(o[..., 3] > 0).float().mean().item() for o in outs[0]]) > 0.05
    for c in caches:
        c.destroy()


@pytest.mark.parametrize("storage,sparse", [("f32", False), ("f16", False), ("fp8", False),
                                            ("f32", True), ("fp8", True)])
def test_split_single_views_of_any_size(storage, sparse):
    """Split rays (4x4 tiles, four lanes per ray) on single views whose sides
    are not multiples of 4 (partial tiles at the right and bottom edges), in
    the box and between near and far: bitwise the tile schedule's image, and
    the oracle's within the kernel parity tolerance."""
    import torch
    import paper_2103_10380_amd as fn
    sig, u, beta = G.config1_scene()
    for in_box in (False, True):
        cache = G.make_cache(sig, u, beta, storage=storage, in_box=in_box, sparse=sparse)
        sc = G.oracle_scene(sig, u, beta, storage=storage, in_box=in_box)
        for (W, H) in [(37, 29), (1, 3), (8, 8), (13, 66)]:
            v = synth.orbit_view(3.2, 0.9, 0.3, W, H, 0.0 if in_box else 2.0,
                                 100.0 if in_box else 4.5)
            out = {}
            for sch in ("tiles", "split"):
                fn.set_schedule(sch)
                out[sch] = fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, 96, 1e-3)
                torch.cuda.synchronize()
            assert torch.equal(out["tiles"], out["split"]), (storage, in_box, H, W)
            res = G.oracle_render(sc, v, 96, 1e-3)
            err, failing, _ = G.compare(out["split"].cpu().numpy().reshape(-1, 4)
                                        .astype(np.float64), res, G.PARITY_TOL)
            assert failing == 0, (storage, in_box, H, W, err)
        cache.destroy()


def _rect_views():
    """Views that exercise the render rectangle (the pixels whose rays can meet
    the box): far (a small rectangle), near (the box overfills the image), the
    camera inside the box (no rectangle), the box half off the image and wholly
    off it (principal point moved), a corner behind the camera."""
    import dataclasses
    vs = [synth.orbit_view(7.0, 0.3, 0.2, 120, 96, 2.0, 12.0),
          synth.orbit_view(1.9, 1.1, 0.5, 96, 120, 0.0, 100.0),
          synth.orbit_view(0.4, 2.0, 0.3, 64, 64, 0.0, 100.0)]
    base = synth.orbit_view(3.0, 0.7, 0.4, 100, 80, 0.0, 100.0)
    for shift in (50.0, 400.0):
        K = base.K.copy()
        K[0, 2] += shift
        vs.append(dataclasses.replace(base, K=K))
    c2w = synth.look_at(synth.orbit_eye(1.3, 0.2, 0.1), target=(5.0, 3.0, 0.0))
    vs.append(synth.View(synth.intrinsics(72, 56), c2w, 56, 72, 0.0, 100.0))
    return vs


@pytest.mark.parametrize("in_box", [False, True])
def test_render_rectangle_cases(in_box):
    """Pixels outside a single view's render rectangle are written as
    background by the kernel's fill pass, the others by the tiles; single views
    (every schedule) and the voxel traversal match the oracle, and a batch of
    the same views (which covers whole images) equals the single renders
    bitwise."""
    import torch
    import paper_2103_10380_amd as fn
    sig, u, beta = G.config1_scene()
    cache = G.make_cache(sig, u, beta, in_box=in_box)
    sc = G.oracle_scene(sig, u, beta, in_box=in_box)
    views = _rect_views()
    for v in views:
        if not in_box:
            v.near, v.far = max(v.near, 0.05), min(v.far, 12.0)
    singles = []
    for v in views:
        res = G.oracle_render(sc, v, 64, 1e-3)
        outs = {}
        for sch in ("tiles", "wide", "split", "refill"):
            fn.set_schedule(sch)
            outs[sch] = fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, 64, 1e-3)
            torch.cuda.synchronize()
        for sch, o in outs.items():
            assert torch.equal(o, outs["tiles"]), (sch, v.W, v.H)
        err, failing, _ = G.compare(outs["tiles"].cpu().numpy().reshape(-1, 4)
                                    .astype(np.float64), res, G.PARITY_TOL)
        assert failing == 0, (v.W, v.H, err)
        singles.append(outs["tiles"])
    fn.set_schedule("auto")
    batch = fn.render_batch(cache, views, 64, 1e-3)
    torch.cuda.synchronize()
    for x, y in zip(batch, singles):
        assert torch.equal(x, y)
    # N = 0 (voxel traversal) takes the same rectangles
    for v in views[:2]:
        res = oracle.render(sc, v.K, v.c2w, v.H, v.W, v.near, v.far, 0, 1e-3,
                            tol=oracle.DEFAULT_TOL)
        out = fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, 0, 1e-3)
        torch.cuda.synchronize()
        err, failing, _ = G.compare(out.cpu().numpy().reshape(-1, 4).astype(np.float64), res,
                                    G.PARITY_TOL)
        assert failing == 0, ("vox", v.W, v.H, err)
    cache.destroy()


def test_schedule_argument_checked():
    import paper_2103_10380_amd as fn
    with pytest.raises(ValueError):
        fn.set_schedule("sideways")
    with pytest.raises(fn.FastNeRFError):
        fn._lib.check(fn.lib().fastnerf_set_schedule(5))
    assert fn.get_schedule() == "auto"
