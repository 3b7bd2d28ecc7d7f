"""The refill schedule (the wave-level ray queue: retired lanes refilled from
a per-wave pool of set-up rays in LDS) and the wide kernel (more records in
flight per lane) against one tile per wave: every ray is computed by one lane
with the same arithmetic, so images are bitwise equal, for every storage
format, dense and brick-sparse caches, both lookups, both sample modes, single
views and batches of uneven views."""
import numpy as np
import pytest

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
    wide kernel's render is checked against the tile one here too."""
    import torch
    import paper_2103_10380_amd as fn
    out = {}
    for sch in ("tiles", "refill", "wide"):
        fn.set_schedule(sch)
        out[sch] = fn_render()
        torch.cuda.synchronize()
    a, w = out["tiles"], out["wide"]
    for x, y in (zip(a, w) if isinstance(a, list) else [(a, w)]):
        assert torch.equal(x, y)
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


def test_schedule_argument_checked():
    import paper_2103_10380_amd as fn
    with pytest.raises(ValueError):
        fn.set_schedule("sideways")
    with pytest.raises(fn.FastNeRFError):
        fn._lib.check(fn.lib().fastnerf_set_schedule(4))
    assert fn.get_schedule() == "auto"
