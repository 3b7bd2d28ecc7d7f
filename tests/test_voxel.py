"""The voxel traversal (N = 0: every voxel a ray crosses, each with its own
length) of the HIP path against the oracle's plane-crossing traversal, closed
forms and invariants."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["f32", "f16", "fp8"])
@pytest.mark.parametrize("in_box", [False, True])
def test_voxel_traversal_parity_plain_scene(storage, in_box):
    """Plain scene (k=128), one 200x200 view: every pixel within 1e-4 of the
    oracle on the same (dequantised) values; the traversal ignores the sample
    mode (it always stays inside the box)."""
    sig, u, beta = G.config1_scene()
    v = G.config1_view()
    cache = G.make_cache(sig, u, beta, storage=storage, in_box=in_box)
    gpu = G.render_gpu(cache, v, 0, 1e-4)
    res = G.oracle_render(G.oracle_scene(sig, u, beta, storage=storage, in_box=in_box), v, 0,
                          1e-4)
    err, failing, _ = G.compare(gpu, res, G.PARITY_TOL)
    print(f"{storage} in_box={in_box}: max err {err:.2e}")
    assert failing == 0, err
    assert res["counts"]["hit"] > 10000


def test_voxel_traversal_homogeneous_chord():
    """A box of constant sigma, u, beta: every pixel is
    c (1 - exp(-sigma L)) + exp(-sigma L) bg with L the analytic chord."""
    k, D, l, s = 9, 2, 4, 3.5
    uval = np.array([[0.3, -0.2, 0.9], [0.5, 0.1, -0.4]], np.float32)
    bval = np.array([0.25, 0.75], np.float32)
    sig = np.full((k, k, k), s, np.float32)
    u = np.broadcast_to(uval, (k, k, k, D, 3)).copy()
    beta = np.broadcast_to(bval, (l, l, D)).copy()
    bg = np.array([0.1, 0.6, 0.35])
    cache = G.make_cache(sig, u, beta, bg=tuple(bg), brick=0)
    v = synth.orbit_view(3.5, 0.3, 0.2, 24, 24, 0.0, 100.0, f=20.0)
    out = G.render_gpu(cache, v, 0, 0.0)
    c = bval.astype(np.float64) @ uval.astype(np.float64)
    sc = oracle.Scene(beta, sig, u, in_box=True)
    for p in range(24 * 24):
        o, d = oracle.pixel_ray(v.K, v.c2w, 24, 24, p % 24, p // 24)
        hit, t0, t1 = oracle.interval(sc, o, d, 0.0, 100.0)
        if not hit:
            assert np.array_equal(out[p], np.concatenate([bg, [0.0]]).astype(np.float32))
            continue
        T = math.exp(-s * (t1 - t0))
        expect = np.concatenate([c * (1 - T) + T * bg, [1 - T]])
        np.testing.assert_allclose(out[p], expect, atol=1e-4)


@pytest.mark.parametrize("storage", ["f32", "fp8"])
def test_voxel_traversal_skipping_is_exact(storage):
    """Restarting past proven-empty space changes no bit of the result."""
    sig, u, beta = G.config1_scene()
    v = G.config1_view()
    outs = [G.render_gpu(G.make_cache(sig, u, beta, storage=storage, brick=b), v, 0, 1e-4)
            for b in (0, 4, 8, 16)]
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_voxel_traversal_batch_equals_single():
    import paper_2103_10380_amd as fn
    import torch
    sig, u, beta = G.config1_scene()
    cache = G.make_cache(sig, u, beta, in_box=True)
    views = synth.random_views(5, 4, [(37, 29), (64, 64), (100, 77)], (3.0, 4.5), (-0.8, 0.8),
                               0.0, 100.0)
    outs = fn.render_batch(cache, views, 0, 1e-4)
    torch.cuda.synchronize()
    for v, o in zip(views, outs):
        single = G.render_gpu(cache, v, 0, 1e-4)
        assert np.array_equal(o.cpu().numpy().reshape(-1, 4).astype(np.float64), single)


def test_voxel_traversal_argument_errors():
    import paper_2103_10380_amd as fn
    sig, u, beta = G.config1_scene()
    v = G.config1_view()
    lin = G.make_cache(sig, u, beta, pos_linear=True)
    with pytest.raises(fn.FastNeRFError):
        fn.render(lin, v.K, v.c2w, v.H, v.W, v.near, v.far, 0, 1e-4)
    with pytest.raises(fn.FastNeRFError):
        fn.render(lin, v.K, v.c2w, v.H, v.W, v.near, v.far, -1, 1e-4)
    nn = G.make_cache(sig, u, beta)
    srv = fn.Server([nn], arena_bytes=1 << 24)
    try:
        with pytest.raises(fn.FastNeRFError):
            srv.submit(0, v.K, v.c2w, v.H, v.W, v.near, v.far, 0, 1e-4)
    finally:
        srv.destroy()
