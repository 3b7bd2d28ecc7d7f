"""HIP render path against the FP64 oracle, element by element, through the C ABI."""
import numpy as np
import pytest

import oracle
import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def _tiny(seed, k, D, l, density=0.5):
    rng = np.random.default_rng(seed)
    sig = (rng.uniform(0, 30, (k, k, k)) * (rng.uniform(size=(k, k, k)) < density)).astype(
        np.float32)
    sig[[0, -1], :, :] = 0
    sig[:, [0, -1], :] = 0
    sig[:, :, [0, -1]] = 0
    u = rng.uniform(-1, 1, (k, k, k, D, 3)).astype(np.float32)
    beta = rng.dirichlet(np.ones(D), (l, l)).astype(np.float32)
    return sig, u, beta


@pytest.mark.parametrize("pos_linear", [False, True])
@pytest.mark.parametrize("dir_linear", [False, True])
@pytest.mark.parametrize("in_box", [False, True])
@pytest.mark.parametrize("W,H", [(16, 16), (13, 11)])
def test_tiny_scenes_all_modes(pos_linear, dir_linear, in_box, W, H):
    """Several tiles and a ragged edge, every lookup and sampling mode, FP32."""
    sig, u, beta = _tiny(1, 8, 3, 6)
    v = synth.orbit_view(2.6, 0.9, 0.3, W, H, 1.2, 4.0, f=1.1 * W)
    for brick in (0, 2, 4):
        cache = G.make_cache(sig, u, beta, pos_linear=pos_linear, dir_linear=dir_linear,
                             brick=brick, in_box=in_box, bg=(0.2, 0.4, 0.9))
        gpu = G.render_gpu(cache, v, 40, 1e-3)
        sc = G.oracle_scene(sig, u, beta, pos_linear=pos_linear, dir_linear=dir_linear,
                            in_box=in_box, bg=(0.2, 0.4, 0.9))
        res = G.oracle_render(sc, v, 40, 1e-3)
        err, failing, _ = G.compare(gpu, res, G.PARITY_TOL)
        assert failing == 0, (brick, err)


def test_config1_fp32_parity():
    """The plain-method workload (k=128, D=8, l=64, 200x200, N=128, eps=1e-4)."""
    sig, u, beta = G.config1_scene()
    v = G.config1_view()
    cache = G.make_cache(sig, u, beta, brick=8)
    gpu = G.render_gpu(cache, v, 128, 1e-4)
    res = G.oracle_render(G.oracle_scene(sig, u, beta), v, 128, 1e-4)
    err, failing, unchecked = G.compare(gpu, res, G.F32_COST_TOL)
    print(f"config1 f32: max err {err:.2e}, ambiguous {res['counts']['ambiguous_pixels']}, "
          f"unchecked {unchecked}")
    assert failing == 0
    # against the admissible result each pixel matched; against the oracle's
    # primary result it is lower where the kernel took the other admissible
    # voxel of a sample within FP32 rounding of a face (reading R13)
    p_matched, p_primary = G.psnr(gpu, G.matched(gpu, res)), G.psnr(gpu, res["rgba"])
    print(f"PSNR {p_matched:.1f} dB against the matched admissible results, "
          f"{p_primary:.1f} dB against the primary ones")
    assert p_matched > 100 and p_primary > 50


@pytest.mark.parametrize("storage", ["f16", "bf16", "fp8"])
def test_config1_reduced_precision_kernel_parity(storage):
    """Each storage format against the oracle run on its own dequantised copy."""
    sig, u, beta = G.config1_scene()
    v = G.config1_view()
    cache = G.make_cache(sig, u, beta, storage=storage, brick=8)
    gpu = G.render_gpu(cache, v, 128, 1e-4)
    res = G.oracle_render(G.oracle_scene(sig, u, beta, storage=storage), v, 128, 1e-4)
    err, failing, _ = G.compare(gpu, res, G.PARITY_TOL)
    assert failing == 0, err


def test_config1_precision_cost():
    """Reduced-precision caches against the FP32-input oracle: FP16 within 2e-3
    max-abs, FP8 at PSNR >= 40 dB; BF16 is reported."""
    sig, u, beta = G.config1_scene()
    v = G.config1_view()
    res = G.oracle_render(G.oracle_scene(sig, u, beta), v, 128, 1e-4)
    out = {}
    for storage in ("f16", "bf16", "fp8"):
        gpu = G.render_gpu(G.make_cache(sig, u, beta, storage=storage), v, 128, 1e-4)
        err, _ = oracle.matches(gpu, res, 1.0)
        out[storage] = (float(err.max()), G.psnr(gpu, G.matched(gpu, res)))
    print("precision cost (max-abs, PSNR):", out)
    assert out["f16"][0] <= G.F16_COST_TOL
    assert out["fp8"][1] >= G.FP8_MIN_PSNR


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16", "fp8"])
def test_readback_equals_oracle_quantiser(storage):
    """The stored cache, decoded, is bit-identical to the oracle's own quantiser."""
    sig, u, beta = _tiny(2, 16, 4, 4)
    u[..., 1, 2] = 0.0
    cache = G.make_cache(sig, u, beta, storage=storage)
    s_g, u_g, sc_g = cache.readback()
    s_o, u_o, sc_o = oracle.dequant_cache(storage, sig, u)
    assert np.array_equal(s_g.cpu().numpy(), s_o)
    assert np.array_equal(u_g.cpu().numpy(), u_o)
    assert np.array_equal(sc_g, sc_o)


def test_fp8_every_code_decodes_exactly():
    """Every finite E4M3 code, stored and read back: each of the 25 channels of
    a k=8, D=8 cache cycles through all 254 finite codes and contains 448, so
    its scale is exactly 1 and the stored code is the input's; the decoded
    cache equals the OCP E4M3 value table (the oracle's decoder) bitwise."""
    codes = [c for c in range(256) if c not in (0x7F, 0xFF)]
    table = np.array([oracle.e4m3_decode(c) for c in codes], np.float32)
    k, D, nch = 8, 8, 25
    vals = np.empty((k ** 3, nch), np.float32)
    for ch in range(nch):
        vals[:, ch] = table[(np.arange(k ** 3) + 7 * ch) % len(codes)]
        vals[ch, ch] = 448.0
    sig = vals[:, 0].reshape(k, k, k).copy()
    u = vals[:, 1:].reshape(k, k, k, D, 3).copy()
    beta = np.full((4, 4, D), 1.0 / D, np.float32)
    cache = G.make_cache(sig, u, beta, storage="fp8")
    s_g, u_g, sc_g = cache.readback()
    assert np.array_equal(sc_g, np.ones(nch, np.float32))
    assert np.array_equal(s_g.cpu().numpy().reshape(-1), vals[:, 0])
    assert np.array_equal(u_g.cpu().numpy().reshape(k ** 3, nch - 1), vals[:, 1:])
    seen = set(np.unique(vals).tolist())
    assert len(seen) == len(set(table.tolist()))  # every value, +-0 counted once


@pytest.mark.parametrize("pos_linear", [False, True])
@pytest.mark.parametrize("dir_linear", [False, True])
def test_debug_lookup_matches_oracle(pos_linear, dir_linear):
    import torch
    import paper_2103_10380_amd as fn
    sig, u, beta = _tiny(3, 16, 5, 12, density=1.0)
    cache = G.make_cache(sig, u, beta, pos_linear=pos_linear, dir_linear=dir_linear)
    rng = np.random.default_rng(4)
    pts = rng.uniform(-1.1, 1.1, (4000, 3))
    # stay away from cell boundaries (nearest) so FP32 and FP64 pick the same voxel
    g = (pts + 1) * 8
    keep = np.all(np.abs(g - np.round(g)) > 1e-3, axis=1)
    pts = pts[keep]
    dirs = rng.standard_normal((3000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    su, _ = fn.debug_lookup(cache, pts=torch.tensor(pts, dtype=torch.float32, device="cuda"))
    _, bo = fn.debug_lookup(cache, dirs=torch.tensor(dirs, dtype=torch.float32, device="cuda"))
    sc = oracle.Scene(beta, sig, u, pos_linear=pos_linear, dir_linear=dir_linear)
    s_o, u_o = oracle.lookup_pos(sc, pts.astype(np.float32).astype(np.float64))
    su = su.cpu().numpy()
    np.testing.assert_allclose(su[:, 0], s_o, atol=2e-5 * 30, rtol=0)
    np.testing.assert_allclose(su[:, 1:], u_o.reshape(len(pts), -1), atol=2e-5, rtol=0)
    b_o = oracle.lookup_dir(sc, dirs.astype(np.float32).astype(np.float64))
    bo = bo.cpu().numpy()
    if dir_linear:
        np.testing.assert_allclose(bo, b_o, atol=1e-5)
    else:  # nearest cells: identical away from cell borders
        same = np.all(np.abs(bo - b_o) < 1e-7, axis=1)
        assert same.mean() > 0.99


def test_render_batch_equals_single_renders():
    import torch
    import paper_2103_10380_amd as fn
    sig, u, beta = G.config1_scene()
    cache = G.make_cache(sig, u, beta, storage="f16", pos_linear=True, in_box=True)
    views = synth.random_views(6, 2, [(64, 64), (40, 24), (33, 17)], (3.0, 5.0), (-1.0, 1.0),
                               0.0, 10.0)
    # uneven sizes (views one after another) and one size (tiles of the views
    # interleaved in the launch)
    same = synth.random_views(5, 3, [(48, 40)], (3.0, 5.0), (-1.0, 1.0), 0.0, 10.0)
    for batch in (views, same):
        outs = fn.render_batch(cache, batch, 96, 1e-4)
        torch.cuda.synchronize()
        for v, o in zip(batch, outs):
            single = fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, 96, 1e-4)
            torch.cuda.synchronize()
            assert torch.equal(o, single)


@pytest.mark.parametrize("n", [11, 16])
def test_interleaved_batches_equal_single_renders(n):
    """Batches of one view size deal their tiles in groups of 8 interleaved
    views: 11 views (a group of 8 and one of 3) and 16 (two groups), under the
    tile and refill schedules and with N = 0, equal the single renders
    bitwise."""
    import torch
    import paper_2103_10380_amd as fn
    sig, u, beta = G.config1_scene()
    cache = G.make_cache(sig, u, beta, in_box=True)
    views = synth.random_views(n, 9, [(40, 24)], (2.5, 5.0), (-1.0, 1.0), 0.0, 10.0)
    try:
        for sch in ("tiles", "refill"):
            fn.set_schedule(sch)
            for N in (64, 0):
                outs = fn.render_batch(cache, views, N, 1e-4)
                torch.cuda.synchronize()
                for v, o in zip(views, outs):
                    single = fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, N, 1e-4)
                    torch.cuda.synchronize()
                    assert torch.equal(o, single), (sch, N)
    finally:
        fn.set_schedule("auto")
        cache.destroy()


def test_concurrent_streams_equal_serial_renders():
    """One cache rendered from two streams at once (each stream has its own
    tile counters and descriptor staging): every image equals the one
    rendered alone, bit for bit."""
    import torch
    import paper_2103_10380_amd as fn
    sig, u, beta = G.config1_scene()
    cache = G.make_cache(sig, u, beta, storage="fp8")
    views = synth.random_views(8, 4, [(96, 80), (64, 64), (50, 30)], (3.0, 5.0), (-1.0, 1.0),
                               0.0, 10.0)
    ref = []
    for v in views:
        ref.append(fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, 128, 1e-4))
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = [None] * len(views)
    for rep in range(3):
        for i, v in enumerate(views):
            st = s1 if i % 2 == 0 else s2
            with torch.cuda.stream(st):
                outs[i] = fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, 128, 1e-4,
                                    stream=st)
        with torch.cuda.stream(s1):
            b1 = fn.render_batch(cache, views[:4], 128, 1e-4, stream=s1)
        with torch.cuda.stream(s2):
            b2 = fn.render_batch(cache, views[4:], 128, 1e-4, stream=s2)
        torch.cuda.synchronize()
        for i in range(len(views)):
            assert torch.equal(outs[i], ref[i]), (rep, i)
        for o, r in zip(b1 + b2, ref):
            assert torch.equal(o, r), rep
