"""Batched uneven renders (64 views of the plain scene at resolutions drawn
from {256^2, 512^2, 800^2, 1024^2, 1280x720}, radii U[3, 5], elevations
U[-1, 1], seed 2; trilinear position lookup, samples inside the box, N = 128,
eps = 1e-4) in the one persistent launch the benchmark times, checked on
sampled pixels of views of every resolution against the FP64 oracle
(Sec. 3.1 Eq. 1, Sec. 3.2 Eq. 5, Sec. 4): kernel parity against the oracle on
its own dequantised copy of the cache, and the storage format's precision
cost against the oracle on the FP32 inputs. Also: batched launches enqueue
without waiting for earlier work on the stream."""
import time

import numpy as np
import pytest

import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

N, EPS = 128, 1e-4
RES = [(256, 256), (512, 512), (800, 800), (1024, 1024), (1280, 720)]


def _views():
    return synth.random_views(64, 2, RES, (3.0, 5.0), (-1.0, 1.0), 0.0, 100.0)


def _checked_views(views, extra):
    """The first view of every resolution plus `extra` more, in view order."""
    pick, seen = [], set()
    for i, v in enumerate(views):
        if (v.W, v.H) not in seen:
            seen.add((v.W, v.H))
            pick.append(i)
    rest = [i for i in range(len(views)) if i not in pick]
    pick += rest[:: max(1, len(rest) // extra)][:extra]
    return sorted(pick)


def _launch(storage):
    import torch
    import paper_2103_10380_amd as fn
    sig, u, beta = G.config1_scene()
    cache = G.make_cache(sig, u, beta, storage=storage, pos_linear=True, in_box=True)
    views = _views()
    outs = fn.render_batch(cache, views, N, EPS)
    torch.cuda.synchronize()
    cache.destroy()
    return views, outs


def _gpu_pixels(out, pix):
    import torch
    return out.reshape(-1, 4)[torch.as_tensor(pix, device=out.device)].cpu().numpy().astype(
        np.float64)


@pytest.mark.parametrize("storage,n_extra,n_pix", [("f16", 5, 2000), ("bf16", 1, 800),
                                                   ("fp8", 1, 800)])
def test_batched_uneven_trilinear_parity(storage, n_extra, n_pix):
    sig, u, beta = G.config1_scene()
    views, outs = _launch(storage)
    assert len(views) == 64
    idx = _checked_views(views, n_extra)
    sizes = {(views[i].W, views[i].H) for i in idx}
    assert (1280, 720) in sizes and (1024, 1024) in sizes
    own = G.oracle_scene(sig, u, beta, storage=storage, pos_linear=True, in_box=True)
    f32 = G.oracle_scene(sig, u, beta, storage="f32", pos_linear=True, in_box=True)
    rng = np.random.default_rng(40)
    worst, worst_cost, se, n, hit = 0.0, 0.0, 0.0, 0, 0
    for i in idx:
        v = views[i]
        pix = np.sort(rng.choice(v.H * v.W, min(n_pix, v.H * v.W), replace=False))
        print(f"{storage} view {i} {v.W}x{v.H}: {len(pix)} pixels", flush=True)
        g = _gpu_pixels(outs[i], pix)
        res = G.oracle_render(own, v, N, EPS, pix=pix)
        err, failing, _ = G.compare(g, res, G.PARITY_TOL)
        assert failing == 0, (i, err)
        worst = max(worst, err)
        hit += res["counts"]["hit"]
        ref = G.oracle_render(f32, v, N, EPS, pix=pix)
        worst_cost = max(worst_cost, float(np.abs(g - ref["rgba"]).max()))
        se += float(np.sum((g[:, :3] - ref["rgba"][:, :3]) ** 2))
        n += 3 * len(pix)
    psnr = float("inf") if se == 0 else 10 * np.log10(n / se)
    print(f"{storage}: parity max err {worst:.2e}; against the FP32-input oracle max err "
          f"{worst_cost:.2e}, PSNR {psnr:.1f} dB over {n // 3} pixels ({hit} hit)")
    assert hit > 1000
    if storage == "f16":
        assert worst_cost <= G.F16_COST_TOL
    elif storage == "fp8":
        assert psnr >= G.FP8_MIN_PSNR


def test_render_batch_does_not_wait_for_earlier_work():
    """With a long job queued first on the stream, four batched launches
    enqueue and return while that job still runs (the host never waits for a
    launch), and each batch's images equal the same views rendered alone."""
    import torch
    import paper_2103_10380_amd as fn
    sig, u, beta = G.config1_scene()
    cache = G.make_cache(sig, u, beta, storage="f16", pos_linear=True, in_box=True)
    views = synth.random_views(6, 5, [(64, 64), (48, 40)], (3.0, 5.0), (-1.0, 1.0), 0.0, 10.0)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        fn.render_batch(cache, views, 64, 1e-4, stream=s)  # the stream's state is created here
        a = torch.randn(4096, 4096, device="cuda")
        torch.cuda.synchronize()
        for _ in range(60):  # tens of milliseconds of matrix products ahead of the batches
            a = a @ a
            a = a / a.norm()
        long_done = torch.cuda.Event()
        long_done.record(s)
        t0 = time.perf_counter()
        outs = [fn.render_batch(cache, views, 64, 1e-4, stream=s) for _ in range(4)]
        host_ms = (time.perf_counter() - t0) * 1e3
        returned_early = not long_done.query()
    torch.cuda.synchronize()
    print(f"4 batches enqueued in {host_ms:.2f} ms host time; the job ahead was still running: "
          f"{returned_early}")
    assert returned_early
    for v_i, v in enumerate(views):
        single = fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, 64, 1e-4)
        torch.cuda.synchronize()
        for o in outs:
            assert torch.equal(o[v_i], single)
    cache.destroy()
