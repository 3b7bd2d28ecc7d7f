"""Shared helpers of the GPU tests: scene construction through the C ABI and
comparison against the oracle under the pass protocol (a pixel passes when it is
within tolerance of at least one admissible oracle result)."""
from __future__ import annotations

import numpy as np

import oracle
import synth

PARITY_TOL = 1e-4          # kernel parity, every storage format (oracle on dequantised values)
F32_COST_TOL = 1e-4        # FP32 cache against the FP32-input oracle
F16_COST_TOL = 2e-3        # FP16 cache against the FP32-input oracle
FP8_MIN_PSNR = 40.0        # FP8 cache against the FP32-input oracle (dB, MAX = 1)


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def make_cache(sig, u, beta, *, storage="f32", pos_linear=False, dir_linear=True, brick=8,
               in_box=False, bg=(1.0, 1.0, 1.0), sparse=False):
    import paper_2103_10380_amd as fn
    k, D = sig.shape[0], u.shape[-2]
    l = beta.shape[0]
    desc = fn.make_desc(k, D, l, storage=storage,
                        pos_interp=fn.LINEAR if pos_linear else fn.NEAREST,
                        dir_interp=fn.LINEAR if dir_linear else fn.NEAREST, brick=brick,
                        sample_mode=fn.IN_BOX if in_box else fn.NEAR_FAR, background=bg,
                        sparse=sparse)
    return fn.Cache.create(desc, sig, u, beta)


def oracle_scene(sig, u, beta, *, storage="f32", pos_linear=False, dir_linear=True,
                 in_box=False, bg=(1.0, 1.0, 1.0), occ_brick=0):
    if storage != "f32":
        sig, u, _ = oracle.dequant_cache(storage, sig, u)
    return oracle.Scene(beta, sig, u, pos_linear=pos_linear, dir_linear=dir_linear,
                        in_box=in_box, bg=bg, occ_brick=occ_brick)


def render_gpu(cache, view, N, eps):
    import paper_2103_10380_amd as fn
    import torch
    out = fn.render(cache, view.K, view.c2w, view.H, view.W, view.near, view.far, N, eps)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(-1, 4).astype(np.float64)


def oracle_render(scene, view, N, eps, pix=None):
    """The oracle with the default admissibility bands (reading R13)."""
    return oracle.render(scene, view.K, view.c2w, view.H, view.W, view.near, view.far, N, eps,
                         pix=pix, tol=oracle.DEFAULT_TOL)


def compare(gpu_rgba, res, tol, max_unchecked=0.01):
    """Returns (max error, number failing, count of pixels with too many
    ambiguous lookups to enumerate). Those are checked against the oracle's
    interval bounds of all their admissible results; the error reported is
    over the enumerated pixels."""
    err, ok = oracle.matches(gpu_rgba, res, tol)
    unchecked = (res["flags"] & oracle.UNCHECKED) != 0
    failing = int((~ok).sum())
    assert unchecked.mean() <= max_unchecked, f"{unchecked.sum()} unchecked pixels"
    return float(err[~unchecked].max()) if (~unchecked).any() else 0.0, failing, \
        int(unchecked.sum())


def matched(gpu_rgba, res):
    """Per pixel, the admissible oracle result nearest to the GPU's (the one
    the pass protocol matches it with): the reference for PSNR, since the
    oracle's primary result is only one of the admissible ones (reading R13)."""
    return oracle.matched(gpu_rgba, res)


def psnr(a, b):
    mse = float(np.mean((np.asarray(a)[:, :3] - np.asarray(b)[:, :3]) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


_C1 = None


def config1_scene():
    """Plain-method scene: k=128, D=8, l=64, 6 ellipsoids, seed 0 (dense FP32)."""
    global _C1
    if _C1 is None:
        spec = synth.SceneSpec(k=128, D=8, l=64, n_ellipsoids=6, seed=0)
        sig, u, beta, _ = synth.scene_arrays(spec)
        _C1 = (sig, u, beta)
    return _C1


def config1_view():
    return synth.orbit_view(3.0, 0.7, 0.4, 200, 200, 2.0, 4.0)
