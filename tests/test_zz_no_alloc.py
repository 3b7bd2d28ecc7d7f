"""The allocation-free render (fastnerf_render_noalloc: the render's queue
counters in a fixed device array of the library) against fastnerf_render,
through the C ABI: bitwise the same image on two calls in a row, the second
with a smaller image, for a dense and a brick-sparse cache, both schedules and
the voxel traversal."""
import ctypes

import numpy as np
import pytest

import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def _call(fn, L, cache, v, N, eps, out, stream):
    K = np.ascontiguousarray(np.asarray(v.K, np.float32).reshape(9))
    C = np.ascontiguousarray(np.asarray(v.c2w, np.float32).reshape(12))
    pf = ctypes.POINTER(ctypes.c_float)
    rc = L.fastnerf_render_noalloc(cache.handle, K.ctypes.data_as(pf), C.ctypes.data_as(pf),
                                   v.H, v.W, v.near, v.far, N, eps,
                                   ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0, L.fastnerf_last_error()


@pytest.mark.parametrize("storage,sparse,schedule", [("f32", False, "auto"),
                                                     ("fp8", True, "tiles"),
                                                     ("f16", False, "refill")])
def test_noalloc_equals_render(storage, sparse, schedule):
    import torch
    import paper_2103_10380_amd as fn
    L = fn.lib()
    sig, u, beta = G.config1_scene()
    cache = G.make_cache(sig, u, beta, storage=storage, in_box=True, sparse=sparse)
    fn.set_schedule(schedule)
    try:
        s = torch.cuda.current_stream()
        big = synth.orbit_view(3.0, 0.7, 0.4, 200, 200, 0.0, 10.0)
        small = synth.orbit_view(3.5, 2.1, -0.3, 61, 35, 0.0, 10.0)
        for v, N in ((big, 128), (small, 96), (small, 0)):
            ref = fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, N, 1e-4)
            out = torch.full((v.H, v.W, 4), float("nan"), dtype=torch.float32, device="cuda")
            print(f"{storage} sparse={sparse} {schedule}: {v.W}x{v.H} N={N}", flush=True)
            _call(fn, L, cache, v, N, 1e-4, out, s)
            torch.cuda.synchronize()
            assert torch.equal(out, ref)
            assert (ref[..., 3] > 0).any()
    finally:
        fn.set_schedule("auto")
        cache.destroy()


def test_noalloc_argument_errors():
    import torch
    import paper_2103_10380_amd as fn
    L = fn.lib()
    sig, u, beta = G.config1_scene()
    cache = G.make_cache(sig, u, beta)
    v = synth.orbit_view(3.0, 0.7, 0.4, 16, 16, 2.0, 4.0)
    out = torch.empty((16, 16, 4), dtype=torch.float32, device="cuda")
    K = np.ascontiguousarray(np.asarray(v.K, np.float32).reshape(9))
    C = np.ascontiguousarray(np.asarray(v.c2w, np.float32).reshape(12))
    pf = ctypes.POINTER(ctypes.c_float)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    o = ctypes.c_void_p(out.data_ptr())
    for H, W, N, eps, near, far in ((0, 16, 64, 1e-4, 2.0, 4.0), (16, 70000, 64, 1e-4, 2.0, 4.0),
                                    (16, 16, 5000, 1e-4, 2.0, 4.0), (16, 16, 64, 1.0, 2.0, 4.0),
                                    (16, 16, 64, 1e-4, 4.0, 2.0)):
        rc = L.fastnerf_render_noalloc(cache.handle, K.ctypes.data_as(pf), C.ctypes.data_as(pf),
                                       H, W, near, far, N, eps, o, s)
        assert rc == -1, (H, W, N, eps)
    assert L.fastnerf_render_noalloc(None, K.ctypes.data_as(pf), C.ctypes.data_as(pf), 16, 16,
                                     2.0, 4.0, 64, 1e-4, o, s) == -1
    cache.destroy()
