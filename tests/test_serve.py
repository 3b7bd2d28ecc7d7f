"""The render server on the GPU: continuous batching over several resident
scenes of different storage formats; every result equals its standalone render
bitwise (same kernel arithmetic, no cross-ray reductions)."""
import threading

import numpy as np
import pytest

import synth
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


def _scenes():
    out = []
    for seed, storage, k in ((10, "f16", 32), (11, "fp8", 48), (12, "f32", 40)):
        spec = synth.SceneSpec(k=k, D=8, l=16, n_ellipsoids=5, seed=seed)
        sig, u, beta, _ = synth.scene_arrays(spec)
        out.append(G.make_cache(sig, u, beta, storage=storage, in_box=True))
    return out


def test_mixed_requests_equal_standalone_renders():
    import torch
    import paper_2103_10380_amd as fn
    caches = _scenes()
    views = synth.random_views(24, 3, [(40, 40), (64, 48), (100, 60), (23, 17)], (3.0, 5.0),
                               (-1.0, 1.0), 0.0, 100.0)
    scenes = [i % 3 for i in range(len(views))]
    srv = fn.Server(caches, arena_bytes=4 << 20, max_inflight=6)
    try:
        tickets = [None] * len(views)

        def submit(lo, hi):
            for i in range(lo, hi):
                v = views[i]
                tickets[i] = srv.submit(scenes[i], v.K, v.c2w, v.H, v.W, v.near, v.far, 96,
                                        1e-4)

        th = [threading.Thread(target=submit, args=(j * 8, j * 8 + 8)) for j in range(3)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        lat = []
        for i, v in enumerate(views):
            got, ms = srv.result(tickets[i], v.H, v.W)
            lat.append(ms)
            alone = fn.render(caches[scenes[i]], v.K, v.c2w, v.H, v.W, v.near, v.far, 96, 1e-4)
            torch.cuda.synchronize()
            assert torch.equal(got, alone), i
        st = srv.stats()
        assert st["completed"] == len(views)
        assert st["max_batch"] >= 2  # requests shared steps
        assert min(lat) > 0
    finally:
        srv.destroy()


def test_request_larger_than_arena_is_rejected():
    import paper_2103_10380_amd as fn
    caches = _scenes()[:1]
    srv = fn.Server(caches, arena_bytes=1 << 16, max_inflight=2)
    try:
        v = synth.orbit_view(3.0, 0.1, 0.2, 128, 128, 0.0, 100.0)
        with pytest.raises(fn.FastNeRFError) as e:
            srv.submit(0, v.K, v.c2w, v.H, v.W, v.near, v.far, 64, 1e-4)
        assert e.value.status == -2
        with pytest.raises(fn.FastNeRFError):
            srv.submit(5, v.K, v.c2w, 8, 8, v.near, v.far, 64, 1e-4)
    finally:
        srv.destroy()


def test_requests_split_across_steps_equal_standalone_renders():
    """Two 4096x4096 requests (262,144 tiles each: more than a step's share of
    the tile budget when they run together) in the FP16 and FP8 scenes, with
    small FP32 requests among them: the large ones span several steps in both
    slots while the format groups run concurrently; every result equals its
    standalone render bitwise."""
    import torch
    import paper_2103_10380_amd as fn
    caches = _scenes()
    reqs = [(0, synth.orbit_view(3.0, 0.3, 0.2, 4096, 4096, 0.0, 100.0)),
            (1, synth.orbit_view(3.5, 2.1, -0.4, 4096, 4096, 0.0, 100.0))]
    reqs += [(2, synth.orbit_view(3.0 + 0.2 * i, 0.5 * i, 0.1, 64 + 8 * i, 48, 0.0, 100.0))
             for i in range(4)]
    srv = fn.Server(caches, arena_bytes=1 << 30, max_inflight=8)
    try:
        tickets = [srv.submit(s, v.K, v.c2w, v.H, v.W, v.near, v.far, 64, 1e-4) for s, v in reqs]
        for (s, v), t in zip(reqs, tickets):
            got, _ = srv.result(t, v.H, v.W)
            alone = fn.render(caches[s], v.K, v.c2w, v.H, v.W, v.near, v.far, 64, 1e-4)
            torch.cuda.synchronize()
            assert torch.equal(got, alone), (s, v.H, v.W)
            del got, alone
        st = srv.stats()
        assert st["completed"] == len(reqs)
        assert st["steps"] >= 3, st  # the large requests were split
    finally:
        srv.destroy()


def test_arena_sized_from_free_device_memory():
    """arena_bytes = 0: the server's arena is a quarter of the device memory
    free at creation (admission by free memory); requests render as alone."""
    import torch
    import paper_2103_10380_amd as fn
    caches = _scenes()
    free_before, _ = torch.cuda.mem_get_info()
    srv = fn.Server(caches, arena_bytes=0, max_inflight=4)
    try:
        free_after, _ = torch.cuda.mem_get_info()
        taken = free_before - free_after
        assert abs(taken - free_before / 4) <= (1 << 30), (free_before, taken)
        views = [synth.orbit_view(3.0 + 0.3 * i, 0.7 * i, 0.2, 96, 80, 0.0, 100.0)
                 for i in range(3)]
        tickets = [srv.submit(i % len(caches), v.K, v.c2w, v.H, v.W, v.near, v.far, 64, 1e-4)
                   for i, v in enumerate(views)]
        for i, (v, t) in enumerate(zip(views, tickets)):
            got, _ = srv.result(t, v.H, v.W)
            alone = fn.render(caches[i % len(caches)], v.K, v.c2w, v.H, v.W, v.near, v.far, 64,
                              1e-4)
            torch.cuda.synchronize()
            assert torch.equal(got, alone)
    finally:
        srv.destroy()
