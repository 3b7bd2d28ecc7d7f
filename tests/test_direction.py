"""Direction-cache filtering and level-of-detail rendering on the GPU against
the oracle (oracle/direction.py, and the render oracle for the renders)."""
import numpy as np
import pytest

import synth
from oracle import direction as odir
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

# FP32: weights from expf (relative error ~1e-7) and two nested sums of at
# most 61 terms each of values in [0, 1]: worst case about 61 * 2 * 6e-8
FILTER_TOL = 1e-5


@pytest.mark.parametrize("l,D,sigma", [(1, 1, 1.0), (7, 3, 0.4), (7, 8, 10.0), (64, 8, 1.5),
                                       (64, 16, 0.0), (33, 5, 3.3)])
def test_filter_parity(l, D, sigma):
    import torch
    import paper_2103_10380_amd as fn
    rng = np.random.default_rng(l * 100 + D)
    b = rng.uniform(0, 1, (l, l, D)).astype(np.float32)
    got = fn.filter_direction(torch.as_tensor(b, device="cuda"), sigma)
    torch.cuda.synchronize()
    ref = odir.filter_direction(b, sigma)
    err = np.abs(got.cpu().numpy() - ref).max()
    assert err <= FILTER_TOL, err
    if sigma == 0.0:
        assert np.array_equal(got.cpu().numpy(), b)


def test_filter_rejects_bad_arguments():
    import torch
    import paper_2103_10380_amd as fn
    b = torch.zeros((8, 8, 3), device="cuda")
    with pytest.raises(fn.FastNeRFError):
        fn.filter_direction(b, -1.0)
    with pytest.raises(fn.FastNeRFError):
        fn.filter_direction(b, 11.0)
    with pytest.raises(fn.FastNeRFError):
        fn.filter_direction(b, 1.0, out=b)  # in place: overlapping
    with pytest.raises(fn.FastNeRFError):
        fn.filter_direction(b.cpu(), 1.0, out=torch.zeros((8, 8, 3)))  # host arrays


def test_filtered_direction_cache_renders_like_the_oracle():
    """The plain scene with its direction table smoothed (sigma = 2 cells) on
    the GPU renders within the parity tolerance of the oracle rendering with
    the table smoothed by the oracle."""
    import torch
    import paper_2103_10380_amd as fn
    sig, u, beta = G.config1_scene()
    bf = fn.filter_direction(torch.as_tensor(beta, device="cuda"), 2.0)
    torch.cuda.synchronize()
    cache = G.make_cache(sig, u, bf.cpu().numpy())
    v = G.config1_view()
    gpu = G.render_gpu(cache, v, 128, 1e-4)
    res = G.oracle_render(G.oracle_scene(sig, u, odir.filter_direction(beta, 2.0)), v, 128, 1e-4)
    err, failing, _ = G.compare(gpu, res, G.PARITY_TOL)
    assert failing == 0, err


def test_level_of_detail_render():
    """One scene at k = 32, 64 and 128 (the same analytic fields sampled at
    each resolution): lod_select picks the coarsest level that resolves the
    pixel footprint, and that level's render passes the oracle."""
    import paper_2103_10380_amd as fn
    levels = {}
    for k in (32, 64, 128):
        sig, u, beta, _ = synth.scene_arrays(synth.SceneSpec(k=k, D=8, l=64, n_ellipsoids=6,
                                                             seed=0))
        levels[k] = (sig, u, beta)
    ks = list(levels)
    # footprint 3 / f against voxel edges 2 / k: f = 20 -> 32, 50 -> 64, 100 -> 128;
    # f = 1000 resolves finer than any level: the finest
    for r, f, expect in ((3.0, 20.0, 32), (3.0, 50.0, 64), (3.0, 100.0, 128), (3.0, 1000.0, 128)):
        v = synth.orbit_view(r, 0.7, 0.4, 64, 64, 2.0, 4.0, f=f)
        i = fn.lod_select(ks, (-1.0,) * 3, (1.0,) * 3, v.K, v.c2w, 1.0)
        assert ks[i] == expect, (f, ks[i])
        sig, u, beta = levels[ks[i]]
        gpu = G.render_gpu(G.make_cache(sig, u, beta), v, 96, 1e-4)
        res = G.oracle_render(G.oracle_scene(sig, u, beta), v, 96, 1e-4)
        err, failing, _ = G.compare(gpu, res, G.PARITY_TOL)
        assert failing == 0, (ks[i], err)
