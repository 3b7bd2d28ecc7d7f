"""Cache bake on the matrix cores against the FP64 oracle (oracle/mlp.py).

Tolerances: the kernel rounds the Fourier features and every hidden activation
to binary16 (unit roundoff 2^-11) and accumulates in FP32. Emulating exactly
that rounding in numpy on 40,000 voxel centres of two random 8 x 384 networks
gives at most 2.3e-3 on sigma (raw outputs up to 4.8), 7.1e-4 on u and 5.3e-4
on beta; the bounds below are four times those."""
import numpy as np
import pytest

import synth
from oracle import mlp

pytestmark = pytest.mark.gpu

SIGMA_TOL = (8e-3, 2e-3)   # |d| <= a + r |sigma|
U_TOL = 3e-3
BETA_TOL = 2.5e-3
BOX = ((-1.0, -1.0, -1.0), (1.0, 1.0, 1.0))


def _net(spec):
    import paper_2103_10380_amd as fn
    w = synth.mlp_weights(spec)
    return fn.Mlp(spec, w), w


def _check_position(spec, w, k, z0, nz, sig, u, idx=None, box=BOX):
    sig = sig.cpu().numpy().reshape(-1)
    u = u.cpu().numpy().reshape(-1, spec.D, 3)
    if idx is None:
        idx = mlp.slab_indices(k, z0, nz)
        rows = np.arange(len(idx))
    else:
        rows = (idx[:, 2] - z0) * k * k + idx[:, 1] * k + idx[:, 0]
    s_ref, u_ref = mlp.bake_position(w, spec, k, box[0], box[1], idx)
    ds = np.abs(sig[rows] - s_ref)
    du = np.abs(u[rows] - u_ref)
    assert np.all(np.isfinite(sig)) and np.all(np.isfinite(u))
    assert np.all(ds <= SIGMA_TOL[0] + SIGMA_TOL[1] * np.abs(s_ref)), ds.max()
    assert du.max() <= U_TOL, du.max()
    return ds.max(), du.max()


def test_bake_position_parity_default_network():
    """8 x 384 with the skip at layer 5, L = 10, D = 8 at every voxel centre of
    k = 21 (9,261 points: 73 workgroups, the last one ragged)."""
    spec = synth.MlpSpec()
    net, w = _net(spec)
    sig, u = net.bake_position(21, *BOX, 0, 21)
    ds, du = _check_position(spec, w, 21, 0, 21, sig, u)
    print(f"sigma err {ds:.2e}, u err {du:.2e}")


@pytest.mark.parametrize("kw", [
    dict(D=1, pos_hidden=32, pos_layers=1, pos_skip=-1, pos_freqs=1),
    dict(D=3, pos_hidden=128, pos_layers=2, pos_skip=1, pos_freqs=4),
    dict(D=16, pos_hidden=256, pos_layers=8, pos_skip=5, pos_freqs=10),
    dict(D=6, pos_hidden=96, pos_layers=4, pos_skip=-1, pos_freqs=7),
])
def test_bake_position_parity_shapes(kw):
    spec = synth.MlpSpec(seed=11, **kw)
    net, w = _net(spec)
    k, box = 12, ((-0.5, -2.0, 0.0), (1.5, 1.0, 0.25))
    sig, u = net.bake_position(k, *box, 3, 7)
    _check_position(spec, w, k, 3, 7, sig, u, box=box)


def test_bake_direction_parity():
    for spec, l in ((synth.MlpSpec(), 37), (synth.MlpSpec(D=16, dir_hidden=384, dir_layers=2,
                                                          dir_freqs=10, seed=3), 20),
                    (synth.MlpSpec(D=1, dir_hidden=32, dir_layers=1, dir_freqs=1, seed=4), 5)):
        net, w = _net(spec)
        beta = net.bake_direction(l).cpu().numpy().reshape(-1, spec.D)
        ref = mlp.bake_direction(w, spec, l, mlp.grid_indices(l))
        err = np.abs(beta - ref).max()
        assert err <= BETA_TOL, (l, err)
        np.testing.assert_allclose(beta.sum(axis=1), 1.0, atol=1e-5)


def test_bake_slab_equals_whole_bitwise():
    """A slab bake gives exactly the rows of the whole-grid bake."""
    import torch
    spec = synth.MlpSpec(seed=9)
    net, _ = _net(spec)
    k = 16
    s_all, u_all = net.bake_position(k, *BOX, 0, k)
    s_sl, u_sl = net.bake_position(k, *BOX, 5, 6)
    torch.cuda.synchronize()
    assert torch.equal(s_sl, s_all[5:11]) and torch.equal(u_sl, u_all[5:11])


def test_bake_paper_scale_sampled():
    """k = 768: four layers of the position grid (2.36M points) and the whole
    l = 384 direction grid, checked on 3,000 sampled outputs each."""
    spec = synth.MlpSpec()
    net, w = _net(spec)
    k, z0, nz = 768, 380, 4
    sig, u = net.bake_position(k, *BOX, z0, nz)
    rng = np.random.default_rng(1)
    idx = np.stack([rng.integers(0, k, 3000), rng.integers(0, k, 3000),
                    rng.integers(z0, z0 + nz, 3000)], axis=1)
    _check_position(spec, w, k, z0, nz, sig, u, idx=idx)
    l = 384
    beta = net.bake_direction(l).cpu().numpy().reshape(-1, spec.D)
    cells = mlp.grid_indices(l)[rng.choice(l * l, 3000, replace=False)]
    ref = mlp.bake_direction(w, spec, l, cells)
    assert np.abs(beta[cells[:, 0] * l + cells[:, 1]] - ref).max() <= BETA_TOL


def test_bake_feeds_cache_build():
    """Baked slabs go straight into a cache (device arrays, slab API); the cache
    reads back exactly the baked values and renders."""
    import torch
    import paper_2103_10380_amd as fn
    spec = synth.MlpSpec(seed=12)
    net, _ = _net(spec)
    k, l = 32, 16
    beta = net.bake_direction(l)
    c = fn.Cache.create_empty(fn.make_desc(k, spec.D, l), beta.cpu().numpy())
    slabs = []
    for z0 in range(0, k, 8):
        s, u = net.bake_position(k, *BOX, z0, 8)
        c.upload_slab(z0, s, u)
        slabs.append((s, u))
    c.finalize()
    s_back, u_back, _ = c.readback()
    torch.cuda.synchronize()
    assert torch.equal(s_back, torch.cat([s for s, _ in slabs]))
    assert torch.equal(u_back, torch.cat([u for _, u in slabs]))
    v = synth.orbit_view(3.0, 0.5, 0.4, 48, 40, 2.0, 4.0)
    img = fn.render(c, v.K, v.c2w, v.H, v.W, v.near, v.far, 64, 1e-4)
    torch.cuda.synchronize()
    assert torch.isfinite(img).all() and float(img[..., 3].max()) > 0.5


def test_bake_errors():
    import paper_2103_10380_amd as fn
    spec = synth.MlpSpec(seed=2)
    net, w = _net(spec)
    with pytest.raises(fn.FastNeRFError):
        net.bake_position(8, *BOX, 6, 3)   # slab past k
    with pytest.raises(fn.FastNeRFError):
        net.bake_position(8, (0, 0, 0), (0, 1, 1), 0, 1)  # empty box
    with pytest.raises(fn.FastNeRFError):  # host output arrays
        net.bake_position(4, *BOX, 0, 4, sigma=np.zeros((4, 4, 4), np.float32),
                          u=np.zeros((4, 4, 4, spec.D, 3), np.float32))
    with pytest.raises(fn.FastNeRFError):
        net.bake_direction(0)
    w2 = dict(w)
    w2["pos"] = w["pos"][:-1]
    with pytest.raises(fn.FastNeRFError):  # parameter count mismatch
        fn.Mlp(spec, w2)
    bad = synth.mlp_weights(spec)
    bad["dir"][0][0][0, 0] = np.nan
    with pytest.raises(fn.FastNeRFError):
        fn.Mlp(spec, bad)
