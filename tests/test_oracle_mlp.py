"""Pins of the bake oracle (oracle/mlp.py) against closed forms, a hand-derived
example and invariants of ReLU networks, so that a dropped term, a swapped
sin/cos, a wrong frequency, a misplaced skip input or a transposed output
column fails here."""
import json
import math
import os

import numpy as np

from oracle import mlp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mlp_tiny.json")


def test_fourier_features_closed_forms():
    L = 4
    f = mlp.fourier_features(np.zeros((1, 3)), L)[0]
    for j in range(L):
        assert np.array_equal(f[6 * j:6 * j + 3], [0, 0, 0])
        assert np.array_equal(f[6 * j + 3:6 * j + 6], [1, 1, 1])
    # x = 1/2 on every axis: sin(2^j pi / 2) = 1, 0, 0, ...; cos = 0, -1, 1, 1, ...
    f = mlp.fourier_features(np.full((1, 3), 0.5), L)[0]
    sin_expect = [1.0, 0.0, 0.0, 0.0]
    cos_expect = [0.0, -1.0, 1.0, 1.0]
    for j in range(L):
        np.testing.assert_allclose(f[6 * j:6 * j + 3], sin_expect[j], atol=1e-15)
        np.testing.assert_allclose(f[6 * j + 3:6 * j + 6], cos_expect[j], atol=1e-15)
    # distinct axes and frequencies: (1/6, 1/4, 1/3)
    f = mlp.fourier_features(np.array([[1 / 6, 1 / 4, 1 / 3]]), 3)[0]
    r2, r3 = math.sqrt(2) / 2, math.sqrt(3) / 2
    np.testing.assert_allclose(f[0:6], [0.5, r2, r3, r3, r2, 0.5], atol=1e-15)
    # j = 2: sin(4 pi x): sin(2pi/3), sin(pi), sin(4pi/3)
    np.testing.assert_allclose(f[12:15], [r3, 0.0, -r3], atol=1e-14)
    np.testing.assert_allclose(f[15:18], [-0.5, -1.0, -0.5], atol=1e-14)


def test_fourier_features_period_two():
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, (50, 3))
    np.testing.assert_allclose(mlp.fourier_features(x + 2.0, 10), mlp.fourier_features(x, 10),
                               atol=1e-11)


def test_hand_derived_network():
    g = json.load(open(GOLDEN))
    layers = [(np.array(l["W"], float), np.array(l["b"], float)) for l in g["layers"]]
    f = np.array(g["features"])
    assert np.array_equal(mlp.trunk(layers[:-1], f, g["skip"]), np.array(g["trunk"]))
    assert np.array_equal(mlp.network(layers, f, g["skip"]), np.array(g["raw"]))


def test_nonnegative_network_is_one_affine_map():
    """With non-negative inputs, weights and biases no ReLU clips, so the
    network is the composition of its affine maps: x (W0 W1 W2) + bias terms,
    the matrices multiplied together first."""
    rng = np.random.default_rng(1)
    Ws = [rng.uniform(0, 1, s) for s in [(6, 5), (5, 7), (7, 3)]]
    bs = [rng.uniform(0, 1, s) for s in (5, 7, 3)]
    x = rng.uniform(0, 1, (20, 6))
    got = mlp.network(list(zip(Ws, bs)), x)
    M = Ws[0] @ Ws[1] @ Ws[2]
    c = (bs[0] @ Ws[1] + bs[1]) @ Ws[2] + bs[2]
    np.testing.assert_allclose(got, x @ M + c, rtol=1e-12)


def test_positive_homogeneity_without_bias():
    """A bias-free ReLU network (skip included) satisfies f(a x) = a f(x), a > 0."""
    rng = np.random.default_rng(2)
    n_in, h = 6, 9
    shapes = [(n_in, h), (h, h), (h + n_in, h), (h, 4)]
    layers = [(rng.normal(size=s), np.zeros(s[1])) for s in shapes]
    x = rng.normal(size=(30, n_in))
    np.testing.assert_allclose(mlp.network(layers, 3.5 * x, skip=2),
                               3.5 * mlp.network(layers, x, skip=2), rtol=1e-12, atol=1e-12)


def test_skip_input_enters_at_its_layer():
    """Zero weights and biases before the skip layer: its input is [0, f], so
    its output is relu(f W_f + b) with W_f the feature rows (after the hidden
    rows)."""
    rng = np.random.default_rng(3)
    n_in, h, skip = 5, 7, 2
    layers = [(np.zeros((n_in, h)), np.zeros(h)), (np.zeros((h, h)), np.zeros(h)),
              (rng.normal(size=(h + n_in, h)), rng.normal(size=h))]
    x = rng.normal(size=(12, n_in))
    got = mlp.trunk(layers, x, skip)
    W = layers[2][0]
    np.testing.assert_allclose(got, np.maximum(x @ W[h:] + layers[2][1], 0.0), rtol=1e-13)


def test_heads():
    D = 4
    t = (np.arange(3 * D) + 1) / (3 * D + 2)
    raw = np.concatenate([[-1.0], np.log(t / (1 - t))])[None, :]
    sigma, u = mlp.position_heads(raw, D)
    assert sigma[0] == 0.0
    np.testing.assert_allclose(u[0], t.reshape(D, 3), rtol=1e-14)  # u[d][c] = column 1 + 3d + c
    sigma, _ = mlp.position_heads(np.array([[2.5] + [0.0] * 3 * D]), D)
    assert sigma[0] == 2.5
    b = mlp.direction_head(np.log(np.array([[1.0, 2.0, 3.0]])))
    np.testing.assert_allclose(b[0], [1 / 6, 2 / 6, 3 / 6], rtol=1e-14)
    z = np.random.default_rng(4).normal(size=(5, 8))
    np.testing.assert_allclose(mlp.direction_head(z + 1000.0), mlp.direction_head(z), rtol=1e-12)
    np.testing.assert_allclose(mlp.direction_head(z).sum(axis=1), 1.0, rtol=1e-14)


def test_zero_output_layer_gives_its_bias():
    """With a zero output layer the bake is its bias through the heads,
    whatever the trunk: sigma = max(b0, 0), u = sigmoid(b), beta = softmax(b)."""
    import synth
    spec = synth.MlpSpec(D=3, pos_hidden=32, pos_layers=3, pos_skip=2, pos_freqs=2,
                         dir_hidden=32, dir_layers=2, dir_freqs=2, seed=5)
    w = synth.mlp_weights(spec)
    bp = np.array([0.7] + list(np.linspace(-2, 2, 9)))
    bd = np.array([0.1, 0.2, 0.3])
    w["pos"][-1] = (np.zeros_like(w["pos"][-1][0]), bp)
    w["dir"][-1] = (np.zeros_like(w["dir"][-1][0]), bd)
    sigma, u = mlp.bake_position(w, spec, 4, (-1, -1, -1), (1, 1, 1), mlp.slab_indices(4, 1, 2))
    assert np.all(sigma == 0.7)
    np.testing.assert_allclose(u, np.broadcast_to((1 / (1 + np.exp(-bp[1:]))).reshape(3, 3),
                                                  u.shape), rtol=1e-14)
    beta = mlp.bake_direction(w, spec, 3, mlp.grid_indices(3))
    e = np.exp(bd)
    np.testing.assert_allclose(beta, np.broadcast_to(e / e.sum(), beta.shape), rtol=1e-14)


def test_sample_points():
    p = mlp.voxel_centres(4, (-1, -1, -1), (1, 1, 1), [[0, 1, 3]])
    np.testing.assert_allclose(p, [[-0.75, -0.25, 0.75]], rtol=0, atol=1e-15)
    p = mlp.voxel_centres(5, (0, -2, 1), (1, 2, 3), [[2, 0, 4]])
    np.testing.assert_allclose(p, [[0.5, -1.6, 2.8]], atol=1e-15)
    # the voxel index of a centre under the nearest rule (the cell that holds
    # the point) is the voxel itself
    k = 7
    idx = mlp.slab_indices(k, 0, k)
    g = (mlp.voxel_centres(k, (-1, -1, -1), (1, 1, 1), idx) + 1) / 2 * k
    assert np.array_equal(np.minimum(np.floor(g), k - 1).astype(int), idx)
    d = mlp.direction_centres(2, [[0, 0]])
    np.testing.assert_allclose(d, [[0.0, math.sqrt(2) / 2, math.sqrt(2) / 2]], atol=1e-15)
    l = 9
    cells = mlp.grid_indices(l)
    d = mlp.direction_centres(l, cells)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, rtol=1e-14)
    th = np.arccos(d[:, 2])
    ph = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2 * np.pi)
    back = np.stack([np.floor(th / np.pi * l), np.floor(ph / (2 * np.pi) * l)], axis=1)
    assert np.array_equal(back.astype(int), cells)


def test_index_orders():
    idx = mlp.slab_indices(5, 2, 3)
    assert idx.shape == (75, 3)
    assert list(idx[0]) == [0, 0, 2] and list(idx[1]) == [1, 0, 2] and list(idx[5]) == [0, 1, 2]
    assert list(idx[25]) == [0, 0, 3]
    g = mlp.grid_indices(4)
    assert list(g[1]) == [0, 1] and list(g[4]) == [1, 0]
