"""FP64 CPU oracle of the cache bake -- TEST INFRASTRUCTURE ONLY.

Evaluates FastNeRF's two networks where the caches sample them: the position
network F_pos at every voxel centre of the k^3 grid and the direction network
F_dir at every (theta, phi) cell centre of the l x l grid (Sec. 3.2, Eqs. 3-4;
Sec. 3.3, caching). Plain numpy in float64, one layer after the other. Only
the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; it shares no code with the HIP library.

Readings where the paper is silent (the same in the library):

* Fourier features (supplementary, "Motion smoothness": R -> R^{2L} per input
  coordinate; Sec. 4: the view direction is a 3-D unit vector): feature 6j + a
  is sin(2^j pi x_a) and feature 6j + 3 + a is cos(2^j pi x_a), for frequency
  j = 0..L-1 and coordinate a = 0..2. No raw coordinate is appended.
* "n-layer MLP with h hidden units" (Sec. 4): n fully connected layers of width
  h with ReLU, then a linear output layer. The position network feeds its
  input features again into layer ``skip`` (the layer after the fifth, as in
  NeRF, which FastNeRF trains identically); that layer's weight rows are the
  hidden units first, then the features.
* outputs: sigma = max(raw, 0) (NeRF's density activation); (u, v, w) =
  sigmoid(raw) and beta = softmax(raw) over the D components, so that the
  colour of Eq. 5 is a convex combination of values in [0, 1]. Output column
  0 is sigma, column 1 + 3d + c is component d of channel c.
* sample points: voxel centres bmin + (i + 1/2) h on every axis (the cell
  centres of the cache, reading R6 of the renderer); direction cells at
  theta = (j + 1/2) pi / l, phi = (m + 1/2) 2 pi / l with
  d = (sin theta cos phi, sin theta sin phi, cos theta) (reading R5).
"""
from __future__ import annotations

import numpy as np


def fourier_features(x, L):
    """[n, 3] coordinates -> [n, 6L] features (layout in the module header)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((x.shape[0], 6 * L), dtype=np.float64)
    for j in range(L):
        arg = (2.0 ** j) * np.pi * x
        out[:, 6 * j:6 * j + 3] = np.sin(arg)
        out[:, 6 * j + 3:6 * j + 6] = np.cos(arg)
    return out


def trunk(layers, feats, skip=-1):
    """Hidden layers of a network: ``layers`` is the list of (W, b) without the
    output layer. Returns the last hidden activation [n, h]."""
    f = np.asarray(feats, dtype=np.float64)
    h = f
    for i, (W, b) in enumerate(layers):
        x = np.concatenate([h, f], axis=1) if (i == skip and i > 0) else h
        h = np.maximum(x @ np.asarray(W, np.float64) + np.asarray(b, np.float64), 0.0)
    return h


def network(layers, feats, skip=-1):
    """Raw outputs [n, n_out]: the trunk, then the linear output layer."""
    h = trunk(layers[:-1], feats, skip)
    W, b = layers[-1]
    return h @ np.asarray(W, np.float64) + np.asarray(b, np.float64)


def position_heads(raw, D):
    """sigma [n], u [n, D, 3] from raw position-network outputs."""
    sigma = np.maximum(raw[:, 0], 0.0)
    u = 1.0 / (1.0 + np.exp(-raw[:, 1:1 + 3 * D]))
    return sigma, u.reshape(-1, D, 3)


def direction_head(raw):
    """beta [n, D] = softmax of the raw direction-network outputs."""
    z = raw - raw.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def voxel_centres(k, bbox_min, bbox_max, idx):
    """Centres of voxels idx [n, 3] (x, y, z) of a k^3 grid over the box."""
    lo = np.asarray(bbox_min, np.float64)
    hi = np.asarray(bbox_max, np.float64)
    h = (hi - lo) / k
    return lo + (np.asarray(idx, np.float64) + 0.5) * h


def direction_centres(l, idx):
    """Unit directions of cells idx [n, 2] (theta row j, phi column m)."""
    idx = np.asarray(idx, np.float64)
    th = (idx[:, 0] + 0.5) * np.pi / l
    ph = (idx[:, 1] + 0.5) * 2.0 * np.pi / l
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)


def bake_position(weights, spec, k, bbox_min, bbox_max, idx):
    """sigma [n], u [n, D, 3] of F_pos at the centres of voxels idx [n, 3]."""
    p = voxel_centres(k, bbox_min, bbox_max, idx)
    raw = network(weights["pos"], fourier_features(p, spec.pos_freqs), spec.pos_skip)
    return position_heads(raw, spec.D)


def bake_direction(weights, spec, l, idx):
    """beta [n, D] of F_dir at the centres of direction cells idx [n, 2]."""
    d = direction_centres(l, idx)
    return direction_head(network(weights["dir"], fourier_features(d, spec.dir_freqs)))


def slab_indices(k, z0, nz):
    """Voxel indices (x fastest, then y, then z) of layers z0..z0+nz-1: [nz k k, 3]."""
    z, y, x = np.meshgrid(np.arange(z0, z0 + nz), np.arange(k), np.arange(k), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def grid_indices(l):
    """Direction cells in row-major (theta row, phi column) order: [l l, 2]."""
    j, m = np.meshgrid(np.arange(l), np.arange(l), indexing="ij")
    return np.stack([j.ravel(), m.ravel()], axis=1)
