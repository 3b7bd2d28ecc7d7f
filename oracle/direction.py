"""FP64 CPU oracle of direction-cache filtering and the level-of-detail
choice -- TEST INFRASTRUCTURE ONLY (only the tests, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it; it shares no code with
the HIP library).

Readings (the paper only allows smoothing the direction cache with a filter
kernel such as a Gaussian, Sec. 4, and compares caches of several resolutions
to levels of detail, Sec. 5):

* filter: a separable Gaussian over the table's cells with standard deviation
  sigma cells, taps |t| <= ceil(3 sigma) with weights exp(-t^2 / (2 sigma^2))
  normalised to sum 1; phi (columns) periodic, theta (rows) clamped to the
  edge rows, as the bilinear lookup clamps theta. sigma = 0 is the identity.
* level of detail: the coarsest cache whose voxel edge (longest box side / k)
  is at most `ratio` times the world footprint of one pixel at the box centre
  (camera-to-centre distance / focal length); the finest if none is.
"""
from __future__ import annotations

import math

import numpy as np


def gaussian_taps(sigma):
    """(radius, weights[2r+1]) of the normalised truncated Gaussian."""
    r = int(math.ceil(3.0 * sigma))
    t = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-t * t / (2.0 * sigma * sigma))
    return r, g / g.sum()


def filter_direction(beta, sigma):
    """beta [l, l, D] (theta row, phi column) smoothed: theta pass, then phi pass."""
    b = np.asarray(beta, dtype=np.float64)
    if sigma == 0:
        return b.copy()
    l = b.shape[0]
    r, g = gaussian_taps(sigma)
    rows = np.zeros_like(b)
    for a in range(-r, r + 1):
        idx = np.clip(np.arange(l) + a, 0, l - 1)
        rows += g[a + r] * b[idx]
    out = np.zeros_like(b)
    for c in range(-r, r + 1):
        idx = (np.arange(l) + c) % l
        out += g[c + r] * rows[:, idx]
    return out


def lod_select(ks, bbox_min, bbox_max, K, c2w, ratio):
    """Index of the chosen level among caches of resolutions ks."""
    lo = np.asarray(bbox_min, np.float64)
    hi = np.asarray(bbox_max, np.float64)
    side = float((hi - lo).max())
    eye = np.asarray(c2w, np.float64).reshape(3, 4)[:, 3]
    footprint = float(np.linalg.norm((lo + hi) / 2 - eye)) / float(np.asarray(K).reshape(-1)[0])
    ok = [i for i, k in enumerate(ks) if side / k <= ratio * footprint]
    if ok:
        return min(ok, key=lambda i: ks[i])
    return max(range(len(ks)), key=lambda i: ks[i])
