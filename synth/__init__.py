"""Seeded synthetic inputs for FastNeRF's cached render.

This module serves both the HIP library and the oracle. It draws random scene
parameters with numpy (PCG64, fixed draw order: primitives, radiance fields,
direction fields; cameras come from their own generators) and evaluates the
fields at voxel centres and direction-cell centres. It holds none of the
rendering arithmetic: no rays, no lookups, no compositing.

Recipe (stands in for the paper's trained caches of the NeRF synthetic and LLFF
scenes, which are not available):

* density: a union of solid ellipsoids and thin ellipsoidal shells, each with a
  constant density drawn from U(5, 50); sigma is the maximum over the
  primitives containing a voxel centre, 0 elsewhere, and 0 in a 2-voxel margin
  at the box faces. Centres ~ U[-0.5, 0.5]^3, semi-axes ~ U[0.1, 0.35]^3 times a
  global factor (found by bisection when a target occupancy is given),
  rotations from normalised Gaussian quaternions; shells keep the normalised
  radius band [1 - w, 1] with w giving about 2 voxels of thickness.
* radiance map: each of the 3D channels is a normalised sum of 4 sinusoids
  a_f sin(pi f <n_f, x> + psi_f) / sum a_f with a ~ U(0.5, 1), n a random unit
  vector and psi ~ U(0, 2 pi), so values lie in [-1, 1].
* direction weights: logits 3 sum_f b_f sin(pi f <m_f, w> + chi_f) / sum b_f of
  the unit direction w at each cell centre, softmax over the D components.
* cameras: on a sphere of radius r looking at the origin with +z up, OpenCV
  axes (columns right, down, forward, eye), pinhole focal 1.2 W, principal
  point at the image centre.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class SceneSpec:
    k: int
    D: int = 8
    l: int = 64
    n_ellipsoids: int = 6
    n_shells: int = 0
    seed: int = 0
    occupancy: tuple | None = None   # (lo, hi) target voxel occupancy
    margin: int = 2                  # empty voxels kept at every box face
    bbox: tuple = (-1.0, 1.0)


@dataclasses.dataclass
class SceneParams:
    spec: SceneSpec
    centres: np.ndarray      # [P,3]
    axes: np.ndarray         # [P,3] semi-axes (after the global factor)
    rot: np.ndarray          # [P,3,3] columns = principal axes in world space
    dens: np.ndarray         # [P]
    shell_w: np.ndarray      # [P] 0 for solids
    ua: np.ndarray           # [3D,4]
    un: np.ndarray           # [3D,4,3]
    upsi: np.ndarray         # [3D,4]
    bb: np.ndarray           # [D,4]
    bm: np.ndarray           # [D,4,3]
    bchi: np.ndarray         # [D,4]
    factor: float = 1.0


def _unit(rng, shape):
    v = rng.standard_normal(shape + (3,))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _quat_rot(q):
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def draw(spec: SceneSpec) -> SceneParams:
    rng = np.random.default_rng(spec.seed)
    P = spec.n_ellipsoids + spec.n_shells
    centres = rng.uniform(-0.5, 0.5, (P, 3))
    axes = rng.uniform(0.1, 0.35, (P, 3))
    rot = np.stack([_quat_rot(rng.standard_normal(4)) for _ in range(P)]) if P else \
        np.zeros((0, 3, 3))
    dens = rng.uniform(5.0, 50.0, P)
    is_shell = np.zeros(P, dtype=bool)
    is_shell[spec.n_ellipsoids:] = True
    C = 3 * spec.D
    ua = rng.uniform(0.5, 1.0, (C, 4))
    un = _unit(rng, (C, 4))
    upsi = rng.uniform(0.0, 2 * math.pi, (C, 4))
    bb = rng.uniform(0.5, 1.0, (spec.D, 4))
    bm = _unit(rng, (spec.D, 4))
    bchi = rng.uniform(0.0, 2 * math.pi, (spec.D, 4))
    p = SceneParams(spec, centres, axes, rot, dens, np.zeros(P), ua, un, upsi, bb, bm, bchi)
    factor = 1.0
    if spec.occupancy is not None:
        factor = _bisect_factor(p, spec, rng)
    _apply_factor(p, factor)
    return p


def _apply_factor(p: SceneParams, factor: float):
    spec = p.spec
    p.factor = factor
    p.axes = p.axes * factor
    h = (spec.bbox[1] - spec.bbox[0]) / spec.k
    w = np.zeros(len(p.dens))
    shell = np.arange(len(p.dens)) >= spec.n_ellipsoids
    w[shell] = np.minimum(2.0 * h / p.axes[shell].mean(axis=1), 1.0)
    p.shell_w = w


def _inside_np(p: SceneParams, axes, shell_w, x):
    """Density at points x [M,3] (numpy, float64) for given semi-axes."""
    sig = np.zeros(x.shape[0])
    for e in range(len(p.dens)):
        q = (x - p.centres[e]) @ p.rot[e] / axes[e]
        r2 = (q * q).sum(axis=1)
        inside = r2 <= 1.0
        if shell_w[e] > 0:
            inside &= r2 >= (1.0 - shell_w[e]) ** 2
        sig = np.where(inside, np.maximum(sig, p.dens[e]), sig)
    return sig


def _bisect_factor(p: SceneParams, spec: SceneSpec, rng) -> float:
    k, m = spec.k, spec.margin
    lo_b, hi_b = spec.bbox
    h = (hi_b - lo_b) / k
    idx = rng.integers(0, k, (1 << 16, 3))
    x = lo_b + (idx + 0.5) * h
    keep = np.all((idx >= m) & (idx < k - m), axis=1)
    target = 0.5 * (spec.occupancy[0] + spec.occupancy[1])
    shell = np.arange(len(p.dens)) >= spec.n_ellipsoids
    a, b = 0.2, 3.0
    for _ in range(20):
        f = 0.5 * (a + b)
        axes = p.axes * f
        w = np.zeros(len(p.dens))
        w[shell] = np.minimum(2.0 * h / axes[shell].mean(axis=1), 1.0)
        occ = np.mean((_inside_np(p, axes, w, x) > 0) & keep)
        if occ < target:
            a = f
        else:
            b = f
    return 0.5 * (a + b)


def _torch():
    import torch
    return torch


def density(p: SceneParams, z0: int, nz: int, device="cpu"):
    """sigma for voxel layers z0..z0+nz-1: torch float32 [nz,k,k] (x fastest)."""
    torch = _torch()
    spec = p.spec
    k, m = spec.k, spec.margin
    lo_b, hi_b = spec.bbox
    h = (hi_b - lo_b) / k
    sig = torch.zeros((nz, k, k), dtype=torch.float32, device=device)
    for e in range(len(p.dens)):
        half = np.sqrt(((p.rot[e] * p.axes[e][None, :]) ** 2).sum(axis=1))
        lo = np.floor((p.centres[e] - half - lo_b) / h - 0.5).astype(int) - 1
        hi = np.ceil((p.centres[e] + half - lo_b) / h - 0.5).astype(int) + 2
        lo = np.maximum(lo, 0)
        hi = np.minimum(hi, k)
        zl, zh = max(lo[2], z0), min(hi[2], z0 + nz)
        if zl >= zh or lo[0] >= hi[0] or lo[1] >= hi[1]:
            continue
        xs = lo_b + (torch.arange(lo[0], hi[0], device=device, dtype=torch.float64) + 0.5) * h
        ys = lo_b + (torch.arange(lo[1], hi[1], device=device, dtype=torch.float64) + 0.5) * h
        zs = lo_b + (torch.arange(zl, zh, device=device, dtype=torch.float64) + 0.5) * h
        Z, Y, X = torch.meshgrid(zs, ys, xs, indexing="ij")
        R = torch.tensor(p.rot[e], dtype=torch.float64, device=device)
        c = p.centres[e]
        dx, dy, dz = X - c[0], Y - c[1], Z - c[2]
        r2 = torch.zeros_like(X)
        for j in range(3):
            qj = (dx * R[0, j] + dy * R[1, j] + dz * R[2, j]) / float(p.axes[e][j])
            r2 = r2 + qj * qj
        inside = r2 <= 1.0
        if p.shell_w[e] > 0:
            inside &= r2 >= (1.0 - float(p.shell_w[e])) ** 2
        blk = sig[zl - z0:zh - z0, lo[1]:hi[1], lo[0]:hi[0]]
        blk.copy_(torch.where(inside, torch.clamp(blk, min=float(p.dens[e])), blk))
    # empty margin at the box faces
    zi = torch.arange(z0, z0 + nz, device=device)
    sig[(zi < m) | (zi >= k - m)] = 0.0
    sig[:, :m, :] = 0.0
    sig[:, k - m:, :] = 0.0
    sig[:, :, :m] = 0.0
    sig[:, :, k - m:] = 0.0
    return sig


def radiance(p: SceneParams, z0: int, nz: int, device="cpu", chunk=1 << 20):
    """Deep radiance map u for layers z0..z0+nz-1: torch float32 [nz,k,k,D,3]."""
    torch = _torch()
    spec = p.spec
    k, D = spec.k, spec.D
    lo_b, hi_b = spec.bbox
    h = (hi_b - lo_b) / k
    C = 3 * D
    freq = np.arange(1, 5, dtype=np.float64)
    Nm = (math.pi * freq[None, :, None] * p.un).reshape(C * 4, 3)
    Nm = torch.tensor(Nm, dtype=torch.float32, device=device)
    psi = torch.tensor(p.upsi.reshape(C * 4), dtype=torch.float32, device=device)
    A = p.ua / p.ua.sum(axis=1, keepdims=True)
    Wm = np.zeros((C * 4, C))
    for c in range(C):
        Wm[4 * c:4 * c + 4, c] = A[c]
    Wm = torch.tensor(Wm, dtype=torch.float32, device=device)
    out = torch.empty((nz * k * k, C), dtype=torch.float32, device=device)
    coords = lo_b + (torch.arange(k, device=device, dtype=torch.float32) + 0.5) * h
    zc = lo_b + (torch.arange(z0, z0 + nz, device=device, dtype=torch.float32) + 0.5) * h
    Z, Y, X = torch.meshgrid(zc, coords, coords, indexing="ij")
    pts = torch.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], dim=1)
    for s in range(0, pts.shape[0], chunk):
        ph = pts[s:s + chunk] @ Nm.T + psi
        out[s:s + chunk] = torch.sin(ph) @ Wm
    return out.reshape(nz, k, k, D, 3)


def beta_table(p: SceneParams):
    """Direction weights at cell centres: numpy float32 [l,l,D] (theta row, phi column)."""
    spec = p.spec
    l, D = spec.l, spec.D
    th = (np.arange(l) + 0.5) * math.pi / l
    ph = (np.arange(l) + 0.5) * 2 * math.pi / l
    T, Ph = np.meshgrid(th, ph, indexing="ij")
    w = np.stack([np.sin(T) * np.cos(Ph), np.sin(T) * np.sin(Ph), np.cos(T)], axis=-1)
    z = np.zeros((l, l, D))
    for d in range(D):
        acc = np.zeros((l, l))
        for f in range(4):
            acc += p.bb[d, f] * np.sin(math.pi * (f + 1) * (w @ p.bm[d, f]) + p.bchi[d, f])
        z[..., d] = 3.0 * acc / p.bb[d].sum()
    z -= z.max(axis=-1, keepdims=True)
    e = np.exp(z)
    return (e / e.sum(axis=-1, keepdims=True)).astype(np.float32)


def scene_arrays(spec: SceneSpec, device="cpu"):
    """Dense (sigma [k,k,k], u [k,k,k,D,3], beta [l,l,D]) as numpy float32."""
    p = draw(spec)
    sig = density(p, 0, spec.k, device).cpu().numpy()
    u = radiance(p, 0, spec.k, device).cpu().numpy()
    return sig, u, beta_table(p), p


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


# --------------------------------------------------------------------------- cameras

def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)):
    """3x4 camera-to-world with OpenCV axes: columns right, down, forward, eye."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r /= np.linalg.norm(r)
    dn = np.cross(f, r)
    return np.stack([r, dn, f, eye], axis=1)


def orbit_eye(r, az, el):
    return (r * math.cos(el) * math.cos(az), r * math.cos(el) * math.sin(az), r * math.sin(el))


def intrinsics(W, H, f=None):
    f = 1.2 * W if f is None else f
    return np.array([[f, 0.0, W / 2.0], [0.0, f, H / 2.0], [0.0, 0.0, 1.0]])


@dataclasses.dataclass
class View:
    K: np.ndarray
    c2w: np.ndarray
    H: int
    W: int
    near: float
    far: float


def orbit_view(r, az, el, W, H, near, far, f=None):
    return View(intrinsics(W, H, f), look_at(orbit_eye(r, az, el)), H, W, near, far)


def random_views(n, seed, resolutions, r_range, el_range, near, far):
    """n views at random poses and resolutions drawn uniformly from a list."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        W, H = resolutions[rng.integers(len(resolutions))]
        r = rng.uniform(*r_range)
        az = rng.uniform(0.0, 2 * math.pi)
        el = rng.uniform(*el_range)
        out.append(orbit_view(r, az, el, W, H, near, far))
    return out


# ------------------------------------------------------------------ brick-sparse copies

def brick_sparse_slab(sig_slab, u_slab, sb):
    """Bricks of one slab of sb layers that hold any sigma > 0.

    Returns (brick indices within the slab's brick layer, sigma [n,sb^3],
    u [n,sb^3,D,3]) as numpy; brick-local order is x fastest.
    """
    torch = _torch()
    nz, k, _ = sig_slab.shape
    assert nz == sb and k % sb == 0
    nb = k // sb
    s = sig_slab.reshape(sb, nb, sb, nb, sb).permute(1, 3, 0, 2, 4)  # by,bx,z,y,x
    occ = (s.reshape(nb * nb, -1) > 0).any(dim=1)
    idx = torch.nonzero(occ).flatten()
    D = u_slab.shape[-2]
    uu = u_slab.reshape(sb, nb, sb, nb, sb, D, 3).permute(1, 3, 0, 2, 4, 5, 6)
    ss = s.reshape(nb * nb, sb ** 3)[idx]
    us = uu.reshape(nb * nb, sb ** 3, D, 3)[idx]
    return idx.cpu().numpy(), ss.cpu().numpy(), us.cpu().numpy()


def brick_sparse(p: SceneParams, sb: int, device="cpu", on_slab=None):
    """Brick-sparse copy of a whole scene, generated layer by layer.

    Returns (slot [(k/sb)^3] int32, sigma [n,sb^3], u [n,sb^3,D,3]); calls
    ``on_slab(z0, sig_slab, u_slab)`` with every dense slab (torch) first.
    """
    k = p.spec.k
    nb = k // sb
    slot = np.full(nb ** 3, -1, dtype=np.int32)
    sl, ul = [], []
    n = 0
    for bz in range(nb):
        z0 = bz * sb
        sig = density(p, z0, sb, device)
        u = radiance(p, z0, sb, device)
        if on_slab is not None:
            on_slab(z0, sig, u)
        idx, ss, us = brick_sparse_slab(sig, u, sb)
        slot[bz * nb * nb + idx] = np.arange(n, n + len(idx), dtype=np.int32)
        n += len(idx)
        sl.append(ss)
        ul.append(us)
        del sig, u
    D = p.spec.D
    ss = np.concatenate(sl) if sl else np.zeros((0, sb ** 3), np.float32)
    us = np.concatenate(ul) if ul else np.zeros((0, sb ** 3, D, 3), np.float32)
    return slot, ss, us


# --------------------------------------------------------------- named workloads

def plain_scene_spec():
    """Plain-method scene: k=128, D=8, l=64, 6 ellipsoids, seed 0."""
    return SceneSpec(k=128, D=8, l=64, n_ellipsoids=6, seed=0)


def plain_view():
    """One 200x200 view at radius 3 (az 0.7, el 0.4 rad), samples in [2, 4]."""
    return orbit_view(3.0, 0.7, 0.4, 200, 200, 2.0, 4.0)


def paper_scene_spec(k=768, seed=1):
    """Paper-scale scene: D=8, l=384, 28 ellipsoids and 12 thin shells scaled to
    7.5-8.5% voxel occupancy."""
    return SceneSpec(k=k, D=8, l=384, n_ellipsoids=28, n_shells=12, seed=seed,
                     occupancy=(0.075, 0.085))


def paper_orbit(n=40, W=800, H=800, r=4.0, el=0.5):
    """n views on an orbit at radius r, elevation el, az = 2 pi v / n + 0.1,
    focal 1.2 W; samples span [0, 100] clipped to the box."""
    return [orbit_view(r, 2 * math.pi * v / n + 0.1, el, W, H, 0.0, 100.0) for v in range(n)]


# --------------------------------------------------------------------------- networks

@dataclasses.dataclass(frozen=True)
class MlpSpec:
    """Shapes of the factorised networks (Sec. 4: an 8-layer, 384-wide position
    network and a 4-layer, 128-wide direction network, Fourier features with
    L = 10 and L = 4 frequencies) and the seed of their random weights."""
    D: int = 8
    pos_hidden: int = 384
    pos_layers: int = 8
    pos_skip: int = 5
    pos_freqs: int = 10
    dir_hidden: int = 128
    dir_layers: int = 4
    dir_freqs: int = 4
    seed: int = 7


def _layer_shapes(n_in, hidden, layers, skip, n_out):
    shapes = []
    for i in range(layers):
        fan_in = n_in if i == 0 else hidden + (n_in if i == skip else 0)
        shapes.append((fan_in, hidden))
    shapes.append((hidden, n_out))
    return shapes


def mlp_shapes(spec: MlpSpec):
    """(pos, dir) lists of weight shapes [fan_in, fan_out], output layer last."""
    pos = _layer_shapes(6 * spec.pos_freqs, spec.pos_hidden, spec.pos_layers, spec.pos_skip,
                        1 + 3 * spec.D)
    dirs = _layer_shapes(6 * spec.dir_freqs, spec.dir_hidden, spec.dir_layers, -1, spec.D)
    return pos, dirs


def mlp_weights(spec: MlpSpec):
    """Random weights of both networks: dict(pos=[(W, b), ...], dir=[...]) as
    float32, W [fan_in, fan_out]. W ~ U(-a, a) with a = sqrt(6 / fan_in) (the
    variance-preserving uniform draw for ReLU layers), rounded to the nearest
    binary16 value so that every consumer sees the same weights; b ~ U(-0.1,
    0.1) in float32. Draw order: position layers, then direction layers."""
    rng = np.random.default_rng(spec.seed)
    out = {}
    for name, shapes in zip(("pos", "dir"), mlp_shapes(spec)):
        layers = []
        for fan_in, fan_out in shapes:
            a = math.sqrt(6.0 / fan_in)
            W = rng.uniform(-a, a, (fan_in, fan_out)).astype(np.float16).astype(np.float32)
            b = rng.uniform(-0.1, 0.1, fan_out).astype(np.float32)
            layers.append((W, b))
        out[name] = layers
    return out
