"""FP64 CPU oracle for FastNeRF's cached render -- TEST INFRASTRUCTURE ONLY.

The arithmetic lives in ``fastnerf_oracle.c`` (plain C, double precision, one
thread); this module only marshals numpy arrays into it through ctypes. Only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it. It shares no code with the HIP library and never imports it.

Paper passages: Sec. 3.1 Eq. 1 (quadrature), Sec. 3.2 Eq. 5 (colour as the
inner product of beta with the deep radiance map), Sec. 3.3 (the two caches),
Sec. 4 (rays per pixel, nearest position lookup, interpolated direction lookup),
supplementary S3 (termination). The readings taken where the paper is silent
are listed in the C source header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
MAXCAND = 32
HIT, AMBIG, UNCHECKED = 1, 2, 4

# Default admissibility bands (reading R13): a sample within 1e-3 voxel of a
# voxel face (but not on it) may take either voxel (FP32 grid coordinates are
# good to about 1.3e-4 voxel at k = 768); a stop point within 1e-3 of ln(1/eps)
# in optical depth may be taken or not; nearest direction cells within 1e-5 rad.
DEFAULT_TOL = (1e-3, 1e-5, 1e-3)
ON_FACE = 1e-9  # a grid coordinate this close to a face lies on it (reading R6b)


def build(verbose: bool = False) -> str:
    """Compiles the oracle with gcc (strict IEEE double, no contraction)."""
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-pthread",
           "-ffp-contract=off", "-fno-fast-math", "-o", LIB_PATH + ".tmp",
           os.path.join(_HERE, "fastnerf_oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Scene(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("D", ctypes.c_int32), ("l", ctypes.c_int32),
                ("bmin", ctypes.c_double * 3), ("bmax", ctypes.c_double * 3),
                ("pos_linear", ctypes.c_int32), ("dir_linear", ctypes.c_int32),
                ("in_box", ctypes.c_int32), ("bg", ctypes.c_double * 3),
                ("sigma", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("sb", ctypes.c_int32), ("slot", ctypes.c_void_p),
                ("ssigma", ctypes.c_void_p), ("su", ctypes.c_void_p),
                ("beta", ctypes.c_void_p),
                ("ob", ctypes.c_int32), ("occ", ctypes.c_void_p)]


class _View(ctypes.Structure):
    _fields_ = [("K", ctypes.c_double * 9), ("c2w", ctypes.c_double * 12),
                ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("near", ctypes.c_double), ("far", ctypes.c_double),
                ("N", ctypes.c_int32), ("eps", ctypes.c_double)]


class _Tol(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("gamma_dir", ctypes.c_double),
                ("tau_band", ctypes.c_double), ("max_choice", ctypes.c_int32)]


class _Counts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("rays", "hit", "samples", "occ_samples", "nonzero_samples",
                 "ambiguous_pixels", "unchecked_pixels")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        L.orc_render.argtypes = [P(_Scene), P(_View), P(_Tol), ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p, P(_Counts)]
        L.orc_render.restype = ctypes.c_int
        L.orc_render_mt.argtypes = L.orc_render.argtypes + [ctypes.c_int32]
        L.orc_render_mt.restype = ctypes.c_int
        L.orc_pixel_ray.argtypes = [P(_View), ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_interval.argtypes = [P(_Scene), P(_View), dp, dp, dp, dp]
        L.orc_interval.restype = ctypes.c_int
        L.orc_lookup_pos.argtypes = [P(_Scene), ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
        L.orc_lookup_dir.argtypes = [P(_Scene), ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p]
        L.orc_trace.argtypes = [P(_Scene), P(_View), ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, dp]
        L.orc_trace.restype = ctypes.c_int
        L.orc_occupancy.argtypes = [P(_Scene), ctypes.c_int32, ctypes.c_void_p]
        L.orc_round_to.argtypes = [ctypes.c_int32, ctypes.c_double]
        L.orc_round_to.restype = ctypes.c_double
        L.orc_e4m3_decode.argtypes = [ctypes.c_uint32]
        L.orc_e4m3_decode.restype = ctypes.c_double
        L.orc_e4m3_encode.argtypes = [ctypes.c_float]
        L.orc_e4m3_encode.restype = ctypes.c_uint32
        L.orc_dequant_cache.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class Scene:
    """A position cache, a direction cache and the lookup/sampling options.

    Dense source: ``sigma`` [k,k,k] and ``u`` [k,k,k,D,3] (x fastest).
    Brick-sparse source: ``sparse=(sb, slot[(k/sb)^3], ssigma[nslot,sb^3],
    su[nslot,sb^3,D,3])``; voxels of absent bricks read as zero.
    ``beta`` is [l,l,D] (theta row, phi column).
    """

    def __init__(self, beta, sigma=None, u=None, *, k=None, bbox=(-1.0, 1.0),
                 pos_linear=False, dir_linear=True, in_box=False, bg=(1.0, 1.0, 1.0),
                 sparse=None, occ_brick=0):
        self.beta = _f32(beta)
        l, l2, D = self.beta.shape
        assert l == l2
        s = _Scene()
        if sparse is None:
            self.sigma = _f32(sigma)
            self.u = _f32(u)
            k = self.sigma.shape[0]
            assert self.sigma.shape == (k, k, k) and self.u.shape == (k, k, k, D, 3)
            s.sigma, s.u = _ptr(self.sigma), _ptr(self.u)
        else:
            sb, slot, ss, su = sparse
            self.slot = np.ascontiguousarray(slot, dtype=np.int32)
            self.ssigma, self.su = _f32(ss), _f32(su)
            assert k is not None and k % sb == 0
            s.sb, s.slot = sb, _ptr(self.slot)
            s.ssigma, s.su = _ptr(self.ssigma), _ptr(self.su)
        s.k, s.D, s.l = k, D, l
        lo, hi = bbox
        lo = np.broadcast_to(np.asarray(lo, dtype=np.float64), (3,))
        hi = np.broadcast_to(np.asarray(hi, dtype=np.float64), (3,))
        s.bmin[:] = list(lo)
        s.bmax[:] = list(hi)
        s.pos_linear, s.dir_linear, s.in_box = int(pos_linear), int(dir_linear), int(in_box)
        s.bg[:] = list(bg)
        s.beta = _ptr(self.beta)
        self.k, self.D, self.l = k, D, l
        self._s = s
        self.occ = None
        if occ_brick:
            nb = (k + occ_brick - 1) // occ_brick
            self.occ = np.zeros(nb ** 3, dtype=np.uint8)
            lib().orc_occupancy(ctypes.byref(s), occ_brick, _ptr(self.occ))
            s.ob, s.occ = occ_brick, _ptr(self.occ)

    @property
    def struct(self):
        return self._s


def _view(K, c2w, H, W, near, far, N, eps):
    v = _View()
    v.K[:] = [float(x) for x in np.asarray(K, dtype=np.float64).ravel()]
    v.c2w[:] = [float(x) for x in np.asarray(c2w, dtype=np.float64).ravel()]
    v.H, v.W, v.near, v.far, v.N, v.eps = int(H), int(W), float(near), float(far), int(N), \
        float(eps)
    return v


def _tol(tol):
    """(gamma, gamma_dir, tau_band[, max_choice]) -> the C struct."""
    t = _Tol()
    t.gamma, t.gamma_dir, t.tau_band = tol[:3]
    t.max_choice = int(tol[3]) if len(tol) > 3 else 0
    return t


def render(scene: Scene, K, c2w, H, W, near, far, N, eps, pix=None, tol=DEFAULT_TOL,
           candidates=True, threads=1):
    """Renders pixels (all when ``pix`` is None). Returns a dict with ``rgba``
    [n,4] (primary result), ``cand`` [n,MAXCAND,4] / ``ncand`` [n] (every
    admissible result), ``env`` [n,2,4] (lower and upper RGBA bounds of every
    admissible result: the hull of the enumerated ones, or interval bounds for
    a pixel with too many ambiguous lookups to enumerate), ``flags`` [n] and
    ``counts`` (dict). ``threads`` > 1 splits the pixel list into that many
    contiguous bands, one thread each (bitwise the same result)."""
    v = _view(K, c2w, H, W, near, far, N, eps)
    if pix is None:
        n, pp = H * W, None
    else:
        pp = np.ascontiguousarray(pix, dtype=np.int64)
        n = pp.size
    rgba = np.zeros((n, 4), dtype=np.float64)
    cand = np.zeros((n, MAXCAND, 4), dtype=np.float64) if candidates else None
    ncand = np.zeros(n, dtype=np.int32) if candidates else None
    flags = np.zeros(n, dtype=np.int32)
    env = np.zeros((n, 2, 4), dtype=np.float64)
    cnt = _Counts()
    t = _tol(tol) if tol is not None else _tol((0.0, 0.0, 0.0))
    args = (ctypes.byref(scene.struct), ctypes.byref(v), ctypes.byref(t), n, _ptr(pp),
            _ptr(rgba), _ptr(cand), _ptr(ncand), _ptr(flags), _ptr(env), ctypes.byref(cnt))
    if threads > 1:
        rc = lib().orc_render_mt(*args, int(threads))
    else:
        rc = lib().orc_render(*args)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    counts = {f: getattr(cnt, f) for f, _ in _Counts._fields_}
    return dict(rgba=rgba, cand=cand, ncand=ncand, flags=flags, env=env, counts=counts)


def pixel_ray(K, c2w, H, W, x, y):
    v = _view(K, c2w, H, W, 0.0, 1.0, 1, 0.0)
    o = (ctypes.c_double * 3)()
    d = (ctypes.c_double * 3)()
    lib().orc_pixel_ray(ctypes.byref(v), float(x), float(y), o, d)
    return np.array(o[:]), np.array(d[:])


def interval(scene: Scene, o, d, near, far):
    v = _view(np.eye(3), np.zeros(12), 1, 1, near, far, 1, 0.0)
    oo = (ctypes.c_double * 3)(*[float(x) for x in o])
    dd = (ctypes.c_double * 3)(*[float(x) for x in d])
    t0, t1 = ctypes.c_double(), ctypes.c_double()
    hit = lib().orc_interval(ctypes.byref(scene.struct), ctypes.byref(v), oo, dd,
                             ctypes.byref(t0), ctypes.byref(t1))
    return bool(hit), t0.value, t1.value


def lookup_pos(scene: Scene, pts):
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    n = pts.shape[0]
    sig = np.zeros(n, dtype=np.float64)
    uu = np.zeros((n, scene.D, 3), dtype=np.float64)
    lib().orc_lookup_pos(ctypes.byref(scene.struct), n, _ptr(pts), _ptr(sig), _ptr(uu))
    return sig, uu


def lookup_dir(scene: Scene, dirs):
    dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    n = dirs.shape[0]
    beta = np.zeros((n, scene.D), dtype=np.float64)
    lib().orc_lookup_dir(ctypes.byref(scene.struct), n, _ptr(dirs), _ptr(beta))
    return beta


def trace(scene: Scene, K, c2w, H, W, near, far, N, x, y):
    """All N samples of pixel (x, y): t, sigma, colour and delta (no termination)."""
    v = _view(K, c2w, H, W, near, far, N, 0.0)
    t = np.zeros(N)
    sig = np.zeros(N)
    rgb = np.zeros((N, 3))
    dl = ctypes.c_double()
    n = lib().orc_trace(ctypes.byref(scene.struct), ctypes.byref(v), x, y, _ptr(t), _ptr(sig),
                        _ptr(rgb), ctypes.byref(dl))
    if n <= 0:
        return None
    return t, sig, rgb, dl.value


def round_to(fmt: int, x: float) -> float:
    return lib().orc_round_to(fmt, float(x))


def e4m3_decode(code: int) -> float:
    return lib().orc_e4m3_decode(code)


def e4m3_encode(y: float) -> int:
    return lib().orc_e4m3_encode(y)


FMT = {"f32": 0, "f16": 1, "bf16": 2, "fp8": 3}


def dequant_cache(fmt: str, sigma, u):
    """The oracle's own dequantised copy of a position cache (reading R12)."""
    sigma = _f32(sigma)
    u = _f32(u)
    D = u.shape[-2]
    nvox = sigma.size
    sq = np.empty_like(sigma)
    uq = np.empty_like(u)
    sc = np.zeros(1 + 3 * D, dtype=np.float32)
    lib().orc_dequant_cache(FMT[fmt], nvox, D, _ptr(sigma), _ptr(u), _ptr(sq), _ptr(uq),
                            _ptr(sc))
    return sq, uq, sc


def matches(rgba_gpu, res, tol):
    """Pass protocol: a pixel passes when its result lies within ``tol``
    (max-abs over RGBA) of at least one admissible oracle result; a pixel with
    too many ambiguous lookups to enumerate (UNCHECKED) passes when it lies
    within ``tol`` of the enclosure of all its admissible results. Returns
    (per-pixel error, pass mask)."""
    g = np.asarray(rgba_gpu, dtype=np.float64).reshape(-1, 4)
    cand, ncand = res["cand"], res["ncand"]
    err = np.abs(cand - g[:, None, :]).max(axis=2)
    mask = np.arange(cand.shape[1])[None, :] < ncand[:, None]
    err = np.where(mask, err, np.inf).min(axis=1)
    if "env" in res and "flags" in res:
        unchecked = (res["flags"] & UNCHECKED) != 0
        if unchecked.any():
            lo, hi = res["env"][:, 0], res["env"][:, 1]
            out = np.maximum(np.maximum(lo - g, g - hi), 0.0).max(axis=1)
            err = np.where(unchecked, out, err)
    return err, err <= tol


def matched(rgba_gpu, res):
    """Per pixel, the admissible oracle result nearest (max-abs over RGBA) to
    the given one: the result the pass protocol matches it with."""
    g = np.asarray(rgba_gpu, dtype=np.float64).reshape(-1, 4)
    cand, ncand = res["cand"], res["ncand"]
    err = np.abs(cand - g[:, None, :]).max(axis=2)
    err = np.where(np.arange(cand.shape[1])[None, :] < ncand[:, None], err, np.inf)
    return cand[np.arange(len(g)), err.argmin(axis=1)]
