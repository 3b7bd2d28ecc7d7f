"""ctypes binding of libfastnerf.so (the C ABI in include/fastnerf.h).

Argument marshalling only: every step of the render runs in the library's HIP
kernels. PyTorch provides device memory (output tensors) and the current HIP
stream. torch is imported before the library is loaded so that the process
holds a single HIP runtime. There is no fallback: if the library is missing or
fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfastnerf.so")

F32, F16, BF16, FP8 = 0, 1, 2, 3
DTYPES = {"f32": F32, "f16": F16, "bf16": BF16, "fp8": FP8}
NEAREST, LINEAR = 0, 1
NEAR_FAR, IN_BOX = 0, 1

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EBUSY", -5: "ECANCELED",
          -6: "ESHUTDOWN", -7: "ETIMEDOUT"}


class FastNeRFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("D", ctypes.c_int32), ("l", ctypes.c_int32),
                ("bbox_min", ctypes.c_float * 3), ("bbox_max", ctypes.c_float * 3),
                ("storage", ctypes.c_int32), ("pos_interp", ctypes.c_int32),
                ("dir_interp", ctypes.c_int32), ("brick", ctypes.c_int32),
                ("sample_mode", ctypes.c_int32), ("background", ctypes.c_float * 3),
                ("sparse", ctypes.c_int32)]


class MlpDesc(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("pos_hidden", ctypes.c_int32),
                ("pos_layers", ctypes.c_int32), ("pos_skip", ctypes.c_int32),
                ("pos_freqs", ctypes.c_int32), ("dir_hidden", ctypes.c_int32),
                ("dir_layers", ctypes.c_int32), ("dir_freqs", ctypes.c_int32)]


# every symbol the header declares: (name, restype, argtypes)
_vp, _i32, _u64, _f32, _i64, _dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64,
                                     ctypes.c_float, ctypes.c_int64, ctypes.c_double)
_pf = ctypes.POINTER(ctypes.c_float)
SYMBOLS = {
    "fastnerf_cache_create": (_i32, [ctypes.POINTER(Desc), _vp, _vp, _vp, _vp, _vp]),
    "fastnerf_cache_create_empty": (_i32, [ctypes.POINTER(Desc), _vp, _vp, _vp]),
    "fastnerf_cache_scan_slab": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "fastnerf_cache_upload_slab": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "fastnerf_cache_finalize": (_i32, [_vp, _vp]),
    "fastnerf_cache_bytes": (_i32, [_vp, ctypes.POINTER(_u64)]),
    "fastnerf_cache_record_bytes": (_i32, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "fastnerf_cache_readback": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "fastnerf_cache_occupancy": (_i32, [_vp, _vp, ctypes.POINTER(_i32)]),
    "fastnerf_cache_skip_distance": (_i32, [_vp, _vp, ctypes.POINTER(_i32)]),
    "fastnerf_cache_destroy": (_i32, [_vp]),
    "fastnerf_render": (_i32, [_vp, _pf, _pf, _i32, _i32, _f32, _f32, _i32, _f32, _vp, _vp]),
    "fastnerf_render_batch": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _f32, _vp,
                                     _vp]),
    "fastnerf_render_noalloc": (_i32, [_vp, _pf, _pf, _i32, _i32, _f32, _f32, _i32, _f32, _vp,
                                       _vp]),
    "fastnerf_set_schedule": (_i32, [_i32]),
    "fastnerf_get_schedule": (_i32, []),
    "fastnerf_debug_lookup": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "fastnerf_model_bytes": (_dbl, [_dbl, _i64, _i64, _i32, _dbl, _dbl, _dbl]),
    "fastnerf_server_create": (_i32, [_vp, _i32, _u64, _i32, _vp]),
    "fastnerf_serve_submit": (_i32, [_vp, _i32, _pf, _pf, _i32, _i32, _f32, _f32, _i32, _f32,
                                     ctypes.POINTER(_u64)]),
    "fastnerf_serve_wait": (_i32, [_vp, _u64, _i64, ctypes.POINTER(_vp),
                                   ctypes.POINTER(_dbl)]),
    "fastnerf_serve_release": (_i32, [_vp, _u64]),
    "fastnerf_serve_cancel": (_i32, [_vp, _u64]),
    "fastnerf_server_stats": (_i32, [_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64),
                                     ctypes.POINTER(_u64)]),
    "fastnerf_server_destroy": (_i32, [_vp]),
    "fastnerf_mlp_create": (_i32, [ctypes.POINTER(MlpDesc), _vp, _vp, _vp]),
    "fastnerf_mlp_param_count": (_i64, [ctypes.POINTER(MlpDesc), _i32]),
    "fastnerf_bake_position": (_i32, [_vp, _i32, _pf, _pf, _i32, _i32, _vp, _vp, _vp]),
    "fastnerf_bake_direction": (_i32, [_vp, _i32, _vp, _vp]),
    "fastnerf_mlp_destroy": (_i32, [_vp]),
    "fastnerf_filter_direction": (_i32, [_vp, _i32, _i32, _f32, _vp, _vp]),
    "fastnerf_lod_select": (_i32, [ctypes.POINTER(_i32), _i32, _pf, _pf, _pf, _pf, _f32]),
    "fastnerf_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Loads the library (building it first only if no build exists)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (one HIP runtime per process: torch's)
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
        for name, (res, args) in SYMBOLS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != 0:
        msg = lib().fastnerf_last_error()
        raise FastNeRFError(status, msg.decode() if msg else "")


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _arr9(a, n):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1))
    assert a.size == n
    return a, a.ctypes.data_as(_pf)


def _ptr(x):
    """Data pointer of a numpy array or a torch tensor (must be contiguous FP32)."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        assert x.is_contiguous()
        return ctypes.c_void_p(x.data_ptr())
    assert x.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(x.ctypes.data)


def make_desc(k, D, l, *, storage="f32", pos_interp=NEAREST, dir_interp=LINEAR, brick=8,
              sample_mode=NEAR_FAR, bbox=(-1.0, 1.0), background=(1.0, 1.0, 1.0), sparse=False):
    d = Desc()
    d.k, d.D, d.l = k, D, l
    lo, hi = bbox
    d.bbox_min[:] = list(np.broadcast_to(np.asarray(lo, np.float32), (3,)))
    d.bbox_max[:] = list(np.broadcast_to(np.asarray(hi, np.float32), (3,)))
    d.storage = DTYPES[storage] if isinstance(storage, str) else int(storage)
    d.pos_interp, d.dir_interp, d.brick, d.sample_mode = pos_interp, dir_interp, brick, sample_mode
    d.background[:] = list(background)
    d.sparse = 1 if sparse else 0
    return d


class Cache:
    """A resident position + direction cache (fastnerf_cache)."""

    def __init__(self, desc: Desc, handle):
        self.desc = desc
        self.handle = handle

    @classmethod
    def create(cls, desc: Desc, sigma, u, beta, stream=None):
        h = ctypes.c_void_p()
        keep = [np.ascontiguousarray(x, dtype=np.float32) if isinstance(x, np.ndarray) else x
                for x in (sigma, u, beta)]
        check(lib().fastnerf_cache_create(ctypes.byref(desc), _ptr(keep[0]), _ptr(keep[1]),
                                          _ptr(keep[2]), _stream(stream), ctypes.byref(h)))
        return cls(desc, h)

    @classmethod
    def create_empty(cls, desc: Desc, beta, stream=None):
        h = ctypes.c_void_p()
        b = np.ascontiguousarray(beta, dtype=np.float32) if isinstance(beta, np.ndarray) else beta
        check(lib().fastnerf_cache_create_empty(ctypes.byref(desc), _ptr(b), _stream(stream),
                                                ctypes.byref(h)))
        return cls(desc, h)

    def scan_slab(self, z0, sigma, u, stream=None):
        check(lib().fastnerf_cache_scan_slab(self.handle, z0, sigma.shape[0], _ptr(sigma),
                                             _ptr(u), _stream(stream)))

    def upload_slab(self, z0, sigma, u, stream=None):
        check(lib().fastnerf_cache_upload_slab(self.handle, z0, sigma.shape[0], _ptr(sigma),
                                               _ptr(u), _stream(stream)))

    def finalize(self, stream=None):
        check(lib().fastnerf_cache_finalize(self.handle, _stream(stream)))

    @property
    def resident_bytes(self):
        v = ctypes.c_uint64()
        check(lib().fastnerf_cache_bytes(self.handle, ctypes.byref(v)))
        return v.value

    @property
    def record_bytes(self):
        s, p = ctypes.c_int32(), ctypes.c_int32()
        check(lib().fastnerf_cache_record_bytes(self.handle, ctypes.byref(s), ctypes.byref(p)))
        return s.value, p.value

    def readback(self, stream=None):
        import torch
        k, D = self.desc.k, self.desc.D
        sig = torch.empty((k, k, k), dtype=torch.float32, device="cuda")
        u = torch.empty((k, k, k, D, 3), dtype=torch.float32, device="cuda")
        sc = np.zeros(1 + 3 * D, np.float32)
        check(lib().fastnerf_cache_readback(self.handle, _ptr(sig), _ptr(u), _ptr(sc),
                                            _stream(stream)))
        return sig, u, sc

    def occupancy(self):
        n = ctypes.c_int32()
        check(lib().fastnerf_cache_occupancy(self.handle, None, ctypes.byref(n)))
        nb = n.value
        words = np.zeros(max(1, (nb ** 3 + 31) // 32), np.uint32)
        check(lib().fastnerf_cache_occupancy(self.handle, _ptr(words), ctypes.byref(n)))
        bits = np.unpackbits(words.view(np.uint8), bitorder="little")[:nb ** 3]
        return bits.reshape(nb, nb, nb).astype(bool)

    def skip_distance(self):
        """Per-brick max-norm distance (in bricks) to the nearest occupied
        brick, capped at 63: uint8 [nb, nb, nb] indexed [z, y, x]."""
        n = ctypes.c_int32()
        check(lib().fastnerf_cache_skip_distance(self.handle, None, ctypes.byref(n)))
        nb = n.value
        d = np.zeros(max(1, nb ** 3), np.uint8)
        check(lib().fastnerf_cache_skip_distance(self.handle, _ptr(d), ctypes.byref(n)))
        return d[:nb ** 3].reshape(nb, nb, nb)

    def destroy(self):
        if self.handle:
            check(lib().fastnerf_cache_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.fastnerf_cache_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def render(cache: Cache, K, c2w, H, W, near, far, N, eps, out=None, stream=None):
    """Renders one view; returns the [H, W, 4] FP32 device tensor (asynchronous)."""
    import torch
    if out is None:
        out = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
    k_, kp = _arr9(K, 9)
    c_, cp = _arr9(c2w, 12)
    check(lib().fastnerf_render(cache.handle, kp, cp, H, W, near, far, N, eps, _ptr(out),
                                _stream(stream)))
    return out


def render_noalloc(cache: Cache, K, c2w, H, W, near, far, N, eps, out, stream=None):
    """fastnerf_render_noalloc: renders one view into the caller's [H, W, 4] FP32
    device tensor with no allocation in the library (asynchronous)."""
    if tuple(out.shape) != (H, W, 4) or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous [H, W, 4] device tensor")
    k_, kp = _arr9(K, 9)
    c_, cp = _arr9(c2w, 12)
    check(lib().fastnerf_render_noalloc(cache.handle, kp, cp, H, W, near, far, N, eps,
                                        _ptr(out), _stream(stream)))
    return out


def render_batch(cache: Cache, views, N, eps, outs=None, stream=None):
    """Renders a list of views (objects with K, c2w, H, W, near, far) in one launch."""
    import torch
    n = len(views)
    K = np.ascontiguousarray(np.stack([np.asarray(v.K, np.float32).reshape(9) for v in views]))
    C = np.ascontiguousarray(np.stack([np.asarray(v.c2w, np.float32).reshape(12)
                                       for v in views]))
    H = np.array([v.H for v in views], np.int32)
    W = np.array([v.W for v in views], np.int32)
    nr = np.array([v.near for v in views], np.float32)
    fr = np.array([v.far for v in views], np.float32)
    if outs is None:
        outs = [torch.empty((v.H, v.W, 4), dtype=torch.float32, device="cuda") for v in views]
    ptrs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    check(lib().fastnerf_render_batch(cache.handle, n, _ptr(K), _ptr(C), _ptr(H), _ptr(W),
                                      _ptr(nr), _ptr(fr), N, eps, ptrs, _stream(stream)))
    return outs


SCHEDULES = {"auto": 0, "tiles": 1, "refill": 2, "wide": 3, "split": 4}


def set_schedule(name: str):
    """Process-wide schedule of fixed-N render launches: "auto", "tiles",
    "refill", "wide" or "split" (see fastnerf_set_schedule)."""
    if name not in SCHEDULES:
        raise ValueError(f"unknown schedule {name!r}")
    check(lib().fastnerf_set_schedule(SCHEDULES[name]))


def get_schedule() -> str:
    return {v: k for k, v in SCHEDULES.items()}[lib().fastnerf_get_schedule()]


def debug_lookup(cache: Cache, pts=None, dirs=None, stream=None):
    """The kernels' own lookups: returns (sigma_u [n,1+3D], beta [n,D]) device tensors."""
    import torch
    D = cache.desc.D
    n = (pts if pts is not None else dirs).shape[0]
    for a in (pts, dirs):
        if a is not None and (tuple(a.shape) != (n, 3) or not a.is_cuda or
                              a.dtype != torch.float32 or not a.is_contiguous()):
            raise ValueError("pts and dirs must be contiguous float32 [n, 3] device tensors "
                             "with the same n")
    su = torch.empty((n, 1 + 3 * D), dtype=torch.float32, device="cuda") if pts is not None \
        else None
    bo = torch.empty((n, D), dtype=torch.float32, device="cuda") if dirs is not None else None
    check(lib().fastnerf_debug_lookup(cache.handle, n, _ptr(pts), _ptr(dirs), _ptr(su),
                                      _ptr(bo), _stream(stream)))
    return su, bo


def model_bytes(alpha, k, l, D, s_sigma, s_uvw, s_beta):
    return lib().fastnerf_model_bytes(alpha, k, l, D, s_sigma, s_uvw, s_beta)


class Server:
    """Continuous-batching render server over resident caches (fastnerf_server)."""

    def __init__(self, caches, arena_bytes, max_inflight=16):
        self.caches = list(caches)  # keep the caches alive while the server runs
        arr = (ctypes.c_void_p * len(self.caches))(*[c.handle.value for c in self.caches])
        h = ctypes.c_void_p()
        check(lib().fastnerf_server_create(arr, len(self.caches), arena_bytes, max_inflight,
                                           ctypes.byref(h)))
        self.handle = h

    def submit(self, scene, K, c2w, H, W, near, far, N, eps):
        """Returns a ticket; raises FastNeRFError (EBUSY, ENOMEM, ...) otherwise."""
        k_, kp = _arr9(K, 9)
        c_, cp = _arr9(c2w, 12)
        t = ctypes.c_uint64()
        check(lib().fastnerf_serve_submit(self.handle, scene, kp, cp, H, W, near, far, N, eps,
                                          ctypes.byref(t)))
        return t.value

    def wait(self, ticket, timeout_us=-1):
        """Returns (device pointer of the H*W*4 floats, latency in ms)."""
        p = ctypes.c_void_p()
        ms = ctypes.c_double()
        check(lib().fastnerf_serve_wait(self.handle, ticket, timeout_us, ctypes.byref(p),
                                        ctypes.byref(ms)))
        return p.value, ms.value

    def result(self, ticket, H, W, timeout_us=-1):
        """Waits, copies the result into a new [H, W, 4] device tensor, releases."""
        import torch
        ptr, ms = self.wait(ticket, timeout_us)
        out = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
        _copy_device(out.data_ptr(), ptr, H * W * 16)
        self.release(ticket)
        return out, ms

    def release(self, ticket):
        check(lib().fastnerf_serve_release(self.handle, ticket))

    def cancel(self, ticket):
        check(lib().fastnerf_serve_cancel(self.handle, ticket))

    def stats(self):
        s, c, m = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        check(lib().fastnerf_server_stats(self.handle, ctypes.byref(s), ctypes.byref(c),
                                          ctypes.byref(m)))
        return dict(steps=s.value, completed=c.value, max_batch=m.value)

    def destroy(self):
        if self.handle:
            check(lib().fastnerf_server_destroy(self.handle))
            self.handle = None


_hip = None


def _copy_device(dst, src, nbytes):
    """Device-to-device copy through the HIP runtime torch already loaded."""
    global _hip
    import torch
    if _hip is None:
        # the runtime torch loaded (same soname): no second HIP runtime in the process
        _hip = ctypes.CDLL("libamdhip64.so.7", mode=os.RTLD_NOLOAD | os.RTLD_GLOBAL)
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    torch.cuda.synchronize()
    rc = _hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, 3)
    if rc != 0:
        raise FastNeRFError(-3, f"hipMemcpy failed ({rc})")


def mlp_desc(spec):
    """MlpDesc from any object with the descriptor's field names (e.g. synth.MlpSpec)."""
    d = MlpDesc()
    for name, _ in MlpDesc._fields_:
        setattr(d, name, int(getattr(spec, name)))
    return d


def _flat(layers):
    return np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(),
                                           np.asarray(b, np.float32).ravel()])
                           for W, b in layers]).astype(np.float32)


class Mlp:
    """Both factorised networks on the device (fastnerf_mlp), for cache bakes."""

    def __init__(self, spec, weights):
        self.desc = mlp_desc(spec)
        self.D = self.desc.D
        pos, dirs = _flat(weights["pos"]), _flat(weights["dir"])
        for arr, which in ((pos, 0), (dirs, 1)):
            n = lib().fastnerf_mlp_param_count(ctypes.byref(self.desc), which)
            if n != arr.size:
                raise FastNeRFError(-1, f"network {which}: {arr.size} parameters, expected {n}")
        h = ctypes.c_void_p()
        check(lib().fastnerf_mlp_create(ctypes.byref(self.desc), _ptr(pos), _ptr(dirs),
                                        ctypes.byref(h)))
        self.handle = h

    def bake_position(self, k, bbox_min, bbox_max, z0, nz, sigma=None, u=None, stream=None):
        """sigma [nz,k,k], u [nz,k,k,D,3] device float32 tensors (new ones if None)."""
        import torch
        if sigma is None:
            sigma = torch.empty((nz, k, k), dtype=torch.float32, device="cuda")
        if u is None:
            u = torch.empty((nz, k, k, self.D, 3), dtype=torch.float32, device="cuda")
        lo, lp = _arr9(bbox_min, 3)
        hi, hp = _arr9(bbox_max, 3)
        check(lib().fastnerf_bake_position(self.handle, k, lp, hp, z0, nz, _ptr(sigma), _ptr(u),
                                           _stream(stream)))
        return sigma, u

    def bake_direction(self, l, beta=None, stream=None):
        """beta [l,l,D] device float32 tensor."""
        import torch
        if beta is None:
            beta = torch.empty((l, l, self.D), dtype=torch.float32, device="cuda")
        check(lib().fastnerf_bake_direction(self.handle, l, _ptr(beta), _stream(stream)))
        return beta

    def destroy(self):
        if self.handle:
            check(lib().fastnerf_mlp_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.fastnerf_mlp_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def filter_direction(beta, sigma, out=None, stream=None):
    """Gaussian-smoothed copy of a device direction table beta [l, l, D]."""
    import torch
    l, D = beta.shape[0], beta.shape[-1]
    if out is None:
        out = torch.empty_like(beta)
    check(lib().fastnerf_filter_direction(_ptr(beta), l, D, float(sigma), _ptr(out),
                                          _stream(stream)))
    return out


def lod_select(ks, bbox_min, bbox_max, K, c2w, ratio=1.0):
    """Index of the level of detail among caches of resolutions ks (-1: bad arguments)."""
    arr = (ctypes.c_int32 * len(ks))(*[int(k) for k in ks])
    lo, lp = _arr9(bbox_min, 3)
    hi, hp = _arr9(bbox_max, 3)
    k_, kp = _arr9(K, 9)
    c_, cp = _arr9(c2w, 12)
    return lib().fastnerf_lod_select(arr, len(ks), lp, hp, kp, cp, float(ratio))
