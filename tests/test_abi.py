"""The C-ABI library loads, exports every symbol the header declares, and
rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fastnerf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fastnerf_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2103_10380_amd import _lib
    return _lib.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2103_10380_amd import _lib
    assert sorted(_lib.SYMBOLS) == _declared()


def test_model_bytes_worked_example(L):
    """Supplementary S4 (second printing): k = l = 1024, D = 8, half floats."""
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "cache_size_s4.json")))
    from paper_2103_10380_amd import model_bytes
    # s_uvw = one (u, v, w) triple of half floats, s_sigma = s_beta = one half float
    pos = model_bytes(1.0, g["k"], g["l"], g["D"], 2, 6, 2) - model_bytes(0.0, g["k"], g["l"],
                                                                          g["D"], 2, 6, 2)
    assert pos == g["position_bytes_per_unit_alpha"]
    assert model_bytes(0.0, g["k"], g["l"], g["D"], 2, 6, 2) == g["direction_bytes"]
    assert model_bytes(0.01, 1024, 1024, 8, 2, 6, 2) == pytest.approx(
        0.01 * g["position_bytes_per_unit_alpha"] + g["direction_bytes"])


def test_bad_descriptors_rejected_without_device(L):
    import paper_2103_10380_amd as fn
    from paper_2103_10380_amd._lib import Desc
    h = ctypes.c_void_p()
    for kw in (dict(k=0), dict(D=0), dict(D=17), dict(l=0), dict(brick=3), dict(brick=16, k=24),
               dict(storage=7),
               # brick-sparse caches: nearest lookups, brick 8, k a multiple of 8
               dict(sparse=True, pos_interp=fn.LINEAR), dict(sparse=True, brick=16),
               dict(sparse=True, brick=0), dict(sparse=True, k=36, brick=4)):
        args = dict(k=kw.pop("k", 32), D=kw.pop("D", 8), l=kw.pop("l", 8))
        d = fn.make_desc(args["k"], args["D"], args["l"], **kw)
        st = L.fastnerf_cache_create_empty(ctypes.byref(d), ctypes.c_void_p(1), None,
                                           ctypes.byref(h))
        assert st == -1, kw
        assert L.fastnerf_last_error()
    d = fn.make_desc(32, 8, 8)
    d.sparse = 2
    assert L.fastnerf_cache_create_empty(ctypes.byref(d), ctypes.c_void_p(1), None,
                                         ctypes.byref(h)) == -1
    st = L.fastnerf_cache_create_empty(None, None, None, ctypes.byref(h))
    assert st == -1
    d = Desc()
    assert L.fastnerf_cache_create_empty(ctypes.byref(d), None, None, ctypes.byref(h)) == -1


def test_null_handles_rejected(L):
    K = (ctypes.c_float * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1)
    C = (ctypes.c_float * 12)()
    assert L.fastnerf_render(None, K, C, 8, 8, 1.0, 2.0, 8, 0.0, ctypes.c_void_p(1), None) == -1
    assert L.fastnerf_cache_destroy(None) == -1
    assert L.fastnerf_cache_finalize(None, None) == -1
    v = ctypes.c_uint64()
    assert L.fastnerf_cache_bytes(None, ctypes.byref(v)) == -1


def test_mlp_descriptors_checked_without_device(L):
    import synth
    from paper_2103_10380_amd import _lib
    d = _lib.mlp_desc(synth.MlpSpec())
    # 60x384 + 4 x 384x384 + 444x384 + 2 x 384x384 + 384x25, plus biases
    n_pos = 60 * 384 + 6 * 384 * 384 + 444 * 384 + 384 * 25 + 8 * 384 + 25
    assert L.fastnerf_mlp_param_count(ctypes.byref(d), 0) == n_pos
    assert L.fastnerf_mlp_param_count(ctypes.byref(d), 1) == 24 * 128 + 3 * 128 * 128 + \
        128 * 8 + 4 * 128 + 8
    assert L.fastnerf_mlp_param_count(ctypes.byref(d), 2) == -1
    w = synth.mlp_weights(synth.MlpSpec())
    assert sum(W.size + b.size for W, b in w["pos"]) == n_pos
    h = ctypes.c_void_p()
    for field, bad in (("D", 0), ("D", 17), ("pos_hidden", 48), ("pos_hidden", 416),
                       ("dir_hidden", 0), ("pos_layers", 0), ("pos_layers", 17),
                       ("pos_skip", 0), ("pos_skip", 8), ("pos_freqs", 11), ("dir_freqs", 0)):
        d = _lib.mlp_desc(synth.MlpSpec())
        setattr(d, field, bad)
        assert L.fastnerf_mlp_param_count(ctypes.byref(d), 0) == -1, field
        assert L.fastnerf_mlp_create(ctypes.byref(d), ctypes.c_void_p(1), ctypes.c_void_p(1),
                                     ctypes.byref(h)) == -1, field
    assert L.fastnerf_mlp_destroy(None) == -1
    assert L.fastnerf_bake_direction(None, 8, None, None) == -1


def test_lod_select_matches_oracle(L):
    """Host-only: the library's level-of-detail choice equals the oracle's on
    random cameras, boxes and level sets."""
    import numpy as np
    import synth
    from oracle import direction as odir
    from paper_2103_10380_amd import _lib
    rng = np.random.default_rng(3)
    for _ in range(200):
        n = int(rng.integers(1, 6))
        ks = list(rng.choice([64, 128, 256, 384, 512, 768, 1024], n, replace=False))
        lo = rng.uniform(-2, 0, 3)
        hi = lo + rng.uniform(0.5, 3, 3)
        v = synth.orbit_view(float(rng.uniform(2, 30)), float(rng.uniform(0, 6)),
                             float(rng.uniform(-1, 1)), 64, 64, 0.1, 50.0,
                             f=float(rng.uniform(20, 2000)))
        ratio = float(rng.uniform(0.1, 4))
        assert _lib.lod_select(ks, lo, hi, v.K, v.c2w, ratio) == \
            odir.lod_select(ks, lo, hi, v.K, v.c2w, ratio)
    v = synth.orbit_view(3.0, 0.0, 0.0, 8, 8, 0.1, 5.0)
    assert _lib.lod_select([], (-1,) * 3, (1,) * 3, v.K, v.c2w) == -1
    assert _lib.lod_select([256, 0], (-1,) * 3, (1,) * 3, v.K, v.c2w) == -1
    assert _lib.lod_select([256], (-1,) * 3, (1,) * 3, v.K, v.c2w, 0.0) == -1
    assert _lib.lod_select([256], (1,) * 3, (1,) * 3, v.K, v.c2w) == -1
    assert L.fastnerf_filter_direction(None, 8, 3, ctypes.c_float(1.0), None, None) == -1
