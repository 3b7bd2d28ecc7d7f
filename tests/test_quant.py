"""Pins of the oracle's storage formats against library conversions and the
format definitions (reading R12: FP16/BF16 round to nearest even from FP32;
FP8 is OCP E4M3 "fn", round to nearest even, saturating at +-448)."""
import numpy as np
import pytest
import torch

import oracle


def _probe_floats(n=20000, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n) * np.exp2(rng.integers(-30, 20, n))
    bits = rng.integers(0, 2 ** 31, n, dtype=np.uint32).view(np.float32)
    x = np.concatenate([x.astype(np.float32), bits[np.isfinite(bits)]])
    return x


def test_fp16_matches_numpy():
    x = _probe_floats()
    ties = (np.arange(1, 3000, dtype=np.float32) + np.float32(0.5)) * np.float32(2.0 ** -10)
    sub = np.arange(1, 2000, dtype=np.float32) * np.float32(2.0 ** -25)  # subnormal halves
    x = np.concatenate([x, ties, -ties, sub, [65504, 65519.99, 65520, 1e9, -1e9]]).astype(
        np.float32)
    ours = np.array([oracle.round_to(1, float(v)) for v in x])
    ref = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(ours, ref)


def test_bf16_matches_torch():
    x = _probe_floats(seed=1)
    ties = (np.arange(1, 3000, dtype=np.float32) + np.float32(0.5)) * np.float32(2.0 ** -7)
    x = np.concatenate([x, ties, -ties]).astype(np.float32)
    ours = np.array([oracle.round_to(2, float(v)) for v in x])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_e4m3_decode_all_codes_match_torch():
    codes = torch.arange(256, dtype=torch.uint8)
    ref = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    ours = np.array([oracle.e4m3_decode(c) for c in range(256)])
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan) and nan.sum() == 2  # S.1111.111 only
    assert np.array_equal(ours[~nan], ref[~nan])
    assert ours[0x7E] == 448.0 and ours[0x01] == 2.0 ** -9 and ours[0x08] == 2.0 ** -6


def test_e4m3_encode_matches_torch_in_range():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.uniform(-463.9, 463.9, 20000),
                        rng.standard_normal(20000) * np.exp2(rng.integers(-12, 6, 20000))]
                       ).astype(np.float32)
    mids = []  # exact midpoints between neighbouring codes: ties to even
    vals = sorted({oracle.e4m3_decode(c) for c in range(0x7F)})
    for a, b in zip(vals[:-1], vals[1:]):
        mids.append((a + b) / 2)
    x = np.concatenate([x, np.array(mids, np.float32), -np.array(mids, np.float32)])
    ours = np.array([oracle.e4m3_encode(float(v)) for v in x], dtype=np.uint8)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)


def test_e4m3_saturates():
    for y, code in [(448.0, 0x7E), (449.0, 0x7E), (463.9, 0x7E), (464.0, 0x7E), (480.0, 0x7E),
                    (1e30, 0x7E), (-1e30, 0xFE), (float("inf"), 0x7E)]:
        assert oracle.e4m3_encode(y) == code, y
    assert oracle.e4m3_encode(0.0) == 0x00 and oracle.e4m3_encode(-0.0) == 0x80
    assert oracle.e4m3_encode(2.0 ** -10) == 0x00          # half of the smallest subnormal
    assert oracle.e4m3_encode(3 * 2.0 ** -10) == 0x02      # 1.5 ulp -> even (2 ulp)


@pytest.mark.parametrize("fmt,bound", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_dequant_cache_relative_error(fmt, bound):
    rng = np.random.default_rng(3)
    sig = rng.uniform(0, 50, (4, 4, 4)).astype(np.float32)
    u = rng.uniform(-1, 1, (4, 4, 4, 3, 3)).astype(np.float32)
    sq, uq, sc = oracle.dequant_cache(fmt, sig, u)
    assert np.all(sc == 1)
    assert np.all(np.abs(sq - sig) <= bound * np.abs(sig))
    assert np.all(np.abs(uq - u) <= bound * np.abs(u))


def test_dequant_cache_e4m3_scales():
    rng = np.random.default_rng(4)
    D = 2
    sig = rng.uniform(0, 37, (5, 5, 5)).astype(np.float32)
    u = (rng.uniform(-1, 1, (5, 5, 5, D, 3)) * np.array([1, 0.5, 0.25])).astype(np.float32)
    u[..., 1, 2] = 0.0  # an all-zero channel keeps scale 1
    sq, uq, sc = oracle.dequant_cache("fp8", sig, u)
    amax = np.concatenate([[np.abs(sig).max()], np.abs(u).reshape(-1, 3 * D).max(0)])
    expect = np.where(amax > 0, (amax / np.float32(448)).astype(np.float32), 1).astype(
        np.float32)
    assert np.array_equal(sc, expect)
    # absmax maps to the largest code, so every value is within half a step of
    # its binade: |x - q| <= 2^-4 |x| for normals, <= 2^-10 s below 2^-6 s
    for x, q, s in [(sig.ravel(), sq.ravel(), sc[0])] + [
            (u.reshape(-1, 3 * D)[:, j], uq.reshape(-1, 3 * D)[:, j], sc[1 + j])
            for j in range(3 * D)]:
        err = np.abs(x.astype(np.float64) - q)
        assert np.all(err <= np.maximum(2.0 ** -4 * np.abs(x), 2.0 ** -10 * s) * (1 + 1e-6))
    assert np.all(uq[..., 1, 2] == 0)
