"""Pins of the oracle's storage codes: bfloat16 (RNE) and OCP FP8 e4m3 with a
per-Gaussian scale, against torch's own casts (a library routine) and the
format's defining values."""

import numpy as np
import pytest
import torch

from oracle import quant


def test_bf16_matches_torch_cast():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(100_000).astype(np.float32),
                        rng.uniform(-1e-3, 1e-3, 10_000).astype(np.float32),
                        np.array([0.0, -0.0, 1.0, 65504.0, 1e-30], np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(quant.bf16_encode(x), want)
    np.testing.assert_array_equal(quant.bf16_decode(want),
                                  torch.from_numpy(want.view(np.int16)).view(torch.bfloat16).float().numpy())


def test_e4m3_defining_values():
    assert quant.e4m3_decode_code(0x7E) == 448.0
    assert quant.e4m3_decode_code(0x01) == 2.0 ** -9
    assert quant.e4m3_decode_code(0x38) == 1.0
    assert quant.e4m3_decode_code(0x08) == 2.0 ** -6
    assert quant.e4m3_decode_code(0xB8) == -1.0
    assert np.isnan(quant.e4m3_decode_code(0x7F)) and np.isnan(quant.e4m3_decode_code(0xFF))


@pytest.mark.skipif(not hasattr(torch, "float8_e4m3fn"), reason="torch without float8_e4m3fn")
def test_e4m3_decode_and_encode_match_torch():
    codes = np.arange(256, dtype=np.uint8)
    t = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    np.testing.assert_array_equal(np.isnan(t), np.isnan(quant.E4M3_TABLE))
    ok = ~np.isnan(t)
    np.testing.assert_array_equal(t[ok], quant.E4M3_TABLE[ok])
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-448, 448, 50_000), rng.standard_normal(50_000) * 0.01,
                        quant.E4M3_TABLE[ok],  # exact values
                        (quant.E4M3_TABLE[1:0x7E] + quant.E4M3_TABLE[2:0x7F]) / 2]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = quant.e4m3_encode(x)
    np.testing.assert_array_equal(got, want)


def test_e4m3_row_scales_and_roundtrip_error():
    rng = np.random.default_rng(2)
    f = rng.standard_normal((200, 64)).astype(np.float32)
    f[3] = 0.0
    codes, s = quant.e4m3_quantize(f)
    assert s[3] == 1.0
    np.testing.assert_allclose(s[:3], np.abs(f[:3]).max(1) / 448.0, rtol=1e-7)
    back = quant.e4m3_dequantize(codes, s)
    # each row's largest entry maps to +-448 exactly
    i = np.abs(f[0]).argmax()
    assert abs(back[0, i]) == pytest.approx(abs(f[0, i]), rel=1e-6)
    # 3 mantissa bits: relative error <= 2^-4 for normal codes
    big = np.abs(f) > 2.0 ** -6 * s[:, None]
    rel = np.abs(back - f)[big] / np.abs(f)[big]
    assert rel.max() <= 2.0 ** -4 + 1e-7
