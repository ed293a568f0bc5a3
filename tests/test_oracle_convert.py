"""Pins of the BF16 / FP8-e4m3 conversion oracle."""
import numpy as np
import pytest

import synth
from oracle import convert as cv

torch = pytest.importorskip("torch")


def _values(n=1_000_000):
    x = synth.uniform_operand(77, n).astype(np.float32)
    scale = np.float32(2.0) ** (synth.uniform_operand(78, n) * 20).astype(np.int32).astype(np.float32)
    return (x * scale).astype(np.float32)


def test_bf16_vs_torch():
    x = _values()
    edge = np.array([0.0, -0.0, 1.0, -1.0, 3.4e38, -3.4e38, 1e-40, np.inf, -np.inf,
                     1.00390625, 1.01171875, 1.0078125, 1.0234375], dtype=np.float32)
    x = np.concatenate([x, edge])
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(cv.bf16_rne(x), want)


def test_bf16_ties_to_even():
    # 1 + 2**-8 lies exactly between bf16 1.0 and 1 + 2**-7: rounds to even (1.0)
    assert cv.bf16_rne(np.array([1.00390625], np.float32))[0] == 0x3F80
    # 1 + 3*2**-8 lies between 1+2**-7 (odd) and 1+2**-6 (even): rounds up
    assert cv.bf16_rne(np.array([1.01171875], np.float32))[0] == 0x3F82
    assert np.isnan(cv.bf16_decode(cv.bf16_rne(np.array([np.nan], np.float32))))


def test_e4m3_decode_exhaustive():
    t = cv.E4M3_TABLE
    assert t[0x7E] == 448.0 and t[0xFE] == -448.0
    assert np.isnan(t[0x7F]) and np.isnan(t[0xFF])
    assert t[0x01] == 2.0 ** -9 and t[0x07] == 7 * 2.0 ** -9 and t[0x08] == 2.0 ** -6
    assert t[0x38] == 1.0 and t[0x40] == 2.0
    pos = t[:0x7F]
    assert np.all(np.diff(pos) > 0)
    # against torch's decode of every code
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8).view(torch.float8_e4m3fn)
    td = codes.to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(np.isnan(td), np.isnan(t))
    ok = ~np.isnan(t)
    assert np.array_equal(td[ok], t[ok])


def test_e4m3_encode_vs_torch_in_range():
    x = _values()
    x = np.clip(x, -448, 448).astype(np.float32)
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(cv.e4m3_encode(x), want)


def test_e4m3_midpoints_round_to_even_and_saturate():
    pos = cv.E4M3_TABLE[:0x7F]
    mids = ((pos[:-1] + pos[1:]) / 2).astype(np.float32)
    got = cv.e4m3_encode(mids).astype(np.int64)
    lo = np.arange(0, 0x7E)
    want = np.where(lo % 2 == 0, lo, lo + 1)
    assert np.array_equal(got, want)
    assert cv.e4m3_encode(np.array([449.0, 464.0, 1e9, -1e9], np.float32)).tolist() == [0x7E, 0x7E, 0x7E, 0xFE]


def test_quantize_scale():
    x = synth.uniform_operand(5, 1000)
    q, s = cv.quantize_fp8(x)
    amax = np.abs(x).max()
    assert s == np.float32(448.0) / np.float32(amax)
    d = cv.e4m3_decode(q) / np.float64(s)
    assert np.max(np.abs(d - x)) <= amax * 2 ** -4        # half an e4m3 ulp at the top binade
    assert cv.quantize_fp8(np.zeros(4, np.float32))[1] == 1.0
