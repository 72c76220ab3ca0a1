"""Pins for the oracle's number formats (Table 2 and the published format
definitions): exhaustive code round trips, agreement with NumPy / torch casts,
hand-made ties.  CPU only."""
import numpy as np
import pytest
import torch

import oracle as O


def test_unit_roundoffs_table2(orc):
    # Table 2: half 2^-11, single 2^-24, double 2^-53; u = 1 means "drop".
    assert orc.unit_roundoff(O.FP16) == 2.0 ** -11
    assert orc.unit_roundoff(O.FP32) == 2.0 ** -24
    assert orc.unit_roundoff(O.FP64) == 2.0 ** -53
    assert orc.unit_roundoff(O.BF16) == 2.0 ** -8
    assert orc.unit_roundoff(O.FP8) == 2.0 ** -4
    assert orc.unit_roundoff(O.DROP) == 1.0


def test_fp16_all_codes_match_numpy(orc):
    codes = np.arange(1 << 16, dtype=np.uint32)
    ref = codes.astype(np.uint16).view(np.float16).astype(np.float64)
    got = orc.decode(O.FP16, codes)
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    assert np.array_equal(np.isinf(got), np.isinf(ref))
    back = orc.encode(O.FP16, got[fin])
    assert np.array_equal(back, codes[fin])


def test_bf16_all_codes_match_torch(orc):
    codes = np.arange(1 << 16, dtype=np.uint32)
    ref = torch.from_numpy(codes.astype(np.uint16).view(np.int16)).view(torch.bfloat16).double().numpy()
    got = orc.decode(O.BF16, codes)
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])
    back = orc.encode(O.BF16, got[fin])
    assert np.array_equal(back, codes[fin])


def test_fp8_all_codes_match_torch(orc):
    codes = np.arange(256, dtype=np.uint32)
    ref = torch.from_numpy(codes.astype(np.uint8)).view(torch.float8_e4m3fn).double().numpy()
    got = orc.decode(O.FP8, codes)
    fin = np.isfinite(ref)
    assert np.array_equal(got[fin], ref[fin])
    assert np.isnan(got[0x7F]) and np.isnan(got[0xFF])
    assert got[0x7E] == 448.0
    back = orc.encode(O.FP8, got[fin])
    assert np.array_equal(back, codes[fin])


def _samples(rng, n, lo, hi):
    e = rng.uniform(lo, hi, size=n)
    return np.where(rng.random(n) < 0.5, -1, 1) * np.exp2(e) * (1 + rng.random(n))


def test_fp16_rounding_from_double_matches_numpy(orc):
    # NumPy converts float64 -> float16 directly (no float32 intermediate).
    rng = np.random.default_rng(0)
    x = _samples(rng, 200000, -26, 15)
    assert np.array_equal(orc.round_to(O.FP16, x), x.astype(np.float16).astype(np.float64))


def test_fp32_rounding_matches_numpy(orc):
    rng = np.random.default_rng(1)
    x = _samples(rng, 200000, -150, 120)
    assert np.array_equal(orc.round_to(O.FP32, x), x.astype(np.float32).astype(np.float64))


def test_bf16_fp8_rounding_matches_torch_on_fp32_inputs(orc):
    # For inputs that are exactly binary32, torch's float32 -> bf16 / e4m3fn casts
    # are single roundings, so they must agree with the oracle's direct rounding.
    rng = np.random.default_rng(2)
    x = _samples(rng, 100000, -130, 120).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).double().numpy()
    assert np.array_equal(orc.round_to(O.BF16, x.astype(np.float64)), ref)
    y = _samples(rng, 100000, -12, 8).astype(np.float32)
    y = y[np.abs(y) <= 448]
    ref8 = torch.from_numpy(y).to(torch.float8_e4m3fn).double().numpy()
    assert np.array_equal(orc.round_to(O.FP8, y.astype(np.float64)), ref8)


@pytest.mark.parametrize("prec,p", [(O.FP16, 11), (O.BF16, 8), (O.FP8, 4)])
def test_ties_round_to_even_and_no_double_rounding(orc, prec, p):
    one = 1.0
    ulp = 2.0 ** (1 - p)
    # exact tie between 1 and 1+ulp -> even (1.0); tie between 1+ulp and 1+2ulp -> 1+2ulp
    assert orc.round_to(prec, one + ulp / 2)[0] == 1.0
    assert orc.round_to(prec, one + 1.5 * ulp)[0] == 1.0 + 2 * ulp
    # just above a tie by far less than a binary32 ulp: must round up
    # (a float32 intermediate would collapse it onto the tie and round to even)
    assert orc.round_to(prec, one + ulp / 2 + 2.0 ** -40)[0] == 1.0 + ulp
    assert orc.round_to(prec, -(one + ulp / 2 + 2.0 ** -40))[0] == -(1.0 + ulp)


def test_subnormals_kept(orc):
    # smallest fp16 subnormal 2^-24, fp8 e4m3 2^-9
    assert orc.round_to(O.FP16, 2.0 ** -24)[0] == 2.0 ** -24
    assert orc.round_to(O.FP16, 2.0 ** -25)[0] == 0.0  # tie -> even (zero)
    assert orc.round_to(O.FP16, 1.5 * 2.0 ** -25)[0] == 2.0 ** -24
    assert orc.round_to(O.FP8, 3 * 2.0 ** -9)[0] == 3 * 2.0 ** -9
    assert orc.round_to(O.FP8, 2.0 ** -10)[0] == 0.0
