"""The shared input generators: shapes, seeding and BF16 rounding (pinned to
torch's round-to-nearest-even FP32 -> BF16 conversion)."""
import numpy as np
import torch

import synth


def test_bf16_round_matches_torch():
    g = np.random.Generator(np.random.PCG64(3))
    x = np.concatenate([g.standard_normal(100000).astype(np.float32) * 37,
                        np.array([0.0, -0.0, 1.0, 65504.0, 1e-40, -3.4e38, np.inf, -np.inf], np.float32)])
    # exact ties: low 16 bits = 0x8000
    ties = (g.integers(0, 1 << 15, 1000, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    x = np.concatenate([x, ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    mine = synth.bf16_round(x)
    nan = np.isnan(x)
    assert np.array_equal(mine[~nan], ref[~nan])          # NaN payloads are not compared
    assert np.all(np.isnan(synth.bf16_to_f32(mine[nan])))
    back = synth.bf16_to_f32(ref)
    tb = torch.from_numpy(ref.view(np.int16)).view(torch.bfloat16).float().numpy()
    assert np.array_equal(back[~nan], tb[~nan])


def test_generators_seeded_and_shaped():
    a = synth.ses_gaussian_outliers(5000, 7, 1)
    b = synth.ses_gaussian_outliers(5000, 7, 1)
    assert a.shape == (5000, 7) and np.array_equal(a, b)
    X, u = synth.svm_planted(400, 300, 5, 2)
    assert X.shape == (700, 5) and abs(np.linalg.norm(u) - 1) < 1e-15
    assert np.all(X[:400] @ u >= 0.05) and np.all(X[400:] @ u <= -0.05)
    E = synth.ses_ellipsoid(1000, 3, 4)
    assert E.shape == (1000, 3)


# ---------------------------------------------------------------- FP8 E4M3
def test_fp8_decode_matches_torch_for_every_code():
    import torch
    codes = np.arange(256, dtype=np.uint8)
    mine = synth.fp8_e4m3_decode(codes)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float32).numpy()
    assert np.array_equal(np.isnan(mine), np.isnan(ref))
    assert np.array_equal(mine[~np.isnan(mine)], ref[~np.isnan(ref)])
    assert synth.fp8_e4m3_decode(np.array([0x7E], np.uint8))[0] == synth.FP8_E4M3_MAX


def test_fp8_encode_matches_torch_round_to_nearest_even():
    """torch's FP32 -> float8_e4m3fn conversion (nearest, ties to even) on
    random values of every scale up to the 464 tie and on the ties and
    boundaries themselves."""
    import torch
    r = np.random.default_rng(0)
    v = np.concatenate([r.uniform(-463.9, 463.9, 100000), r.standard_normal(100000) * 0.01,
                        r.standard_normal(50000) * 1e-4,
                        [0.0, -0.0, 448.0, 447.99, 463.99, 2 ** -9, 2 ** -10, 1.5 * 2 ** -10, 2.5 * 2 ** -9,
                         1.0625, 1.1875, 2 ** -6, 2 ** -6 * 0.999, -416.0 - 16.0]]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(synth.fp8_e4m3_encode(v), ref)


def test_fp8_encode_saturates_and_keeps_nan():
    v = np.array([464.0, 1e30, -500.0, np.nan], np.float32)
    c = synth.fp8_e4m3_encode(v)
    assert list(c[:3]) == [0x7E, 0x7E, 0xFE] and (c[3] & 0x7F) == 0x7F


def test_fp8_rows_scale_and_error_bound():
    """Per-row scales put the row's largest magnitude at 448; every stored
    value is within half a code step of the original (2^-4 relative in the
    normal range, 2^-10 * scale among subnormals)."""
    X = synth.ses_gaussian_outliers(2000, 37, 3, dtype=np.float32)
    X[5] = 0.0
    c, s = synth.fp8_rows(X)
    assert c.dtype == np.uint8 and s.dtype == np.float32 and s[5] == 1.0
    dec = synth.fp8_e4m3_decode(c).astype(np.float64)
    nz = np.max(np.abs(X), axis=1) > 0
    assert np.all(np.max(np.abs(dec[nz]), axis=1) == synth.FP8_E4M3_MAX)
    Xt = synth.fp8_values(c, s)
    err = np.abs(Xt - X)
    bound = np.maximum(2.0 ** -4 * np.abs(X), 2.0 ** -10 * s[:, None].astype(np.float64))
    assert np.all(err <= bound * (1 + 1e-6))
