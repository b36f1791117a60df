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
