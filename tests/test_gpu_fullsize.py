"""Parity at the full workload sizes, in the launch configuration bench.py
times (default grid, one workgroup per compute unit).

The FP64 oracle takes a few seconds per iteration at these sizes, so each
test runs the GPU for a number of iterations, reads its state (the running
sums), and compares the next iteration against one oracle step from that
same state: the ORACLE output, its objective, ln of the trace, and the
monitor value f of the mean -- every output of the iteration.
"""
import math

import numpy as np
import pytest

import synth
from oracle import ses as oses
from oracle import svm as osvm

pytestmark = pytest.mark.gpu

TIGHT = 1e-9


def _ses_case(V32, Vref64, storage, alpha_fn, tol=TIGHT):
    import torch
    import paper_2405_09157_amd as scp
    P = oses.setup(Vref64)
    alpha = alpha_fn(P)
    T = 20000
    eta = math.sqrt(math.log(P.r) / T)
    m = scp.MWU(torch.from_numpy(V32).cuda(), "ses", flags=scp.SCP_MWU_FLAG_NO_EARLY_STOP,
                storage=storage, chunk=64)
    assert abs(m.D - P.D) <= 1e-12 * P.D
    m.step(alpha, T, 37)
    sums, t = m.get_state()
    assert t == 37
    info = m.step(alpha, T, 1)
    u_gpu = np.array(m.vector(2))
    m.close()
    st = oses.step(P, np.array(sums), t, alpha, eta)
    assert np.linalg.norm(u_gpu - st["u"]) / alpha <= tol
    assert abs(info["value"] - st["value"]) / st["scale"] <= tol
    assert abs(info["log_trace"] - st["logC"]) / abs(st["logC"]) <= tol
    assert abs(info["f_last"] - st["f_prev"]) / st["f_prev"] <= tol
    assert (info["outcome_name"] == "separated") == st["separated"]


def test_ses_1m_d100_f32_fullsize():
    V = synth.ses_gaussian_outliers(1_000_000, 100, 0, dtype=np.float32)
    _ses_case(V, V.astype(np.float64), None, lambda P: 0.8 * P.D)


def test_ses_1m_d100_bf16_fullsize():
    V = synth.ses_gaussian_outliers(1_000_000, 100, 0, dtype=np.float32)
    Vq = synth.bf16_to_f32(synth.bf16_round(V)).astype(np.float64)
    # binary32 per-element arithmetic with BF16 storage (bound derived in test_gpu_parity)
    _ses_case(V, Vq, "bf16", lambda P: 0.8 * P.D, tol=2e-4)


def test_ses_1m_d100_fp8_fullsize():
    V = synth.ses_gaussian_outliers(1_000_000, 100, 0, dtype=np.float32)
    codes, scales = synth.fp8_rows(V)
    # binary32 per-element arithmetic, as with BF16 storage (same bound)
    _ses_case(V, synth.fp8_values(codes, scales), "fp8", lambda P: 0.8 * P.D, tol=2e-4)


@pytest.mark.parametrize("storage", [None, "bf16", "fp8"])
def test_svm_500k_d256_fullsize(storage):
    import torch
    import paper_2405_09157_amd as scp
    X, _ = synth.svm_planted(250_000, 250_000, 256, 0, dtype=np.float32)
    if storage is None:
        X64 = X.astype(np.float64)
    elif storage == "bf16":
        X64 = synth.bf16_to_f32(synth.bf16_round(X)).astype(np.float64)
    else:
        X64 = synth.fp8_values(*synth.fp8_rows(X))
    tol = TIGHT  # the SVM pass is binary64 for every storage type
    Pb = osvm.setup(X64, 250_000)
    alpha, T = 0.12, 20000            # near the planted margin
    eta = math.sqrt(math.log(Pb.r) / T)
    m = scp.MWU(torch.from_numpy(X).cuda(), "svm", n_pos=250_000,
                flags=scp.SCP_MWU_FLAG_NO_EARLY_STOP, storage=storage, chunk=64)
    assert abs(m.D - Pb.D) <= 1e-12 * Pb.D
    m.step(alpha, T, 29)
    sums, t = m.get_state()
    info = m.step(alpha, T, 1)
    y = np.array(m.vector(2))
    m.close()
    sums = np.array(sums)
    st = osvm.step(Pb, sums[:256], sums[256], sums[257], t, alpha, eta)
    assert np.linalg.norm(y[:256] - st["w"]) <= tol
    assert abs(y[256] - st["s1"]) <= tol * Pb.D and abs(y[257] - st["s2"]) <= tol * Pb.D
    assert abs(info["value"] - st["value"]) / st["scale"] <= tol
    assert abs(info["log_trace"] - st["logC"]) / max(1.0, abs(st["logC"])) <= tol
    if st["f_prev"] > 0:
        assert abs(info["f_last"] - st["f_prev"]) / st["f_prev"] <= tol
