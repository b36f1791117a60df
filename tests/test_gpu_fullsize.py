"""Parity at the full workload sizes, in the launch configuration bench.py
times (default grid, one workgroup per compute unit).

The FP64 oracle takes a few seconds per iteration at these sizes, so each
test runs the GPU for a number of iterations, reads its state (the running
sums), and compares the next iteration against one oracle step from that
same state: the ORACLE output, its objective, ln of the trace, and the
monitor value f of the mean -- every output of the iteration.
"""
import json
import math
import os

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


@pytest.mark.parametrize("rows_per_group", [8192, 16384])
def test_batched_4096_fullsize(rows_per_group):
    """The batched configuration at full size (4,096 instances, 86.7 M points)
    at the workgroup shares the bench's autotuner picks on this workload
    (8192 or 16384 rows per share): after 37 iterations of every
    instance, the next iteration of sampled instances (the largest of each
    dimension and a few seeded others) against one oracle step from that
    instance's state (running sum = mean x t)."""
    import torch
    import paper_2405_09157_amd as scp
    n, d = synth.ses_batch_sizes(4096, 1000, 100_000, [2, 3, 16, 64], 0)
    pts, off = synth.ses_batch_points_device(n, d, 0)
    m = len(n)
    T = 20000
    with scp.MWUBatch(pts, n, d, off, flags=scp.SCP_MWU_FLAG_NO_EARLY_STOP,
                      rows_per_group=rows_per_group) as b:
        alphas = list(b.D)             # the ball at v1 of radius D encloses every point
        b.step(alphas, [T] * m, 37)
        before = b.step(alphas, [T] * m, 0)
        means = b.vectors(0)
        infos = b.step(alphas, [T] * m, 1)
        us = b.vectors(2)
        D = list(b.D)
    sample = {int(np.flatnonzero(d == dd)[np.argmax(n[d == dd])]) for dd in (2, 3, 16, 64)}
    sample |= set(int(k) for k in np.random.default_rng(3).choice(m, 4, replace=False))
    for k in sorted(sample):
        V = pts[int(off[k]):int(off[k]) + int(n[k] * d[k])].reshape(int(n[k]), int(d[k])).cpu().double().numpy()
        P = oses.setup(V)
        assert abs(D[k] - P.D) <= 1e-12 * P.D
        t = before[k]["t"]
        assert t == 37 and infos[k]["outcome_name"] == "running"
        st = oses.step(P, np.array(means[k]) * t, t, alphas[k], math.sqrt(math.log(P.r) / T))
        assert np.linalg.norm(np.array(us[k]) - st["u"]) / alphas[k] <= TIGHT, k
        assert abs(infos[k]["value"] - st["value"]) / st["scale"] <= TIGHT, k
        assert abs(infos[k]["log_trace"] - st["logC"]) / abs(st["logC"]) <= TIGHT, k
        assert abs(infos[k]["f_last"] - st["f_prev"]) / st["f_prev"] <= TIGHT, k


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _grad_fixture(T):
    path = os.path.join(GOLDEN, f"grad_200k_d64_T{T}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written (tests/golden/make_grad_200k_d64.py {T})")
    with open(path) as f:
        return json.load(f)


def _grad_run(Xt, alpha, T, gv=1.0):
    import paper_2405_09157_amd as scp
    with scp.MWU(Xt, "ses", flags=scp.SCP_MWU_FLAG_NO_EARLY_STOP) as m:
        m.step(alpha, T, 0, reset=True)
        return m.backward(gv)


def _grad_points(fx):
    import torch
    V32 = synth.ses_gaussian_outliers(fx["n"], fx["d"], fx["seed"], frac=0.0, dtype=np.float32)
    return V32, torch.from_numpy(V32).cuda()


def test_grad_200k_d64_against_oracle_fixture():
    """The gradient workload's points and alpha (n = 200,000, d = 64, alpha
    the oracle's solved radius, eps = 1e-2) at T = 500 against the FP64
    oracle's own run (tests/golden/grad_200k_d64_T500.json, written by a
    script that calls only the oracle): R within 1e-9; the gradient rows of
    64 seeded rows plus the active row, v1 and D's far row element by element
    within 1e-6 max|g| (the FP32 result bar of the reverse pass); the
    directional derivative sum_ij g_ij z_ij along the seeded N(0, 1)
    direction within 1e-6 sum_ij |g_ij z_ij|.

    T = 500 because the map is reproducible there: perturbing alpha by 1e-13
    (relative) moves R by 1e-14 and the gradient by 6e-9 max|g|, while at
    T = 1000 and 2000 the same perturbation moves the gradient by O(1) and R
    by up to 2.5e-4 (the unrolled iterations amplify rounding where ||W_t||
    is small), so no two implementations agree there (the T = 2000 fixture is
    compared by its radius alone, below).

    Dual weights (eq. (ses_qp) and its dual, Section 5): the optimal radius
    has gradient pi_i (v_i - c*) / R* (Danskin), pi the optimal dual weights.
    The fixture holds that vector at the same rows, with pi from the MWU trace
    weights of iteration T + 1 and c = ubar_T, and the cosine the oracle's
    gradient makes with it; the HIP gradient's cosine with those rows must
    equal the oracle's within 1e-4."""
    fx = _grad_fixture(500)
    V32, X = _grad_points(fx)
    R, g = _grad_run(X, fx["alpha"], fx["T"])
    G = g.cpu().double().numpy()
    assert abs(R - fx["R"]) <= TIGHT * fx["R"], (R, fx["R"])
    rows = np.asarray(fx["rows"])
    G0 = np.asarray(fx["grad_rows"])
    err = np.abs(G[rows] - G0).max()
    assert err <= 1e-6 * fx["max_abs_grad"], (err, fx["max_abs_grad"])
    assert abs(np.abs(G).max() - fx["max_abs_grad"]) <= 1e-6 * fx["max_abs_grad"]
    z = np.random.default_rng(fx["dir_seed"]).standard_normal(G.shape, dtype=np.float32).astype(np.float64)
    dd = float(np.sum(G * z))
    assert abs(dd - fx["dir_deriv"]) <= 1e-6 * float(np.sum(np.abs(G * z))), (dd, fx["dir_deriv"])
    Dk = np.asarray(fx["danskin_rows"])
    cos = float(np.sum(G[rows] * Dk) / (np.linalg.norm(G[rows]) * np.linalg.norm(Dk)))
    assert abs(cos - fx["danskin_cos"]) <= 1e-4, (cos, fx["danskin_cos"])


def test_grad_200k_d64_T2000_radius_against_oracle():
    """The gradient workload itself (T = 2000, alpha the oracle's solved
    radius): the map's value against the oracle's (the T = 2000 fixture)
    within 1e-3 of R.  Rounding decides the trajectory here (a 1e-13 change of
    alpha moves R by up to 2.5e-4 and the gradient by O(1), measured on this
    library), so R is compared at that bar and the gradient by the properties
    that hold for any trajectory: it is finite, and the two rigid-motion
    invariances hold (sum_i g_i = 0; sum_i v_i g_i^T symmetric) to 1e-6 of
    the corresponding sums of magnitudes."""
    fx = _grad_fixture(2000)
    V32, X = _grad_points(fx)
    R, g = _grad_run(X, fx["alpha"], fx["T"])
    assert abs(R - fx["R"]) <= 1e-3 * fx["R"], (R, fx["R"])
    G = g.cpu().double().numpy()
    assert np.all(np.isfinite(G))
    V = V32.astype(np.float64)
    A = np.abs(G)
    assert np.all(np.abs(G.sum(axis=0)) <= 1e-6 * A.sum(axis=0))
    M = V.T @ G
    assert np.all(np.abs(M - M.T) <= 1e-6 * (np.abs(V).T @ A + A.T @ np.abs(V)))


def test_grad_200k_d64_fullsize():
    """The gradient workload's points and alpha at T = 500 (where the map is
    reproducible, above) through the reverse pass, checked by properties that
    hold at any size: the two rigid-motion invariances of R (sum_i g_i = 0;
    sum_i v_i g_i^T symmetric) and the directional derivative along a fixed
    direction against central differences of the same map evaluated by the
    library in binary64 (R returned by the reverse pass on binary64 copies of
    V +- h Delta).  The unrolled map is rough: iterations where ||W_t|| is
    small amplify perturbations, so its derivative is a very local quantity
    and central differences approach it only for small h (on the oracle at
    n = 2000, d = 64, T = 1000 the difference quotient is off by 99% at
    h = 1e-5, 7e-4 at 1e-8 and 4e-5 at 1e-9, where the binary64 rounding of
    R, ~1e-15 R / h, is still far below the slope); hence the steps 1e-8 and
    1e-9 and a 1e-3 bar on the better of the two."""
    import torch
    fx = _grad_fixture(500)
    n, d, T = fx["n"], fx["d"], fx["T"]
    V32, X = _grad_points(fx)
    alpha = fx["alpha"]

    def run(Xt, gv=1.0):
        return _grad_run(Xt, alpha, T, gv)

    R, g = run(X)
    G = g.cpu().double().numpy()
    V = V32.astype(np.float64)
    A = np.abs(G)
    assert np.all(np.abs(G.sum(axis=0)) <= 1e-6 * A.sum(axis=0))
    M = V.T @ G
    assert np.all(np.abs(M - M.T) <= 1e-6 * (np.abs(V).T @ A + A.T @ np.abs(V)))
    # direction: the gradient itself plus a seeded random part, unit norm
    rnd = np.random.default_rng(5).standard_normal((n, d))
    Dl = G / np.linalg.norm(G) + 0.5 * rnd / np.linalg.norm(rnd)
    Dl /= np.linalg.norm(Dl)
    slope = float(np.sum(G * Dl))
    X64 = torch.from_numpy(V).cuda()
    Dt = torch.from_numpy(Dl).cuda()
    errs = []
    for h in (1e-8, 1e-9):
        Rp, _ = run(X64 + h * Dt)
        Rm, _ = run(X64 - h * Dt)
        errs.append(abs((Rp - Rm) / (2 * h) - slope))
    R64, _ = run(X64)
    assert abs(R - R64) <= 1e-12 * R64
    assert min(errs) <= 1e-3 * abs(slope), (errs, slope)
