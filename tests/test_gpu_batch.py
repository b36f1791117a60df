"""Batched SES on the GPU (one pass launch per column layout and one epilogue
launch per iteration for all instances) against the FP64 oracle run on each
instance alone.

Per instance the arithmetic is that of the single-problem path (binary64 for
F32 storage, so the 1e-9 bar of test_gpu_parity applies; binary32 per element
with BF16 storage, at its BF16_STEP bar), so every instance's sequence of
ORACLE outputs, objectives, log-traces and monitor values must match the
oracle's, whatever the other instances of the batch do.
"""
import math

import numpy as np
import pytest

import synth
from oracle import ses as oses

pytestmark = pytest.mark.gpu

TIGHT = 1e-9
BF16_STEP = 2e-4
SEP_SLACK = 5  # iterations per test by which a slow separation may move
# The radius of a solve is the least f over tests of up to thousands of
# iterations; summation order perturbs a trajectory at the rounding level and
# the perturbation grows along a test, so which iteration attains the least f
# (and its value) can differ.  Near OPT f fluctuates along a test at the 1e-4
# level (the least f of the final tests of one oracle search spread by 7e-5),
# so results are compared at SOLVE_TOL, 50x below the solves' eps = 1e-2, and
# the returned centre must realise its radius exactly.
SOLVE_TOL = 2e-4

# (n, d): one and several workgroup shares, ragged last batches, every column
# layout the batched config uses (d in {2, 3, 16, 64}) and a few others, up to
# d = 512 (a record with more column pairs than the batched epilogue's threads)
SHAPES = [(1000, 2), (3001, 3), (517, 16), (2049, 64), (40, 5), (20000, 3), (777, 100), (4500, 64), (2, 7),
          (1301, 33), (600, 512)]


def _instances(shapes, seed, bf16=False):
    pts, vals = [], []
    for k, (n, d) in enumerate(shapes):
        V = synth.ses_ellipsoid(n, d, seed + k).astype(np.float32)
        pts.append(V.ravel())
        vals.append(synth.bf16_to_f32(synth.bf16_round(V)).astype(np.float64) if bf16 else V.astype(np.float64))
    return np.concatenate(pts), vals


def _batch(flat, shapes, **kw):
    import torch
    import paper_2405_09157_amd as scp
    return scp.MWUBatch(torch.from_numpy(flat).cuda(), [s[0] for s in shapes], [s[1] for s in shapes], **kw)


def _compare_steps(b, vals, alphas, Ts, K, tol):
    m = len(vals)
    P = [oses.setup(V) for V in vals]
    for k in range(m):
        assert abs(b.D[k] - P[k].D) <= 1e-12 * P[k].D
    S = [np.zeros(V.shape[1]) for V in vals]
    done = [False] * m
    worst = dict(u=0.0, value=0.0, logC=0.0, f=0.0, ubar=0.0)
    for t in range(1, K + 1):
        infos = b.step(alphas, Ts, 1)
        us = b.vectors(2)
        means = b.vectors(0)
        for k in range(m):
            if done[k]:
                assert infos[k]["outcome_name"] == "separated"
                continue
            eta = math.sqrt(math.log(P[k].r) / Ts[k])
            st = oses.step(P[k], S[k], t - 1, alphas[k], eta)
            info = infos[k]
            worst["u"] = max(worst["u"], np.linalg.norm(np.array(us[k]) - st["u"]) / alphas[k])
            worst["value"] = max(worst["value"], abs(info["value"] - st["value"]) / st["scale"])
            worst["logC"] = max(worst["logC"], abs(info["log_trace"] - st["logC"]) / max(1.0, abs(st["logC"])))
            if st["f_prev"] is not None:
                worst["f"] = max(worst["f"], abs(info["f_last"] - st["f_prev"]) / st["f_prev"])
            if st["separated"]:
                assert info["outcome_name"] == "separated" and info["t_end"] == t, (k, t, info)
                done[k] = True
                continue
            assert info["outcome_name"] == "running", (k, t, info)
            S[k] = st["S"]
            worst["ubar"] = max(worst["ubar"], np.linalg.norm(np.array(means[k]) - st["ubar"]) / alphas[k])
    for key, v in worst.items():
        assert v <= tol, (key, v, worst)
    return done


@pytest.mark.parametrize("rows_per_group", [0, 700])
def test_batch_step_parity_f32(rows_per_group):
    """Every instance of a mixed batch follows its own oracle sequence at the
    1e-9 bar; two instances run far below OPT with a short cap (large step)
    and must separate at the oracle's iteration (8 and 15) while the others
    keep running."""
    import paper_2405_09157_amd as scp
    flat, vals = _instances(SHAPES, 100)
    b = _batch(flat, SHAPES, flags=scp.SCP_MWU_FLAG_NO_EARLY_STOP, chunk=4, rows_per_group=rows_per_group)
    alphas = [0.8 * D for D in b.D]
    Ts = [3000] * len(SHAPES)
    alphas[1], Ts[1] = 0.1 * b.D[1], 100
    alphas[5], Ts[5] = 0.2 * b.D[5], 100
    done = _compare_steps(b, vals, alphas, Ts, 30, TIGHT)
    b.close()
    assert done[1] and done[5]


def test_batch_step_parity_bf16():
    import paper_2405_09157_amd as scp
    flat, vals = _instances(SHAPES, 200, bf16=True)
    b = _batch(flat, SHAPES, flags=scp.SCP_MWU_FLAG_NO_EARLY_STOP, storage="bf16", rows_per_group=900)
    _compare_steps(b, vals, [0.8 * D for D in b.D], [3000] * len(SHAPES), 15, BF16_STEP)
    b.close()


def test_batch_solve_matches_oracle():
    """The alpha searches of a batch, run concurrently, against the oracle's
    solve of each instance alone: the same number of tests, iterations within
    SEP_SLACK per test, radius and certified lower bound within SOLVE_TOL, and
    a centre whose farthest point is at the returned radius.  eps = 1e-2 and a cap of 1500
    iterations per test keep the oracle's share short; the instances' tests
    end in every way (separated, f below alpha, stabilised, cap reached).
    A test that separates after ~1000 iterations does so where the ORACLE
    objective crosses zero very slowly, so the iteration moves by a few under
    any change of summation order (the single-problem path moves too): the
    iteration totals are compared with SEP_SLACK iterations per test."""
    shapes = [(2000, 3), (1500, 2), (1200, 16), (900, 3), (700, 64)]
    flat, vals = _instances(shapes, 300)
    refs = [oses.solve(V, eps=1e-2, t_cap=1500) for V in vals]
    b = _batch(flat, shapes, eps=1e-2, t_cap=1500, chunk=8)
    code, out = b.solve()
    b.close()
    import paper_2405_09157_amd as scp
    assert code == scp.SCP_MWU_OK
    for o, ref, V in zip(out, refs, vals):
        assert o["tests"] == len(ref.steps)
        assert abs(o["iters"] - ref.iters) <= SEP_SLACK * o["tests"], (o["iters"], ref.iters)
        far = np.max(np.linalg.norm(V - np.array(o["center"]), axis=1))
        assert abs(far - o["radius"]) <= 1e-9 * o["radius"]
        assert abs(o["radius"] - ref.radius) / ref.radius <= SOLVE_TOL
        assert abs(o["lower"] - ref.lower) / ref.radius <= SOLVE_TOL
        assert bool(o["converged"]) == ref.converged


def test_batch_solve_matches_single_problem_contexts():
    """Each instance of a batch solve against the single-problem entry point
    on the same points: the same search and results (the two differ only in
    how the pass splits rows over workgroups, i.e. in summation order)."""
    import torch
    import paper_2405_09157_amd as scp
    shapes = [(5000, 64), (3000, 16), (8000, 2), (1000, 3), (2500, 40)]
    flat, vals = _instances(shapes, 400)
    b = _batch(flat, shapes, eps=1e-2, t_cap=3000)
    code, out = b.solve()
    b.close()
    o = 0
    for (n, d), r in zip(shapes, out):
        X = torch.from_numpy(flat[o:o + n * d].reshape(n, d)).cuda()
        o += n * d
        m = scp.MWU(X, "ses", eps=1e-2, t_cap=3000)
        s = m.solve()
        m.close()
        assert r["tests"] == s["tests"]
        assert abs(r["iters"] - s["iters"]) <= SEP_SLACK * r["tests"], (r["iters"], s["iters"])
        assert abs(r["radius"] - s["radius"]) / s["radius"] <= SOLVE_TOL
        assert abs(r["lower"] - s["lower"]) / s["radius"] <= SOLVE_TOL


def test_batch_invalid_descriptors():
    import torch
    import paper_2405_09157_amd as scp
    X = torch.from_numpy(np.random.default_rng(0).standard_normal(3000).astype(np.float32)).cuda()
    for n, d in (([1, 10], [3, 3]), ([10, 10], [3, 600]), ([], [])):
        with pytest.raises((scp.ScpMwuError, ValueError)):
            scp.MWUBatch(X, n, d)
    with pytest.raises(scp.ScpMwuError):
        scp.MWUBatch(X, [10, 10], [3, 3], offset=[0, -3])
    Z = torch.zeros(3000, dtype=torch.float32, device="cuda")
    with pytest.raises(scp.ScpMwuError) as e:
        scp.MWUBatch(Z, [10, 10], [3, 3])      # all points coincide
    assert e.value.code == scp.SCP_MWU_E_INVAL
    Xn = X.clone()
    Xn[35] = float("nan")
    for storage in (None, "bf16"):
        with pytest.raises(scp.ScpMwuError) as e:
            scp.MWUBatch(Xn, [10, 100], [3, 5], storage=storage)
        assert e.value.code == scp.SCP_MWU_E_NUMERIC
    b = scp.MWUBatch(X, [10, 100], [3, 5])
    with pytest.raises(scp.ScpMwuError):
        b.vectors(0)                            # no test yet
    with pytest.raises(scp.ScpMwuError):
        b.step([1.0, -1.0], [10, 10], 1)
    b.close()


# ------------------------------------------------------- k-way alpha search
@pytest.mark.parametrize("n,d,seed,k", [(1500, 3, 500, 2), (1200, 16, 501, 3)])
def test_kway_search_matches_oracle(n, d, seed, k):
    """The k-way search (k tests per round sharing the passes) against the
    oracle's k-way search on the same points: the same number of tests,
    iterations and shared passes within SEP_SLACK per test, radius and lower
    bound within SOLVE_TOL, and a centre that realises the radius."""
    import torch
    import paper_2405_09157_amd as scp
    V = synth.ses_ellipsoid(n, d, seed).astype(np.float32)
    V64 = V.astype(np.float64)
    ref = oses.solve_kway(V64, k, eps=1e-2, t_cap=1500)
    with scp.MWUBatch.kway(torch.from_numpy(V).cuda(), k, eps=1e-2, t_cap=1500, chunk=8) as b:
        out = b.solve_kway()
    assert out["code"] == scp.SCP_MWU_OK and out["converged"] == int(ref.converged)
    assert out["tests"] == len(ref.steps)
    assert abs(out["iters"] - ref.iters) <= SEP_SLACK * out["tests"], (out["iters"], ref.iters)
    assert abs(out["passes"] - ref.passes) <= SEP_SLACK * out["tests"], (out["passes"], ref.passes)
    far = np.max(np.linalg.norm(V64 - np.array(out["center"]), axis=1))
    assert abs(far - out["radius"]) <= 1e-9 * out["radius"]
    assert abs(out["radius"] - ref.radius) / ref.radius <= SOLVE_TOL
    assert abs(out["lower"] - ref.lower) / ref.radius <= SOLVE_TOL


def test_kway_search_with_one_slot_is_the_paper_search():
    """k = 1 against the oracle's search of Section 3 (the k-way search with
    one test per round is that search, pinned step for step on the CPU)."""
    import torch
    import paper_2405_09157_amd as scp
    V = synth.ses_ellipsoid(2000, 3, 300).astype(np.float32)
    ref = oses.solve(V.astype(np.float64), eps=1e-2, t_cap=1500)
    with scp.MWUBatch.kway(torch.from_numpy(V).cuda(), 1, eps=1e-2, t_cap=1500) as b:
        out = b.solve_kway()
    assert out["tests"] == len(ref.steps) and out["passes"] == out["iters"]
    assert abs(out["iters"] - ref.iters) <= SEP_SLACK * out["tests"]
    assert abs(out["radius"] - ref.radius) / ref.radius <= SOLVE_TOL


def test_kway_search_needs_one_point_set():
    import torch
    import paper_2405_09157_amd as scp
    X = torch.from_numpy(np.random.default_rng(5).standard_normal(4000).astype(np.float32)).cuda()
    with scp.MWUBatch(X, [100, 100], [3, 3], [0, 300]) as b:
        with pytest.raises(scp.ScpMwuError) as e:
            b.solve_kway()
        assert e.value.code == scp.SCP_MWU_E_INVAL
