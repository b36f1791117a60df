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
RESULT = 1e-6
# End-to-end solves are compared where the search path is pinned.  Two things
# unpin it, and the oracle records both per search (oracle/ses.py):
#  * tie_margin, the least relative distance of any decision value
#    (separation, f below alpha, stabilisation) to its threshold: a change of
#    the state moves a decision only where it is that small;
#  * cancel_max, the largest cancellation ratio sum_i ||w_i|| / ||W|| of the
#    ORACLE's weighted sum: where W passes near zero its direction, hence the
#    ORACLE output u, amplifies any rounding difference by that factor, and
#    from there on two correct implementations (two summation orders) follow
#    different trajectories (measured: a d = 3 test drifts from 1e-13 to 1e-2
#    in f within 300 iterations; well-conditioned d = 64 tests stay below
#    1e-9).  Tests that end by separation pass near W = 0.
# Pinned instances (tie_margin >= PINNED, cancel_max <= CANCEL_MAX, chosen by
# the oracle alone) must reproduce the oracle's path exactly: the same tests
# and iteration counts, and radius and lower bound within the 1e-6 result bar.
# Unpinned searches are compared by what both sides certify: each side's
# returned radius is f of its returned centre (an upper bound on OPT) and its
# lower bound comes from separations (a lower bound), so each side's lower
# bound must not exceed the other's radius.
PINNED = 1e-4
CANCEL_MAX = 1e3


def _brackets(out_lower, out_radius, ref):
    assert out_lower <= ref.radius * (1 + 1e-9) and ref.lower <= out_radius * (1 + 1e-9), \
        (out_lower, out_radius, ref.lower, ref.radius)

# (n, d): one and several workgroup shares, ragged last batches, every column
# layout the batched config uses (d in {2, 3, 16, 64}) and a few others, up to
# d = 512 (a record with more column pairs than the batched epilogue's threads)
SHAPES = [(1000, 2), (3001, 3), (517, 16), (2049, 64), (40, 5), (20000, 3), (777, 100), (4500, 64), (2, 7),
          (1301, 33), (600, 512)]


def _instances(shapes, seed, bf16=False):
    """Instances (n, d) with seeds seed + k, or (n, d, seed) with their own."""
    pts, vals = [], []
    for k, shp in enumerate(shapes):
        n, d = shp[0], shp[1]
        V = synth.ses_ellipsoid(n, d, shp[2] if len(shp) > 2 else seed + k).astype(np.float32)
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


def test_batch_solve_matches_oracle_pinned():
    """The alpha searches of a batch, run concurrently, against the oracle's
    solve of each instance alone on pinned instances: the same number of
    tests and iterations, radius and certified lower bound within RESULT, and
    a centre whose farthest point is at the returned radius (eps = 1e-2, a
    cap of 300 iterations per test)."""
    shapes = [(700, 64, 700), (700, 64, 701), (700, 64, 702), (700, 64, 709)]
    flat, vals = _instances(shapes, 0)
    refs = [oses.solve(V, eps=1e-2, t_cap=300) for V in vals]
    for ref in refs:
        assert ref.tie_margin >= PINNED and ref.cancel_max <= CANCEL_MAX
    b = _batch(flat, [s[:2] for s in shapes], eps=1e-2, t_cap=300, chunk=8)
    code, out = b.solve()
    b.close()
    import paper_2405_09157_amd as scp
    assert code == scp.SCP_MWU_OK
    for o, ref, V in zip(out, refs, vals):
        assert o["tests"] == len(ref.steps) and o["iters"] == ref.iters, (o["tests"], o["iters"], ref.iters)
        far = np.max(np.linalg.norm(V - np.array(o["center"]), axis=1))
        assert abs(far - o["radius"]) <= 1e-9 * o["radius"]
        assert abs(o["radius"] - ref.radius) / ref.radius <= RESULT
        assert abs(o["lower"] - ref.lower) / ref.radius <= RESULT
        assert bool(o["converged"]) == ref.converged


def test_batch_solve_brackets_oracle_unpinned():
    """Unpinned searches (tests ending in every way: separated, f below alpha,
    stabilised, cap reached; low dimensions, near-zero W): each instance's
    centre realises its radius, and the GPU's and the oracle's certified
    bounds are consistent (each lower bound at most the other's radius)."""
    shapes = [(2000, 3, 607), (1500, 2, 605), (1200, 16, 612), (900, 3, 608), (700, 64, 602)]
    flat, vals = _instances(shapes, 0)
    refs = [oses.solve(V, eps=1e-2, t_cap=1500) for V in vals]
    outcomes = set(st[2] for ref in refs for st in ref.steps)
    assert outcomes == {oses.SEPARATED, oses.BEAT, oses.STABILIZED, oses.T_REACHED}
    b = _batch(flat, [s[:2] for s in shapes], eps=1e-2, t_cap=1500, chunk=8)
    code, out = b.solve()
    b.close()
    import paper_2405_09157_amd as scp
    assert code == scp.SCP_MWU_OK
    for o, ref, V in zip(out, refs, vals):
        far = np.max(np.linalg.norm(V - np.array(o["center"]), axis=1))
        assert abs(far - o["radius"]) <= 1e-9 * o["radius"]
        assert o["lower"] <= o["radius"]
        _brackets(o["lower"], o["radius"], ref)


def test_batch_solve_matches_single_problem_contexts():
    """Each instance of a batch solve against the single-problem entry point
    on the same points: the same search and results (the two differ only in
    how the pass splits rows over workgroups, i.e. in summation order)."""
    import torch
    import paper_2405_09157_amd as scp
    # pinned instances (tie_margin >= PINNED, cancel_max <= CANCEL_MAX)
    shapes = [(700, 64, 700), (700, 64, 701), (700, 64, 702), (700, 64, 709)]
    flat, vals = _instances(shapes, 0)
    b = _batch(flat, [s[:2] for s in shapes], eps=1e-2, t_cap=300)
    code, out = b.solve()
    b.close()
    o = 0
    for (n, d, _), r in zip(shapes, out):
        X = torch.from_numpy(flat[o:o + n * d].reshape(n, d)).cuda()
        o += n * d
        m = scp.MWU(X, "ses", eps=1e-2, t_cap=300)
        s = m.solve()
        m.close()
        assert r["tests"] == s["tests"] and r["iters"] == s["iters"], (r["iters"], s["iters"])
        assert abs(r["radius"] - s["radius"]) / s["radius"] <= RESULT
        assert abs(r["lower"] - s["lower"]) / s["radius"] <= RESULT


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
@pytest.mark.parametrize("n,d,seed,k", [(1000, 64, 742, 2), (900, 64, 747, 3), (900, 64, 775, 4)])
def test_kway_search_matches_oracle(n, d, seed, k):
    """The k-way search (k tests per round sharing the passes; four tests in
    two shared pairs) against the oracle's k-way search on the same points (a
    pinned search path; the k = 4 case stops 6 of its 16 tests as moot): the
    same number of tests, iterations and shared passes, radius and lower
    bound within RESULT, and a centre that realises the radius."""
    import torch
    import paper_2405_09157_amd as scp
    V = synth.ses_ellipsoid(n, d, seed).astype(np.float32)
    V64 = V.astype(np.float64)
    ref = oses.solve_kway(V64, k, eps=1e-2, t_cap=300)
    assert ref.tie_margin >= PINNED and ref.cancel_max <= CANCEL_MAX
    with scp.MWUBatch.kway(torch.from_numpy(V).cuda(), k, eps=1e-2, t_cap=300, chunk=8) as b:
        out = b.solve_kway()
    assert out["code"] == scp.SCP_MWU_OK and out["converged"] == int(ref.converged)
    assert out["tests"] == len(ref.steps)
    assert out["iters"] == ref.iters and out["passes"] == ref.passes, (out["iters"], ref.iters, out["passes"])
    far = np.max(np.linalg.norm(V64 - np.array(out["center"]), axis=1))
    assert abs(far - out["radius"]) <= 1e-9 * out["radius"]
    assert abs(out["radius"] - ref.radius) / ref.radius <= RESULT
    assert abs(out["lower"] - ref.lower) / ref.radius <= RESULT


def test_kway_search_brackets_oracle_unpinned():
    """An unpinned k-way search (d = 3, separations): the centre realises the
    radius and the certified bounds are consistent with the oracle's k-way
    search."""
    import torch
    import paper_2405_09157_amd as scp
    V = synth.ses_ellipsoid(1500, 3, 548).astype(np.float32)
    V64 = V.astype(np.float64)
    ref = oses.solve_kway(V64, 2, eps=1e-2, t_cap=1500)
    with scp.MWUBatch.kway(torch.from_numpy(V).cuda(), 2, eps=1e-2, t_cap=1500, chunk=8) as b:
        out = b.solve_kway()
    assert out["code"] == scp.SCP_MWU_OK
    far = np.max(np.linalg.norm(V64 - np.array(out["center"]), axis=1))
    assert abs(far - out["radius"]) <= 1e-9 * out["radius"]
    _brackets(out["lower"], out["radius"], ref)


def test_kway_search_with_one_slot_is_the_paper_search():
    """k = 1 against the oracle's search of Section 3 (the k-way search with
    one test per round is that search, pinned step for step on the CPU)."""
    import torch
    import paper_2405_09157_amd as scp
    V = synth.ses_ellipsoid(700, 64, 700).astype(np.float32)
    ref = oses.solve(V.astype(np.float64), eps=1e-2, t_cap=300)
    assert ref.tie_margin >= PINNED and ref.cancel_max <= CANCEL_MAX
    with scp.MWUBatch.kway(torch.from_numpy(V).cuda(), 1, eps=1e-2, t_cap=300) as b:
        out = b.solve_kway()
    assert out["tests"] == len(ref.steps) and out["passes"] == out["iters"] == ref.iters
    assert abs(out["radius"] - ref.radius) / ref.radius <= RESULT


def test_kway_search_needs_one_point_set():
    import torch
    import paper_2405_09157_amd as scp
    X = torch.from_numpy(np.random.default_rng(5).standard_normal(4000).astype(np.float32)).cuda()
    with scp.MWUBatch(X, [100, 100], [3, 3], [0, 300]) as b:
        with pytest.raises(scp.ScpMwuError) as e:
            b.solve_kway()
        assert e.value.code == scp.SCP_MWU_E_INVAL
