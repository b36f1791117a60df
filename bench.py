"""Benchmark of the MWU iteration on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-solve] [--no-cpu]

Workload: smallest enclosing sphere, n = 1,000,000 points in d = 100, i.i.d.
N(0, I) with 1 % of the rows scaled x5 (seed 0), resident in HBM as FP32.
One step = one MWU iteration of an alpha-feasibility test: one streaming pass
over the 400 MB point matrix fused with the SCMWU update, plus its FP64
epilogue (ORACLE, running mean, monitor).  K steps are timed between two
device synchronisations; the reported value is MWU iterations per second.

The same JSON line also carries
  roofline      bytes the pass must read (n d sizeof) over its mean HIP-event
                duration, against the 8 TB/s HBM peak and against the
                library's plain streaming-read kernel over the same number of
                bytes; HBM traffic from the committed rocprofv3 counter
                summary when it matches the kernel;
  bf16, fp8     the same measurement with BF16 storage (library-rounded copy)
                and with FP8 E4M3 storage (library-quantized codes, one FP32
                scale per row);
  solve         eps = 1e-3 solves (FP32, BF16 and FP8 storage) with the paper's
                Section 5 early stopping: wall time, iterations, tests,
                certified bounds;
  batched       the batched workload: 4,096 independent SES instances, n
                log-uniform in [1e3, 1e5], d from {2, 3, 16, 64}, points
                uniform in seeded random ellipsoids (86.7 M points, 7.4 GB as
                FP32), drawn on the device; the rows per workgroup share are
                picked by the library's autotuner; batched iterations/s (every
                instance advances one MWU iteration), the pass's bytes over its
                HIP-event time, FP32 and BF16 storage, and the eps = 1e-3 solve
                of all 4,096 instances (solves/s);
  solve_kway    eps = 1e-3 solves of the 1e6 x 100 workload by the k-way alpha
                search (k tests per round sharing the passes), FP32 storage;
  cpu_baseline  the FP64 reference implementation timed on this host on a
                bounded sample (a few iterations at the full size), one
                thread and all cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = dict(name="ses_1m_d100", n=1_000_000, d=100, seed=0, outlier_frac=0.01, outlier_scale=5.0)
METRIC = "MWU iters/sec + ε=1e-3 solves/sec (MEB n=1M,d=100), HBM GB/s frac; BF16 vs FP32"
KERNEL_SOURCES = ["paper_2405_09157_amd/csrc/mwu_kernels.hpp", "paper_2405_09157_amd/csrc/mwu_common.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_ses_pass_1m_d100.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(storage: str):
    """HBM bytes per pass from the committed counter summary, if it was taken
    on the current kernel source (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    rec = t.get(storage)
    return None if rec is None else rec.get("bytes_per_pass")


def measure(X, storage, steps, warmup, alpha, T=20000):
    """Time `steps` MWU iterations of one alpha-test.  alpha is an actual
    enclosing radius (>= OPT), so the test cannot separate and, with the
    Section 5 exits off, runs every iteration; the pass costs the same for
    any alpha."""
    import torch
    import paper_2405_09157_amd as scp
    m = scp.MWU(X, "ses", flags=scp.SCP_MWU_FLAG_NO_EARLY_STOP, storage=storage, chunk=64)
    m.step(alpha, T, max(warmup, 1), reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = m.step(alpha, T, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert info["outcome_name"] == "running" and info["t"] == max(warmup, 1) + steps, info
    # per-pass HIP-event timing on the launch stream (the dominant kernel)
    kms, ims = m.time_passes(min(steps, 200))
    m.close()
    return dict(ms_per_step=1e3 * dt / steps, kernel_ms=kms, iter_event_ms=ims, f_last=info["f_last"])


def copy_probe(X, reps=10):
    """A plain elementwise copy of the same 400 MB (torch.neg into a second
    tensor, a kernel of its own name): the kernel of known size whose
    rocprofv3 FETCH_SIZE / WRITE_SIZE readings scale the counters."""
    import torch
    Y = torch.empty_like(X)
    torch.neg(X, out=Y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(X, out=Y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    moved = X.numel() * X.element_size() * 2
    del Y
    return dict(ms=round(ms, 5), GBs=round(moved / (ms * 1e-3) / 1e9, 1), bytes=moved)


def read_reference(nbytes, X=None, reps=20):
    """Achievable read bandwidth: the library's plain streaming-read kernel over
    nbytes of device memory (the point matrix itself when given)."""
    import torch
    import paper_2405_09157_amd as scp
    buf = X if X is not None else torch.empty(nbytes // 2, dtype=torch.int16, device="cuda")
    ms = scp.scp_mwu_read_reference(buf.data_ptr(), nbytes, reps, torch.cuda.current_stream().cuda_stream)
    return dict(ms=round(ms, 5), GBs=round(nbytes / (ms * 1e-3) / 1e9, 1), bytes=nbytes)


def solve_kway(X, k):
    """eps = 1e-3 solve of the headline workload by the k-way alpha search."""
    import torch
    import paper_2405_09157_amd as scp
    with scp.MWUBatch.kway(X, k, eps=1e-3, chunk=32) as b:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = b.solve_kway()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    return dict(k=k, seconds=round(dt, 3), solves_per_s=round(1.0 / dt, 4), tests=out["tests"], iters=out["iters"],
                passes=out["passes"], radius=out["radius"], lower=out["lower"], converged=bool(out["converged"]))


def solve(X, storage):
    """eps = 1e-3 solve with the Section 5 exits and weight certificates (the
    dual lower bound of eq.(ses_qp) from the pass's weights, taken once per
    graph chunk): wall time, iterations, tests, radius and certified bounds.
    The partial sums are combined in a fixed order, so that the search path
    (which rounding decides near a test's decision points) and the figures
    are the same from run to run."""
    import torch
    import paper_2405_09157_amd as scp
    m = scp.MWU(X, "ses", eps=1e-3, storage=storage, chunk=64,
                flags=scp.SCP_MWU_FLAG_CERTIFICATES | scp.SCP_MWU_FLAG_DETERMINISTIC)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = m.solve()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    m.close()
    # the returned centre evaluated on the original FP32 points (the radius a
    # user of the original data gets from this solve)
    c = torch.tensor(out["center"], dtype=torch.float64, device=X.device)
    r_orig = float(torch.linalg.vector_norm(X.double() - c, dim=1).max())
    return dict(seconds=dt, solves_per_s=1.0 / dt, iters=out["iters"], tests=out["tests"],
                radius=out["radius"], radius_on_original_points=r_orig, lower=out["lower"], upper=out["upper"],
                cert_gap=(out["upper"] - out["lower"]) / out["lower"], converged=bool(out["converged"]))


BATCH = dict(name="ses_batched_4096", instances=4096, n_lo=1000, n_hi=100_000, dims=[2, 3, 16, 64], seed=0)


def batched(steps, warmup, solve_storages):
    """Batched SES: iteration rate and pass bandwidth for FP32 and BF16
    storage, then eps = 1e-3 solves of the whole batch."""
    import torch
    import synth
    import paper_2405_09157_amd as scp
    B = BATCH
    n, d = synth.ses_batch_sizes(B["instances"], B["n_lo"], B["n_hi"], B["dims"], B["seed"])
    pts, off = synth.ses_batch_points_device(n, d, B["seed"])
    torch.cuda.synchronize()
    m = len(n)
    nbytes = int((n * d).sum()) * 4
    rpg, tune = scp.autotune_rows_per_group(pts, n, d, off)
    print(f"# batched: {m} instances, {int(n.sum())} points, {nbytes / 1e9:.2f} GB; rows per group {rpg} "
          f"(pass ms {tune})", file=sys.stderr, flush=True)
    out = dict(workload=B["name"], instances=m, points=int(n.sum()), fp32_bytes=nbytes, rows_per_group=rpg,
               autotune_pass_ms={str(k): round(v, 4) for k, v in tune.items()})
    for storage in (None, "bf16"):
        key = storage or "f32"
        with scp.MWUBatch(pts, n, d, off, flags=scp.SCP_MWU_FLAG_NO_EARLY_STOP, storage=storage,
                          rows_per_group=rpg) as b:
            b.step(b.D, [20000] * m, max(warmup, 32), reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = b.step(b.D, [20000] * m, steps)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            assert all(i["outcome_name"] == "running" for i in info)
            mp, mi = b.time_iters(20)
        nb = nbytes // (2 if storage else 1)
        out[key] = dict(batched_iters_per_s=round(1.0 / dt, 1), instance_iters_per_s=round(m / dt, 0),
                        ms_per_batched_iter=round(dt * 1e3, 4), pass_ms=round(mp, 4), bytes_per_pass=nb,
                        pass_GBs=round(nb / (mp * 1e-3) / 1e9, 1),
                        pass_hbm_frac=round(nb / (mp * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
        print(f"# batched {key}: {out[key]}", file=sys.stderr, flush=True)
    for storage in solve_storages:
        key = storage or "f32"
        with scp.MWUBatch(pts, n, d, off, eps=1e-3, storage=storage, rows_per_group=rpg) as b:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            code, res = b.solve()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        its = np.array([r["iters"] for r in res])
        out[key]["solve"] = dict(seconds=round(dt, 2), solves_per_s=round(m / dt, 2),
                                 converged=int(sum(r["converged"] for r in res)), code=code,
                                 iters_mean=round(float(its.mean()), 1), iters_max=int(its.max()),
                                 instance_iters_per_s=round(float(its.sum()) / dt, 0))
        print(f"# batched solve {key}: {out[key]['solve']}", file=sys.stderr, flush=True)
    del pts
    torch.cuda.empty_cache()
    return out


SVM = dict(name="svm_500k_d256", n_pos=250_000, n_neg=250_000, d=256, seed=0)


def svm_leg(steps, warmup, solve_budget=60_000):
    """Hard-margin SVM at 500k x 256 (planted margin, P rows then Q rows):
    MWU iterations/s and the pass's bytes over its HIP-event time for FP32 and
    BF16 storage, then eps = 1e-3 solves (the search of Section 3 mirrored for
    the min form, Section 5 exits) within an iteration budget (none when the
    budget is 0), with their certified margin (lower) and polytope-distance
    upper bound."""
    import torch
    import paper_2405_09157_amd as scp
    import synth
    c = SVM
    X, _ = synth.svm_planted(c["n_pos"], c["n_neg"], c["d"], seed=c["seed"], dtype=np.float32)
    Xd = torch.from_numpy(X).cuda()
    del X
    n = c["n_pos"] + c["n_neg"]
    out = dict(workload=c["name"], n=n, d=c["d"])
    for storage in (None, "bf16"):
        key = storage or "f32"
        m = scp.MWU(Xd, "svm", n_pos=c["n_pos"], flags=scp.SCP_MWU_FLAG_NO_EARLY_STOP, storage=storage, chunk=64)
        m.step(0.05, 20000, max(warmup, 1), reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.step(0.05, 20000, steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        kms, ims = m.time_passes(min(steps, 100))
        m.close()
        nb = n * c["d"] * (2 if storage else 4)
        ach = nb / (kms * 1e-3) / 1e9
        out[key] = dict(iters_per_s=round(1.0 / dt, 1), ms_per_iter=round(dt * 1e3, 5),
                        roofline=dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                                      frac=round(ach / HBM_PEAK_GBS, 4), traffic=traffic_for("svm_" + key),
                                      kernel_ms=round(kms, 5),
                                      kernel=f"svm_pass_kernel<{'uint16_t' if storage else 'float'},16,"
                                             f"{8 if storage else 4},0>", bytes_per_launch=nb))
        if not solve_budget:
            print(f"# svm {key}: {out[key]}", file=sys.stderr, flush=True)
            continue
        m = scp.MWU(Xd, "svm", n_pos=c["n_pos"], eps=1e-3, storage=storage, chunk=64, max_iters=solve_budget)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = m.solve()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        m.close()
        out[key]["solve"] = dict(seconds=round(sec, 3), iters=r["iters"], tests=r["tests"], margin=r["value"],
                                 lower=r["lower"], upper=r["upper"],
                                 cert_gap=(r["upper"] - r["lower"]) / r["upper"] if r["upper"] > 0 else None,
                                 converged=bool(r["converged"]), code=r["code"], iter_budget=solve_budget)
        print(f"# svm {key}: {out[key]}", file=sys.stderr, flush=True)
    if "f32" in out and "bf16" in out:
        out["bf16_over_f32_iteration_rate"] = round(out["bf16"]["iters_per_s"] / out["f32"]["iters_per_s"], 4)
    del Xd
    torch.cuda.empty_cache()
    return out


SMALL = dict(name="ses_2000_d3_f64", n=2000, d=3, seeds=list(range(10)))


def small_config():
    """SES 2000 x 3 uniform in [-1, 1]^3 with FP64 storage, eps = 1e-3: the GPU
    solve of each of 10 seeds (solves/s from the median wall time).  The CPU
    baseline's full solve of seed 0 is in cpu_baseline."""
    import torch
    import paper_2405_09157_amd as scp
    import synth
    times, res = [], []
    for seed in SMALL["seeds"]:
        V = synth.ses_uniform(SMALL["n"], SMALL["d"], seed)
        Vd = torch.from_numpy(V).cuda()
        m = scp.MWU(Vd, "ses", eps=1e-3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = m.solve()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        m.close()
        res.append(r)
    med = float(np.median(times))
    out = dict(workload=SMALL["name"], solves=len(times), median_s=round(med, 5), solves_per_s=round(1.0 / med, 2),
               iters_mean=float(np.mean([r["iters"] for r in res])), radius_seed0=res[0]["radius"],
               converged=int(sum(bool(r["converged"]) for r in res)))
    print(f"# small config: {out}", file=sys.stderr, flush=True)
    return out


def beyond_cache(steps):
    """The 1e6 x 100 measurement at n = 2e6 (BF16 400 MB, FP32 800 MB): every
    matrix larger than the 256 MB Infinity Cache, so the pass rate is HBM's."""
    import torch
    import paper_2405_09157_amd as scp
    import synth
    V = synth.ses_gaussian_outliers(2_000_000, 100, 1, dtype=np.float32)
    X = torch.from_numpy(V).cuda()
    del V
    alpha = 1.02 * float(torch.linalg.vector_norm(X - X.mean(0, keepdim=True), dim=1).max())
    out = dict(n=2_000_000, d=100)
    for storage, es in ((None, 4), ("bf16", 2)):
        r = measure(X, storage, steps, 8, alpha)
        nb = 2_000_000 * 100 * es
        ach = nb / (r["kernel_ms"] * 1e-3) / 1e9
        out[storage or "f32"] = dict(ms_per_iter=round(r["ms_per_step"], 5), kernel_ms=round(r["kernel_ms"], 5),
                                     bytes=nb, GBs=round(ach, 1), hbm_frac=round(ach / HBM_PEAK_GBS, 4),
                                     traffic=traffic_for((storage or "f32") + "_2e6"))
    out["bf16_over_f32_iteration_rate"] = round(out["f32"]["ms_per_iter"] / out["bf16"]["ms_per_iter"], 4)
    print(f"# beyond cache: {out}", file=sys.stderr, flush=True)
    del X
    torch.cuda.empty_cache()
    return out


GRAD = dict(name="ses_grad_200k_d64_T2000", n=200_000, d=64, T=2000, seed=0)
GRAD_FIXTURE = os.path.join(ROOT, "tests", "golden", "grad_200k_d64_T2000.json")


def gradient(reps=3):
    """Reverse pass of the radius after T fixed-alpha iterations (FP32 points
    N(0, I)), alpha held at the solved radius (the FP64 oracle's, from its
    fixture, else this library's eps = 1e-2 solve): wall time of
    scp_mwu_backward with running sums kept every 50 iterations (forward,
    per-segment recomputation, reverse iterations), of the same call keeping
    the whole tape, and, beside them, T forward iterations of the streaming
    pass at the same alpha."""
    import numpy as np
    import torch
    import paper_2405_09157_amd as scp
    import synth
    g = GRAD
    V = synth.ses_gaussian_outliers(g["n"], g["d"], g["seed"], frac=0.0, dtype=np.float32)
    X = torch.from_numpy(V).cuda()
    out = torch.empty_like(X)
    try:
        with open(GRAD_FIXTURE) as f:
            alpha, alpha_src = float(json.load(f)["alpha"]), "oracle solved radius (eps 1e-2)"
    except (OSError, ValueError, KeyError):
        with scp.MWU(X, "ses", eps=1e-2) as ms:
            alpha, alpha_src = float(ms.solve()["radius"]), "library solved radius (eps 1e-2)"
    with scp.MWU(X, "ses", flags=scp.SCP_MWU_FLAG_NO_EARLY_STOP) as m:
        m.step(alpha, g["T"], 0, reset=True)
        R, _ = m.backward(1.0, out)           # warm-up
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m.backward(1.0, out)
            times.append(time.perf_counter() - t0)
        m.backward(1.0, out, checkpoint_every=0)       # warm-up of the whole-tape mode
        times_full = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m.backward(1.0, out, checkpoint_every=0)
            times_full.append(time.perf_counter() - t0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.step(alpha, g["T"], g["T"], reset=True)
        torch.cuda.synchronize()
        fwd = time.perf_counter() - t0
    bwd = min(times)
    return dict(workload=g["name"], n=g["n"], d=g["d"], T=g["T"], checkpoint_every=50,
                storage="f32", alpha=alpha, alpha_source=alpha_src, radius=R, backward_s=round(bwd, 4),
                reverse_iters_per_s=round(g["T"] / bwd, 1),
                forward_s=round(fwd, 4), backward_over_forward=round(bwd / fwd, 2),
                whole_tape=dict(backward_s=round(min(times_full), 4),
                                reverse_iters_per_s=round(g["T"] / min(times_full), 1)),
                grad_abs_sum=float(out.abs().sum()))


PRODUCT = dict(name="product_cone_orthant1e7_1e5x64", n_orth=10_000_000, blocks=100_000, d=64, seed=0, eta=0.05)


def product_cone(reps=20):
    """SCMWU iterate over R^{1e7}_+ (+) 1e5 Lorentz blocks Q^{65} (16.5 M binary64
    values) through one validated ProductCone handle: HIP-event time of the
    three launches of an iterate (enqueued back to back, no host work between
    them), the wall time of one call that also reads ln Tr back, and the rate
    of the algorithmic bytes (m read twice, p written, then read and written
    once more: 5 x 8 bytes per value)."""
    import numpy as np
    import torch
    import paper_2405_09157_amd as scp
    c = PRODUCT
    total = c["n_orth"] + c["blocks"] * (c["d"] + 1)
    g = torch.Generator(device="cuda").manual_seed(c["seed"])
    m = torch.randn(total, dtype=torch.float64, device="cuda", generator=g)
    p = torch.empty_like(m)
    dims = [c["d"]] * c["blocks"]
    with scp.ProductCone(c["n_orth"], dims) as pc:
        pc.exp(m, c["eta"], out=p)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            pc.exp(m, c["eta"], out=p, log_trace=False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        walls = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pc.exp(m, c["eta"], out=p)
            walls.append(time.perf_counter() - t0)
    nbytes = 5 * 8 * total
    return dict(workload=c["name"], values=total, kernels_ms=round(ms, 4), algorithmic_bytes=nbytes,
                GBs=round(nbytes / (ms * 1e-3) / 1e9, 1), hbm_frac=round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                wall_ms_with_readback=round(float(np.median(walls)) * 1e3, 4))


def _oracle_iters(V64, threads, warm, timed, budget_s):
    """Median seconds per FP64 oracle iteration of the benchmarked alpha-test."""
    from threadpoolctl import threadpool_limits
    from oracle import ses as oses
    with threadpool_limits(threads):
        P = oses.setup(V64)
        alpha, T = 0.8 * P.D, 20000
        eta = math.sqrt(math.log(P.r) / T)
        S = np.zeros(V64.shape[1])
        t_prev, times = 0, []
        t_start = time.perf_counter()
        while len(times) < warm + timed:
            t0 = time.perf_counter()
            st = oses.step(P, S, t_prev, alpha, eta)
            times.append(time.perf_counter() - t0)
            S, t_prev = st["S"], t_prev + 1
            if time.perf_counter() - t_start > budget_s and len(times) > warm:
                break
    tt = sorted(times[warm:]) if len(times) > warm else sorted(times)
    return tt[len(tt) // 2], len(times) - min(warm, len(times) - 1)


def cpu_baseline(V32):
    """The FP64 reference implementation (numpy) on the host at the full size,
    on a bounded sample: a few iterations of the same alpha-test, one thread,
    then with every core available to its BLAS calls."""
    V64 = V32.astype(np.float64)
    one, n1 = _oracle_iters(V64, 1, 1, 2, 15.0)
    ncpu = os.cpu_count() or 1
    allc, n2 = _oracle_iters(V64, ncpu, 1, 2, 12.0)
    # the small configuration's full eps = 1e-3 solve (SES 2000 x 3, seed 0)
    import synth
    from threadpoolctl import threadpool_limits
    from oracle import ses as oses
    Vs = synth.ses_uniform(SMALL["n"], SMALL["d"], 0)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        ref = oses.solve(Vs, eps=1e-3)
        dts = time.perf_counter() - t0
    return dict(value=round(1.0 / one, 4), unit="iters/s", cores=1, kind="oracle",
                small_config_solve=dict(workload=SMALL["name"], seconds=round(dts, 3), solves_per_s=round(1.0 / dts, 4),
                                        cores=1, iters=ref.iters, radius=ref.radius),
                sample=f"median of {n1} FP64 oracle iterations (after 1 warm-up) of the same "
                       f"n=1e6, d=100 alpha-test, numpy on one thread",
                all_cores=dict(value=round(1.0 / allc, 4), cores=ncpu,
                               note=f"median of {n2} iterations with {ncpu} threads allowed "
                                    f"(only the BLAS calls are threaded)"))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-fp8", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--batch-solve", default="f32",
                    help="storage types of the batched eps solves: comma list of f32, bf16, or none")
    ap.add_argument("--no-grad", action="store_true", help="skip the reverse-pass workload")
    ap.add_argument("--no-cone", action="store_true", help="skip the product-cone iterate")
    ap.add_argument("--no-svm", action="store_true", help="skip the SVM 500k x 256 workload")
    ap.add_argument("--no-small", action="store_true", help="skip the SES 2000 x 3 FP64 solves")
    ap.add_argument("--no-big", action="store_true", help="skip the n = 2e6 (beyond-cache) measurement")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also time a plain copy of the matrix (counter calibration)")
    a = ap.parse_args(argv)
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(sharding would split the point rows and all-reduce each iteration's sums)", file=sys.stderr)
        return 2
    import numpy as np
    import torch
    import synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = WORKLOAD
    V = synth.ses_gaussian_outliers(w["n"], w["d"], w["seed"], frac=w["outlier_frac"],
                                    scale=w["outlier_scale"], dtype=np.float32)
    X = torch.from_numpy(V).cuda()
    # an enclosing radius: the sphere at the centroid with this radius holds every point
    alpha = 1.02 * float(torch.linalg.vector_norm(X - X.mean(0, keepdim=True), dim=1).max())
    print(f"# data ready: {w['n']} x {w['d']} float32, alpha {alpha:.4f}", file=sys.stderr, flush=True)
    f32 = measure(X, None, a.steps, a.warmup, alpha)
    print(f"# f32: {f32}", file=sys.stderr, flush=True)
    # narrow storage types: bytes one pass must read (FP8: codes and row scales)
    narrow = {k: v for k, v in (("bf16", w["n"] * w["d"] * 2), ("fp8", w["n"] * (w["d"] + 4)))
              if not getattr(a, "no_" + k)}
    res = {}
    for k in narrow:
        res[k] = measure(X, k, a.steps, a.warmup, alpha)
        print(f"# {k}: {res[k]}", file=sys.stderr, flush=True)
    rref = dict(f32=read_reference(w["n"] * w["d"] * 4, X))
    for k, nb in narrow.items():
        rref[k] = read_reference(nb)
    print(f"# read reference: {rref}", file=sys.stderr, flush=True)
    probe = copy_probe(X) if a.copy_probe else None
    if probe:
        print(f"# copy: {probe}", file=sys.stderr, flush=True)
    sol = {}
    if not a.no_solve:
        sol["f32"] = solve(X, None)
        print(f"# solve f32: {sol['f32']}", file=sys.stderr, flush=True)
        for k in narrow:
            sol[k] = solve(X, k)
            rel = sol[k]["radius"] / sol["f32"]["radius"] - 1.0
            sol[k]["radius_rel_to_f32"] = rel
            print(f"# solve {k}: {sol[k]}", file=sys.stderr, flush=True)
            # a solve-rate ratio counts as at equal accuracy when the narrow-
            # storage solve's centre encloses the ORIGINAL points within 1e-3
            # of the FP32 solve's radius (or better), or both certified gaps
            # are within eps
            rel_orig = sol[k]["radius_on_original_points"] / sol["f32"]["radius_on_original_points"] - 1.0
            sol[k]["radius_on_original_points_rel_to_f32"] = rel_orig
            equal = rel_orig <= 1e-3 or (sol[k]["cert_gap"] <= 1e-3 and sol["f32"]["cert_gap"] <= 1e-3)
            sol[f"{k}_over_f32_solve_rate"] = dict(
                ratio=round(sol[k]["solves_per_s"] / sol["f32"]["solves_per_s"], 4), equal_accuracy=bool(equal),
                note="its centre encloses the original points within 1e-3 of the FP32 solve's radius, or better"
                if equal else "NOT at equal accuracy: its centre's radius on the original points is more than "
                              "1e-3 above the FP32 solve's")
            # the same comparison at equal iteration counts: the iteration rates
            sol[f"{k}_over_f32_iteration_rate"] = round(f32["ms_per_step"] / res[k]["ms_per_step"], 4)
        # the BF16 / FP32 solve-rate comparison over two more instances of the
        # workload's distribution (seeds 1 and 2): rounding decides where a
        # test separates or stabilises, so the search path and its iteration
        # count differ between storage types instance by instance
        if "bf16" in narrow:
            per_seed = [dict(seed=w["seed"], ratio=sol["bf16_over_f32_solve_rate"]["ratio"],
                             equal_accuracy=sol["bf16_over_f32_solve_rate"]["equal_accuracy"],
                             f32_iters=sol["f32"]["iters"], bf16_iters=sol["bf16"]["iters"])]
            for sd in (1, 2):
                Vs = synth.ses_gaussian_outliers(w["n"], w["d"], sd, frac=w["outlier_frac"],
                                                 scale=w["outlier_scale"], dtype=np.float32)
                Xs = torch.from_numpy(Vs).cuda()
                del Vs
                rf, rb = solve(Xs, None), solve(Xs, "bf16")
                rel = rb["radius_on_original_points"] / rf["radius_on_original_points"] - 1.0
                per_seed.append(dict(seed=sd, ratio=round(rf["seconds"] / rb["seconds"], 4),
                                     equal_accuracy=bool(rel <= 1e-3 or (rb["cert_gap"] <= 1e-3 and rf["cert_gap"] <= 1e-3)),
                                     f32_iters=rf["iters"], bf16_iters=rb["iters"],
                                     f32_s=round(rf["seconds"], 3), bf16_s=round(rb["seconds"], 3)))
                del Xs
                torch.cuda.empty_cache()
            sol["bf16_over_f32_solve_rate_over_seeds"] = dict(
                per_seed=per_seed, median_ratio=float(np.median([r["ratio"] for r in per_seed])),
                all_equal_accuracy=all(r["equal_accuracy"] for r in per_seed))
            print(f"# solve bf16/f32 over seeds: {sol['bf16_over_f32_solve_rate_over_seeds']}", file=sys.stderr,
                  flush=True)
        kway = [solve_kway(X, k) for k in (2, 4)]
        for r in kway:
            r["over_f32_solve_rate"] = round(r["solves_per_s"] / sol["f32"]["solves_per_s"], 3)
            print(f"# solve k-way: {r}", file=sys.stderr, flush=True)
        sol["kway"] = kway
    del X
    torch.cuda.empty_cache()
    bsolve = [] if a.batch_solve == "none" else [None if s == "f32" else s for s in a.batch_solve.split(",")]
    batch = None if a.no_batch else batched(min(a.steps, 320), a.warmup, bsolve)
    grad = None if a.no_grad else gradient()
    if grad:
        print(f"# gradient: {grad}", file=sys.stderr, flush=True)
    cone = None if a.no_cone else product_cone()
    if cone:
        print(f"# product cone: {cone}", file=sys.stderr, flush=True)
    svm = None if a.no_svm else svm_leg(min(a.steps, 640), a.warmup, solve_budget=0 if a.no_solve else 60_000)
    small = None if a.no_small else small_config()
    big = None if a.no_big else beyond_cache(min(max(a.steps, 64), 640))
    cpu = None if a.no_cpu else cpu_baseline(V)
    if cpu:
        print(f"# cpu: {cpu}", file=sys.stderr, flush=True)

    algo_bytes = w["n"] * w["d"] * 4
    ach = algo_bytes / (f32["kernel_ms"] * 1e-3) / 1e9
    roof = dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(ach / HBM_PEAK_GBS, 4), traffic=traffic_for("f32"),
                kernel="ses_fused_kernel<float,8,4,false,0,true>", kernel_ms=round(f32["kernel_ms"], 5),
                bytes_per_launch=algo_bytes, read_reference_GBs=rref["f32"]["GBs"],
                frac_of_read_reference=round(ach / rref["f32"]["GBs"], 4))
    line = dict(metric=METRIC, value=round(1e3 / f32["ms_per_step"], 1), unit="iters/s", n_gpus=1,
                steps=a.steps, warmup=a.warmup, ms_per_step=round(f32["ms_per_step"], 5),
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
                data="synthetic",
                config=dict(workload=w["name"], n=w["n"], d=w["d"], storage="f32",
                            points="N(0,I), 1% rows x5, seed 0", problem="SES"),
                roofline=roof, cpu_baseline=cpu)
    kname = dict(bf16="ses_fused_kernel<uint16_t,8,4,false,0,true>", fp8="ses_fused_kernel<uint8_t,8,4,false,0,true>")
    for k, nb in narrow.items():
        r = res[k]
        b_ach = nb / (r["kernel_ms"] * 1e-3) / 1e9
        line[k] = dict(value=round(1e3 / r["ms_per_step"], 1), unit="iters/s",
                       ms_per_step=round(r["ms_per_step"], 5),
                       speedup_vs_f32=round(f32["ms_per_step"] / r["ms_per_step"], 3),
                       roofline=dict(bound="hbm", achieved=round(b_ach, 1), peak=HBM_PEAK_GBS,
                                     unit="GB/s", frac=round(b_ach / HBM_PEAK_GBS, 4),
                                     traffic=traffic_for(k), kernel=kname[k],
                                     kernel_ms=round(r["kernel_ms"], 5), bytes_per_launch=nb,
                                     read_reference_GBs=rref[k]["GBs"],
                                     frac_of_read_reference=round(b_ach / rref[k]["GBs"], 4)))
    if sol:
        line["solve"] = sol
    if batch:
        line["batched"] = batch
    if grad:
        line["gradient"] = grad
    if cone:
        line["product_cone"] = cone
    if svm:
        line["svm"] = svm
    if small:
        line["small_config"] = small
    if big:
        line["beyond_cache"] = big
    if probe:
        line["copy_reference"] = probe
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
