"""Writes grad_200k_d64_T<T>.json (T = 2000 by default): the FP64 oracle's
reference for the gradient workload (n = 200,000 points N(0, I) in d = 64,
FP32, seed 0; T fixed-alpha iterations; alpha held at the oracle's solved
radius).  With T other than 2000 the solved radius is read from
grad_200k_d64_T2000.json (written by this script) when that file exists.

Calls only oracle/ and synth/ (test infrastructure):
  1. the radius R* of the oracle's adaptive search, eps = 1e-2 (Section 3
     search with the Section 5 exits; its certified radius, the least f seen),
     taken as alpha and held fixed (detached);
  2. ses_grad.radius_grad at that alpha and T: R and dR/dV (every row);
  3. a compact record: R, the rows of the gradient at 64 seeded rows plus the
     rows that carry R's and D's own terms (the active row i*, v1 = row 0 and
     D's far row), the directional derivative sum_ij g_ij z_ij for a seeded
     N(0, 1) direction z (float32, seed 1), and the dual-weight gradient at
     the same rows (pi_i (v_i - c) / R from the MWU weights of the last
     iteration, c = ubar_T), for the loose Danskin comparison.

    python tests/golden/make_grad_200k_d64.py [T]   (T = 2000: about 1.5 h on
                                                     one core; T = 500 with the
                                                     stored radius: about 10 min)
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import ses, ses_grad  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main(T=2000):
    t0 = time.time()
    out_path = os.path.join(HERE, f"grad_200k_d64_T{T}.json")
    ref_path = os.path.join(HERE, "grad_200k_d64_T2000.json")
    V = synth.ses_gaussian_outliers(200_000, 64, 0, frac=0.0, dtype=np.float32).astype(np.float64)
    if T != 2000 and os.path.exists(ref_path):
        with open(ref_path) as f:
            ref = json.load(f)
        alpha, lower = float(ref["alpha"]), float(ref["solve_lower"])
        print(f"solved radius from {ref_path}: {alpha:.12g}", flush=True)
    else:
        sol = ses.solve(V, eps=1e-2)
        alpha, lower = float(sol.radius), float(sol.lower)
        print(f"solve: radius {alpha:.12g} lower {lower:.12g} tests {len(sol.steps)} iters {sol.iters} "
              f"({time.time() - t0:.0f} s)", flush=True)
    fw = ses_grad.forward(V, alpha, T)
    R, G = ses_grad.radius_grad(V, alpha, T, fw=fw)
    print(f"grad: R {R:.12g} ({time.time() - t0:.0f} s)", flush=True)
    P = fw.P
    eta = fw.eta
    # the final mean and the weights of iteration T + 1 (the dual weights pi)
    c = fw.S[T] / T
    W, s, _ = ses.hyperplane(P, c, alpha, T, eta)
    pi = np.zeros(V.shape[0])
    pi[P.F] = s / np.sum(s)                    # trace weights of the blocks, normalised
    dist = np.linalg.norm(V - c[None, :], axis=1)
    istar = int(np.argmax(dist))
    jstar = int(np.argmax(np.linalg.norm(V[0] - V, axis=1)))
    rng = np.random.default_rng(7)
    rows = sorted(set(rng.choice(V.shape[0], 64, replace=False).tolist()) | {0, istar, jstar})
    z = np.random.default_rng(1).standard_normal(V.shape, dtype=np.float32).astype(np.float64)
    danskin = pi[rows, None] * (V[rows] - c[None, :]) / R
    out = dict(
        source="FP64 oracle (oracle/ses.py solve, oracle/ses_grad.py radius_grad); "
               "written by tests/golden/make_grad_200k_d64.py",
        n=200_000, d=64, seed=0, T=T, eps_solve=1e-2, alpha=alpha, solve_lower=lower,
        R=float(R), istar=istar, jstar=jstar, rows=rows,
        grad_rows=G[rows].tolist(), max_abs_grad=float(np.abs(G).max()),
        dir_seed=1, dir_deriv=float(np.sum(G * z)),
        grad_sum=np.sum(G, axis=0).tolist(),
        danskin_rows=danskin.tolist(), pi_top=float(np.max(pi)),
        danskin_cos=float(np.sum(G[rows] * danskin) / (np.linalg.norm(G[rows]) * np.linalg.norm(danskin))),
    )
    with open(out_path, "w") as f:
        json.dump(out, f)
    print(f"wrote {out_path} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2000)
