"""Hard-margin SVM / polytope distance by the min-form meta-algorithm, FP64.

Test infrastructure (see package header).  Written from Section 3
("Extension to minimization problems", eq.(min_scp), eq.(min_oracle),
eq.(min_implement), Theorem min_meta) with Section 4.2:

* (SVM): max s1 + s2  s.t.  P^T w >= s1 1, -Q^T w >= s2 1, ||w|| <= 1, with
  P, Q holding the two classes' points (stored here as rows: X = [P rows; Q
  rows], rows [0, n_pos) are class +1).
* split eq.(svm_dual_scp): K = R^n_+ (hard, one coordinate per point),
  K' = Q^{d+1} x R^2_+ (easy: ||w|| <= 1, s1 <= D, s2 <= D, Lemma svm_bound).
  c - sum_j a_j y_j = (P^T w - s1 1 ; -Q^T w - s2 1), the per-point slack.
* D = max_i ||x_i||, width rho = 2D, R = 2, rank r = n, OPT in (0, 2D].
* hyperplane update eq.(min_implement): p(t+1) = exp(-(eta t/rho)(c - sum_j
  a_j ybar_j(t))) / C, i.e. weights exp(-(eta t / rho) slack_i(ybar)).
* ORACLE eq.(svm_oracle): w = (P mu - Q gamma)/||P mu - Q gamma||,
  s1 = D if Tr(mu) <= Tr(gamma) else alpha - D, s2 = alpha - s1.  Its value
  (P mu - Q gamma).w - Tr(mu) s1 - Tr(gamma) s2 < 0 certifies OPT < alpha, and
  then (mu/Tr mu ; gamma/Tr gamma) is a polytope-distance solution of value
  < alpha (the Claim in Section 4.2).
* T = ceil(64 D^2 ln n / (eps^2 alpha^2)), eta = sqrt(ln n / T).
* monitor f(t) = max{(min_{x in P} x.wbar - max_{x in Q} x.wbar)/||wbar||, 0}
  (Section 5; the paper's names for the two classes are swapped there).

Readings where the paper is silent (listed with reasons in the design notes):
  S1  rows, not columns, of the stored matrices are the points (the
      "j-th column" wording of eq.(svm_dual_scp) indexes coordinates).
  S2  search mirrors the max form: alpha_i = U - (U-L)/3,
      eps_i = (U-L)/(3 alpha_i), so (1 - eps_i) alpha_i = L + (U-L)/3.
  S3  separation: value < -tau * (||V|| + Tr(mu)|s1| + Tr(gamma)|s2|), tau = 1e-12.
  S4  T_k = min(T_theory, t_cap) raised to at least ceil(ln n).
  S5  after a stabilised / capped test, L <- max(f_best, L + (U-L)/3)
      (the paper's conclusion), the reported margin is the certified
      max_t f(t); every PD value ||P mu/Tr mu - Q gamma/Tr gamma|| seen is a
      certified upper bound and tightens U.
  S6  V = 0 (measure zero) gives w = 0.
  S7  stop when U - L <= eps * U.

Pins: tests/test_oracle_svm.py (ORACLE against brute force over s1 and random
unit w, width bound, PD claim on separation, exact 2-D maximum margin by
direction enumeration).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import eja

SEPARATED, BEAT, STABILIZED, T_REACHED = "separated", "beat_alpha", "stabilized", "t_reached"


@dataclass
class SvmSetup:
    X: np.ndarray
    n_pos: int
    D: float
    rho: float
    R: float
    r: int


def setup(X, n_pos: int) -> SvmSetup:
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    if not (1 <= n_pos <= n - 1):
        raise ValueError("both classes must be non-empty")
    D = float(np.max(np.linalg.norm(X, axis=1)))
    return SvmSetup(X=X, n_pos=n_pos, D=D, rho=2.0 * D, R=2.0, r=n)


def slack(Pb: SvmSetup, wbar: np.ndarray, s1: float, s2: float) -> np.ndarray:
    """c - sum_j a_j y_j = (P^T w - s1 1 ; -Q^T w - s2 1)."""
    P, Q = Pb.X[:Pb.n_pos], Pb.X[Pb.n_pos:]
    return np.concatenate([P @ wbar - s1, -(Q @ wbar) - s2])


def hyperplane(Pb: SvmSetup, ybar, t_prev: int, eta: float):
    """p(t_prev + 1) in R^n_+ from eq.(min_implement); returns (mu, gam, logC)."""
    n = Pb.X.shape[0]
    if t_prev == 0:
        x = np.zeros(n)
    else:
        wbar, s1, s2 = ybar
        x = -(eta * t_prev / Pb.rho) * slack(Pb, wbar, s1, s2)
    shift = float(np.max(x))
    e = eja.orthant_exp(x, shift)
    C = float(np.sum(e))
    p = e / C
    return p[:Pb.n_pos], p[Pb.n_pos:], shift + math.log(C)


def oracle(Pb: SvmSetup, mu: np.ndarray, gam: np.ndarray, alpha: float):
    """Closed form of eq.(svm_oracle).  Returns (w, s1, s2, value, scale, V, degenerate)."""
    P, Q = Pb.X[:Pb.n_pos], Pb.X[Pb.n_pos:]
    V = P.T @ mu - Q.T @ gam
    nV = float(np.linalg.norm(V))
    degenerate = not (nV > 0.0)
    w = np.zeros_like(V) if degenerate else V / nV
    trm, trg = float(np.sum(mu)), float(np.sum(gam))
    s1 = Pb.D if trm <= trg else alpha - Pb.D
    s2 = alpha - s1
    value = float(V @ w) - trm * s1 - trg * s2
    scale = nV + trm * abs(s1) + trg * abs(s2)
    return w, s1, s2, value, scale, V, degenerate


def pd_value(Pb: SvmSetup, mu: np.ndarray, gam: np.ndarray) -> float:
    """||P mu/Tr mu - Q gamma/Tr gamma||: a polytope-distance value, hence an
    upper bound on the maximum margin for any non-negative mu, gamma."""
    P, Q = Pb.X[:Pb.n_pos], Pb.X[Pb.n_pos:]
    return float(np.linalg.norm(P.T @ (mu / np.sum(mu)) - Q.T @ (gam / np.sum(gam))))


def monitor(Pb: SvmSetup, wbar: np.ndarray) -> float:
    """f = max{(min_P x.wbar - max_Q x.wbar)/||wbar||, 0} (Section 5)."""
    nw = float(np.linalg.norm(wbar))
    if not (nw > 0.0):
        return 0.0
    P, Q = Pb.X[:Pb.n_pos], Pb.X[Pb.n_pos:]
    return max((float(np.min(P @ wbar)) - float(np.max(Q @ wbar))) / nw, 0.0)


def theory_T(Pb: SvmSetup, eps: float, alpha: float) -> int:
    """T = ceil(4 R^2 rho^2 ln r/(eps^2 alpha^2)) = ceil(64 D^2 ln n/(eps^2 alpha^2))."""
    return int(math.ceil(4.0 * Pb.R ** 2 * Pb.rho ** 2 * math.log(Pb.r) / (eps ** 2 * alpha ** 2)))


def min_T(Pb: SvmSetup) -> int:
    return max(1, int(math.ceil(math.log(Pb.r))))


@dataclass
class FtpResult:
    outcome: str
    t: int
    Sw: np.ndarray
    S1: float
    S2: float
    t_done: int
    f_best: float
    wbar_best: Optional[np.ndarray]
    t_best: int
    ub_best: float
    f_traj: List[float] = field(default_factory=list)
    values: List[float] = field(default_factory=list)
    logC: List[float] = field(default_factory=list)
    # closest approach of the test's decisions to their thresholds, relative
    # (as in the SES oracle): separation in units of scale, f above alpha in
    # units of alpha, the stabilisation ratio in units of delta
    tie_margin: float = math.inf


def step(Pb: SvmSetup, Sw: np.ndarray, S1: float, S2: float, t_prev: int,
         alpha: float, eta: float, tau: float = 1e-12):
    """One iteration t = t_prev + 1 from the running sums of past ORACLE outputs."""
    ybar = (Sw / t_prev, S1 / t_prev, S2 / t_prev) if t_prev > 0 else None
    mu, gam, logC = hyperplane(Pb, ybar, t_prev, eta)
    w, s1, s2, value, scale, V, degenerate = oracle(Pb, mu, gam, alpha)
    return dict(w=w, s1=s1, s2=s2, value=value, scale=scale, logC=logC, V=V,
                mu=mu, gam=gam, degenerate=degenerate,
                separated=value < -tau * scale, ub=pd_value(Pb, mu, gam),
                f_prev=monitor(Pb, ybar[0]) if t_prev > 0 else None,
                Sw=Sw + w, S1=S1 + s1, S2=S2 + s2)


def ftp(Pb: SvmSetup, alpha: float, T: int, eta: float, delta: float = 1e-4,
        patience: int = 10, tau: float = 1e-12, early_stop: bool = True,
        record: bool = False) -> FtpResult:
    """alpha-feasibility test of the min form (Theorem min_meta) for SVM."""
    d = Pb.X.shape[1]
    Sw, S1, S2 = np.zeros(d), 0.0, 0.0
    f_prev = None
    cnt = 0
    res = FtpResult(outcome=T_REACHED, t=T, Sw=Sw, S1=S1, S2=S2, t_done=0,
                    f_best=-math.inf, wbar_best=None, t_best=0, ub_best=math.inf)
    for t in range(1, T + 1):
        ybar = (Sw / (t - 1), S1 / (t - 1), S2 / (t - 1)) if t > 1 else None
        mu, gam, logC = hyperplane(Pb, ybar, t - 1, eta)
        w, s1, s2, value, scale, _, _ = oracle(Pb, mu, gam, alpha)
        res.ub_best = min(res.ub_best, pd_value(Pb, mu, gam))
        if record:
            res.values.append(value)
            res.logC.append(logC)
        if scale > 0.0:
            res.tie_margin = min(res.tie_margin, abs(value + tau * scale) / scale)
        if value < -tau * scale:
            res.outcome, res.t = SEPARATED, t
            break
        Sw, S1, S2 = Sw + w, S1 + s1, S2 + s2
        res.Sw, res.S1, res.S2, res.t_done = Sw, S1, S2, t
        wbar = Sw / t
        f = monitor(Pb, wbar)
        if record:
            res.f_traj.append(f)
        if f > res.f_best:
            res.f_best, res.wbar_best, res.t_best = f, wbar.copy(), t
        if not early_stop:
            continue
        res.tie_margin = min(res.tie_margin, abs(f - alpha) / alpha)
        if f > alpha:
            res.outcome, res.t = BEAT, t
            break
        if f_prev is not None:
            if f_prev > 0.0:
                res.tie_margin = min(res.tie_margin, abs(abs(f - f_prev) / f_prev - delta) / delta)
            if f_prev > 0.0 and abs(f - f_prev) / f_prev < delta:
                cnt += 1
            else:
                cnt = 0
        f_prev = f
        if cnt >= patience:
            res.outcome, res.t = STABILIZED, t
            break
    return res


@dataclass
class SolveResult:
    margin: float
    w: Optional[np.ndarray]
    lower: float
    upper: float
    L: float
    U: float
    iters: int
    steps: list
    converged: bool
    tie_margin: float = math.inf  # least FtpResult.tie_margin over the search's tests


def solve(X, n_pos: int, eps: float = 1e-3, t_cap: Optional[int] = None,
          delta: float = 1e-4, patience: int = 10, tau: float = 1e-12,
          max_iters: Optional[int] = None, max_steps: int = 400,
          theory: bool = False) -> SolveResult:
    """(1-eps)-approximate maximum margin by the mirrored alpha search on (0, 2D].

    ``theory=True``: full T_theory iterations per test, no early exit."""
    Pb = setup(X, n_pos)
    n = Pb.X.shape[0]
    if t_cap is None:
        t_cap = min(int(math.ceil(math.log(n) / eps ** 2)), 20000)
    L, U = 0.0, 2.0 * Pb.D
    Lc, Uc = 0.0, U
    w_best = None
    iters = 0
    steps = []
    converged = False
    tie_margin = math.inf
    for _ in range(max_steps):
        if U - L <= eps * U:
            converged = True
            break
        if max_iters is not None and iters >= max_iters:
            break
        alpha = U - (U - L) / 3.0
        eps_k = (U - L) / (3.0 * alpha)
        T = theory_T(Pb, eps_k, alpha) if theory else min(theory_T(Pb, eps_k, alpha), t_cap)
        T = max(T, min_T(Pb))
        eta = math.sqrt(math.log(Pb.r) / T)
        r = ftp(Pb, alpha, T, eta, delta, patience, tau, early_stop=not theory)
        tie_margin = min(tie_margin, r.tie_margin)
        iters += r.t
        steps.append((alpha, T, r.outcome, r.t, r.f_best))
        Uc = min(Uc, r.ub_best)
        if r.wbar_best is not None and r.f_best > Lc:
            Lc, w_best = r.f_best, r.wbar_best / np.linalg.norm(r.wbar_best)
        if r.outcome == SEPARATED:
            U = alpha
        elif r.outcome == BEAT:
            L = max(L, r.f_best)
        else:
            L = max(L, r.f_best, L + (U - L) / 3.0)
        U = min(U, Uc)
        L = max(L, Lc)
    else:
        converged = U - L <= eps * U
    return SolveResult(margin=Lc, w=w_best, lower=Lc, upper=Uc, L=L, U=U,
                       iters=iters, steps=steps, converged=converged, tie_margin=tie_margin)
