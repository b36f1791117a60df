"""Smallest enclosing sphere (SES) by the primal-dual meta-algorithm, FP64.

Test infrastructure (see package header).  Written from Sections 3 and 4.1 of
the paper in its order and notation:

* split (Section 4.1, proof of the SES theorem): C = {||u - v1|| <= gamma - gamma1}
  (easy), F = all other constraints (hard); K = product over i != 1 of
  Q^{d+1}, K' = Q^{d+1}.
* dual SCP eq.(dualses): y = (u; gamma), a_j = (+)(e_j; 0), a_{d+1} = (+)(0; 1),
  c = (+)(v_i; gamma_i), b = (0; 1).  Hence sum_j a_j y_j - c is the block
  vector (+)_i (u - v_i ; gamma - gamma_i).
* bounds: D = max_{i>=2} ||v1 - v_i|| + gamma1 + gamma_i, OPT in [D/2, D];
  width rho = 3D/sqrt2, R = sqrt2, rank r = 2(n-1).
* hyperplane update eq.(implement): p(t+1) = exp(-(eta t / rho)
  (sum_j a_j ybar_j(t) - c)) / C with C the trace normaliser.
* ORACLE eq.(ses_oracle): gamma = alpha and u = v1 + (alpha - gamma1) W/||W||
  with W = sum_i w_i (linear objective over a ball).  The objective value is
  sum_i (u - v_i).w_i + (alpha - gamma_i) s_i; a negative value separates,
  i.e. certifies OPT > alpha (Section 3, "Testing of separation").
* T = ceil(36 D^2 ln(2n-2) / (eps^2 alpha^2)), eta = sqrt(ln r / T)
  (SES theorem with the meta theorem).
* monitor f(t) = max_i ||ubar(t) - v_i|| + gamma_i, early "better than alpha"
  exit and the stabilisation rule |f(t)-f(t-1)|/f(t-1) < delta for
  ``patience`` consecutive iterations (Section 5, implementation strategies).
* adaptive search (Section 3, "From feasibility to optimization"):
  alpha_i = L + (U-L)/3, eps_i = (U-L)/(3 alpha_i).

Readings where the paper is silent (each is listed with its reason in the
design notes shipped with the library):
  R1  v1 is input row ``v1`` (default 0).
  R2  at t = 1 (and whenever W = 0) every point of the ball is an ORACLE
      maximiser; u = v1 is taken.
  R3  T_k = min(T_theory, t_cap), raised to at least ceil(ln r) so that
      eta <= 1 as the SCMWU theorem requires.
  R4  separation is declared when value < -tau * alpha (||W|| + 1/sqrt2),
      tau = 1e-12, so rounding-level ties count as "not separated".
  R5  f(t-1) = 0 skips the stabilisation ratio and resets the run count.
  R6  after a stabilised or capped test that did not separate, the search
      takes the paper's conclusion OPT <= (1+eps_i) alpha_i for its interval
      (U <- L + 2(U-L)/3), while the reported radius is the certified
      min_t f(t) and its centre; every observed f tightens U.
  R7  the search stops when U - L <= eps * L (additive eps*OPT in the paper,
      with L <= OPT) or when the iteration budget is spent.

Pins: tests/test_oracle_ses.py (closed-form ORACLE checked against a generic
convex solver and KKT, width bound, trace-one and cone membership of p(t),
the cumulative-loss identity against explicit SCMWU over the stored losses,
the meta theorem's certificate on tiny inputs, and final radii against
Welzl's algorithm / brute force).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import eja

SQRT2 = math.sqrt(2.0)

SEPARATED, BEAT, STABILIZED, T_REACHED = "separated", "beat_alpha", "stabilized", "t_reached"


@dataclass
class SesSetup:
    V: np.ndarray          # n x d, float64
    gamma: np.ndarray      # n, float64
    v1: int
    D: float
    rho: float
    R: float
    r: int
    F: np.ndarray          # indices of the hard blocks (i != v1)


def setup(V, gamma=None, v1: int = 0) -> SesSetup:
    """Bounds and constants of the SES split (Section 4.1)."""
    V = np.asarray(V, dtype=np.float64)
    n, d = V.shape
    if n < 2:
        raise ValueError("SES needs at least two input spheres")
    g = np.zeros(n) if gamma is None else np.asarray(gamma, dtype=np.float64)
    F = np.array([i for i in range(n) if i != v1], dtype=np.int64)
    D = float(np.max(np.linalg.norm(V[v1] - V[F], axis=1) + g[F]) + g[v1])
    return SesSetup(V=V, gamma=g, v1=v1, D=D, rho=3.0 * D / SQRT2, R=SQRT2,
                    r=2 * (n - 1), F=F)


def hyperplane(P: SesSetup, ubar: Optional[np.ndarray], alpha: float, t_prev: int,
               eta: float):
    """p(t_prev + 1) from eq.(implement): the Loewner exponential of
    -(eta t_prev / rho) * (+)_i (ubar - v_i ; alpha - gamma_i), normalised to
    trace one.  Returns (W, s, logC): the blocks (w_i; s_i) of p for the hard
    indices F, and the log of the unnormalised trace C."""
    F = P.F
    if t_prev == 0:
        # the cumulative loss is empty: exp(0) = e, so p(1) = e / r
        XU = np.zeros((F.size, P.V.shape[1]))
        x0 = np.zeros(F.size)
    else:
        k = eta * t_prev / P.rho
        XU = -k * (ubar[None, :] - P.V[F])
        x0 = -k * (alpha - P.gamma[F])
    lam1, _, _ = eja.soc_spectral_blocks(XU, x0)
    shift = float(np.max(lam1))
    W, s = eja.soc_exp_blocks(XU, x0, shift)
    C = float(np.sum(eja.soc_trace_blocks(s)))
    return W / C, s / C, shift + math.log(C)


def oracle(P: SesSetup, W: np.ndarray, s: np.ndarray, alpha: float, tau: float = 1e-12):
    """Closed-form solution of eq.(ses_oracle) and its objective value.

    Returns (u, value, scale, Wsum, degenerate).  ``value`` is
    sum_i (u - v_i).w_i + (alpha - gamma_i) s_i at the maximiser (u; alpha);
    ``scale`` = alpha (||Wsum|| + sum_i s_i) is the magnitude against which
    reading R4 compares it."""
    F = P.F
    v1 = P.V[P.v1]
    Wsum = np.sum(W, axis=0)
    nW = float(np.linalg.norm(Wsum))
    degenerate = not (nW > 0.0)
    if degenerate:
        u = v1.copy()
    else:
        u = v1 + (alpha - P.gamma[P.v1]) * Wsum / nW
    value = float(np.sum((u[None, :] - P.V[F]) * W) + np.sum((alpha - P.gamma[F]) * s))
    scale = alpha * (nW + float(np.sum(s)))
    return u, value, scale, Wsum, degenerate


def monitor(P: SesSetup, ubar: np.ndarray) -> float:
    """f = max_i ||ubar - v_i|| + gamma_i (Section 5)."""
    return float(np.max(np.linalg.norm(P.V - ubar[None, :], axis=1) + P.gamma))


def theory_T(P: SesSetup, eps: float, alpha: float) -> int:
    """T = ceil(4 R^2 rho^2 ln r / (eps^2 alpha^2)) = ceil(36 D^2 ln(2n-2) / (eps^2 alpha^2))."""
    return int(math.ceil(4.0 * P.R ** 2 * P.rho ** 2 * math.log(P.r) / (eps ** 2 * alpha ** 2)))


def min_T(P: SesSetup) -> int:
    return max(1, int(math.ceil(math.log(P.r))))


@dataclass
class FtpResult:
    outcome: str
    t: int                      # iteration at which the test ended
    S: np.ndarray               # sum of the ORACLE centres u(1..t_done)
    t_done: int                 # number of centres averaged into S
    f_best: float
    ubar_best: Optional[np.ndarray]
    t_best: int
    f_traj: List[float] = field(default_factory=list)
    values: List[float] = field(default_factory=list)
    scales: List[float] = field(default_factory=list)
    logC: List[float] = field(default_factory=list)
    # closest approach of the test's decisions to their thresholds, relative:
    # the separation test (value against -tau * scale, in units of scale), the
    # f < alpha exit (in units of alpha) and the stabilisation ratio (in units
    # of delta), over every iteration the test ran; a rounding-level change
    # can flip a decision only where its margin is that small
    tie_margin: float = math.inf
    # largest cancellation ratio sum_i ||w_i|| / ||sum_i w_i|| of the ORACLE's
    # weighted sum over the test's iterations: the factor by which a relative
    # change of the weights moves the direction of W, hence u (a trajectory
    # through a near-zero W is sensitive to rounding from there on)
    cancel_max: float = 1.0


def step(P: SesSetup, S: np.ndarray, t_prev: int, alpha: float, eta: float,
         tau: float = 1e-12):
    """One iteration t = t_prev + 1 from the running sum S of past centres.

    Returns a dict with the new centre u, the ORACLE value / scale, log C, the
    separation flag, the mean ubar(t) and f(t_prev) (None when t_prev = 0)."""
    ubar_prev = S / t_prev if t_prev > 0 else None
    W, s, logC = hyperplane(P, ubar_prev, alpha, t_prev, eta)
    u, value, scale, Wsum, degenerate = oracle(P, W, s, alpha, tau)
    sep = value < -tau * scale
    out = dict(u=u, value=value, scale=scale, logC=logC, separated=sep, W=W, s=s,
               Wsum=Wsum, degenerate=degenerate,
               f_prev=monitor(P, ubar_prev) if t_prev > 0 else None)
    S_new = S + u
    out["S"] = S_new
    out["ubar"] = S_new / (t_prev + 1)
    return out


def ftp(P: SesSetup, alpha: float, T: int, eta: float, delta: float = 1e-4,
        patience: int = 10, tau: float = 1e-12, early_stop: bool = True,
        record: bool = False) -> FtpResult:
    """The alpha-feasibility test (meta-algorithm box, Section 3) for SES."""
    d = P.V.shape[1]
    S = np.zeros(d)
    f_prev = None
    cnt = 0
    res = FtpResult(outcome=T_REACHED, t=T, S=S, t_done=0, f_best=math.inf,
                    ubar_best=None, t_best=0)
    for t in range(1, T + 1):
        ubar_prev = S / (t - 1) if t > 1 else None
        W, s, logC = hyperplane(P, ubar_prev, alpha, t - 1, eta)
        u, value, scale, Wsum, _ = oracle(P, W, s, alpha, tau)
        nWs = float(np.linalg.norm(Wsum))
        if t > 1:
            res.cancel_max = max(res.cancel_max, float(np.sum(np.linalg.norm(W, axis=1))) / nWs if nWs > 0.0 else math.inf)
        if record:
            res.values.append(value)
            res.scales.append(scale)
            res.logC.append(logC)
        if scale > 0.0:
            res.tie_margin = min(res.tie_margin, abs(value + tau * scale) / scale)
        if value < -tau * scale:
            res.outcome, res.t = SEPARATED, t
            break
        S = S + u
        res.S, res.t_done = S, t
        ubar = S / t
        f = monitor(P, ubar)
        if record:
            res.f_traj.append(f)
        if f < res.f_best:
            res.f_best, res.ubar_best, res.t_best = f, ubar.copy(), t
        if not early_stop:
            continue
        res.tie_margin = min(res.tie_margin, abs(f - alpha) / alpha)
        if f < alpha:
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
    radius: float
    center: np.ndarray
    lower: float
    upper: float
    L: float
    U: float
    iters: int
    steps: list
    converged: bool
    passes: int = 0             # k-way search: sum over rounds of the longest test
    tie_margin: float = math.inf  # least FtpResult.tie_margin over the search's tests
    cancel_max: float = 1.0       # largest FtpResult.cancel_max over the search's tests
    stopped: Optional[list] = None  # k-way search: per step, whether the round stopped the test (moot)


def solve(V, gamma=None, v1: int = 0, eps: float = 1e-3, t_cap: Optional[int] = None,
          delta: float = 1e-4, patience: int = 10, tau: float = 1e-12,
          max_iters: Optional[int] = None, max_steps: int = 200,
          theory: bool = False) -> SolveResult:
    """(1+eps)-approximate SES by the adaptive alpha search over [D/2, D].

    ``theory=True`` runs every test for its full T_theory iterations with no
    early exit, as the meta theorem assumes; otherwise Section 5's practice
    (cap, f < alpha exit, stabilisation) applies."""
    P = setup(V, gamma, v1)
    n = P.V.shape[0]
    if t_cap is None:
        t_cap = min(int(math.ceil(math.log(n) / eps ** 2)), 20000)
    L, U = P.D / 2.0, P.D
    Lc, Uc = L, U
    center = P.V[v1].copy()
    iters = 0
    steps = []
    converged = False
    tie_margin = math.inf
    cancel_max = 1.0
    for _ in range(max_steps):
        if U - L <= eps * L:
            converged = True
            break
        if max_iters is not None and iters >= max_iters:
            break
        alpha = L + (U - L) / 3.0
        eps_k = (U - L) / (3.0 * alpha)
        T = theory_T(P, eps_k, alpha) if theory else min(theory_T(P, eps_k, alpha), t_cap)
        T = max(T, min_T(P))
        eta = math.sqrt(math.log(P.r) / T)
        r = ftp(P, alpha, T, eta, delta, patience, tau, early_stop=not theory)
        tie_margin = min(tie_margin, r.tie_margin)
        cancel_max = max(cancel_max, r.cancel_max)
        iters += r.t
        steps.append((alpha, T, r.outcome, r.t, r.f_best))
        if r.f_best < Uc:
            Uc, center = r.f_best, r.ubar_best.copy()
        if r.outcome == SEPARATED:
            L = alpha
            Lc = max(Lc, alpha)
        elif r.outcome == BEAT:
            U = r.f_best
        else:
            U = min(U, L + 2.0 * (U - L) / 3.0)
        U = min(U, Uc)
    else:
        converged = U - L <= eps * L
    return SolveResult(radius=Uc, center=center, lower=Lc, upper=Uc, L=L, U=U,
                       iters=iters, steps=steps, converged=converged, tie_margin=tie_margin,
                       cancel_max=cancel_max)


def solve_kway(V, k: int, gamma=None, v1: int = 0, eps: float = 1e-3, t_cap: Optional[int] = None,
               delta: float = 1e-4, patience: int = 10, tau: float = 1e-12,
               max_iters: Optional[int] = None, max_rounds: int = 200,
               theory: bool = False) -> SolveResult:
    """k-way alpha search (Section 3 names other searching methods besides
    the one it spells out; reading K1): each round cuts [L, U] into 2k + 1
    equal parts and runs the k alpha-feasibility tests at
    alpha_i = L + (2i - 1)(U - L)/(2k + 1) with eps_i = (U - L)/((2k + 1) alpha_i),
    so that (1 + eps_i) alpha_i = L + 2i (U - L)/(2k + 1).  The tests advance
    together; in the order in which they end (ties: the lower alpha first), an
    ended test stops the tests its outcome makes moot: a separated test those
    below it (their alphas are below a certified lower bound), any other test
    those above it (their alphas are above the conclusion (1 + eps_i) alpha_i).
    A stopped test decides nothing.  After the round, every separated test
    raises L to its alpha (a certificate); every other deciding test whose
    alpha is not below the new L lowers U to its conclusion (f_best when f
    beat alpha, else L + 2i (U - L)/(2k + 1)); every deciding test's f tightens
    U and the certified radius.  k = 1 is solve()'s search.  A stopped test
    counts the iterations it ran until it was stopped; `passes` counts the
    iterations of the rounds when the k tests advance together (each round
    lasts until its last deciding test ends)."""
    P = setup(V, gamma, v1)
    n = P.V.shape[0]
    if t_cap is None:
        t_cap = min(int(math.ceil(math.log(n) / eps ** 2)), 20000)
    L, U = P.D / 2.0, P.D
    Lc, Uc = L, U
    center = P.V[v1].copy()
    iters = passes = 0
    steps = []
    stopped_steps = []
    converged = False
    tie_margin = math.inf
    cancel_max = 1.0
    g = 2 * k + 1
    for _ in range(max_rounds):
        if U - L <= eps * L:
            converged = True
            break
        if max_iters is not None and iters >= max_iters:
            break
        round_ = []
        for i in range(1, k + 1):
            alpha = L + (2 * i - 1) * (U - L) / g
            eps_i = (U - L) / (g * alpha)
            T = theory_T(P, eps_i, alpha) if theory else min(theory_T(P, eps_i, alpha), t_cap)
            T = max(T, min_T(P))
            eta = math.sqrt(math.log(P.r) / T)
            r = ftp(P, alpha, T, eta, delta, patience, tau, early_stop=not theory)
            tie_margin = min(tie_margin, r.tie_margin)
            cancel_max = max(cancel_max, r.cancel_max)
            round_.append((alpha, L + 2 * i * (U - L) / g, T, r))
            steps.append((alpha, T, r.outcome, r.t, r.f_best))
        # the moot tests, in the order in which the tests end
        stop = [None] * k
        live = set(range(k))
        for i in sorted(range(k), key=lambda i: (round_[i][3].t, i)):
            if i not in live:
                continue
            live.discard(i)
            moot = range(i) if round_[i][3].outcome == SEPARATED else range(i + 1, k)
            for j in moot:
                if j in live:
                    live.discard(j)
                    stop[j] = round_[i][3].t
        stopped_steps += [stop[i] is not None for i in range(k)]
        ran = [r.t if stop[i] is None else min(r.t, stop[i]) for i, (_, _, _, r) in enumerate(round_)]
        iters += sum(ran)
        passes += max(ran)
        deciding = [x for i, x in enumerate(round_) if stop[i] is None]
        for alpha, concl, T, r in deciding:
            if r.f_best < Uc:
                Uc, center = r.f_best, r.ubar_best.copy()
        L_new = max([L] + [a for a, _, _, r in deciding if r.outcome == SEPARATED])
        Lc = max(Lc, L_new)
        U_new = min(U, Uc)
        for alpha, concl, T, r in deciding:
            if r.outcome != SEPARATED and alpha >= L_new:
                U_new = min(U_new, r.f_best if r.outcome == BEAT else concl)
        L, U = L_new, U_new
    else:
        converged = U - L <= eps * L
    return SolveResult(radius=Uc, center=center, lower=Lc, upper=Uc, L=L, U=U, iters=iters,
                       steps=steps, converged=converged, passes=passes, tie_margin=tie_margin,
                       cancel_max=cancel_max, stopped=stopped_steps)
