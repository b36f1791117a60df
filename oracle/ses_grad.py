"""Gradient of the SES radius after a fixed number of MWU iterations, FP64.

Test infrastructure (see package header).

The map (point sets, all gamma_i = 0): the points V (n x d) go through T
iterations of one alpha-feasibility test of the SES split (Section 4.1) at a
fixed alpha and fixed T, eta = sqrt(ln r / T), with no early exit (Section 5's
rules off), exactly as ``ses.step`` computes them; the result is the Section 5
monitor at the final mean,

    R(V) = f(ubar_T) = max_i ||v_i - ubar_T||,   ubar_T = S_T / T,
    S_t = S_{t-1} + u(t),   u(t) = v1 + alpha W_t / ||W_t||   (eq. ses_oracle),
    W_t = sum_{i != v1} a_i(t) (v_i - c_t),   c_t = ubar_{t-1},
    a_i(t) = sinh(kappa_t d_i) / d_i,   d_i = ||v_i - c_t||,
    kappa_t = eta (t - 1) / (rho sqrt2) = eta (t - 1) / (3 D).

a_i is the vector part of the Loewner exponential of the block
-(eta (t-1)/rho)(c_t - v_i ; alpha) (Section 2.1: spectral values
(x0 +- ||x||)/sqrt2) up to factors common to every block, which cancel in
W_t / ||W_t||.  D = max_{i != v1} ||v1 - v_i|| is a function of the points too.

The gradient dR/dV is taken by the adjoint (reverse) recursion through the
iterations, every partial derivative written out from the formulas above:

* R: the active point i* gets (v_i* - ubar_T)/R; the adjoint of S_T is
  lambda_T = (ubar_T - v_i*) / (R T).
* u(t) = v1 + alpha What: v1 gets lambda_t; the adjoint of W_t is
  lambda_W = alpha (I - What What^T) lambda_t / ||W_t||.
* W_t: with delta_i = v_i - c_t, the adjoint of delta_i is
  a_i lambda_W + beta_i delta_i, beta_i = a_i'(d_i) (delta_i . lambda_W) / d_i,
  a_i'(d) = (kappa cosh(kappa d) d - sinh(kappa d)) / d^2.  Row i gets it,
  c_t gets minus their sum, and lambda_{t-1} = lambda_t + (adjoint of c_t)/(t-1).
* kappa_t through D: dW_t/dkappa = sum_i cosh(kappa d_i) delta_i and
  dkappa_t/dD = -kappa_t / D; the accumulated adjoint of D goes to v1 and
  to the row j attaining D, along (v1 - v_j)/D.
* t = 1: W_1 = 0 and u(1) = v1 (reading R2 of ``ses``); only v1 depends on it.

Readings (listed with reasons in the design notes):
  G1  the differentiated map is R(V) above: fixed alpha and T (constants of the
      map), D recomputed from the points (so the map is that of the forward
      pass run on V), ties in the two maxima broken by the first index (the
      map is differentiable where both maxima are unique).
  G2  the workloads take alpha = 2D/3, the first guess of the search of
      Section 3 on [D/2, D], evaluated once and then held fixed.

Pins: tests/test_oracle_ses_grad.py (central finite differences of the
forward map ``radius`` on small inputs, translation invariance sum_i dR/dv_i = 0,
rotation invariance sum_i (v_i g_i^T - g_i v_i^T) = 0, the forward map's
trajectory against ``ses.ftp`` with early exits off, and, loosely, the optimal
radius's gradient from the dual weights of Welzl's ball as T grows).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import ses


@dataclass
class Forward:
    P: ses.SesSetup
    alpha: float
    T: int
    eta: float
    S: np.ndarray       # (T + 1) x d running sums S_0 .. S_T
    R: float
    i_star: int         # argmax_i ||v_i - ubar_T||


def forward(V, alpha: float, T: int, v1: int = 0) -> Forward:
    """T fixed-alpha iterations of ``ses.step`` (no early exit) and R = f(ubar_T)."""
    P = ses.setup(V, None, v1)
    eta = math.sqrt(math.log(P.r) / T)
    d = P.V.shape[1]
    S = np.zeros((T + 1, d))
    for t in range(1, T + 1):
        st = ses.step(P, S[t - 1], t - 1, alpha, eta)
        S[t] = st["S"]
    ubar = S[T] / T
    dist = np.linalg.norm(P.V - ubar[None, :], axis=1)
    i_star = int(np.argmax(dist))
    return Forward(P=P, alpha=alpha, T=T, eta=eta, S=S, R=float(dist[i_star]), i_star=i_star)


def radius(V, alpha: float, T: int, v1: int = 0) -> float:
    """The map R(V) (reading G1)."""
    return forward(V, alpha, T, v1).R


def radius_grad(V, alpha: float, T: int, v1: int = 0, fw: Forward | None = None):
    """(R, dR/dV) by the adjoint recursion through the T iterations."""
    if fw is None:
        fw = forward(V, alpha, T, v1)
    P, S = fw.P, fw.S
    V = P.V
    F = P.F
    n, d = V.shape
    G = np.zeros((n, d))
    ubar = S[T] / T
    g = (ubar - V[fw.i_star]) / fw.R          # dR/d ubar_T
    G[fw.i_star] -= g                          # the direct term (v_i* - ubar_T)/R
    lam = g / T                                # adjoint of S_T
    lam_D = 0.0
    for t in range(T, 0, -1):
        G[P.v1] += lam                         # u(t) = v1 + ...
        if t == 1:
            break                              # u(1) = v1
        c = S[t - 1] / (t - 1)
        kap = fw.eta * (t - 1) / (P.rho * ses.SQRT2)
        delta = V[F] - c[None, :]
        dist = np.linalg.norm(delta, axis=1)
        m = float(np.max(kap * dist))          # common factor e^{-m}, cancels
        ep = np.exp(kap * dist - m)
        em = np.exp(-kap * dist - m)
        sh, ch = 0.5 * (ep - em), 0.5 * (ep + em)
        a = sh / dist
        W = a @ delta
        nW = float(np.linalg.norm(W))
        Wh = W / nW
        lam_W = fw.alpha * (lam - Wh * float(Wh @ lam)) / nW
        dot = delta @ lam_W
        a1 = (kap * ch * dist - sh) / dist ** 2
        beta = a1 * dot / dist
        adj_delta = a[:, None] * lam_W[None, :] + beta[:, None] * delta
        G[F] += adj_delta
        lam_D += float(ch @ dot) * (-kap / P.D)
        lam = lam - adj_delta.sum(axis=0) / (t - 1)
    dv = np.linalg.norm(V[P.v1][None, :] - V[F], axis=1)
    j = int(F[int(np.argmax(dv))])
    e = (V[P.v1] - V[j]) / P.D
    G[P.v1] += lam_D * e
    G[j] -= lam_D * e
    return fw.R, G
