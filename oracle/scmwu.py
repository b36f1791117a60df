"""SCMWU online learner (Section 2.3, eq. SCMWU) over a product of second-order
cone blocks or over the orthant.

Test infrastructure (see package header).

    p(t+1) = exp(-eta sum_{tau<=t} m(tau)) / Tr(exp(-eta sum_{tau<=t} m(tau))),
    p(1)   = e / r.

Pins (tests/test_oracle_scmwu.py): on the orthant it is the textbook
multiplicative-weights softmax; for both cone types the regret bound of the
SCMWU theorem (Section 2.3) holds on random loss sequences with
||m||_inf <= 1; every iterate has trace one and lies in the cone.
"""
from __future__ import annotations

import numpy as np

from . import eja


def soc_iterate(MU: np.ndarray, mu0: np.ndarray, eta: float):
    """p = exp(-eta * M) / Tr(...) for a cumulative loss M = (MU; mu0) given
    blockwise (n blocks of Q^{d+1}).  Returns (W, s) with sum_i sqrt2 s_i = 1.

    The largest eigenvalue of -eta*M is used as a common shift (exact, see
    ``eja.soc_exp_blocks``)."""
    XU, x0 = -eta * MU, -eta * mu0
    lam1, _, _ = eja.soc_spectral_blocks(XU, x0)
    shift = float(np.max(lam1))
    W, s = eja.soc_exp_blocks(XU, x0, shift)
    tr = float(np.sum(eja.soc_trace_blocks(s)))
    return W / tr, s / tr


def orthant_iterate(m: np.ndarray, eta: float) -> np.ndarray:
    """p = exp(-eta m) / sum(exp(-eta m)) on R^n_+."""
    x = -eta * m
    e = eja.orthant_exp(x, float(np.max(x)))
    return e / np.sum(e)


def soc_run(losses, eta: float):
    """Play SCMWU against a fixed sequence of blockwise losses
    [(MU_t, mu0_t)] and return the iterates [(W_t, s_t)] (p(1) = e/r)."""
    n, d = losses[0][0].shape
    MU = np.zeros((n, d))
    mu0 = np.zeros(n)
    out = []
    for (LU, l0) in losses:
        out.append(soc_iterate(MU, mu0, eta))
        MU = MU + LU
        mu0 = mu0 + l0
    return out


def orthant_run(losses, eta: float):
    m = np.zeros_like(losses[0])
    out = []
    for l in losses:
        out.append(orthant_iterate(m, eta))
        m = m + l
    return out
