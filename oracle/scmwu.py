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


def product_iterate(m: np.ndarray, n_orth: int, offsets, eta: float):
    """p = exp(-eta m) / Tr(exp(-eta m)) over the product cone
    R^{n_orth}_+ (+) Q^{d_1+1} (+) ... (+) Q^{d_k+1} (Section 2.1: the Loewner
    exponential and the trace of a direct sum act blockwise).

    m holds the orthant coordinates first, then block j in
    m[offsets[j]:offsets[j+1]] as its vector part followed by its scalar part
    (offsets[0] = n_orth).  One shift, the largest eigenvalue over all blocks,
    keeps the exponentials in range and cancels in the normalisation.
    Returns (p, logC) with logC = ln Tr(exp(-eta m))."""
    m = np.asarray(m, dtype=np.float64)
    x = -eta * m
    xo = x[:n_orth]
    blocks = [(x[offsets[j]:offsets[j + 1] - 1], x[offsets[j + 1] - 1]) for j in range(len(offsets) - 1)]
    lam = [float(np.max(xo))] if n_orth > 0 else []
    for U, u0 in blocks:
        l1, _, _ = eja.soc_spectral_blocks(U[None, :], np.array([u0]))
        lam.append(float(l1[0]))
    shift = max(lam)
    p = np.empty_like(x)
    tr = 0.0
    if n_orth > 0:
        e = eja.orthant_exp(xo, shift)
        p[:n_orth] = e
        tr += float(np.sum(e))
    for j, (U, u0) in enumerate(blocks):
        W, s = eja.soc_exp_blocks(U[None, :], np.array([u0]), shift)
        p[offsets[j]:offsets[j + 1] - 1] = W[0]
        p[offsets[j + 1] - 1] = s[0]
        tr += float(eja.soc_trace_blocks(s)[0])
    return p / tr, shift + float(np.log(tr))
