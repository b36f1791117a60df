"""Certified bounds on OPT for any candidate (FP64).

Test infrastructure (see package header).

SES (points and spheres):
  upper(c)       = max_i ||c - v_i|| + gamma_i  -- the sphere at c with this
                   radius encloses every input sphere, so OPT <= upper(c).
SES (points, gamma = 0):
  lower(pi)      = sqrt(sum_i pi_i ||v_i - cbar||^2), cbar = sum_i pi_i v_i, for
                   any simplex weights pi.  For every centre c,
                   sum_i pi_i ||v_i - c||^2 >= sum_i pi_i ||v_i - cbar||^2 and the
                   left side is at most OPT^2 at the optimal centre; this is
                   the objective of the SES quadratic program eq.(ses_qp)
                   evaluated at x = pi (negated), i.e. weak duality.
SVM:
  lower(w)       = max{min_P x.w - max_Q x.w, 0} / ||w||  -- margin of w.
  upper(mu, gam) = ||P mu - Q gam|| for simplex weights (eq.(pd)); by weak
                   duality between (SVM) and (PD) every such value bounds the
                   maximum margin from above.
"""
from __future__ import annotations

import numpy as np


def ses_upper(V, gamma, c) -> float:
    V = np.asarray(V, dtype=np.float64)
    g = np.zeros(V.shape[0]) if gamma is None else np.asarray(gamma, dtype=np.float64)
    return float(np.max(np.linalg.norm(V - np.asarray(c)[None, :], axis=1) + g))


def ses_lower(V, pi) -> float:
    V = np.asarray(V, dtype=np.float64)
    pi = np.asarray(pi, dtype=np.float64)
    pi = pi / np.sum(pi)
    cbar = pi @ V
    return float(np.sqrt(np.sum(pi * np.sum((V - cbar) ** 2, axis=1))))


def svm_lower(X, n_pos, w) -> float:
    X = np.asarray(X, dtype=np.float64)
    nw = float(np.linalg.norm(w))
    if not (nw > 0.0):
        return 0.0
    return max(float(np.min(X[:n_pos] @ w) - np.max(X[n_pos:] @ w)) / nw, 0.0)


def svm_upper(X, n_pos, mu, gam) -> float:
    X = np.asarray(X, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    gam = np.asarray(gam, dtype=np.float64)
    return float(np.linalg.norm(X[:n_pos].T @ (mu / mu.sum()) - X[n_pos:].T @ (gam / gam.sum())))
