"""Exact references that pin the approximate methods.

Test infrastructure (see package header).

* ``welzl``      -- smallest enclosing ball of points (Welzl 1991, cited in
                    Section 4.1 among the exact SES methods), move-to-front
                    form: recursion depth is bounded by d + 2, each level is a
                    loop over the points.
* ``brute_ses``  -- minimum over all subsets of at most d+1 points of their
                    circumscribed ball (centre in the subset's affine hull)
                    that encloses every point; exponential, for n <= 12.
* ``svm2d``      -- exact maximum margin (SVM objective s1 + s2) in the plane:
                    the optimal normal is parallel to a cross-class difference
                    p - q or orthogonal to a within-class edge (the closest
                    points of two convex polygons are vertex-vertex or
                    vertex-edge), so enumerating those directions and scoring
                    each by min_P x.w - max_Q x.w is exact.
* ``circumball`` -- smallest ball having a set of affinely independent points
                    on its boundary.

These are pinned against each other and against closed forms
(tests/test_oracle_exact.py: regular simplices, collinear points, two-point
SVM).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def circumball(R: np.ndarray):
    """Centre and radius of the smallest ball with all rows of R on its
    boundary: c = p0 + sum_j l_j (p_j - p0) with (p_j - p0).(c - p0) =
    ||p_j - p0||^2 / 2."""
    R = np.asarray(R, dtype=np.float64)
    p0 = R[0]
    if R.shape[0] == 1:
        return p0.copy(), 0.0
    A = R[1:] - p0
    G = A @ A.T
    b = 0.5 * np.sum(A * A, axis=1)
    lam = np.linalg.lstsq(G, b, rcond=None)[0]
    c = p0 + lam @ A
    r = float(np.max(np.linalg.norm(R - c, axis=1)))
    return c, r


def _inside(p, c, r, tol):
    return float(np.linalg.norm(p - c)) <= r * (1.0 + tol) + tol


def welzl(V: np.ndarray, seed: int = 0, tol: float = 1e-12):
    """Smallest enclosing ball (centre, radius) of the rows of V."""
    V = np.asarray(V, dtype=np.float64)
    n, d = V.shape
    order = list(np.random.Generator(np.random.PCG64(seed)).permutation(n))

    def mtf(lst, m, boundary):
        if boundary:
            c, r = circumball(V[boundary])
        else:
            c, r = V[lst[0]].copy(), 0.0
        if len(boundary) == d + 1:
            return c, r
        i = 0
        while i < m:
            p = lst[i]
            if not _inside(V[p], c, r, tol):
                c, r = mtf(lst, i, boundary + [p])
                # move p to the front of the list
                lst.pop(i)
                lst.insert(0, p)
            i += 1
        return c, r

    c, r = mtf(order, n, [])
    # final radius measured against every point
    r = float(np.max(np.linalg.norm(V - c, axis=1)))
    return c, r


def brute_ses(V: np.ndarray, tol: float = 1e-10):
    """Exact smallest enclosing ball by enumeration (small n only)."""
    V = np.asarray(V, dtype=np.float64)
    n, d = V.shape
    best = (None, math.inf)
    for k in range(1, min(d + 1, n) + 1):
        for sub in itertools.combinations(range(n), k):
            c, r = circumball(V[list(sub)])
            rr = float(np.max(np.linalg.norm(V - c, axis=1)))
            if rr <= r * (1.0 + tol) + tol and rr < best[1]:
                best = (c, rr)
    return best


def margin(X: np.ndarray, n_pos: int, w: np.ndarray) -> float:
    """min_P x.w - max_Q x.w for a unit vector w (may be negative)."""
    X = np.asarray(X, dtype=np.float64)
    return float(np.min(X[:n_pos] @ w) - np.max(X[n_pos:] @ w))


def svm2d(X: np.ndarray, n_pos: int):
    """Exact maximum margin and its unit normal for planar point sets."""
    X = np.asarray(X, dtype=np.float64)
    assert X.shape[1] == 2
    P, Q = X[:n_pos], X[n_pos:]
    cands = []
    for p in P:
        for q in Q:
            cands.append(p - q)
    for S in (P, Q):
        for a, b in itertools.combinations(range(S.shape[0]), 2):
            e = S[b] - S[a]
            cands.append(np.array([-e[1], e[0]]))
            cands.append(np.array([e[1], -e[0]]))
    best = (-math.inf, None)
    for w in cands:
        nw = np.linalg.norm(w)
        if nw == 0.0:
            continue
        w = w / nw
        m = margin(X, n_pos, w)
        if m > best[0]:
            best = (m, w)
    return best
