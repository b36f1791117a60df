"""Pins of the exact references against closed forms and each other."""
import json
import math
import os

import numpy as np
import pytest

from oracle import exact

GOLD = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.Generator(np.random.PCG64(7))


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("case", load("ses_closed_form.json")["cases"], ids=lambda c: c["name"])
def test_ses_closed_forms(case):
    V = np.array(case["points"], dtype=np.float64)
    c, r = exact.welzl(V)
    assert abs(r - case["radius"]) < 1e-12 * max(1, case["radius"])
    if "center" in case:
        assert np.allclose(c, case["center"], atol=1e-12)
    if V.shape[0] <= 12:
        cb, rb = exact.brute_ses(V)
        assert abs(rb - case["radius"]) < 1e-12 * max(1, case["radius"])


@pytest.mark.parametrize("d", [2, 3])
def test_welzl_matches_brute_force(d):
    for _ in range(12):
        n = int(RNG.integers(3, 11))
        V = RNG.uniform(-1, 1, (n, d))
        c1, r1 = exact.welzl(V, seed=int(RNG.integers(1 << 30)))
        c2, r2 = exact.brute_ses(V)
        assert abs(r1 - r2) < 1e-9
        assert np.max(np.linalg.norm(V - c1, axis=1)) <= r1 * (1 + 1e-12)


def test_welzl_sphere_points():
    # points on the unit sphere including an antipodal pair: radius exactly 1
    V = RNG.standard_normal((300, 3))
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    V = np.vstack([V, [[0, 0, 1.0], [0, 0, -1.0]]])
    c, r = exact.welzl(V)
    assert abs(r - 1.0) < 1e-9 and np.linalg.norm(c) < 1e-8


@pytest.mark.parametrize("case", load("svm_closed_form.json")["cases"], ids=lambda c: c["name"])
def test_svm2d_closed_forms(case):
    X = np.array(case["points"], dtype=np.float64)
    m, w = exact.svm2d(X, case["n_pos"])
    assert abs(m - case["margin"]) < 1e-12


def test_svm2d_beats_random_directions():
    for _ in range(5):
        P = RNG.standard_normal((15, 2)) + [3, 1]
        Q = RNG.standard_normal((15, 2)) - [3, 1]
        X = np.vstack([P, Q])
        m, w = exact.svm2d(X, 15)
        th = RNG.uniform(0, 2 * math.pi, 20000)
        W = np.stack([np.cos(th), np.sin(th)], 1)
        best = np.max(np.min(P @ W.T, 0) - np.max(Q @ W.T, 0))
        assert m >= best - 1e-12
        assert m <= best + 1e-3  # fine sampling gets close to the optimum
