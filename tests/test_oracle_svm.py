"""Pins of the SVM oracle (Section 3 min form with Section 4.2)."""
import math

import numpy as np
import pytest
import scipy.special

import synth
from oracle import certify, exact, svm

RNG = np.random.Generator(np.random.PCG64(77))


def planted2d(n1, n2, seed, gap=1.0):
    g = np.random.Generator(np.random.PCG64(seed))
    P = g.standard_normal((n1, 2)) * 0.6 + [gap + 1.0, 0.3]
    Q = g.standard_normal((n2, 2)) * 0.6 - [gap + 1.0, -0.2]
    P = P[P[:, 0] > gap / 2]
    Q = Q[Q[:, 0] < -gap / 2]
    return np.vstack([P, Q]), P.shape[0]


def test_oracle_closed_form_vs_brute_force():
    X, n_pos = planted2d(20, 20, 1)
    Pb = svm.setup(X, n_pos)
    for t_prev in (0, 5, 60):
        ybar = (RNG.standard_normal(2) * 0.3, 0.1, 0.2) if t_prev else None
        mu, gam, _ = svm.hyperplane(Pb, ybar, t_prev, 0.2)
        for alpha in (0.3 * Pb.D, 1.1 * Pb.D, 1.9 * Pb.D):
            w, s1, s2, value, _, V, _ = svm.oracle(Pb, mu, gam, alpha)
            assert abs(np.linalg.norm(w) - 1) < 1e-14 and s1 + s2 == pytest.approx(alpha)
            assert s1 <= Pb.D + 1e-15 and s2 <= Pb.D + 1e-15
            trm, trg = mu.sum(), gam.sum()
            # feasible set: s1 in [alpha - D, D], s2 = alpha - s1 (tight at optimum), ||w|| <= 1
            for s in np.linspace(alpha - Pb.D, Pb.D, 101):
                th = RNG.uniform(0, 2 * math.pi, 50)
                for ww in np.stack([np.cos(th), np.sin(th)], 1) * RNG.uniform(0, 1, (50, 1)):
                    assert V @ ww - trm * s - trg * (alpha - s) <= value + 1e-12


def test_iterates_are_softmax_and_width_bound():
    X, n_pos = planted2d(30, 25, 2)
    Pb = svm.setup(X, n_pos)
    alpha, T = 1.0, 200
    eta = math.sqrt(math.log(Pb.r) / T)
    Sw, S1, S2 = np.zeros(2), 0.0, 0.0
    for t in range(1, T + 1):
        st = svm.step(Pb, Sw, S1, S2, t - 1, alpha, eta)
        p = np.concatenate([st["mu"], st["gam"]])
        assert abs(p.sum() - 1) < 1e-12 and np.all(p >= 0)
        if t > 1:
            sl = svm.slack(Pb, Sw / (t - 1), S1 / (t - 1), S2 / (t - 1))
            assert np.allclose(p, scipy.special.softmax(-(eta * (t - 1) / Pb.rho) * sl), rtol=1e-12)
        # width: |slack_i(y(t))| <= rho = 2D for the ORACLE output
        sl_now = svm.slack(Pb, st["w"], st["s1"], st["s2"])
        assert np.max(np.abs(sl_now)) <= Pb.rho * (1 + 1e-12)
        # any simplex weights give an upper bound on the margin
        assert st["ub"] >= exact.svm2d(X, n_pos)[0] - 1e-12
        Sw, S1, S2 = st["Sw"], st["S1"], st["S2"]


def test_pd_claim_on_separation():
    X, n_pos = planted2d(25, 25, 3)
    Pb = svm.setup(X, n_pos)
    m_star, _ = exact.svm2d(X, n_pos)
    alpha = 1.5 * m_star
    T = 4000
    r = svm.ftp(Pb, alpha, T, math.sqrt(math.log(Pb.r) / T), early_stop=False)
    assert r.outcome == svm.SEPARATED
    Sw, S1, S2 = r.Sw, r.S1, r.S2
    ybar = (Sw / r.t_done, S1 / r.t_done, S2 / r.t_done)
    mu, gam, _ = svm.hyperplane(Pb, ybar, r.t_done, math.sqrt(math.log(Pb.r) / T))
    assert svm.pd_value(Pb, mu, gam) < alpha
    assert m_star <= svm.pd_value(Pb, mu, gam) + 1e-12


@pytest.mark.slow
def test_theory_solve_within_eps_of_exact_2d():
    X, n_pos = planted2d(8, 8, 4, gap=2.0)
    m_star, _ = exact.svm2d(X, n_pos)
    eps = 0.1
    r = svm.solve(X, n_pos, eps=eps, theory=True)
    assert r.converged
    assert (1 - eps) * m_star <= r.margin <= m_star * (1 + 1e-12)
    assert r.upper >= m_star * (1 - 1e-12)


@pytest.mark.slow
def test_practical_solve_certified_planted():
    X, u = synth.svm_planted(300, 300, 2, seed=5, shift=0.6, margin=0.3)
    m_star, _ = exact.svm2d(X, 300)
    r = svm.solve(X, 300, eps=1e-3)
    assert r.lower <= m_star * (1 + 1e-12) <= r.upper * (1 + 1e-12)
    assert abs(certify.svm_lower(X, 300, r.w) - r.margin) < 1e-12
    # Section 5 practice: an actual margin, below the exact one, within the
    # accuracy the stabilisation rule allows here (a few percent).
    assert 0.9 * m_star <= r.margin <= m_star * (1 + 1e-12)


def test_certify_svm_upper_pins():
    """certify.svm_upper = ||P mu - Q gam|| over normalised simplex weights (the
    dual polytope-distance problem, eq.(pd)): equal to the hull distance at the
    closest points' weights (closed form), and never below the exact maximum
    margin (direction enumeration in 2-D) for random weights, by weak duality."""
    # closed form: the segment P from (0, 1) to (2, 1) and the point (1, -1)
    X = np.array([[0.0, 1.0], [2.0, 1.0], [1.0, -1.0]])
    assert abs(certify.svm_upper(X, 2, [0.5, 0.5], [1.0]) - 2.0) < 1e-15
    assert abs(certify.svm_upper(X, 2, [1.0, 0.0], [1.0]) - np.sqrt(5.0)) < 1e-15
    assert abs(certify.svm_upper(X, 2, [3.0, 3.0], [2.0]) - 2.0) < 1e-15    # weights are normalised
    rng = np.random.default_rng(21)
    for seed in range(5):
        Xs, _ = synth.svm_planted(15, 12, 2, seed=seed, shift=0.6, margin=0.3)
        m_star, _ = exact.svm2d(Xs, 15)
        for _ in range(50):
            mu, gam = rng.random(15), rng.random(12)
            assert certify.svm_upper(Xs, 15, mu, gam) >= m_star * (1 - 1e-12)
        # the weights of the two closest points (a vertex pair) reach the bound
        # only when the hull distance is a vertex-vertex distance; an extreme
        # weight vector is still an upper bound
        i, j = 0, 0
        assert certify.svm_upper(Xs, 15, np.eye(15)[i], np.eye(12)[j]) >= m_star * (1 - 1e-12)
