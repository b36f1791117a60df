"""Pins of the SES oracle (Sections 3 and 4.1) against a generic convex
solver, the SCMWU definition, the meta theorem, and exact enclosing balls."""
import math

import numpy as np
import pytest
import scipy.optimize

import synth
from oracle import certify, eja, exact, scmwu, ses

RNG = np.random.Generator(np.random.PCG64(2024))


def small(n=12, d=3, seed=0, radii=False):
    V = synth.ses_uniform(n, d, seed)
    g = RNG.uniform(0.0, 0.2, n) if radii else None
    return ses.setup(V, g, 0)


def test_setup_bounds():
    P = small(40, 3, 1)
    c, R = exact.welzl(P.V)
    assert P.D / 2 <= R + 1e-12 and R <= P.D + 1e-12
    assert P.r == 2 * 39 and abs(P.rho - 3 * P.D / math.sqrt(2)) < 1e-15


@pytest.mark.parametrize("radii", [False, True])
def test_oracle_closed_form_vs_convex_solver(radii):
    P = small(10, 3, 2, radii)
    alpha = 0.8 * P.D
    ubar = RNG.standard_normal(3) * 0.2
    W, s, _ = ses.hyperplane(P, ubar, alpha, 37, 0.05)
    u, value, _, Wsum, _ = ses.oracle(P, W, s, alpha)
    F = P.F

    def obj(z):
        uu, gg = z[:3], z[3]
        return -(np.sum((uu - P.V[F]) * W) + np.sum((gg - P.gamma[F]) * s))

    cons = [dict(type="ineq", fun=lambda z: alpha - z[3]),
            dict(type="ineq", fun=lambda z: z[3] - P.gamma[0] - np.linalg.norm(z[:3] - P.V[0]))]
    best = None
    for _ in range(6):
        z0 = np.concatenate([P.V[0] + RNG.standard_normal(3) * 0.01, [alpha]])
        r = scipy.optimize.minimize(obj, z0, constraints=cons, method="SLSQP",
                                    options=dict(ftol=1e-14, maxiter=500))
        if best is None or r.fun < best.fun:
            best = r
    assert abs(-best.fun - value) <= 1e-7 * max(1.0, abs(value))
    # KKT: u - v1 parallel to W with norm alpha - gamma1, gamma = alpha
    assert abs(np.linalg.norm(u - P.V[0]) - (alpha - P.gamma[0])) < 1e-12
    assert np.allclose((u - P.V[0]) / np.linalg.norm(u - P.V[0]), Wsum / np.linalg.norm(Wsum), atol=1e-12)
    # no feasible point does better
    for _ in range(2000):
        gg = alpha - abs(RNG.standard_normal()) * 0.1
        dirn = RNG.standard_normal(3)
        uu = P.V[0] + dirn / np.linalg.norm(dirn) * (gg - P.gamma[0]) * RNG.uniform()
        assert -obj(np.concatenate([uu, [gg]])) <= value + 1e-12


def test_first_iterate_and_tiebreak():
    P = small(9, 2, 3)
    W, s, logC = ses.hyperplane(P, None, 1.0, 0, 0.1)
    assert np.allclose(W, 0.0)
    assert np.allclose(s, math.sqrt(2) / P.r)          # e / r blockwise
    assert abs(logC - math.log(P.r)) < 1e-13            # Tr(exp 0) = r
    u, value, _, _, degenerate = ses.oracle(P, W, s, 1.0)
    assert degenerate and np.array_equal(u, P.V[0])


@pytest.mark.parametrize("radii", [False, True])
def test_trace_one_cone_membership_and_width(radii):
    P = small(30, 4, 4, radii)
    alpha = 0.7 * P.D
    T = 300
    eta = math.sqrt(math.log(P.r) / T)
    S = np.zeros(4)
    for t in range(1, T + 1):
        st = ses.step(P, S, t - 1, alpha, eta)
        W, s = st["W"], st["s"]
        assert abs(math.sqrt(2) * s.sum() - 1.0) < 1e-12
        assert np.all(np.linalg.norm(W, axis=1) <= s * (1 + 1e-12))
        # ||m(t)||_inf <= 1 for m = (1/rho)(u - v_i ; alpha - gamma_i)
        lam = (np.abs(alpha - P.gamma[P.F]) + np.linalg.norm(st["u"] - P.V[P.F], axis=1)) / math.sqrt(2)
        assert np.max(lam) / P.rho <= 1.0 + 1e-12
        S = st["S"]


def test_cumulative_loss_identity_matches_explicit_scmwu():
    # p(t+1) computed from the mean of past ORACLE outputs (eq. implement) must
    # equal SCMWU run on the explicit loss sequence m(tau) (eq. SCMWU).
    P = small(15, 3, 5, radii=True)
    alpha, T = 0.75 * P.D, 40
    eta = math.sqrt(math.log(P.r) / 1000)
    S = np.zeros(3)
    losses, ps = [], []
    for t in range(1, T + 1):
        st = ses.step(P, S, t - 1, alpha, eta)
        ps.append((st["W"], st["s"]))
        u = st["u"]
        losses.append(((u - P.V[P.F]) / P.rho, (alpha - P.gamma[P.F]) / P.rho))
        S = st["S"]
    ref = scmwu.soc_run(losses, eta)
    for (W, s), (Wr, sr) in zip(ps, ref):
        assert np.allclose(W, Wr, rtol=1e-10, atol=1e-15)
        assert np.allclose(s, sr, rtol=1e-10, atol=1e-15)


def test_meta_theorem_certificate_tiny():
    # Theorem meta: with T = T_theory and no early exit the test either
    # separates (then OPT > alpha) or ends with every point within (1+eps) alpha.
    V = synth.ses_uniform(8, 2, 11)
    c, R = exact.welzl(V)
    P = ses.setup(V)
    eps = 0.3
    for rel in (1.0, 1.2):
        alpha = rel * R
        T = ses.theory_T(P, eps, alpha)
        r = ses.ftp(P, alpha, T, math.sqrt(math.log(P.r) / T), early_stop=False)
        assert r.outcome == ses.T_REACHED               # alpha >= OPT never separates
        assert ses.monitor(P, r.S / r.t_done) <= (1 + eps) * alpha
    alpha = 0.7 * R                                      # (1+eps) alpha < OPT: must separate
    T = ses.theory_T(P, eps, alpha)
    r = ses.ftp(P, alpha, T, math.sqrt(math.log(P.r) / T), early_stop=False)
    assert r.outcome == ses.SEPARATED


@pytest.mark.slow
def test_theory_solve_within_eps_of_exact():
    V = synth.ses_uniform(8, 2, 12)
    c, R = exact.brute_ses(V)
    eps = 0.1
    r = ses.solve(V, eps=eps, theory=True)
    assert r.converged
    assert R <= r.radius * (1 + 1e-12) and r.radius <= (1 + eps) * R
    assert r.lower <= R * (1 + 1e-12)
    assert certify.ses_upper(V, None, r.center) <= r.radius * (1 + 1e-12)


@pytest.mark.slow
def test_practical_solve_certified_and_accurate():
    # Section 5 practice (cap, f < alpha exit, stabilisation).  The reported
    # radius is an actual enclosing radius (>= R*) and the certified lower
    # bound is below R*; the error is within the paper's reported range
    # (Table "ses_error": mean errors up to about 1e-2).
    V = synth.ses_uniform(400, 3, 3)
    c, R = exact.welzl(V)
    r = ses.solve(V, eps=1e-3)
    assert r.radius >= R * (1 - 1e-12)
    assert r.lower <= R * (1 + 1e-12)
    assert r.radius <= 1.02 * R
    assert abs(certify.ses_upper(V, None, r.center) - r.radius) < 1e-12


def test_weight_lower_bound_is_valid():
    V = synth.ses_uniform(50, 3, 13)
    c, R = exact.welzl(V)
    for _ in range(50):
        pi = RNG.dirichlet(np.ones(50) * 0.3)
        assert certify.ses_lower(V, pi) <= R * (1 + 1e-12)
    # and it is tight for the optimal support weights of a symmetric set
    sq = np.array([[1.0, 0], [-1, 0], [0, 1], [0, -1]])
    assert abs(certify.ses_lower(sq, np.ones(4) / 4) - 1.0) < 1e-15


def test_step_matches_ftp_trajectory():
    P = small(20, 3, 6)
    alpha, T = 0.9 * P.D, 50
    eta = math.sqrt(math.log(P.r) / T)
    r = ses.ftp(P, alpha, T, eta, early_stop=False, record=True)
    S = np.zeros(3)
    for t in range(1, r.t_done + 1):
        st = ses.step(P, S, t - 1, alpha, eta)
        assert st["value"] == r.values[t - 1]
        S = st["S"]
        assert ses.monitor(P, st["ubar"]) == r.f_traj[t - 1]


def test_kway_search_with_one_test_is_the_paper_search():
    V = synth.ses_uniform(300, 3, 21)
    a = ses.solve(V, eps=1e-2)
    b = ses.solve_kway(V, 1, eps=1e-2)
    assert [s[:4] for s in a.steps] == [s[:4] for s in b.steps]
    assert a.iters == b.iters == b.passes
    assert a.radius == b.radius and a.lower == b.lower and np.array_equal(a.center, b.center)
    assert (a.L, a.U) == (b.L, b.U)


@pytest.mark.slow
@pytest.mark.parametrize("k", [2, 3])
def test_kway_theory_solve_within_eps_of_exact(k):
    V = synth.ses_uniform(8, 2, 12)
    c, R = exact.brute_ses(V)
    eps = 0.1
    r = ses.solve_kway(V, k, eps=eps, theory=True)
    assert r.converged
    assert R <= r.radius * (1 + 1e-12) and r.radius <= (1 + eps) * R
    assert r.lower <= R * (1 + 1e-12)
    assert certify.ses_upper(V, None, r.center) <= r.radius * (1 + 1e-12)
    # each round's guesses split the interval into 2k + 1 equal parts
    assert len(r.steps) % k == 0


@pytest.mark.parametrize("k,seed", [(2, 12), (3, 12), (4, 5), (3, 7)])
def test_kway_stopped_tests_are_implied_by_theorem_meta(k, seed):
    """A stopped test decides nothing, which loses nothing only if its own
    outcome follows from the round's deciding tests.  With T = T_theory,
    Theorem meta gives that outcome: a test at alpha >= OPT never separates,
    one with (1 + eps) alpha < OPT always does; a separation certifies
    alpha < OPT.  So a test below a separated deciding test separates
    ((1 + eps_j) alpha_j <= L + 2j (U - L)/(2k + 1) < alpha_i < OPT), and a
    test above a non-separated deciding test i does not
    (OPT <= (1 + eps_i) alpha_i < alpha_j).  The oracle runs every test to its
    end, so each stopped test's own outcome is checked against the deciding
    tests of its round."""
    V = synth.ses_uniform(8, 2, seed)
    r = ses.solve_kway(V, k, eps=0.1, theory=True)
    assert len(r.stopped) == len(r.steps) and len(r.steps) % k == 0
    n_stopped = 0
    for r0 in range(0, len(r.steps), k):
        rnd = list(zip(r.steps[r0:r0 + k], r.stopped[r0:r0 + k]))
        dec = [st for st, s in rnd if not s]
        assert dec, "a round keeps at least one deciding test"
        for st, s in rnd:
            if not s:
                continue
            n_stopped += 1
            above_sep = any(x[2] == ses.SEPARATED and x[0] > st[0] for x in dec)
            below_not = any(x[2] != ses.SEPARATED and x[0] < st[0] for x in dec)
            assert above_sep or below_not
            assert (st[2] == ses.SEPARATED) == above_sep
    assert n_stopped > 0


@pytest.mark.slow
@pytest.mark.parametrize("k", [2, 4])
def test_kway_practical_solve_brackets_exact(k):
    V = synth.ses_uniform(400, 3, 3)
    c, R = exact.welzl(V)
    r = ses.solve_kway(V, k, eps=1e-3)
    assert r.radius >= R * (1 - 1e-12)
    assert r.lower <= R * (1 + 1e-12)
    assert r.radius <= 1.02 * R
    assert abs(certify.ses_upper(V, None, r.center) - r.radius) < 1e-12
    assert r.passes <= r.iters
