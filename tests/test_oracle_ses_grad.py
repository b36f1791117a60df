"""Pins of the gradient oracle (oracle/ses_grad.py): the adjoint recursion
against central finite differences of the forward map itself, the forward map
against the alpha-test with early exits off, and the two invariances of an
enclosing radius under rigid motions."""
import math

import numpy as np
import pytest

import synth
from oracle import ses, ses_grad

# (n, d, T, seed): small inputs on which the map is smooth at the step sizes
# used (the unrolled map can amplify perturbations over many iterations when
# ||W_t|| becomes small, so cases are fixed, not drawn).
CASES = [(10, 3, 30, 0), (12, 3, 40, 3), (9, 5, 25, 4)]


def central_fd(V, alpha, T, h, v1=0):
    G = np.zeros_like(V)
    for i in range(V.shape[0]):
        for k in range(V.shape[1]):
            Vp, Vm = V.copy(), V.copy()
            Vp[i, k] += h
            Vm[i, k] -= h
            G[i, k] = (ses_grad.radius(Vp, alpha, T, v1) - ses_grad.radius(Vm, alpha, T, v1)) / (2 * h)
    return G


@pytest.mark.parametrize("case", CASES)
def test_gradient_vs_central_differences(case):
    n, d, T, seed = case
    V = synth.ses_uniform(n, d, seed)
    alpha = 2.0 * ses.setup(V).D / 3.0
    R, G = ses_grad.radius_grad(V, alpha, T)
    assert R == ses_grad.radius(V, alpha, T)
    # truncation O(h^2) against rounding O(1e-16 / h): the better of two steps
    err = min(np.abs(G - central_fd(V, alpha, T, h)).max() for h in (1e-5, 1e-6))
    assert err <= 2e-6 * np.abs(G).max()


def test_gradient_vs_central_differences_v1_not_first():
    V = synth.ses_uniform(9, 3, 7)
    alpha = 2.0 * ses.setup(V, None, 4).D / 3.0
    _, G = ses_grad.radius_grad(V, alpha, 30, v1=4)
    err = min(np.abs(G - central_fd(V, alpha, 30, h, v1=4)).max() for h in (1e-5, 1e-6))
    assert err <= 2e-6 * np.abs(G).max()


@pytest.mark.parametrize("case", CASES + [(200, 8, 60, 11)])
def test_rigid_motion_invariances(case):
    """R is unchanged when every point moves by the same vector or is rotated
    about the origin, so sum_i g_i = 0 and sum_i v_i g_i^T is symmetric."""
    n, d, T, seed = case
    V = synth.ses_uniform(n, d, seed)
    alpha = 2.0 * ses.setup(V).D / 3.0
    _, G = ses_grad.radius_grad(V, alpha, T)
    scale = np.abs(G).max() * np.abs(V).max()
    assert np.abs(G.sum(axis=0)).max() <= 1e-10 * np.abs(G).max() * n
    M = V.T @ G
    assert np.abs(M - M.T).max() <= 1e-10 * scale * n


def test_forward_is_the_alpha_test_without_exits():
    V = synth.ses_uniform(30, 4, 5)
    P = ses.setup(V)
    alpha, T = 2.0 * P.D / 3.0, 50
    fw = ses_grad.forward(V, alpha, T)
    res = ses.ftp(P, alpha, T, math.sqrt(math.log(P.r) / T), early_stop=False, record=True)
    assert res.outcome in (ses.T_REACHED, ses.SEPARATED)
    np.testing.assert_allclose(fw.S[res.t_done], res.S, rtol=0, atol=1e-12)
    assert abs(res.f_traj[-1] - ses.monitor(P, fw.S[res.t_done] / res.t_done)) <= 1e-12
    if res.outcome == ses.T_REACHED:
        assert abs(fw.R - res.f_traj[-1]) <= 1e-12 * fw.R


def danskin_gradient(V):
    """dR*/dv_i = pi_i (v_i - c*)/R* for the smallest enclosing ball (c*, R*)
    (Welzl) with pi the optimal dual weights: the convex combination of the
    points on the sphere that equals c* (the dual of eq.(ses_qp))."""
    from oracle import exact
    c, R = exact.welzl(V)
    act = np.flatnonzero(np.abs(np.linalg.norm(V - c, axis=1) - R) <= 1e-9 * R)
    A = np.vstack([V[act].T, np.ones(act.size)])
    pi_a = np.linalg.lstsq(A, np.append(c, 1.0), rcond=None)[0]
    assert np.all(pi_a >= -1e-9) and np.abs(A @ pi_a - np.append(c, 1.0)).max() < 1e-9
    pi = np.zeros(V.shape[0])
    pi[act] = pi_a
    return R, pi[:, None] * (V - c) / R


def test_gradient_approaches_the_dual_weight_gradient():
    """At alpha just above R* and growing T, ubar_T approaches the centre and
    the adjoint approaches the optimal value's gradient (Danskin on the dual):
    the gap shrinks with T, and is a small fraction of the gradient once R is
    within a fraction of a percent of R* (a loose check: the unrolled map
    still carries O(gap) terms off the support)."""
    V = synth.ses_uniform(60, 2, 3)
    Rs, Gd = danskin_gradient(V)
    errs = []
    for T in (2000, 8000):
        R, G = ses_grad.radius_grad(V, 1.001 * Rs, T)
        errs.append(np.abs(G - Gd).max())
    assert R / Rs - 1.0 < 3e-3
    assert errs[1] < errs[0] and errs[1] <= 0.2 * np.abs(Gd).max()


@pytest.mark.parametrize("seed,alpha_frac", [(0, 0.55), (1, 0.8), (2, 1.0)])
def test_shift_bound_along_the_map(seed, alpha_frac):
    """Along the map every exponent kappa_t d_i (i != v1) stays at or below
    kappa_t (D + alpha), and the largest stays within 2 kappa_t alpha of it:
    the common shift the reverse pass takes (c_t - v1 is alpha times a mean of
    unit vectors, and the row at distance D from v1 keeps its distance to c_t
    above D - ||v1 - c_t||)."""
    V = synth.ses_gaussian_outliers(400, 6, seed, frac=0.02)
    T = 300
    P = ses.setup(V)
    alpha = alpha_frac * P.D
    fw = ses_grad.forward(V, alpha, T)
    for t in range(2, T + 1):
        c = fw.S[t - 1] / (t - 1)
        assert np.linalg.norm(c - P.V[P.v1]) <= alpha * (1 + 1e-12)
        kap = fw.eta * (t - 1) / (3.0 * P.D)
        top = kap * (P.D + alpha)
        largest = float(np.max(kap * np.linalg.norm(P.V[P.F] - c[None, :], axis=1)))
        assert largest <= top * (1 + 1e-12)
        assert largest >= top - 2.0 * kap * alpha - 1e-12 * top
