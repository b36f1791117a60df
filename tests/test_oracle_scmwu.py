"""Pins of the SCMWU learner (Section 2.3): textbook MWU on the orthant and
the regret theorem on both cone types."""
import math

import numpy as np
import pytest
import scipy.special

from oracle import eja, scmwu

RNG = np.random.Generator(np.random.PCG64(99))


def test_orthant_is_softmax():
    for _ in range(10):
        m = RNG.standard_normal(50) * 30
        eta = float(RNG.uniform(0.01, 1.0))
        assert np.allclose(scmwu.orthant_iterate(m, eta), scipy.special.softmax(-eta * m), rtol=1e-13)


def soc_losses(T, n, d):
    out = []
    for _ in range(T):
        LU = RNG.standard_normal((n, d))
        l0 = RNG.standard_normal(n)
        lam = np.maximum(np.abs(l0 + np.linalg.norm(LU, axis=1)), np.abs(l0 - np.linalg.norm(LU, axis=1))) / math.sqrt(2)
        c = float(RNG.uniform(0.3, 1.0)) / np.max(lam)   # ||m||_inf <= 1
        out.append((LU * c, l0 * c))
    return out


@pytest.mark.parametrize("eta", [0.05, 0.3, 1.0])
def test_soc_regret_bound(eta):
    T, n, d = 60, 7, 3
    losses = soc_losses(T, n, d)
    ps = scmwu.soc_run(losses, eta)
    played = 0.0
    MU, mu0 = np.zeros((n, d)), np.zeros(n)
    for (LU, l0), (W, s) in zip(losses, ps):
        # trace one and membership of the product cone
        assert abs(math.sqrt(2) * s.sum() - 1.0) < 1e-12
        assert np.all(np.linalg.norm(W, axis=1) <= s * (1 + 1e-12))
        played += float(np.sum(LU * W) + np.sum(l0 * s))
        MU, mu0 = MU + LU, mu0 + l0
    lam_min = float(np.min(eja.soc_spectral_blocks(MU, mu0)[1]))
    r = 2 * n
    assert played <= lam_min + eta * T + math.log(r) / eta + 1e-9


@pytest.mark.parametrize("eta", [0.05, 0.5])
def test_orthant_regret_bound(eta):
    T, n = 80, 11
    losses = [RNG.uniform(-1, 1, n) for _ in range(T)]
    ps = scmwu.orthant_run(losses, eta)
    played = sum(float(l @ p) for l, p in zip(losses, ps))
    lam_min = float(np.min(np.sum(losses, axis=0)))
    assert played <= lam_min + eta * T + math.log(n) / eta + 1e-9


def test_first_iterate_is_e_over_r():
    n, d = 5, 4
    W, s = scmwu.soc_iterate(np.zeros((n, d)), np.zeros(n), 0.7)
    assert np.allclose(W, 0.0)
    # e = (0; sqrt2) per block, r = 2n
    assert np.allclose(s, math.sqrt(2) / (2 * n))
