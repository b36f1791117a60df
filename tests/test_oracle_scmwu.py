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


# ------------------------------------------------ product of orthant and SOC blocks
def product_layout(n_orth, dims):
    offs = [n_orth]
    for d in dims:
        offs.append(offs[-1] + d + 1)
    return offs


def test_product_reduces_to_each_cone():
    m = RNG.standard_normal(40) * 5
    p, logC = scmwu.product_iterate(m, 40, [40], 0.3)
    assert np.allclose(p, scmwu.orthant_iterate(m, 0.3), rtol=1e-13)
    assert abs(logC - math.log(np.sum(np.exp(-0.3 * m)))) < 1e-12
    MU, mu0 = RNG.standard_normal((6, 3)), RNG.standard_normal(6)
    flat = np.concatenate([np.append(MU[i], mu0[i]) for i in range(6)])
    p, _ = scmwu.product_iterate(flat, 0, product_layout(0, [3] * 6), 0.7)
    W, s = scmwu.soc_iterate(MU, mu0, 0.7)
    assert np.allclose(p, np.concatenate([np.append(W[i], s[i]) for i in range(6)]), rtol=1e-13, atol=1e-16)


def test_product_blocks_are_exponentials_of_their_parts():
    """Each block of the normalised iterate is the block's own exponential
    (2x2 Hermitian representation for d = 3, against scipy's expm) divided by
    the one trace of the whole product."""
    import scipy.linalg
    dims = [3, 1, 3, 2]
    offs = product_layout(5, dims)
    m = RNG.standard_normal(offs[-1]) * 2
    eta = 0.4
    p, logC = scmwu.product_iterate(m, 5, offs, eta)
    C = math.exp(logC)
    assert np.allclose(p[:5] * C, np.exp(-eta * m[:5]), rtol=1e-12)
    tr = float(np.sum(p[:5]))
    for j, d in enumerate(dims):
        blk = p[offs[j]:offs[j + 1]]
        U, u0 = -eta * m[offs[j]:offs[j + 1] - 1], -eta * m[offs[j + 1] - 1]
        if d == 3:
            E = scipy.linalg.expm(eja.soc_to_hermitian((U, u0)))
            eu, e0 = eja.hermitian_to_soc(E, 3)
            assert np.allclose(blk * C, np.append(eu, e0), rtol=1e-11)
        assert np.linalg.norm(blk[:-1]) <= blk[-1] * (1 + 1e-12)   # in the cone
        tr += math.sqrt(2) * blk[-1]
    assert abs(tr - 1.0) < 1e-12


@pytest.mark.parametrize("eta", [0.05, 0.5])
def test_product_regret_bound(eta):
    """SCMWU theorem on the product cone: regret <= eta T + ln r / eta for
    losses with ||m||_inf <= 1 (r = n_orth + 2 * blocks)."""
    T, n_orth, dims = 70, 6, [2, 5, 1]
    offs = product_layout(n_orth, dims)
    cum = np.zeros(offs[-1])
    played = 0.0
    for _ in range(T):
        p, _ = scmwu.product_iterate(cum, n_orth, offs, eta)
        l = RNG.standard_normal(offs[-1])
        lams = list(np.abs(l[:n_orth]))
        for j in range(len(dims)):
            U, u0 = l[offs[j]:offs[j + 1] - 1], l[offs[j + 1] - 1]
            nu = np.linalg.norm(U)
            lams += [abs(u0 + nu) / math.sqrt(2), abs(u0 - nu) / math.sqrt(2)]
        l *= float(RNG.uniform(0.3, 1.0)) / max(lams)
        # <l, p> in the product's trace inner product: orthant dot + SOC blocks' sqrt2-free dot
        played += float(l @ p)
        cum += l
    lam_min = float(np.min(cum[:n_orth]))
    for j in range(len(dims)):
        U, u0 = cum[offs[j]:offs[j + 1] - 1], cum[offs[j + 1] - 1]
        lam_min = min(lam_min, (u0 - np.linalg.norm(U)) / math.sqrt(2))
    r = n_orth + 2 * len(dims)
    assert played <= lam_min + eta * T + math.log(r) / eta + 1e-9
