"""Pins of the Jordan-algebra primitives (Section 2.1) against things other
than themselves: the matrix exponential of the Pauli embedding (d <= 3), the
Jordan power series, and algebra identities."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import eja

RNG = np.random.Generator(np.random.PCG64(1234))


def rand_soc(d, scale=1.0):
    return RNG.standard_normal(d) * scale, float(RNG.standard_normal() * scale)


def close(x, y, tol=1e-12):
    return np.allclose(x[0], y[0], rtol=tol, atol=tol) and abs(x[1] - y[1]) <= tol * max(1.0, abs(y[1]))


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("scale", [0.1, 1.0, 4.0])
def test_pauli_embedding_is_jordan_isomorphism(d, scale):
    for _ in range(5):
        x, y = rand_soc(d, scale), rand_soc(d, scale)
        X, Y = eja.soc_to_hermitian(x), eja.soc_to_hermitian(y)
        Z = eja.soc_to_hermitian(eja.soc_jordan(x, y))
        assert np.allclose(Z, 0.5 * (X @ Y + Y @ X), atol=1e-12 * scale ** 2)
        assert abs(np.trace(X).real - eja.soc_trace(x)) <= 1e-12 * scale
        ev = np.sort(np.linalg.eigvalsh(X))[::-1]
        lam1, lam2, _, _ = eja.soc_spectral(x)
        assert np.allclose(ev, [lam1, lam2], atol=1e-12 * scale)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("scale", [1e-3, 0.5, 3.0, 20.0])
def test_soc_exp_matches_expm(d, scale):
    for _ in range(5):
        x = rand_soc(d, scale)
        E = scipy.linalg.expm(eja.soc_to_hermitian(x))
        ref = eja.hermitian_to_soc(E, d)
        got = eja.soc_exp(x)
        tol = 1e-12 * max(1.0, abs(ref[1]))
        assert np.allclose(got[0], ref[0], rtol=1e-11, atol=tol)
        assert abs(got[1] - ref[1]) <= 1e-11 * abs(ref[1]) + tol


@pytest.mark.parametrize("d", [4, 7, 100])
def test_soc_exp_matches_jordan_power_series(d):
    for scale in (0.05, 0.3, 1.0):
        x = rand_soc(d, scale / math.sqrt(d))
        acc = eja.soc_identity(d)
        term = eja.soc_identity(d)
        for k in range(1, 40):
            term = eja.soc_jordan(term, x)
            term = (term[0] / k, term[1] / k)
            acc = (acc[0] + term[0], acc[1] + term[1])
        got = eja.soc_exp(x)
        assert close(got, acc, 1e-13)


@pytest.mark.parametrize("d", [1, 3, 17])
def test_exp_identities(d):
    for _ in range(5):
        x = rand_soc(d, 2.0)
        ex = eja.soc_exp(x)
        sq = eja.soc_jordan(ex, ex)
        e2 = eja.soc_exp((2 * x[0], 2 * x[1]))
        assert close(sq, e2, 1e-11)
        lam1, lam2, _, _ = eja.soc_spectral(x)
        assert abs(eja.soc_trace(ex) - (math.exp(lam1) + math.exp(lam2))) <= 1e-12 * eja.soc_trace(ex)
        # interior of the cone: ||w|| < s0
        assert np.linalg.norm(ex[0]) < ex[1]
    z = (np.zeros(d), 0.0)
    assert close(eja.soc_exp(z), eja.soc_identity(d), 1e-15)


@pytest.mark.parametrize("d", [1, 5])
def test_spectral_frame(d):
    x = rand_soc(d, 1.5)
    lam1, lam2, q1, q2 = eja.soc_spectral(x)
    rec = (lam1 * q1[0] + lam2 * q2[0], lam1 * q1[1] + lam2 * q2[1])
    assert close(rec, x, 1e-13)
    assert close(eja.soc_jordan(q1, q1), q1, 1e-14)
    assert close(eja.soc_jordan(q2, q2), q2, 1e-14)
    zero = eja.soc_jordan(q1, q2)
    assert np.allclose(zero[0], 0, atol=1e-15) and abs(zero[1]) < 1e-15
    e = eja.soc_identity(d)
    assert close((q1[0] + q2[0], q1[1] + q2[1]), e, 1e-15)
    # e is the identity of the product; the inner product is Tr(x o y)
    assert close(eja.soc_jordan(e, x), x, 1e-14)
    y = rand_soc(d)
    assert abs(eja.soc_inner(x, y) - eja.soc_trace(eja.soc_jordan(x, y))) < 1e-12


def test_jordan_identity():
    for d in (2, 6):
        x, y = rand_soc(d), rand_soc(d)
        x2 = eja.soc_jordan(x, x)
        lhs = eja.soc_jordan(x2, eja.soc_jordan(x, y))
        rhs = eja.soc_jordan(x, eja.soc_jordan(x2, y))
        assert close(lhs, rhs, 1e-12)


def test_blocks_agree_with_single_and_shift():
    n, d = 9, 4
    U = RNG.standard_normal((n, d)) * 3
    u0 = RNG.standard_normal(n) * 3
    U[2] = 0.0  # a block with zero vector part
    W, s = eja.soc_exp_blocks(U, u0)
    for i in range(n):
        ref = eja.soc_exp((U[i], u0[i]))
        assert np.allclose(W[i], ref[0], rtol=1e-13, atol=1e-13)
        assert abs(s[i] - ref[1]) < 1e-13 * ref[1]
    Ws, ss = eja.soc_exp_blocks(U, u0, shift=2.5)
    assert np.allclose(Ws * math.exp(2.5), W, rtol=1e-13)
    assert np.allclose(ss * math.exp(2.5), s, rtol=1e-13)
