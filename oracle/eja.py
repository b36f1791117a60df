"""Euclidean Jordan algebras of the cones used by SES and SVM (Section 2.1).

Test infrastructure (see package header): FP64, plain numpy, no blocking.

Second-order cone Q^{d+1}: elements are pairs (u; u0) with u in R^d.  Section
2.1 fixes
  * Jordan product  (u; u0) o (v; v0) = (1/sqrt2) (v0 u + u0 v ; u.v + u0 v0)
  * identity        e = (0; sqrt2), rank 2
  * eigenvalues     lambda_{1,2} = (u0 +- ||u||) / sqrt2
  * idempotents     q_{1,2} = (1/sqrt2) (+- u/||u|| ; 1)  (any unit vector if u = 0)
  * trace           Tr(u; u0) = sqrt2 u0 = lambda_1 + lambda_2
  * inner product   x . y = Tr(x o y) = u.v + u0 v0
and the Loewner extension exp(sum lambda_i q_i) = sum exp(lambda_i) q_i.

Non-negative orthant R^d_+: componentwise product, e = 1, rank d, trace = sum.

Product cones: rank, trace and spectral decomposition are blockwise.

A batch of n SOC blocks is stored as (U, u0) with U of shape (n, d) and u0 of
shape (n,).

Pins (tests/test_oracle_eja.py): Q^{d+1} for d <= 3 is Jordan-isomorphic to
2x2 Hermitian matrices through Pauli matrices, so ``soc_exp`` must equal
``scipy.linalg.expm`` there; for any d it must equal the Jordan power series
sum_k x^k / k!; exp(x) o exp(x) = exp(2x); exp(0) = e; Tr exp(x) =
e^lambda1 + e^lambda2; exp(x) lies in the interior of the cone.
"""
from __future__ import annotations

import numpy as np

SQRT2 = np.sqrt(2.0)


# ---------------------------------------------------------------- single SOC
def soc_identity(d: int):
    """Identity element e = (0; sqrt2) of Q^{d+1} (Section 2.1)."""
    return np.zeros(d), SQRT2


def soc_jordan(x, y):
    """Jordan product (u;u0) o (v;v0) = (1/sqrt2)(v0 u + u0 v ; u.v + u0 v0)."""
    u, u0 = x
    v, v0 = y
    return (v0 * u + u0 * v) / SQRT2, (float(u @ v) + u0 * v0) / SQRT2


def soc_inner(x, y) -> float:
    """x . y = Tr(x o y) = u.v + u0 v0 (Section 2.1)."""
    return float(x[0] @ y[0]) + x[1] * y[1]


def soc_trace(x) -> float:
    """Tr(u; u0) = sqrt2 u0."""
    return SQRT2 * x[1]


def soc_spectral(x):
    """Spectral decomposition (lambda1, lambda2, q1, q2) of (u; u0).

    lambda_{1,2} = (u0 +- ||u||)/sqrt2 and q_{1,2} = (1/sqrt2)(+- v; 1) with
    v = u/||u||, or the first unit vector when u = 0 (the paper allows any
    unit vector there)."""
    u, u0 = x
    nu = float(np.linalg.norm(u))
    if nu > 0.0:
        v = u / nu
    else:
        v = np.zeros_like(u)
        if v.size:
            v[0] = 1.0
    lam1 = (u0 + nu) / SQRT2
    lam2 = (u0 - nu) / SQRT2
    q1 = (v / SQRT2, 1.0 / SQRT2)
    q2 = (-v / SQRT2, 1.0 / SQRT2)
    return lam1, lam2, q1, q2


def soc_exp(x):
    """Loewner exponential exp(x) = e^lambda1 q1 + e^lambda2 q2."""
    lam1, lam2, q1, q2 = soc_spectral(x)
    a, b = np.exp(lam1), np.exp(lam2)
    return a * q1[0] + b * q2[0], a * q1[1] + b * q2[1]


def soc_eigmin(x) -> float:
    return soc_spectral(x)[1]


# --------------------------------------------------------- batches of blocks
def soc_spectral_blocks(U: np.ndarray, u0: np.ndarray):
    """Blockwise spectral data of n SOC blocks: (lam1, lam2, V) where row i of
    V is the unit vector of block i.  When a block's vector part is zero its
    two eigenvalues coincide, so any function of it has zero vector part
    whatever unit vector is chosen; V holds a zero row there."""
    nu = np.linalg.norm(U, axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        V = np.where(nu[:, None] > 0.0, U / nu[:, None], 0.0)
    return (u0 + nu) / SQRT2, (u0 - nu) / SQRT2, V


def soc_exp_blocks(U: np.ndarray, u0: np.ndarray, shift: float = 0.0):
    """exp(x_i - shift*e) for every block i, returned as (W, s) with
    W[i] = (1/sqrt2)(e^{l1-shift} - e^{l2-shift}) V[i] and
    s[i]  = (1/sqrt2)(e^{l1-shift} + e^{l2-shift}).

    Because e is the sum of the idempotents of every block, exp(x - c e) =
    e^{-c} exp(x) exactly (same Jordan frame, eigenvalues shifted by c); a
    common shift therefore cancels in any trace normalisation and only keeps
    the exponentials in floating-point range."""
    lam1, lam2, V = soc_spectral_blocks(U, u0)
    a = np.exp(lam1 - shift)
    b = np.exp(lam2 - shift)
    W = ((a - b) / SQRT2)[:, None] * V
    s = (a + b) / SQRT2
    return W, s


def soc_trace_blocks(s: np.ndarray) -> np.ndarray:
    return SQRT2 * s


# ------------------------------------------------------------------- orthant
def orthant_exp(x: np.ndarray, shift: float = 0.0) -> np.ndarray:
    """Loewner exponential on R^d_+ (componentwise, Section 2.1)."""
    return np.exp(x - shift)


# --------------------------------------------------- Pauli embedding (pins)
def soc_to_hermitian(x) -> np.ndarray:
    """phi(u; u0) = (1/sqrt2)(u0 I + u1 s1 + u2 s2 + u3 s3) for d <= 3 with
    s1 = diag(1,-1), s2 = [[0,1],[1,0]], s3 = [[0,-i],[i,0]].  phi maps the
    SOC Jordan product to (XY+YX)/2, the SOC trace to the matrix trace, and so
    the Loewner exponential to the matrix exponential.  Used only to pin
    ``soc_exp`` against scipy.linalg.expm."""
    u, u0 = x
    d = u.shape[0]
    assert d <= 3
    s = [np.array([[1, 0], [0, -1]], dtype=complex),
         np.array([[0, 1], [1, 0]], dtype=complex),
         np.array([[0, -1j], [1j, 0]], dtype=complex)]
    M = u0 * np.eye(2, dtype=complex)
    for k in range(d):
        M = M + u[k] * s[k]
    return M / SQRT2


def hermitian_to_soc(M: np.ndarray, d: int):
    """Inverse of ``soc_to_hermitian`` (coefficients in the Pauli basis)."""
    u0 = np.real(np.trace(M)) / SQRT2
    s = [np.array([[1, 0], [0, -1]], dtype=complex),
         np.array([[0, 1], [1, 0]], dtype=complex),
         np.array([[0, -1j], [1j, 0]], dtype=complex)]
    u = np.array([np.real(np.trace(M @ s[k])) / SQRT2 for k in range(d)])
    return u, u0
