"""Seeded synthetic inputs for the smallest-enclosing-sphere (SES) and
hard-margin SVM workloads.

This module only draws numbers: it holds none of the method's arithmetic and is
shared, unchanged, by the FP64 reference checker and the GPU path's tests and
benchmark.  Every generator takes an explicit seed and uses numpy's PCG64.

Workload shapes follow the paper's experiments (random point sets, Section 5;
n swept 2^10..2^20 at d = 64 and d swept 2..512 at n = 1e5), scaled to the
sizes the library is measured on:

* ``ses_uniform``   -- points uniform in the cube [-1, 1]^d (small SES case).
* ``ses_gaussian_outliers`` -- i.i.d. N(0, I) with a fraction of rows scaled
  (large SES case: n = 1e6, d = 100, 1 % outliers scaled x5).
* ``svm_planted``   -- two Gaussian classes N(+-0.1 u, I) filtered to a planted
  margin |u.x| >= 0.05 about the hyperplane u.x = 0 (rows of class +1 first).
* ``ses_ellipsoid`` -- points uniform in a random ellipsoid (batched case).

``bf16_round`` / ``bf16_to_f32`` give the round-to-nearest-even BF16 storage
of FP32 values, so a checker can be fed exactly the values a BF16-stored
matrix holds without reading them back from the GPU.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng",
    "ses_uniform",
    "ses_gaussian_outliers",
    "svm_planted",
    "ses_ellipsoid",
    "bf16_round",
    "bf16_to_f32",
    "CONFIGS",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def ses_uniform(n: int, d: int, seed: int) -> np.ndarray:
    """n x d points uniform in [-1, 1]^d, FP64, row-major."""
    return rng(seed).uniform(-1.0, 1.0, size=(n, d))


def ses_gaussian_outliers(n: int, d: int, seed: int, frac: float = 0.01,
                          scale: float = 5.0, dtype=np.float64) -> np.ndarray:
    """n x d rows i.i.d. N(0, I); ``round(frac * n)`` distinct rows scaled by
    ``scale``.  Generated in FP64 (or float32 directly when asked, to bound
    host memory at n = 1e6) and returned row-major."""
    g = rng(seed)
    if dtype == np.float32:
        x = g.standard_normal(size=(n, d), dtype=np.float32)
    else:
        x = g.standard_normal(size=(n, d))
    k = int(round(frac * n))
    if k > 0:
        idx = g.choice(n, k, replace=False)
        x[idx] *= scale
    return x


def svm_planted(n_pos: int, n_neg: int, d: int, seed: int, shift: float = 0.1,
                margin: float = 0.05, dtype=np.float64):
    """Two classes drawn N(+shift*u, I) and N(-shift*u, I) for a seeded unit
    vector u, keeping only rows with u.x >= margin (class +1) or
    u.x <= -margin (class -1).  Returns (X, u) with X = [P rows; Q rows]."""
    g = rng(seed)
    u = g.standard_normal(d)
    u /= np.linalg.norm(u)
    uf = u.astype(dtype)

    def draw(count: int, sign: float) -> np.ndarray:
        out = np.empty((count, d), dtype=dtype)
        got = 0
        chunk = max(1024, min(1 << 16, 2 * count))
        while got < count:
            if dtype == np.float32:
                z = g.standard_normal(size=(chunk, d), dtype=np.float32)
            else:
                z = g.standard_normal(size=(chunk, d))
            z += (sign * shift) * uf
            proj = z @ uf
            keep = z[(sign * proj) >= margin]
            take = min(count - got, keep.shape[0])
            out[got:got + take] = keep[:take]
            got += take
        return out

    X = np.concatenate([draw(n_pos, +1.0), draw(n_neg, -1.0)], axis=0)
    return X, u


def ses_ellipsoid(n: int, d: int, seed: int) -> np.ndarray:
    """Points uniform in a seeded random ellipsoid: z uniform in the unit ball
    (Gaussian direction times U^(1/d)), then y = Q diag(sigma) z + c with Q a
    random orthogonal matrix, sigma ~ logU[0.1, 1], c ~ N(0, I)."""
    g = rng(seed)
    z = g.standard_normal(size=(n, d))
    z /= np.linalg.norm(z, axis=1, keepdims=True)
    z *= g.uniform(0.0, 1.0, size=(n, 1)) ** (1.0 / d)
    q, r = np.linalg.qr(g.standard_normal(size=(d, d)))
    q *= np.sign(np.diag(r))
    sigma = np.exp(g.uniform(math.log(0.1), 0.0, size=d))
    c = g.standard_normal(d)
    return (z * sigma) @ q.T + c


def ses_batch_sizes(instances: int, n_lo: int, n_hi: int, dims, seed: int):
    """Sizes of a batch of SES instances: n log-uniform in [n_lo, n_hi]
    (rounded down to an integer), d drawn uniformly from ``dims``."""
    g = rng(seed)
    n = np.floor(np.exp(g.uniform(math.log(n_lo), math.log(n_hi), size=instances))).astype(np.int64)
    d = np.asarray(dims, dtype=np.int64)[g.integers(0, len(dims), size=instances)]
    return n, d


def ses_batch_offsets(n, d, align: int = 8):
    """Element offsets of the instances in one buffer, each instance's rows
    dense and starting at a multiple of `align` elements (so that vector
    loads of every instance are aligned); returns (offsets, total length)."""
    off, o = [], 0
    for nk, dk in zip(n, d):
        o = (o + align - 1) // align * align
        off.append(o)
        o += int(nk) * int(dk)
    return np.asarray(off, dtype=np.int64), o


def ses_batch_points(n, d, seed: int, align: int = 8):
    """Every instance's points in one float32 array at ses_batch_offsets:
    instance k is ses_ellipsoid(n[k], d[k], seed + 1 + k) rounded to float32
    (the gaps hold zeros).  Returns (points, offsets)."""
    off, total = ses_batch_offsets(n, d, align)
    out = np.zeros(total, dtype=np.float32)
    for k, (nk, dk) in enumerate(zip(n, d)):
        out[off[k]:off[k] + nk * dk] = ses_ellipsoid(int(nk), int(dk), seed + 1 + k).astype(np.float32).ravel()
    return out, off


def ses_batch_points_device(n, d, seed: int, device="cuda", align: int = 8):
    """The same recipe and layout as ses_batch_points, drawn on the device
    with torch's generator (a different random stream; for inputs too large
    to draw on the host in reasonable time).  Returns (float32 device tensor,
    offsets)."""
    import torch
    off, total = ses_batch_offsets(n, d, align)
    out = torch.zeros(total, dtype=torch.float32, device=device)
    gen = torch.Generator(device=device)
    for k, (nk, dk) in enumerate(zip(n, d)):
        o = int(off[k])
        nk, dk = int(nk), int(dk)
        g = rng(seed + 1 + k)
        q, r = np.linalg.qr(g.standard_normal(size=(dk, dk)))
        q *= np.sign(np.diag(r))
        sigma = np.exp(g.uniform(math.log(0.1), 0.0, size=dk))
        c = g.standard_normal(dk)
        A = torch.from_numpy((sigma[:, None] * q.T).astype(np.float32)).to(device)
        gen.manual_seed(seed + 1 + k)
        z = torch.randn(nk, dk, generator=gen, device=device)
        z /= torch.linalg.vector_norm(z, dim=1, keepdim=True)
        z *= torch.rand(nk, 1, generator=gen, device=device) ** (1.0 / dk)
        y = z @ A + torch.from_numpy(c.astype(np.float32)).to(device)
        out[o:o + nk * dk] = y.reshape(-1)
    return out, off


def bf16_round(x32: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 bit patterns (uint16), round to nearest, ties to even.
    NaN stays NaN (quiet)."""
    b = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32)
    lsb = (b >> np.uint32(16)) & np.uint32(1)
    r = (b + np.uint32(0x7FFF) + lsb) >> np.uint32(16)
    nan = np.isnan(np.ascontiguousarray(x32, dtype=np.float32))
    r = np.where(nan, (b >> np.uint32(16)) | np.uint32(0x40), r)
    return r.astype(np.uint16)


def bf16_to_f32(h: np.ndarray) -> np.ndarray:
    """BF16 bit patterns (uint16) -> the FP32 values they encode."""
    return (np.asarray(h, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


FP8_E4M3_MAX = 448.0


def fp8_e4m3_decode(codes: np.ndarray) -> np.ndarray:
    """FP8 E4M3 codes (uint8: sign, 4 exponent bits with bias 7, 3 mantissa
    bits; no infinities; S.1111.111 is NaN) -> the FP32 values they encode
    (exactly)."""
    c = np.asarray(codes, dtype=np.uint8).astype(np.int32)
    sign = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 0x7
    mag = np.where(e == 0, m * 2.0 ** -9, (8 + m) * np.exp2(e.astype(np.float64) - 10))
    mag = np.where((e == 0xF) & (m == 0x7), np.nan, mag)
    return (sign * mag).astype(np.float32)


def fp8_e4m3_encode(v32: np.ndarray) -> np.ndarray:
    """FP32 values -> FP8 E4M3 codes, round to nearest, ties to even,
    magnitudes from 464 (the tie above 448) up saturated to 448; NaN -> 0x7F
    (with the sign)."""
    v = np.ascontiguousarray(v32, dtype=np.float32)
    b = v.view(np.uint32)
    sign = ((b >> np.uint32(31)) & np.uint32(1)).astype(np.int32) << 7
    a = np.abs(v)
    ab = a.view(np.uint32).astype(np.int64)
    e = (ab >> 23) - 127
    # normals of the target (|a| >= 2^-6): 3 of the 23 mantissa bits, to nearest even
    m = ab & 0x7FFFFF
    m3 = m >> 20
    rem = m & 0xFFFFF
    up = (rem > 0x80000) | ((rem == 0x80000) & ((m3 & 1) == 1))
    m3 = m3 + up
    e = e + (m3 >> 3)
    m3 = m3 & 0x7
    normal = ((e + 7) << 3) | m3
    # subnormals of the target (|a| < 2^-6): multiples of 2^-9, to nearest even
    sub = np.rint(np.where(a < 2.0 ** -6, a, 0.0).astype(np.float64) * 512.0).astype(np.int64)
    code = np.where(a < 2.0 ** -6, sub, normal)
    code = np.where(a >= 464.0, 0x7E, np.minimum(code, 0x7E))
    code = np.where(np.isnan(v), 0x7F, code)
    return (code | sign).astype(np.uint8)


def fp8_rows(x32: np.ndarray):
    """Per-row scaled FP8 storage of a row-major matrix: scale s_r = max_c
    |x_rc| / 448 in FP32 (1 for an all-zero row) and codes of x_rc / s_r
    (FP32 quotient).  Returns (codes uint8 n x d, scales float32 n); the
    stored value of entry (r, c) is s_r * decode(code), exact in FP64."""
    x = np.ascontiguousarray(x32, dtype=np.float32)
    amax = np.max(np.abs(x), axis=1)
    s = (amax / np.float32(FP8_E4M3_MAX)).astype(np.float32)
    s = np.where(amax > 0, s, np.float32(1.0)).astype(np.float32)
    with np.errstate(invalid="ignore", divide="ignore"):
        q = (x / s[:, None]).astype(np.float32)
    return fp8_e4m3_encode(q), s


def fp8_values(codes: np.ndarray, scales: np.ndarray) -> np.ndarray:
    """The FP64 values held by per-row scaled FP8 storage."""
    return fp8_e4m3_decode(codes).astype(np.float64) * np.asarray(scales, dtype=np.float64)[:, None]


# The five measured workloads, by name.  Sizes, distributions and tolerances
# are what the tests and the benchmark use.
CONFIGS = {
    "ses_small_f64": dict(problem="ses", n=2000, d=3, eps=1e-3, t_cap=20000,
                          gen="uniform", seeds=list(range(10))),
    "ses_1m_d100": dict(problem="ses", n=1_000_000, d=100, eps=1e-3, t_cap=20000,
                        gen="gaussian_outliers", seeds=[0, 1, 2]),
    "svm_500k_d256": dict(problem="svm", n_pos=250_000, n_neg=250_000, d=256,
                          eps=1e-3, t_cap=20000, gen="planted", seeds=[0]),
    "ses_batched": dict(problem="ses", instances=4096, n_lo=1000, n_hi=100_000,
                        dims=[2, 3, 16, 64], gen="ellipsoid", seeds=[0]),
    "ses_diff_d64": dict(problem="ses", n=200_000, d=64, T=2000, checkpoint=50,
                         gen="gaussian", seeds=[0]),
}
