"""Seeded synthetic inputs for O(d) synchronization problems.

This module only *draws* inputs; it contains none of the solver's arithmetic.
Both the FP64 CPU oracle (through the tests) and the GPU path use it, so a
problem is a pure function of its seed.

Measurement model (paper, Sec. 2.2, eq. ``def:measurements``):
    A = Z Z^T + sigma W,  Z = (Z_1; ...; Z_n) with Z_i in O(d),
    W symmetric with i.i.d. standard normal entries in its upper triangle.

* Ground truth Z: Haar-distributed blocks, drawn as the sign-corrected QR
  factor of an i.i.d. Gaussian d x d matrix (Mezzadri's construction).  The
  paper projects a Gaussian matrix onto O(d); both constructions give the Haar
  law, and this one keeps the polar factor (part of the method) out of the
  generator.
* Noise W: element (r, c) of the nd x nd matrix is a pure function of
  (seed, min(r, c), max(r, c)) through the counter-based generator
  Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11) followed by the Box-Muller transform.  Any row
  panel of A can therefore be regenerated without the rest, and the GPU
  library carries its own implementation of the same published generator.
* Diagonal blocks: by default W_ii is drawn like every other block (the dense
  symmetric Gaussian W of the benchmark workloads).  ``zero_diag_blocks=True``
  gives the paper's model W_ii = 0, hence A_ii = Z_i Z_i^T = I.
* Incomplete observations (paper, Sec. 4.1): with ``p < 1`` each off-diagonal
  block pair (i < j) is kept with probability p and otherwise A_ij = A_ji = 0.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "PHILOX_M0", "PHILOX_M1", "PHILOX_W0", "PHILOX_W1",
    "philox4x32_10", "noise_elements", "mask_blocks",
    "haar_blocks", "measurement_matrix", "measurement_rows",
    "perturbed_start", "sigma_for", "TAG_NOISE", "TAG_MASK", "stiefel_start",
]

# Philox4x32 constants from the SC'11 paper / Random123 distribution.
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85

TAG_NOISE = 0  # third counter word for the Gaussian noise stream
TAG_MASK = 1   # third counter word for the observation-mask stream

_U32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32 with 10 rounds.

    All arguments are integer arrays (broadcastable) holding 32-bit values.
    Returns four uint64 arrays holding the 32-bit output words.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & _U32
    c1 = np.asarray(c1, dtype=np.uint64) & _U32
    c2 = np.asarray(c2, dtype=np.uint64) & _U32
    c3 = np.asarray(c3, dtype=np.uint64) & _U32
    k0 = np.asarray(k0, dtype=np.uint64) & _U32
    k1 = np.asarray(k1, dtype=np.uint64) & _U32
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    w0 = np.uint64(PHILOX_W0)
    w1 = np.uint64(PHILOX_W1)
    s32 = np.uint64(32)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + w0) & _U32
            k1 = (k1 + w1) & _U32
        p0 = m0 * c0          # < 2^64, exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> s32, p0 & _U32
        hi1, lo1 = p1 >> s32, p1 & _U32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def _key(seed: int):
    seed = int(seed)
    if seed < 0:
        raise ValueError("seed must be non-negative")
    return seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF


def noise_elements(rows, cols, seed: int):
    """Standard normal W[r, c] for arrays of global element indices.

    W is symmetric: the draw uses (min(r, c), max(r, c)) as the counter.
    u1 in (0, 1] and u2 in [0, 1) are 53-bit uniforms built from output
    words (x0, x1) and (x2, x3); W = sqrt(-2 ln u1) cos(2 pi u2).
    """
    r = np.asarray(rows, dtype=np.int64)
    c = np.asarray(cols, dtype=np.int64)
    lo = np.minimum(r, c)
    hi = np.maximum(r, c)
    k0, k1 = _key(seed)
    x0, x1, x2, x3 = philox4x32_10(hi, lo, TAG_NOISE, 0, k0, k1)
    m1 = (x0 << np.uint64(21)) | (x1 >> np.uint64(11))
    m2 = (x2 << np.uint64(21)) | (x3 >> np.uint64(11))
    u1 = (m1.astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = m2.astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def mask_blocks(bi, bj, seed: int, p: float):
    """Observation indicator for block pairs (paper Sec. 4.1), symmetric.

    Diagonal block pairs are always 'observed' (they never enter the
    gradient; they only shift the spectrum).
    """
    bi = np.asarray(bi, dtype=np.int64)
    bj = np.asarray(bj, dtype=np.int64)
    if p >= 1.0:
        return np.ones(np.broadcast(bi, bj).shape, dtype=bool)
    lo = np.minimum(bi, bj)
    hi = np.maximum(bi, bj)
    k0, k1 = _key(seed)
    x0, _, _, _ = philox4x32_10(hi, lo, TAG_MASK, 0, k0, k1)
    u = x0.astype(np.float64) * 2.0 ** -32
    return (u < p) | (lo == hi)


def haar_blocks(n: int, d: int, seed: int) -> np.ndarray:
    """n Haar-random d x d orthogonal blocks stacked as an (n*d, d) float64 array."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, d, d))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diagonal(r, axis1=1, axis2=2))
    s[s == 0] = 1.0
    q = q * s[:, None, :]
    return np.ascontiguousarray(q.reshape(n * d, d))


def measurement_rows(Z: np.ndarray, sigma: float, seed: int, rows,
                     zero_diag_blocks: bool = False, p: float = 1.0) -> np.ndarray:
    """Rows ``rows`` (global indices) of A = Z Z^T + sigma W in float64.

    Z is (n*d, d).  Each row is a pure function of (Z, sigma, seed, row).
    """
    Z = np.asarray(Z, dtype=np.float64)
    nd, d = Z.shape
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.arange(nd, dtype=np.int64)
    R, C = np.meshgrid(rows, cols, indexing="ij")
    out = Z[rows] @ Z.T
    if sigma != 0.0:
        out = out + sigma * noise_elements(R, C, seed)
    bi, bj = R // d, C // d
    if zero_diag_blocks:
        same = bi == bj
        out[same] = (Z[rows] @ Z.T)[same]
    if p < 1.0:
        keep = mask_blocks(bi, bj, seed, p)
        out = np.where(keep, out, 0.0)
    return out


def measurement_matrix(Z: np.ndarray, sigma: float, seed: int,
                       zero_diag_blocks: bool = False, p: float = 1.0,
                       chunk_rows: int = 2048) -> np.ndarray:
    """The full nd x nd measurement matrix in float64 (small problems only)."""
    Z = np.asarray(Z, dtype=np.float64)
    nd = Z.shape[0]
    A = np.empty((nd, nd), dtype=np.float64)
    for r0 in range(0, nd, chunk_rows):
        r1 = min(nd, r0 + chunk_rows)
        A[r0:r1] = measurement_rows(Z, sigma, seed, np.arange(r0, r1),
                                    zero_diag_blocks=zero_diag_blocks, p=p)
    return A


def perturbed_start(Z: np.ndarray, eps: float, seed: int) -> np.ndarray:
    """A non-orthogonal iterate Z + eps * N(0, 1), as the NS iterates are."""
    rng = np.random.default_rng(seed)
    return np.asarray(Z, dtype=np.float64) + eps * rng.standard_normal(Z.shape)


def sigma_for(c: float, n: int, d: int) -> float:
    """Noise level sigma = c * sqrt(n / d) (the scaling of Theorem 3.1)."""
    return float(c) * math.sqrt(n / d)


def stiefel_start(n: int, d: int, p: int, seed: int) -> np.ndarray:
    """n random d x p blocks with orthonormal rows (S_i S_i^T = I_d), stacked as
    an (n*d, p) float64 array: the transposed Q factor of an i.i.d. Gaussian
    p x d matrix, sign-corrected like ``haar_blocks`` (a Haar point of the
    Stiefel manifold; a random start of the Burer-Monteiro relaxation)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, p, d))
    q, r = np.linalg.qr(g)                       # q: (n, p, d), orthonormal columns
    s = np.sign(np.diagonal(r, axis1=1, axis2=2))
    s[s == 0] = 1.0
    q = q * s[:, None, :]
    return np.ascontiguousarray(np.swapaxes(q, 1, 2).reshape(n * d, p))
