"""Pins of the seeded input generator (CPU only)."""
import math
import os

import numpy as np
import pytest

import synth


def _read_kat(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(t, 16) for t in line.split()])
    return rows


def test_philox_known_answers(golden_dir):
    for row in _read_kat(golden_dir):
        ctr, key, want = row[:4], row[4:6], row[6:]
        got = synth.philox4x32_10(*ctr, *key)
        assert [int(g) for g in got] == want


def test_noise_is_symmetric_standard_normal():
    r = np.arange(0, 400000)
    c = (r * 7919) % 3001
    z = synth.noise_elements(r, c, seed=11)
    zt = synth.noise_elements(c, r, seed=11)
    assert np.array_equal(z, zt)
    assert abs(z.mean()) < 0.01
    assert abs(z.std() - 1.0) < 0.01
    assert abs(np.mean(z ** 4) - 3.0) < 0.06          # Gaussian kurtosis
    z2 = synth.noise_elements(r, c, seed=12)
    assert abs(np.corrcoef(z, z2)[0, 1]) < 0.01


def test_haar_blocks_orthogonal_and_isotropic():
    n, d = 4000, 3
    Z = synth.haar_blocks(n, d, seed=3).reshape(n, d, d)
    err = np.abs(Z @ np.swapaxes(Z, 1, 2) - np.eye(d)).max()
    assert err < 1e-14
    # Haar: E[Z] = 0, E[Z_ab^2] = 1/d, and both determinant signs occur equally.
    assert np.abs(Z.mean(axis=0)).max() < 0.03
    assert np.abs((Z ** 2).mean(axis=0) - 1.0 / d).max() < 0.02
    dets = np.linalg.det(Z)
    assert abs(np.mean(dets > 0) - 0.5) < 0.03


def test_measurement_matrix_structure():
    n, d, sigma = 40, 3, 0.7
    Z = synth.haar_blocks(n, d, seed=5)
    A = synth.measurement_matrix(Z, sigma, seed=9)
    assert np.array_equal(A, A.T)
    W = (A - Z @ Z.T) / sigma
    assert abs(W.std() - 1.0) < 0.05
    # rows regenerate independently of the rest of the matrix
    rows = np.array([0, 17, 119])
    assert np.array_equal(synth.measurement_rows(Z, sigma, 9, rows), A[rows])
    # paper model: W_ii = 0, so A_ii = Z_i Z_i^T = I
    A0 = synth.measurement_matrix(Z, sigma, seed=9, zero_diag_blocks=True)
    for i in range(n):
        s = slice(i * d, (i + 1) * d)
        assert np.allclose(A0[s, s], np.eye(d), atol=1e-14)
    off = np.ones_like(A, dtype=bool)
    for i in range(n):
        off[i * d:(i + 1) * d, i * d:(i + 1) * d] = False
    assert np.array_equal(A0[off], A[off])


def test_noise_norm_lemma_7_2():
    # Lemma 7.2: ||W|| <= 3 sqrt(nd) with high probability (here with margin).
    n, d = 300, 3
    Z = np.zeros((n * d, d))
    W = synth.measurement_matrix(Z, 1.0, seed=2, zero_diag_blocks=False)
    assert np.linalg.norm(W, 2) <= 3.0 * math.sqrt(n * d)
    assert np.linalg.norm(W, 2) >= 1.9 * math.sqrt(n * d)   # semicircle edge 2 sqrt(nd)


@pytest.mark.parametrize("p", [0.5, 0.8])
def test_mask_rate_and_symmetry(p):
    n = 300
    bi, bj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    m = synth.mask_blocks(bi, bj, seed=4, p=p)
    assert np.array_equal(m, m.T)
    assert np.all(np.diag(m))
    off = ~np.eye(n, dtype=bool)
    assert abs(m[off].mean() - p) < 0.01
