"""GPU parity of NS-RGS on the Stiefel manifold St(p, d)^n (sync_step_stiefel,
sync_solve_stiefel, sync_stiefel_round) against the FP64 oracle
(oracle/stiefel.py), through the C ABI."""
import math

import numpy as np
import pytest
import torch

import paper_2604_07372_amd as P
import synth
from oracle import nsrgs as O
from oracle import stiefel as St

from gpu_common import FMT_NAME, host, oracle_matrix, require_gpu, step_tolerance, to_dev, xdtype

pytestmark = pytest.mark.gpu

FMTS = [P.F64, P.F32]
# one and two 16-column tiles, ragged row tiles, p = d, d = 1, the largest d = p = 32
SHAPES = [(37, 3, 5), (200, 3, 7), (29, 8, 17), (31, 16, 32), (45, 1, 2), (61, 25, 32), (50, 3, 3),
          (20, 32, 32), (300, 2, 16), (130, 5, 20), (700, 3, 4)]


def _problem(n, d, p, c=0.3, seed=0, eps=0.01):
    """A random point of St(p, d)^n moved off the manifold by eps N(0, 1), as
    the Newton-Schulz iterates are.  eps keeps ||I - F_i F_i^T||_2 below 1,
    the region where the Newton-Schulz steps converge (Lemma 2.1); outside it
    they amplify every rounding error and no fixed bound holds."""
    Z = synth.haar_blocks(n, d, seed)
    A = synth.measurement_matrix(Z, synth.sigma_for(c, n, d), seed + 1)
    rng = np.random.default_rng(seed + 2)
    S = synth.stiefel_start(n, d, p, seed + 3)
    S = S + eps * rng.standard_normal(S.shape)
    return Z, A, S


def _upload(A, fmt):
    return P.upload(A, fmt)


def _tolerance(As, S, n, d, p, fmt):
    """The product's bound (step_tolerance) plus the FP64 d x p arithmetic of
    the step: about ten products with inner dimension d or p (the projection
    and three Newton-Schulz steps, gain below 2 each), so 8 (p + d) eps64
    max(1, |S|)^3."""
    m = max(1.0, float(np.abs(S).max()))
    return step_tolerance(As, S, n, fmt) + 8.0 * (p + d) * 2.0 ** -52 * m ** 3


@pytest.mark.parametrize("fmt", FMTS, ids=lambda f: FMT_NAME[f])
@pytest.mark.parametrize("n,d,p", SHAPES)
def test_stiefel_step_parity(n, d, p, fmt):
    require_gpu()
    print(f"stiefel step n={n} d={d} p={p} fmt={FMT_NAME[fmt]}", flush=True)
    Z, A, S = _problem(n, d, p, seed=100 * n + 7 * d + p)
    Ad = _upload(A, fmt)
    As = oracle_matrix(A, fmt)
    Sin = to_dev(S, xdtype(fmt))
    Sout = torch.empty_like(Sin)
    ws = P.stiefel_workspace(n, d, p, fmt)
    P.step_stiefel(Ad, n, d, p, Sin, Sout, ws, ns_steps=3)
    info = P.read_info(ws)
    Sh = host(Sin)
    ref = St.step(As, Sh, d, mu=1.0 / n, Ts=3)
    Fb = St.blocks(ref.F, d)
    assert np.linalg.norm(np.eye(d) - Fb @ np.swapaxes(Fb, 1, 2), 2, axis=(1, 2)).max() < 1.0
    err = np.abs(host(Sout) - ref.X).max()
    tol = _tolerance(As, Sh, n, d, p, fmt)
    assert err <= tol, (err, tol)
    assert abs(info["rel_change"] - ref.rel_change) <= 1e-6 * ref.rel_change + 1e-7
    assert abs(info["max_orth_defect"] - ref.max_orth_defect) <= 1e-6 * ref.max_orth_defect + 1e-6
    assert info["nonfinite"] == 0


@pytest.mark.parametrize("n,d", [(40, 3), (64, 16), (33, 20)])
def test_stiefel_step_at_p_equal_d_is_the_orthogonal_step(n, d):
    """At p = d from an exactly orthogonal iterate the Stiefel step is the
    O(d) step of sync_step, up to rounding."""
    require_gpu()
    Z = synth.haar_blocks(n, d, 3)
    A = synth.measurement_matrix(Z, synth.sigma_for(0.3, n, d), 4)
    X = O.sgn_blocks(synth.perturbed_start(Z, 0.2, 5), d)
    Ad = _upload(A, P.F64)
    Xin = to_dev(X, torch.float64)
    Xs, Xo = torch.empty_like(Xin), torch.empty_like(Xin)
    P.step_stiefel(Ad, n, d, d, Xin, Xs, P.stiefel_workspace(n, d, d, P.F64))
    P.step(Ad, n, d, Xin, Xo, P.workspace(n, d, P.F64))
    torch.cuda.synchronize()
    assert np.abs(host(Xs) - host(Xo)).max() <= 1e-12


@pytest.mark.parametrize("fmt", FMTS, ids=lambda f: FMT_NAME[f])
@pytest.mark.parametrize("p", [4, 5, 7])
def test_stiefel_solve_from_random_start(p, fmt):
    """From a random point of St(p, 3)^n the solve follows the oracle's
    trajectory, reaches a rank-3 point, and its rounding to O(3)^n is as
    accurate as the O(d) solve from the spectral initialization."""
    require_gpu()
    n, d, T = 200, 3, 150
    print(f"stiefel solve p={p} fmt={FMT_NAME[fmt]}", flush=True)
    Z = synth.haar_blocks(n, d, 31)
    A = synth.measurement_matrix(Z, synth.sigma_for(0.15, n, d), 32)
    As = oracle_matrix(A, fmt)
    S0 = synth.stiefel_start(n, d, p, 33)
    Ad = _upload(A, fmt)
    S = to_dev(S0, xdtype(fmt))
    ws = P.stiefel_workspace(n, d, p, fmt)
    info = P.solve_stiefel(Ad, n, d, p, S, ws, max_iters=T)
    assert info["iters"] == T and info["nonfinite"] == 0
    ref = St.solve(As, host(to_dev(S0, xdtype(fmt))), d, T=T)
    dev = np.abs(host(S) - ref.X).max()
    print(f"  max |S - S_oracle| {dev:.2e}", flush=True)
    assert dev <= (1e-9 if fmt == P.F64 else 2e-4)
    X = torch.empty((n * d, d), dtype=xdtype(fmt), device="cuda")
    P.stiefel_round(S, n, d, p, fmt, X, ws)
    torch.cuda.synchronize()
    e_gpu = O.alignment_error(host(X), Z)
    e_od = O.alignment_error(O.solve(As, d, T=200).X, Z)
    assert abs(e_gpu - e_od) <= (1e-8 if fmt == P.F64 else 1e-4) * e_od


def test_stiefel_solve_tolerance_stop():
    require_gpu()
    n, d, p = 300, 3, 5
    Z = synth.haar_blocks(n, d, 41)
    A = synth.measurement_matrix(Z, synth.sigma_for(0.15, n, d), 42)
    Ad = _upload(A, P.F64)
    S0 = synth.stiefel_start(n, d, p, 43)
    S = to_dev(S0, torch.float64)
    ws = P.stiefel_workspace(n, d, p, P.F64)
    info = P.solve_stiefel(Ad, n, d, p, S, ws, max_iters=500, tol=1e-10)
    ref = St.solve(A, S0, d, T=500, tol=1e-10)
    assert info["converged"] == 1
    assert abs(info["iters"] - ref.iters) <= 1
    assert info["rel_change"] <= 1e-10


@pytest.mark.parametrize("fmt", FMTS, ids=lambda f: FMT_NAME[f])
@pytest.mark.parametrize("n,d,p", [(30, 3, 6), (100, 1, 4), (17, 16, 32), (50, 8, 8)])
def test_stiefel_rounding(n, d, p, fmt):
    """S = Z Q rounds to a rotated copy of Z; a noisy one rounds to the
    oracle's sgn(S_i V) (up to a global rotation: V is fixed up to the signs
    of its columns)."""
    require_gpu()
    Z = synth.haar_blocks(n, d, 12)
    Q = synth.stiefel_start(1, d, p, 13)
    ws = P.stiefel_workspace(n, d, p, fmt)
    X = torch.empty((n * d, d), dtype=xdtype(fmt), device="cuda")
    P.stiefel_round(to_dev(Z @ Q, xdtype(fmt)), n, d, p, fmt, X, ws)
    torch.cuda.synchronize()
    assert O.alignment_error(host(X), Z) <= (1e-12 if fmt == P.F64 else 1e-5)
    # a point with a well separated top-d subspace of S^T S (a noisy Z Q)
    S = St.polar(St.blocks(Z @ Q + 0.1 * np.random.default_rng(14).standard_normal((n * d, p)), d))
    Sd = to_dev(S.reshape(n * d, p), xdtype(fmt))
    P.stiefel_round(Sd, n, d, p, fmt, X, ws)
    torch.cuda.synchronize()
    ref = St.round_to_od(host(Sd), d)
    assert O.dist_F(host(X), ref) / math.sqrt(n) <= (1e-9 if fmt == P.F64 else 1e-4)
