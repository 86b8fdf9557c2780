"""Pins of the Stiefel-manifold oracle (oracle/stiefel.py) against facts fixed
by the mathematics, not by the oracle itself: the reduction to Algorithm 2
at p = d, the tangent space of St(p, d), the gradient as a directional
derivative, the polar factor from the SVD, the noiseless fixed point, and the
rounding to O(d)^n.  CPU only."""
import numpy as np
import pytest

import synth
from oracle import nsrgs as O
from oracle import stiefel as St


def _problem(n, d, c, seed, symmetric=True):
    Z = synth.haar_blocks(n, d, seed)
    A = synth.measurement_matrix(Z, synth.sigma_for(c, n, d), seed + 1)
    if symmetric:
        A = np.triu(A) + np.triu(A, 1).T
    return Z, A


@pytest.mark.parametrize("d,retraction", [(1, "ns"), (3, "ns"), (4, "polar"), (3, "polar")])
def test_p_equal_d_is_algorithm_2(d, retraction):
    """At p = d, from an exactly orthogonal iterate, the Stiefel step is the
    O(d) step of Algorithm 2 (the two projections agree on O(d))."""
    n = 40
    Z, A = _problem(n, d, 0.3, 5)
    X = O.sgn_blocks(synth.perturbed_start(Z, 0.2, 6), d)
    a = St.step(A, X, d, Ts=3, retraction=retraction)
    b = O.rgs_step(A, X, d, Ts=3, retraction=retraction)
    assert np.abs(a.X - b.X).max() <= 1e-12
    assert np.abs(a.F - b.F).max() <= 1e-12
    assert abs(a.max_orth_defect - b.max_orth_defect) <= 1e-12


@pytest.mark.parametrize("d,p", [(1, 2), (2, 5), (3, 3), (3, 7), (5, 8)])
def test_projection_is_the_orthogonal_projection_onto_the_tangent_space(d, p):
    """P(G) lies in {xi : xi S^T + S xi^T = 0}, P(P(G)) = P(G), and G - P(G)
    is orthogonal to every tangent vector."""
    n = 6
    rng = np.random.default_rng(d * 10 + p)
    S = synth.stiefel_start(n, d, p, 3)
    G = rng.standard_normal(S.shape)
    P = St.tangent_projection(S, G, d)
    Sb, Pb = St.blocks(S, d), St.blocks(P, d)
    tang = Pb @ np.swapaxes(Sb, 1, 2) + Sb @ np.swapaxes(Pb, 1, 2)
    assert np.abs(tang).max() <= 1e-13
    assert np.abs(St.tangent_projection(S, P, d) - P).max() <= 1e-13
    xi = St.tangent_projection(S, rng.standard_normal(S.shape), d)
    assert abs(float(np.sum((G - P) * xi))) <= 1e-12 * np.linalg.norm(G) * np.linalg.norm(xi)
    # normal vectors S_i M (M symmetric) project to zero
    M = rng.standard_normal((n, d, d))
    N = (0.5 * (M + np.swapaxes(M, 1, 2)) @ Sb).reshape(S.shape)
    assert np.abs(St.tangent_projection(S, N, d)).max() <= 1e-13


@pytest.mark.parametrize("d,p", [(2, 3), (3, 5), (3, 3)])
def test_gradient_is_the_derivative_of_the_cost_along_the_manifold(d, p):
    """d/dt cost(polar(S + t xi)) at t = 0 equals <P(G), xi> for a tangent xi
    (central differences): the gradient has the right sign, transposes and
    diagonal-block term."""
    n = 12
    Z, A = _problem(n, d, 0.4, 9)
    S = synth.stiefel_start(n, d, p, 10)
    rng = np.random.default_rng(11)
    xi = St.tangent_projection(S, rng.standard_normal(S.shape), d)
    P = St.tangent_projection(S, St.gradient(A, S, d), d)
    h = 1e-5

    def phi(t):
        return St.cost(A, St.polar(St.blocks(S + t * xi, d)).reshape(S.shape), d)

    fd = (phi(h) - phi(-h)) / (2 * h)
    exact = float(np.sum(P * xi))
    assert abs(fd - exact) <= 1e-6 * max(1.0, abs(exact))


@pytest.mark.parametrize("d,p", [(1, 4), (3, 5), (4, 4), (6, 16)])
def test_newton_schulz_converges_to_the_polar_factor(d, p):
    """Algorithm 1 on d x p matrices with singular values in (0, sqrt 3)
    reaches the SVD's U V^T."""
    rng = np.random.default_rng(d + p)
    U = np.linalg.qr(rng.standard_normal((d, d)))[0]
    V = np.linalg.qr(rng.standard_normal((p, d)))[0]
    s = rng.uniform(0.3, 1.6, d)
    F = U @ np.diag(s) @ V.T
    S = St.newton_schulz(F, 60)
    assert np.abs(S - U @ V.T).max() <= 1e-13
    assert np.abs(St.polar(F) - U @ V.T).max() <= 1e-13
    # one step maps each singular value s to (3 s - s^3) / 2
    S1 = St.newton_schulz(F, 1)
    assert np.allclose(np.linalg.svd(S1, compute_uv=False), np.sort((3 * s - s ** 3) / 2)[::-1], atol=1e-14)


@pytest.mark.parametrize("d,p", [(3, 3), (3, 5), (2, 7)])
def test_noiseless_ground_truth_times_a_stiefel_point_is_a_fixed_point(d, p):
    """sigma = 0, A = Z Z^T: S = Z Q (Q with orthonormal rows) has zero
    Riemannian gradient, and the step leaves it in place."""
    n = 20
    Z = synth.haar_blocks(n, d, 2)
    A = Z @ Z.T
    Q = synth.stiefel_start(1, d, p, 4)
    S = Z @ Q
    P = St.tangent_projection(S, St.gradient(A, S, d), d)
    assert np.abs(P).max() <= 1e-12
    assert np.abs(St.step(A, S, d).X - S).max() <= 1e-12


def test_rounding_returns_a_rotated_ground_truth():
    n, d, p = 30, 3, 6
    Z = synth.haar_blocks(n, d, 12)
    S = Z @ synth.stiefel_start(1, d, p, 13)
    X = St.round_to_od(S, d)
    assert O.alignment_error(X, Z) <= 1e-12
    Xb = O.as_blocks(X, d)
    assert np.abs(np.swapaxes(Xb, 1, 2) @ Xb - np.eye(d)).max() <= 1e-12


@pytest.mark.parametrize("p", [4, 5, 7])
def test_random_starts_reach_the_ground_truth_at_low_noise(p):
    """From a random Stiefel start with p > d (the Burer-Monteiro relaxation),
    the iteration reaches a rank-d point: the singular values of S past d
    vanish, and S S^T and the rounded estimate are those of the O(d) solve
    from the spectral initialization (the relaxation is tight here)."""
    n, d = 60, 3
    Z, A = _problem(n, d, 0.15, 21)
    S0 = synth.stiefel_start(n, d, p, 22)
    res = St.solve(A, S0, d, T=100)
    S = res.X
    sv = np.linalg.svd(S, compute_uv=False)
    assert sv[d:].max(initial=0.0) <= 1e-10 * sv[0]
    ref = O.solve(A, d, T=200)
    e_st = O.alignment_error(St.round_to_od(S, d), Z)
    e_od = O.alignment_error(ref.X, Z)
    assert abs(e_st - e_od) <= 1e-8 * e_od
    assert abs(O.rel_err(S, Z) - O.rel_err(ref.X, Z)) <= 1e-8
