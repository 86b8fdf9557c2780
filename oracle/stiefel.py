"""Plain FP64 CPU oracle for NS-RGS on the Stiefel manifold St(p, d)^n.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library: it never imports the product package and the product never
imports it.

The paper names the extension of its Newton-Schulz retraction framework to
the Stiefel manifold as future work (Sec. 6, Discussion); the manifold is the
one of the Burer-Monteiro relaxation its related work recalls (Sec. 1),
St(p, d) = {S in R^{d x p} : S S^T = I_d}, d <= p.  The paper prints no
algorithm for it.  This module is the library's reading, obtained by
rewriting each step of Algorithm 2 (Sec. 2.2) for d x p blocks:

* iterate S = (S_1; ...; S_n), an (n*d, p) stack, block i rows [i d, (i+1) d);
  for p = d it is the O(d)^n iterate of Algorithm 2;
* Euclidean gradient G_i = (n - 1) S_i - sum_{j != i} A_ij S_j, the expression
  of Algorithm 2.  Its first term is normal to the manifold at S_i (the
  projection below maps S_i to zero), so the Riemannian gradient is that of
  the cost (n - 1)/2 sum_i ||S_i||^2 - (1/2) sum_{i != j} tr(S_i^T A_ij S_j)
  (``cost``), which on O(d)^n differs from the objective of eq. def:f by a
  constant;
* tangent projection onto T_S St = {xi : xi S^T + S xi^T = 0}:
  P_i = G_i - sym(G_i S_i^T) S_i, sym(M) = (M + M^T) / 2.  For S_i in O(d)
  this equals the (G_i - S_i G_i^T S_i) / 2 of Algorithm 2;
* step F_i = S_i - mu P_i, mu = 1/n by default as in Theorem 3.1;
* retraction: Ts steps of Algorithm 1 applied to the d x p matrix F_i,
  S <- (3 S - S S^T S) / 2.  Each step maps every singular value s of F_i to
  (3 s - s^3) / 2 and keeps the singular vectors, so the steps converge to the
  polar factor U V^T of F_i = U Sigma V^T (thin SVD), the point of St(p, d)
  nearest to F_i, for singular values in (0, sqrt 3).

Rounding to O(d)^n (``round_to_od``) is the library's reading too: with V the
p x d matrix of top-d right singular vectors of S, X_i = sgn(S_i V).  When
S = Z Q for a Q with orthonormal rows this returns Z (Q V) exactly, a
globally rotated copy of Z.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "blocks", "polar", "newton_schulz", "gradient", "tangent_projection", "cost",
    "step", "StepResult", "solve", "SolveResult", "round_to_od", "rel_change",
]


def blocks(S: np.ndarray, d: int) -> np.ndarray:
    """View an (n*d, p) stack as (n, d, p) blocks."""
    S = np.asarray(S, dtype=np.float64)
    nd, p = S.shape
    if nd % d or p < d:
        raise ValueError(f"expected an (n*{d}, p >= {d}) stack, got {S.shape}")
    return S.reshape(nd // d, d, p)


def polar(F: np.ndarray) -> np.ndarray:
    """U V^T of F = U Sigma V^T (thin SVD), for a d x p matrix or a stack."""
    U, _, Vt = np.linalg.svd(np.asarray(F, dtype=np.float64), full_matrices=False)
    return U @ Vt


def newton_schulz(F: np.ndarray, Ts: int) -> np.ndarray:
    """Algorithm 1 for d x p matrices: S_0 = F, S_{t+1} = (3 S_t - S_t S_t^T S_t) / 2."""
    S = np.array(F, dtype=np.float64, copy=True)
    for _ in range(int(Ts)):
        S = 1.5 * S - 0.5 * (S @ np.swapaxes(S, -1, -2)) @ S
    return S


def gradient(A: np.ndarray, S: np.ndarray, d: int) -> np.ndarray:
    """G_i = (n - 1) S_i - sum_{j != i} A_ij S_j, as an (n*d, p) stack (the full
    product A S minus each diagonal-block term A_ii S_i)."""
    A = np.asarray(A, dtype=np.float64)
    Sb = blocks(S, d)
    n = Sb.shape[0]
    C = (A @ np.asarray(S, dtype=np.float64)).reshape(Sb.shape)
    for i in range(n):
        s = slice(i * d, (i + 1) * d)
        C[i] -= A[s, s] @ Sb[i]
    return ((n - 1) * Sb - C).reshape(n * d, -1)


def tangent_projection(S: np.ndarray, G: np.ndarray, d: int) -> np.ndarray:
    """P_i = G_i - sym(G_i S_i^T) S_i for every block (projection onto T_S St)."""
    Sb, Gb = blocks(S, d), blocks(G, d)
    M = Gb @ np.swapaxes(Sb, -1, -2)
    sym = 0.5 * (M + np.swapaxes(M, -1, -2))
    return (Gb - sym @ Sb).reshape(S.shape[0], -1)


def cost(A: np.ndarray, S: np.ndarray, d: int) -> float:
    """(n - 1)/2 sum_i ||S_i||_F^2 - (1/2) sum_{i != j} tr(S_i^T A_ij S_j), the
    function whose Euclidean gradient is ``gradient``."""
    A = np.asarray(A, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    n = S.shape[0] // d
    M = S.T @ A @ S
    diag = 0.0
    for i in range(n):
        s = slice(i * d, (i + 1) * d)
        diag += float(np.trace(S[s].T @ A[s, s] @ S[s]))
    return 0.5 * (n - 1) * float(np.sum(S * S)) - 0.5 * (float(np.trace(M)) - diag)


def rel_change(Sn: np.ndarray, S: np.ndarray) -> float:
    return float(np.linalg.norm(Sn - S) / np.linalg.norm(S))


@dataclass
class StepResult:
    X: np.ndarray            # S^{t+1}, (n*d, p)
    F: np.ndarray            # F^t = S^t - mu P(G^t)
    G: np.ndarray            # Euclidean gradient G^t
    max_orth_defect: float   # max_i ||I_d - F_i F_i^T||_F
    rel_change: float        # ||S^{t+1} - S^t||_F / ||S^t||_F


def step(A: np.ndarray, S: np.ndarray, d: int, mu: float | None = None, Ts: int = 3,
         retraction: str = "ns") -> StepResult:
    """One Jacobi sweep over all blocks (every block reads S^t).

    retraction="ns": Ts Newton-Schulz steps; "polar": the exact polar factor.
    """
    S = np.asarray(S, dtype=np.float64)
    n = S.shape[0] // d
    if mu is None:
        mu = 1.0 / n
    G = gradient(A, S, d)
    P = tangent_projection(S, G, d)
    F = S - mu * P
    Fb = blocks(F, d)
    if retraction == "ns":
        Sn = newton_schulz(Fb, Ts).reshape(S.shape)
    elif retraction == "polar":
        Sn = polar(Fb).reshape(S.shape)
    else:
        raise ValueError(retraction)
    defect = np.linalg.norm(np.eye(d) - Fb @ np.swapaxes(Fb, -1, -2), axis=(1, 2))
    return StepResult(X=Sn, F=F, G=G, max_orth_defect=float(defect.max()), rel_change=rel_change(Sn, S))


@dataclass
class SolveResult:
    X: np.ndarray
    iters: int
    rel_changes: list = field(default_factory=list)


def solve(A: np.ndarray, S0: np.ndarray, d: int, mu: float | None = None, Ts: int = 3, T: int = 100,
          tol: float = 0.0) -> SolveResult:
    """At most T steps from S0; with tol > 0, stop after the first step whose
    relative change is <= tol."""
    S = np.array(S0, dtype=np.float64, copy=True)
    res = SolveResult(X=S, iters=0)
    for t in range(int(T)):
        st = step(A, S, d, mu=mu, Ts=Ts)
        S = st.X
        res.iters = t + 1
        res.rel_changes.append(st.rel_change)
        if tol > 0.0 and st.rel_change <= tol:
            break
    res.X = S
    return res


def round_to_od(S: np.ndarray, d: int) -> np.ndarray:
    """X_i = sgn(S_i V), V the top-d right singular vectors of S (p x d)."""
    S = np.asarray(S, dtype=np.float64)
    w, E = np.linalg.eigh(S.T @ S)
    V = E[:, np.argsort(w)[::-1][:d]]
    return polar(blocks(S, d) @ V).reshape(-1, d)
