"""Plain FP64 CPU oracle for NS-RGS (orthogonal group synchronization).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library: it never imports the product package and the product never
imports it.

Everything here follows the paper (Peng, Han, Chen, Huang, "NS-RGS: Newton-
Schulz Based Riemannian Gradient Method for Orthogonal Group
Synchronization") step by step, in float64, with NumPy/SciPy library
routines (matmul, SVD, symmetric eigensolvers) as the only building blocks.
Nothing is blocked, fused or reordered.

Conventions
-----------
* An element of O(d)^n, and every iterate, is an (n*d, d) array
  X = (X_1; ...; X_n); block i is rows [i*d, (i+1)*d).
* A is the symmetric (n*d, n*d) block measurement matrix, A_ij its (i, j)
  d x d block (Sec. 2.2, eq. ``def:measurements``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "as_blocks", "sgn", "sgn_blocks", "newton_schulz", "offdiag_product",
    "euclidean_gradient", "tangent_projection", "rgs_step", "StepResult", "block_step",
    "spectral_subspace", "spectral_init", "solve", "SolveResult", "objective",
    "partial_objective", "procrustes", "dist_F", "alignment_error", "rel_err",
    "mse", "rel_change", "objective_ratio", "gpm_step", "block_gradient",
]


# ---------------------------------------------------------------------------
# d x d primitives (Sec. 2.1)
# ---------------------------------------------------------------------------

def as_blocks(X: np.ndarray, d: int) -> np.ndarray:
    """View an (n*d, d) stack as (n, d, d) blocks."""
    X = np.asarray(X, dtype=np.float64)
    nd, dd = X.shape
    if dd != d or nd % d:
        raise ValueError(f"expected an (n*{d}, {d}) stack, got {X.shape}")
    return X.reshape(nd // d, d, d)


def sgn(M: np.ndarray) -> np.ndarray:
    """Matrix sign function of Sec. 2.1: for M = U Sigma V^T, sgn(M) = U V^T.

    Works on a single d x d matrix or on a stack (..., d, d).
    """
    U, _, Vt = np.linalg.svd(np.asarray(M, dtype=np.float64))
    return U @ Vt


def sgn_blocks(Phi: np.ndarray, d: int) -> np.ndarray:
    """Blockwise sign of an (n*d, d) stack (the operator applied to Y in Alg. 2)."""
    return sgn(as_blocks(Phi, d)).reshape(-1, d)


def newton_schulz(M: np.ndarray, Ts: int) -> np.ndarray:
    """Algorithm 1: S_0 = M, S_{t+1} = (1/2) S_t (3 I - S_t^T S_t), Ts steps.

    Works on one d x d matrix or a stack (..., d, d).  No pre-scaling of M
    (Algorithm 1 starts from M itself).
    """
    S = np.array(M, dtype=np.float64, copy=True)
    d = S.shape[-1]
    eye = np.eye(d)
    for _ in range(int(Ts)):
        S = 0.5 * S @ (3.0 * eye - np.swapaxes(S, -1, -2) @ S)
    return S


# ---------------------------------------------------------------------------
# The Riemannian gradient step of Algorithm 2 (Sec. 2.2)
# ---------------------------------------------------------------------------

def offdiag_product(A: np.ndarray, X: np.ndarray, d: int) -> np.ndarray:
    """C_i = sum_{j != i} A_ij X_j for every block i, as an (n*d, d) stack.

    Written as the full product A X minus each diagonal-block term A_ii X_i.
    """
    A = np.asarray(A, dtype=np.float64)
    Xb = as_blocks(X, d)
    n = Xb.shape[0]
    C = (A @ X).reshape(n, d, d)
    for i in range(n):
        s = slice(i * d, (i + 1) * d)
        C[i] -= A[s, s] @ Xb[i]
    return C.reshape(n * d, d)


def euclidean_gradient(A: np.ndarray, X: np.ndarray, d: int) -> np.ndarray:
    """G_i = sum_{j != i} (X_i - A_ij X_j) = (n - 1) X_i - C_i  (Alg. 2, Sec. 2.2).

    The paper reaches this form from the partial derivative of f_i by
    substituting X_j^T X_j = I; it is applied literally to the (not exactly
    orthogonal) Newton-Schulz iterates.
    """
    Xb = as_blocks(X, d)
    n = Xb.shape[0]
    return (n - 1) * np.asarray(X, dtype=np.float64) - offdiag_product(A, X, d)


def tangent_projection(X: np.ndarray, G: np.ndarray, d: int) -> np.ndarray:
    """P_{T_X}(G)_i = (G_i - X_i G_i^T X_i) / 2 per block (Sec. 2.2).

    For X_i in O(d) this is the orthogonal projection onto the tangent space
    {X_i H : H skew}; for the Newton-Schulz iterates it is the paper's
    pseudo projection, applied as written.
    """
    Xb = as_blocks(X, d)
    Gb = as_blocks(G, d)
    P = 0.5 * (Gb - Xb @ np.swapaxes(Gb, -1, -2) @ Xb)
    return P.reshape(-1, d)


@dataclass
class StepResult:
    X: np.ndarray            # X^{t+1}, (n*d, d)
    F: np.ndarray            # F^t = X^t - mu P(G^t), (n*d, d)
    G: np.ndarray            # Euclidean gradient G^t, (n*d, d)
    max_orth_defect: float   # max_i ||I - F_i^T F_i||_F
    rel_change: float        # ||X^{t+1} - X^t||_F / ||X^t||_F


def rgs_step(A: np.ndarray, X: np.ndarray, d: int, mu: float | None = None,
             Ts: int = 3, retraction: str = "ns") -> StepResult:
    """One Jacobi sweep of Algorithm 2 over all blocks i (every block reads X^t).

    retraction="ns"    : X_i^{t+1} = S(F_i), Ts Newton-Schulz steps (Alg. 1).
    retraction="polar" : X_i^{t+1} = sgn(F_i), the exact retraction
                         (the sequence written with a tilde in Sec. 3).
    mu=None gives the step size 1/n of Theorem 3.1.
    """
    X = np.asarray(X, dtype=np.float64)
    Xb = as_blocks(X, d)
    n = Xb.shape[0]
    if mu is None:
        mu = 1.0 / n
    G = euclidean_gradient(A, X, d)
    P = tangent_projection(X, G, d)
    F = X - mu * P
    Fb = as_blocks(F, d)
    if retraction == "ns":
        Xn = newton_schulz(Fb, Ts).reshape(-1, d)
    elif retraction == "polar":
        Xn = sgn(Fb).reshape(-1, d)
    else:
        raise ValueError(retraction)
    eye = np.eye(d)
    defect = np.linalg.norm(eye - np.swapaxes(Fb, -1, -2) @ Fb, axis=(1, 2))
    return StepResult(X=Xn, F=F, G=G, max_orth_defect=float(defect.max()),
                      rel_change=rel_change(Xn, X))


def block_step(A_rows_i: np.ndarray, X: np.ndarray, d: int, i: int, mu: float | None = None,
               Ts: int = 3) -> np.ndarray:
    """X_i^{t+1} of Algorithm 2 for one block i, from the d rows of A that hold
    the blocks A_i1, ..., A_in (shape (d, n*d)) and the whole iterate X^t.

    The same steps as ``rgs_step``, written for a single i: the gradient sum
    over j != i (the full row product minus the diagonal-block term, as in
    ``offdiag_product``), the pseudo projection, the step and Ts Newton-Schulz
    steps.  Lets a large problem be checked on sampled blocks.
    """
    X = np.asarray(X, dtype=np.float64)
    Xb = as_blocks(X, d)
    n = Xb.shape[0]
    if mu is None:
        mu = 1.0 / n
    G = block_gradient(A_rows_i, X, d, i)
    P = 0.5 * (G - Xb[i] @ G.T @ Xb[i])
    F = Xb[i] - mu * P
    return newton_schulz(F, Ts)


def block_gradient(A_rows_i: np.ndarray, X: np.ndarray, d: int, i: int) -> np.ndarray:
    """G_i = (n - 1) X_i - sum_{j != i} A_ij X_j for one block i, from its d rows
    of A (shape (d, n*d)) and the whole iterate (the gradient of Algorithm 2)."""
    X = np.asarray(X, dtype=np.float64)
    Xb = as_blocks(X, d)
    n = Xb.shape[0]
    Ai = np.asarray(A_rows_i, dtype=np.float64)                        # [A_i1 ... A_in]
    s = slice(i * d, (i + 1) * d)
    C = Ai @ X - Ai[:, s] @ Xb[i]                                      # sum over j != i
    return (n - 1) * Xb[i] - C


def gpm_step(A: np.ndarray, X: np.ndarray, d: int) -> StepResult:
    """One step of the generalized power method that Sec. 4.1 compares against:
    X_i^{t+1} = sgn((A X^t)_i) for every block i.

    The paper cites the method and does not print it; this is its usual form
    (the projection of the power iterate A X^t onto O(d)^n, block by block),
    with the whole block row of A, the diagonal block included (A_ii = I in
    the paper's model, so (A X)_i = X_i + sum_{j != i} A_ij X_j).  The
    returned G and F are the power iterate A X^t; max_orth_defect is that of
    the new iterate.
    """
    X = np.asarray(X, dtype=np.float64)
    P = np.asarray(A, dtype=np.float64) @ X
    Xn = sgn_blocks(P, d)
    Xb = as_blocks(Xn, d)
    eye = np.eye(d)
    defect = np.linalg.norm(eye - np.swapaxes(Xb, -1, -2) @ Xb, axis=(1, 2))
    return StepResult(X=Xn, F=P, G=P, max_orth_defect=float(defect.max()),
                      rel_change=rel_change(Xn, X))


# ---------------------------------------------------------------------------
# Spectral initialization (Sec. 2.2, Algorithm 2)
# ---------------------------------------------------------------------------

def spectral_subspace(A: np.ndarray, d: int, dense_limit: int = 3000):
    """Y = eigenvectors of the d largest (algebraic) eigenvalues of A, Y^T Y = I.

    Returns (Y, eigenvalues descending, lambda_{d+1} or nan).  Dense ``eigh``
    up to ``dense_limit`` rows, ARPACK Lanczos (``eigsh``) above.
    """
    A = np.asarray(A, dtype=np.float64)
    nd = A.shape[0]
    if nd <= dense_limit:
        w, V = np.linalg.eigh(A)
        order = np.argsort(w)[::-1]
        w, V = w[order], V[:, order]
        nxt = float(w[d]) if nd > d else float("nan")
        return V[:, :d].copy(), w[:d].copy(), nxt
    from scipy.sparse.linalg import eigsh
    w, V = eigsh(A, k=d + 1, which="LA", tol=1e-14)
    order = np.argsort(w)[::-1]
    w, V = w[order], V[:, order]
    return V[:, :d].copy(), w[:d].copy(), float(w[d])


def spectral_init(A: np.ndarray, d: int, dense_limit: int = 3000) -> np.ndarray:
    """X^0 = blockwise sgn(Y) with the exact sign function (Alg. 2, initialization)."""
    Y, _, _ = spectral_subspace(A, d, dense_limit)
    return sgn_blocks(Y, d)


# ---------------------------------------------------------------------------
# The objective and stopping quantities (Sec. 1, eq. def:f; Sec. 4.1)
# ---------------------------------------------------------------------------

def objective(A: np.ndarray, X: np.ndarray, d: int) -> float:
    """F(X) = sum_{i != j} (1/2) ||X_i X_j^T - A_ij||_F^2 (eq. ``def:f``)."""
    A = np.asarray(A, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0] // d
    R = X @ X.T - A
    for i in range(n):
        s = slice(i * d, (i + 1) * d)
        R[s, s] = 0.0
    return 0.5 * float(np.sum(R * R))


def partial_objective(A: np.ndarray, X: np.ndarray, d: int, i: int) -> float:
    """f_i(X) = sum_{j != i} (1/2) ||X_i X_j^T - A_ij||_F^2 (Sec. 2.2)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0] // d
    s = slice(i * d, (i + 1) * d)
    tot = 0.0
    for j in range(n):
        if j == i:
            continue
        t = slice(j * d, (j + 1) * d)
        R = X[s] @ X[t].T - A[s, t]
        tot += 0.5 * float(np.sum(R * R))
    return tot


def rel_change(Xn: np.ndarray, X: np.ndarray) -> float:
    """||X^{t+1} - X^t||_F / ||X^t||_F.

    The relative change of the iterate, the stop rule the serving workload
    names ("relative-change tolerance").  The paper's own rule is the
    objective ratio R^t below; this reading of "relative change" as a
    Frobenius ratio of iterates is the library's, not the paper's.
    """
    return float(np.linalg.norm(Xn - X) / np.linalg.norm(X))


def objective_ratio(F_t: float, F_t1: float) -> float:
    """R^t = (F(X^t) - F(X^{t+1})) / F(X^{t+1}) (Sec. 4.1 stopping rule)."""
    return (F_t - F_t1) / F_t1


# ---------------------------------------------------------------------------
# The solve: Algorithm 2
# ---------------------------------------------------------------------------

@dataclass
class SolveResult:
    X: np.ndarray
    X0: np.ndarray
    iters: int
    rel_changes: list = field(default_factory=list)
    max_orth_defects: list = field(default_factory=list)
    objectives: list = field(default_factory=list)


def solve(A: np.ndarray, d: int, mu: float | None = None, Ts: int = 3,
          T: int = 100, retraction: str = "ns", stop: str = "fixed",
          tol: float = 0.0, X0: np.ndarray | None = None,
          dense_limit: int = 3000, method: str = "rgs") -> SolveResult:
    """Algorithm 2: spectral initialization, then at most T Jacobi sweeps.

    method="rgs" : the Riemannian gradient step of Algorithm 2 with the
                   given retraction.
    method="gpm" : the generalized power method of the Sec. 4.1 comparison
                   (``gpm_step``) from the same initialization and with the
                   same stop rules; mu, Ts and retraction are unused.

    stop="fixed"      : run exactly T iterations.
    stop="rel_change" : stop after the first iteration with
                        ||X^{t+1} - X^t||_F / ||X^t||_F <= tol.
    stop="objective"  : the paper's rule, stop after the first iteration with
                        R^t < tol (Sec. 4.1), or at T.
    """
    if X0 is None:
        X0 = spectral_init(A, d, dense_limit)
    X = np.array(X0, dtype=np.float64, copy=True)
    res = SolveResult(X=X, X0=np.array(X0, copy=True), iters=0)
    F_prev = objective(A, X, d) if stop == "objective" else None
    for t in range(int(T)):
        if method == "rgs":
            st = rgs_step(A, X, d, mu=mu, Ts=Ts, retraction=retraction)
        elif method == "gpm":
            st = gpm_step(A, X, d)
        else:
            raise ValueError(method)
        X = st.X
        res.iters = t + 1
        res.rel_changes.append(st.rel_change)
        res.max_orth_defects.append(st.max_orth_defect)
        if stop == "rel_change":
            if st.rel_change <= tol:
                break
        elif stop == "objective":
            F_new = objective(A, X, d)
            res.objectives.append(F_new)
            if objective_ratio(F_prev, F_new) < tol:
                break
            F_prev = F_new
        elif stop != "fixed":
            raise ValueError(stop)
    res.X = X
    return res


# ---------------------------------------------------------------------------
# Metrics (Sec. 1.4 distance, Sec. 4.1 Rel. Err., Sec. 4.2 MSE)
# ---------------------------------------------------------------------------

def procrustes(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Q* = argmin_{Q in O(d)} ||X - Y Q||_F = sgn(Y^T X) (orthogonal Procrustes)."""
    return sgn(np.asarray(Y, dtype=np.float64).T @ np.asarray(X, dtype=np.float64))


def dist_F(X: np.ndarray, Y: np.ndarray) -> float:
    """d_F(X, Y) = min_Q ||X - Y Q||_F, evaluated as the explicit residual.

    The closed form ||X||^2 + ||Y||^2 - 2 ||Y^T X||_* cancels badly when the
    two are close, so the residual at the Procrustes optimum is used.
    """
    Q = procrustes(X, Y)
    return float(np.linalg.norm(np.asarray(X, dtype=np.float64) - np.asarray(Y, dtype=np.float64) @ Q))


def alignment_error(X: np.ndarray, Z: np.ndarray) -> float:
    """d_F(X, Z) / sqrt(n): root mean square blockwise error up to a global O(d)."""
    d = np.asarray(Z).shape[1]
    n = np.asarray(Z).shape[0] // d
    return dist_F(X, Z) / math.sqrt(n)


def mse(Xhat: np.ndarray, X: np.ndarray) -> float:
    """MSE = d_F(Xhat, X)^2 / n (Sec. 4.2)."""
    d = np.asarray(X).shape[1]
    n = np.asarray(X).shape[0] // d
    return dist_F(Xhat, X) ** 2 / n


def rel_err(X: np.ndarray, Z: np.ndarray, form: str = "explicit") -> float:
    """Rel. Err. = ||Z Z^T - X X^T||_F / ||Z Z^T||_F (Sec. 4.1).

    form="explicit" builds the two nd x nd products.  form="gram" uses
    ||Z Z^T - X X^T||^2 = ||Z^T Z||^2 + ||X^T X||^2 - 2 ||Z^T X||^2 with d x d
    Grams only (trace identities); it loses accuracy below about 1e-6.
    """
    X = np.asarray(X, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    if form == "explicit":
        ZZ = Z @ Z.T
        return float(np.linalg.norm(ZZ - X @ X.T) / np.linalg.norm(ZZ))
    if form != "gram":
        raise ValueError(form)
    zz = np.sum((Z.T @ Z) ** 2)
    xx = np.sum((X.T @ X) ** 2)
    zx = np.sum((Z.T @ X) ** 2)
    return float(math.sqrt(max(zz + xx - 2.0 * zx, 0.0) / zz))
