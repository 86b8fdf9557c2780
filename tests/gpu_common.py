"""Helpers shared by the GPU parity tests: building device inputs from the
seeded generator and the oracle's view of the same stored matrix.

Nothing here computes any part of the method; the expected values always come
from ``oracle/``.
"""
import math

import numpy as np
import torch

import paper_2604_07372_amd as P
from oracle import quantize as Q

FMT_NAME = {P.F64: "f64", P.F32: "f32", P.BF16: "bf16", P.BF16_SPLIT: "bf16_split", P.FP8_E4M3: "fp8"}
EPS = {P.F64: 2.0 ** -53}
EPS32 = 2.0 ** -24


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"


def xdtype(fmt):
    return torch.float64 if fmt == P.F64 else torch.float32


def to_dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda").to(dtype).contiguous()


def device_matrix(A64: np.ndarray, fmt: int) -> P.StoredMatrix:
    """Store a float64 host matrix on the device in `fmt` (reduced formats via the
    library's one-time FP32 conversion)."""
    if fmt == P.F64:
        return P.upload(A64, P.F64)
    A32 = P.upload(A64, P.F32)
    if fmt == P.F32:
        return A32
    return P.convert(A32.data, fmt)


def oracle_matrix(A64: np.ndarray, fmt: int) -> np.ndarray:
    """The float64 matrix the stored format actually holds (oracle's rounding)."""
    return Q.stored_value(A64, FMT_NAME[fmt])


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().double().numpy()


def step_tolerance(As: np.ndarray, X: np.ndarray, n: int, fmt: int, mu: float | None = None) -> float:
    """Absolute error bound for one step, from the arithmetic.

    The product sum_j A_ij X_j accumulates in the format's accumulation
    precision (eps): its error is at most ~ eps * (|A| |X|)_i times a modest
    factor (per-lane sums of nd / 64 V terms, then a 6-level tree), here 16.
    The step scales the gradient by mu = 1/n and the three Newton-Schulz steps
    near O(d) pass an error on with gain below 2 each; the d x d arithmetic adds a
    few eps of the O(1) entries.
    """
    eps = EPS.get(fmt, EPS32)
    mu = 1.0 / n if mu is None else mu
    prod = np.abs(As) @ np.abs(X)
    return 16.0 * eps * mu * float(prod.max()) * 8.0 + 64.0 * eps * max(1.0, float(np.abs(X).max()))


def align_err(X, Z):
    from oracle import nsrgs as O
    return O.alignment_error(X, Z)


def rel(a, b):
    return abs(a - b) / abs(b)


def sqrt_n(n):
    return math.sqrt(n)


def check_stop_iteration(gpu_iters: int, ref, tol: float, slack: float) -> None:
    """The GPU's relative-change stop fired where the oracle's sequence says it
    should: at the oracle's own stop iteration, or, when the oracle's relative
    change lies within a factor (1 +- slack) of tol at the boundary, at the
    neighbouring one.  ``slack`` states how far rounding can move the monitor:
    ~1e-6 for FP64 arithmetic, a few tens of percent for FP32 accumulation,
    whose iterate noise (~2^-24 relative) is a visible fraction of a 1e-6 change.
    ``ref`` is an oracle solve run with stop="rel_change" and the same tol,
    long enough to cover gpu_iters."""
    if gpu_iters == ref.iters:
        return
    rc = ref.rel_changes
    assert abs(gpu_iters - ref.iters) == 1, (gpu_iters, ref.iters)
    k = min(gpu_iters, ref.iters) - 1          # the iteration the two disagree on
    assert abs(rc[k] / tol - 1.0) <= slack, (gpu_iters, ref.iters, rc[k], tol)
