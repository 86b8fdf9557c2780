"""NS-RGS on AMD MI355X: Python binding of libnsrgs.so (the C ABI in include/nsrgs.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides device memory and the current HIP stream.  The
binding refuses to work without the compiled library (no CPU fallback).
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

__all__ = [
    "F64", "F32", "BF16", "BF16_SPLIT", "FP8_E4M3", "FORMATS", "NsrgsError",
    "lib", "StoredMatrix", "Workspace", "workspace", "step", "read_info",
    "init_spectral", "solve", "generate", "convert", "stored", "padded_ld",
    "Info", "solve_batched", "batch_rows_per_panel", "set_tuning", "get_tuning", "TuneEntry", "Server",
    "step_variants", "TuneResult", "step_symmetric", "symmetric_workspace_bytes",
    "BsrMatrix", "generate_bsr", "step_bsr", "PACKED_LD", "packed_elems", "stored_packed", "convert_packed",
    "stiefel_workspace", "step_stiefel", "solve_stiefel", "stiefel_round",
]

F64, F32, BF16, BF16_SPLIT, FP8_E4M3 = 0, 1, 2, 3, 4
PACKED_LD = -1   # nsrgs_matrix.ld of the packed upper-block-triangle layout (NSRGS_LD_PACKED)
FORMATS = {"f64": F64, "f32": F32, "bf16": BF16, "bf16_split": BF16_SPLIT, "fp8": FP8_E4M3}

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnsrgs.so")


class NsrgsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"nsrgs status {status}: {message}")
        self.status = status


class _Matrix(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("data", ctypes.c_void_p), ("data_lo", ctypes.c_void_p),
                ("row_scale", ctypes.c_void_p), ("ld", ctypes.c_int64)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("nonfinite", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rel_change", ctypes.c_double), ("max_orth_defect", ctypes.c_double),
                ("init_residual", ctypes.c_double), ("ritz", ctypes.c_double * 16),
                ("ritz_next", ctypes.c_double), ("objective", ctypes.c_double),
                ("objective_ratio", ctypes.c_double), ("ritz_more", ctypes.c_double * 16)]

    def as_dict(self, d: int | None = None) -> dict:
        out = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("ritz", "ritz_more")}
        out["ritz"] = (list(self.ritz) + list(self.ritz_more))[: (d or 16)]
        return out


class _Bsr(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("reserved", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("values", ctypes.c_void_p)]


class _SolveOpts(ctypes.Structure):
    _fields_ = [("init", ctypes.c_int32), ("init_iters", ctypes.c_int32),
                ("init_tol", ctypes.c_double), ("refine_iters", ctypes.c_int32),
                ("A_refine", ctypes.POINTER(_Matrix)), ("check_every", ctypes.c_int32),
                ("symmetric", ctypes.c_int32), ("method", ctypes.c_int32), ("stop_rule", ctypes.c_int32)]


class _Problem(ctypes.Structure):
    _fields_ = [("A", _Matrix), ("n", ctypes.c_int32), ("d", ctypes.c_int32), ("mu", ctypes.c_double),
                ("X", ctypes.c_void_p), ("iters", ctypes.c_int32), ("tol", ctypes.c_double)]


class _ProblemInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("nonfinite", ctypes.c_int32),
                ("status", ctypes.c_int32), ("rel_change", ctypes.c_double),
                ("max_orth_defect", ctypes.c_double)]


class _BatchOpts(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_int32), ("order", ctypes.c_int32), ("init", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("wait_polls", ctypes.c_int32), ("ticket_kb", ctypes.c_int32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("blocks_per_panel", ctypes.c_int32), ("unroll", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("order", ctypes.c_int32), ("ticket_kb", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("fmt", ctypes.c_int32), ("d", ctypes.c_int32),
                ("nd_min", ctypes.c_int32), ("nd_max", ctypes.c_int32),
                ("blocks_per_panel", ctypes.c_int32), ("unroll", ctypes.c_int32), ("waves", ctypes.c_int32)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("max_active", ctypes.c_int32), ("iters_per_tick", ctypes.c_int32),
                ("ns_steps", ctypes.c_int32), ("waves", ctypes.c_int32), ("ingest_workers", ctypes.c_int32),
                ("pool_bytes", ctypes.c_uint64)]


class _Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("d", ctypes.c_int32), ("sigma", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("Z", ctypes.c_void_p), ("tol", ctypes.c_double),
                ("max_iters", ctypes.c_int32), ("X_out", ctypes.c_void_p)]


class _Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("pad", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("rel_change", ctypes.c_double)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("active", ctypes.c_int32), ("max_active_seen", ctypes.c_int32),
                ("p50_latency_s", ctypes.c_double), ("p99_latency_s", ctypes.c_double),
                ("mean_latency_s", ctypes.c_double), ("solves_per_s", ctypes.c_double),
                ("pool_bytes", ctypes.c_uint64), ("pool_peak_bytes", ctypes.c_uint64)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libnsrgs.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_07372_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    pm = ctypes.POINTER(_Matrix)
    sig = {
        "nsrgs_status_string": (ctypes.c_char_p, [i32]),
        "nsrgs_last_error": (ctypes.c_char_p, []),
        "nsrgs_version": (i32, []),
        "sync_workspace_bytes": (sz, [i32, i32, i32]),
        "sync_workspace_init": (i32, [vp, sz, vp]),
        "sync_step": (i32, [pm, i32, i32, dbl, i32, vp, vp, vp, sz, vp]),
        "sync_step_noalloc": (i32, [pm, i32, i32, dbl, i32, vp, vp, vp]),
        "sync_step_polar": (i32, [pm, i32, i32, dbl, vp, vp, vp, sz, vp]),
        "sync_step_gpm": (i32, [pm, i32, i32, vp, vp, vp, sz, vp]),
        "sync_step_symmetric_workspace_bytes": (sz, [i32, i32, i32]),
        "sync_step_symmetric": (i32, [pm, i32, i32, dbl, i32, vp, vp, vp, sz, vp]),
        "nsrgs_bsr_count": (i32, [vp, i32, i32, dbl, ctypes.c_uint64, vp, vp, ctypes.POINTER(i64), vp]),
        "nsrgs_bsr_fill": (i32, [vp, i32, i32, dbl, dbl, ctypes.c_uint64, ctypes.POINTER(_Bsr), vp]),
        "sync_step_bsr": (i32, [ctypes.POINTER(_Bsr), i32, i32, dbl, i32, vp, vp, vp, sz, vp]),
        "sync_step_bsr_workspace_bytes": (sz, [i32, i32]),
        "sync_solve_bsr": (i32, [ctypes.POINTER(_Bsr), i32, i32, dbl, i32, i32, dbl, vp, vp, sz, vp,
                                 ctypes.POINTER(_SolveOpts), ctypes.POINTER(Info)]),
        "sync_read_info": (i32, [vp, sz, i32, i32, i32, ctypes.POINTER(Info), vp]),
        "sync_init_spectral": (i32, [pm, i32, i32, vp, i32, dbl, vp, sz, vp, ctypes.POINTER(Info)]),
        "sync_solve": (i32, [pm, i32, i32, dbl, i32, i32, dbl, vp, vp, sz, vp,
                             ctypes.POINTER(_SolveOpts), ctypes.POINTER(Info)]),
        "nsrgs_generate_measurement": (i32, [vp, i32, i32, dbl, ctypes.c_uint64, i32, dbl, i32, vp, i64, vp]),
        "nsrgs_convert": (i32, [vp, i32, i64, pm, vp]),
        "nsrgs_packed_elems": (i64, [i32, i32]),
        "sync_stiefel_workspace_bytes": (sz, [i32, i32, i32, i32]),
        "sync_step_stiefel": (i32, [pm, i32, i32, i32, dbl, i32, vp, vp, vp, sz, vp]),
        "sync_solve_stiefel": (i32, [pm, i32, i32, i32, dbl, i32, i32, dbl, vp, vp, sz, vp, ctypes.POINTER(Info)]),
        "sync_stiefel_round": (i32, [vp, i32, i32, i32, i32, vp, vp, sz, vp]),
        "nsrgs_convert_packed": (i32, [vp, i32, i32, pm, vp]),
        "nsrgs_set_tuning": (i32, [ctypes.POINTER(TuneEntry), i32]),
        "nsrgs_get_tuning": (i32, [ctypes.POINTER(TuneEntry), i32]),
        "nsrgs_step_variants": (i32, [i32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), i32]),
        "nsrgs_autotune_step": (i32, [pm, i32, i32, vp, vp, vp, sz, vp, i32, ctypes.POINTER(TuneResult), i32,
                                      ctypes.POINTER(i32)]),
        "nsrgs_autotune_batched": (i32, [ctypes.POINTER(_Problem), i32, i32, i32, vp, sz, vp,
                                         ctypes.POINTER(TuneResult), i32, ctypes.POINTER(i32)]),
        "nsrgs_server_create": (i32, [ctypes.POINTER(_ServerOpts), ctypes.POINTER(vp)]),
        "nsrgs_server_submit": (i32, [vp, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_int64)]),
        "nsrgs_server_poll": (i32, [vp, ctypes.POINTER(_Result), i32, ctypes.POINTER(i32)]),
        "nsrgs_server_wait_idle": (i32, [vp, dbl]),
        "nsrgs_server_get_stats": (i32, [vp, ctypes.POINTER(_ServerStats)]),
        "nsrgs_server_clock": (dbl, [vp]),
        "nsrgs_server_destroy": (i32, [vp]),
        "sync_batch_workspace_bytes": (sz, [ctypes.POINTER(_Problem), i32, i32]),
        "sync_solve_batched": (i32, [ctypes.POINTER(_Problem), i32, i32, i32, vp, sz, vp,
                                     ctypes.POINTER(_BatchOpts), ctypes.POINTER(_ProblemInfo)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int, allow=()):
    if status != 0 and status not in allow:
        msg = lib().nsrgs_last_error().decode() or lib().nsrgs_status_string(status).decode()
        raise NsrgsError(status, msg)
    return status


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def set_tuning(entries) -> None:
    """Install a tuning table (list of dicts with the TuneEntry fields)."""
    arr = (TuneEntry * max(1, len(entries)))()
    for i, e in enumerate(entries):
        arr[i] = TuneEntry(*(int(e[k]) for k, _ in TuneEntry._fields_))
    _check(lib().nsrgs_set_tuning(arr, len(entries)))


def get_tuning() -> list:
    n = lib().nsrgs_get_tuning(None, 0)
    arr = (TuneEntry * max(1, n))()
    lib().nsrgs_get_tuning(arr, n)
    return [{k: getattr(arr[i], k) for k, _ in TuneEntry._fields_} for i in range(n)]


def step_variants(d: int) -> list:
    """(blocks_per_panel, unroll) shapes of the step kernel compiled for d."""
    B = (ctypes.c_int32 * 16)()
    U = (ctypes.c_int32 * 16)()
    n = lib().nsrgs_step_variants(int(d), B, U, 16)
    if n < 0:
        raise NsrgsError(1, lib().nsrgs_last_error().decode())
    return [(B[i], U[i]) for i in range(min(n, 16))]


def batch_rows_per_panel(d: int) -> int:
    """Rows per panel of the batched kernel (whole d x d blocks)."""
    return d * (8 if d == 1 else 4 if d in (2, 3) else 2 if d == 4 else 1)


def padded_ld(nd: int) -> int:
    """Smallest leading dimension >= nd that the library accepts (multiple of 16)."""
    return (nd + 15) // 16 * 16


class StoredMatrix:
    """Device storage of A in one format: tensors plus the leading dimension.

    data     : F64 float64 / F32 float32 / BF16 and BF16_SPLIT int16 codes /
               FP8 uint8 codes, shape (nd, ld); packed=True: one dimension of
               packed_elems(n, d) values (the upper block triangle, layout in
               include/nsrgs.h under NSRGS_LD_PACKED)
    data_lo  : BF16_SPLIT low part, same shape
    row_scale: FP8 per-row float32 scales, shape (nd,)
    """

    def __init__(self, fmt: int, data: torch.Tensor, nd: int, data_lo=None, row_scale=None,
                 packed: bool = False):
        self.fmt = int(fmt)
        self.data = data
        self.data_lo = data_lo
        self.row_scale = row_scale
        self.nd = int(nd)
        self.packed = bool(packed)
        self.ld = PACKED_LD if packed else int(data.shape[1])

    def c(self) -> _Matrix:
        return _Matrix(self.fmt, _ptr(self.data), _ptr(self.data_lo), _ptr(self.row_scale), self.ld)

    @property
    def nbytes(self) -> int:
        tot = self.data.numel() * self.data.element_size()
        if self.data_lo is not None:
            tot += self.data_lo.numel() * self.data_lo.element_size()
        if self.row_scale is not None:
            tot += self.row_scale.numel() * 4
        return tot


def stored(A: torch.Tensor, fmt: int = F32) -> StoredMatrix:
    """Wrap a float32/float64 device matrix (nd x ld, ld padded) as F32/F64 storage,
    or convert a float32 one into BF16 / BF16_SPLIT / FP8 on the device."""
    nd = A.shape[0]
    if fmt in (F64, F32):
        want = torch.float64 if fmt == F64 else torch.float32
        if A.dtype != want:
            raise TypeError(f"format {fmt} needs a {want} matrix")
        return StoredMatrix(fmt, A, nd)
    return convert(A, fmt)


class Workspace:
    """Device workspace for one (n, d, precision) problem; prepared on creation."""

    def __init__(self, n: int, d: int, fmt: int, device="cuda", symmetric: bool = False, bsr: bool = False):
        if bsr:
            nbytes = lib().sync_step_bsr_workspace_bytes(n, d)
        elif symmetric:
            nbytes = lib().sync_step_symmetric_workspace_bytes(n, d, fmt)
        else:
            nbytes = lib().sync_workspace_bytes(n, d, fmt)
        if nbytes == 0:
            raise NsrgsError(1, f"invalid workspace request n={n} d={d} fmt={fmt}")
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-buf.data_ptr()) % 256
        self._buf = buf
        self.tensor = buf[off: off + nbytes]
        self.nbytes = nbytes
        self.n, self.d, self.fmt = n, d, fmt
        _check(lib().sync_workspace_init(self.ptr, nbytes, _stream()))

    @property
    def ptr(self) -> int:
        return self.tensor.data_ptr()


def workspace(n: int, d: int, fmt: int, device="cuda", symmetric: bool = False, bsr: bool = False) -> Workspace:
    """symmetric=True sizes it for step_symmetric (which also serves every other call);
    bsr=True for the sliced block-sparse step (sync_step_bsr_workspace_bytes, also a
    valid sync_workspace_bytes(n, d, F32) workspace)."""
    return Workspace(n, d, fmt, device, symmetric, bsr)


def _xdtype(fmt: int):
    return torch.float64 if fmt == F64 else torch.float32


def _check_x(X: torch.Tensor, nd: int, d: int, fmt: int, name: str):
    if not X.is_cuda or X.dtype != _xdtype(fmt) or tuple(X.shape) != (nd, d) or not X.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {_xdtype(fmt)} CUDA tensor of shape ({nd}, {d})")


def step(A: StoredMatrix, n: int, d: int, X_in: torch.Tensor, X_out: torch.Tensor,
         ws: Workspace, mu: float = 0.0, ns_steps: int = 3) -> None:
    """One NS-RGS iteration (sync_step), asynchronous on the current stream."""
    _check_x(X_in, n * d, d, A.fmt, "X_in")
    _check_x(X_out, n * d, d, A.fmt, "X_out")
    m = A.c()
    _check(lib().sync_step(ctypes.byref(m), n, d, float(mu), int(ns_steps), X_in.data_ptr(),
                           X_out.data_ptr(), ws.ptr, ws.nbytes, _stream()))


def step_polar(A: StoredMatrix, n: int, d: int, X_in: torch.Tensor, X_out: torch.Tensor,
               ws: Workspace, mu: float = 0.0) -> None:
    """sync_step_polar: one step with the exact retraction sgn(F_i)."""
    _check_x(X_in, n * d, d, A.fmt, "X_in")
    _check_x(X_out, n * d, d, A.fmt, "X_out")
    m = A.c()
    _check(lib().sync_step_polar(ctypes.byref(m), n, d, float(mu), X_in.data_ptr(), X_out.data_ptr(),
                                 ws.ptr, ws.nbytes, _stream()))


def step_gpm(A: StoredMatrix, n: int, d: int, X_in: torch.Tensor, X_out: torch.Tensor, ws: Workspace) -> None:
    """sync_step_gpm: one generalized-power-method step X_i <- sgn((A X)_i)."""
    _check_x(X_in, n * d, d, A.fmt, "X_in")
    _check_x(X_out, n * d, d, A.fmt, "X_out")
    m = A.c()
    _check(lib().sync_step_gpm(ctypes.byref(m), n, d, X_in.data_ptr(), X_out.data_ptr(), ws.ptr, ws.nbytes,
                               _stream()))


def step_noalloc(A: StoredMatrix, n: int, d: int, X_in: torch.Tensor, X_out: torch.Tensor,
                 mu: float = 0.0, ns_steps: int = 3) -> None:
    """sync_step_noalloc: sync_step with the library's fixed scratch instead of a
    workspace (allocates nothing); asynchronous on the current stream."""
    _check_x(X_in, n * d, d, A.fmt, "X_in")
    _check_x(X_out, n * d, d, A.fmt, "X_out")
    m = A.c()
    _check(lib().sync_step_noalloc(ctypes.byref(m), n, d, float(mu), int(ns_steps), X_in.data_ptr(),
                                   X_out.data_ptr(), _stream()))


def step_symmetric(A: StoredMatrix, n: int, d: int, X_in: torch.Tensor, X_out: torch.Tensor,
                   ws: Workspace, mu: float = 0.0, ns_steps: int = 3) -> None:
    """sync_step_symmetric: the iteration from the blocks above the block diagonal
    only (A must be exactly symmetric); ws from workspace(..., symmetric=True)."""
    _check_x(X_in, n * d, d, A.fmt, "X_in")
    _check_x(X_out, n * d, d, A.fmt, "X_out")
    m = A.c()
    _check(lib().sync_step_symmetric(ctypes.byref(m), n, d, float(mu), int(ns_steps), X_in.data_ptr(),
                                     X_out.data_ptr(), ws.ptr, ws.nbytes, _stream()))


class _StiefelWorkspace(Workspace):
    """Workspace of the Stiefel calls (also a single-problem workspace of (n, d, fmt))."""

    def __init__(self, n: int, d: int, p: int, fmt: int, device="cuda"):
        nbytes = lib().sync_stiefel_workspace_bytes(n, d, p, fmt)
        if nbytes == 0:
            raise NsrgsError(1, f"invalid Stiefel workspace request n={n} d={d} p={p} fmt={fmt}")
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-buf.data_ptr()) % 256
        self._buf = buf
        self.tensor = buf[off: off + nbytes]
        self.nbytes = nbytes
        self.n, self.d, self.p, self.fmt = n, d, p, fmt
        _check(lib().sync_workspace_init(self.ptr, nbytes, _stream()))


def stiefel_workspace(n: int, d: int, p: int, fmt: int, device="cuda") -> Workspace:
    return _StiefelWorkspace(n, d, p, fmt, device)


def _check_s(S: torch.Tensor, nd: int, p: int, fmt: int, name: str):
    if not S.is_cuda or S.dtype != _xdtype(fmt) or tuple(S.shape) != (nd, p) or not S.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {_xdtype(fmt)} CUDA tensor of shape ({nd}, {p})")


def step_stiefel(A: StoredMatrix, n: int, d: int, p: int, S_in: torch.Tensor, S_out: torch.Tensor,
                 ws: Workspace, mu: float = 0.0, ns_steps: int = 3) -> None:
    """sync_step_stiefel: one NS-RGS step on St(p, d)^n (S: n*d x p, rows of each
    d x p block orthonormal); ws from stiefel_workspace(n, d, p, fmt)."""
    _check_s(S_in, n * d, p, A.fmt, "S_in")
    _check_s(S_out, n * d, p, A.fmt, "S_out")
    m = A.c()
    _check(lib().sync_step_stiefel(ctypes.byref(m), n, d, p, float(mu), int(ns_steps), S_in.data_ptr(),
                                   S_out.data_ptr(), ws.ptr, ws.nbytes, _stream()))


def solve_stiefel(A: StoredMatrix, n: int, d: int, p: int, S: torch.Tensor, ws: Workspace, mu: float = 0.0,
                  ns_steps: int = 3, max_iters: int = 100, tol: float = 0.0, check: bool = True) -> dict:
    """sync_solve_stiefel: at most max_iters steps from the start held in S (result in S)."""
    _check_s(S, n * d, p, A.fmt, "S")
    m = A.c()
    info = Info()
    st = lib().sync_solve_stiefel(ctypes.byref(m), n, d, p, float(mu), int(ns_steps), int(max_iters), float(tol),
                                  S.data_ptr(), ws.ptr, ws.nbytes, _stream(), ctypes.byref(info))
    if check:
        _check(st, allow=(5,))
    out = info.as_dict(d)
    out["status"] = st
    return out


def stiefel_round(S: torch.Tensor, n: int, d: int, p: int, fmt: int, X: torch.Tensor, ws: Workspace) -> None:
    """sync_stiefel_round: X_i = sgn(S_i V), V the top-d eigenvectors of S^T S."""
    _check_s(S, n * d, p, fmt, "S")
    _check_x(X, n * d, d, fmt, "X")
    _check(lib().sync_stiefel_round(S.data_ptr(), n, d, p, int(fmt), X.data_ptr(), ws.ptr, ws.nbytes, _stream()))


def symmetric_workspace_bytes(n: int, d: int, fmt: int) -> int:
    return int(lib().sync_step_symmetric_workspace_bytes(n, d, fmt))


class BsrMatrix:
    """Block-sparse A of the incomplete observation model (device arrays; layout
    in include/nsrgs.h): row_ptr (n + 1, int64), col_idx (nnzb, int32), values
    (nnzb d^2, FP32 or BF16 bits), in groups of 64 blocks per block row, entry-major
    within each group."""

    def __init__(self, fmt: int, row_ptr: torch.Tensor, col_idx: torch.Tensor, values: torch.Tensor,
                 n: int, d: int, nnzb: int):
        self.fmt, self.row_ptr, self.col_idx, self.values = fmt, row_ptr, col_idx, values
        self.n, self.d, self.nnzb = n, d, nnzb

    def c(self) -> _Bsr:
        return _Bsr(self.fmt, 0, self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.values.data_ptr())

    @property
    def nbytes(self) -> int:
        return (self.row_ptr.numel() * 8 + self.nnzb * 4
                + self.nnzb * self.d * self.d * (4 if self.fmt == F32 else 2))


def generate_bsr(Z: torch.Tensor, sigma: float, seed: int, p: float, fmt: int = F32) -> BsrMatrix:
    """Block-sparse A on the device for the model and seed of generate(..., p=p)
    (nsrgs_bsr_count + nsrgs_bsr_fill): the observed off-diagonal blocks only."""
    if not Z.is_cuda or Z.dtype != torch.float64 or Z.dim() != 2 or not Z.is_contiguous():
        raise ValueError("Z must be a contiguous float64 CUDA tensor (n*d, d)")
    nd, d = Z.shape
    n = nd // d
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=Z.device)
    counts = torch.empty(n, dtype=torch.int64, device=Z.device)
    nnzb = ctypes.c_int64(0)
    _check(lib().nsrgs_bsr_count(Z.data_ptr(), n, d, float(p), int(seed), row_ptr.data_ptr(), counts.data_ptr(),
                                 ctypes.byref(nnzb), _stream()))
    k = int(nnzb.value)
    col_idx = torch.empty(max(k, 1), dtype=torch.int32, device=Z.device)
    values = torch.empty(max(k, 1) * d * d, dtype=torch.float32 if fmt == F32 else torch.int16, device=Z.device)
    A = BsrMatrix(fmt, row_ptr, col_idx, values, n, d, k)
    m = A.c()
    _check(lib().nsrgs_bsr_fill(Z.data_ptr(), n, d, float(sigma), float(p), int(seed), ctypes.byref(m), _stream()))
    return A


def step_bsr(A: BsrMatrix, n: int, d: int, X_in: torch.Tensor, X_out: torch.Tensor, ws: Workspace,
             mu: float = 0.0, ns_steps: int = 3) -> None:
    """sync_step_bsr: one iteration on block-sparse A (pass mu = 1/(n p) for the
    incomplete observation model); ws = workspace(n, d, F32)."""
    _check_x(X_in, n * d, d, F32, "X_in")
    _check_x(X_out, n * d, d, F32, "X_out")
    m = A.c()
    _check(lib().sync_step_bsr(ctypes.byref(m), n, d, float(mu), int(ns_steps), X_in.data_ptr(), X_out.data_ptr(),
                               ws.ptr, ws.nbytes, _stream()))


def solve_bsr(A: BsrMatrix, n: int, d: int, X: torch.Tensor, ws: Workspace, mu: float = 0.0,
              ns_steps: int = 3, max_iters: int = 100, tol: float = 0.0, init: bool = True,
              init_iters: int = 60, init_tol: float = 0.0, check_every: int = 16, check: bool = True,
              method: str = "ns_rgs", stop: str = "rel_change") -> dict:
    """sync_solve_bsr: Algorithm 2 on block-sparse A (spectral initialization with
    the block-sparse product, then the iterations); ws = workspace(n, d, F32), or
    workspace(n, d, F32, bsr=True) for the sliced product at d <= 6."""
    _check_x(X, n * d, d, F32, "X")
    m = A.c()
    opts = _SolveOpts(int(init), int(init_iters), float(init_tol), 0, None, int(check_every), 0,
                      METHODS[method], STOP_RULES[stop])
    info = Info()
    st = lib().sync_solve_bsr(ctypes.byref(m), n, d, float(mu), int(ns_steps), int(max_iters), float(tol),
                              X.data_ptr(), ws.ptr, ws.nbytes, _stream(), ctypes.byref(opts), ctypes.byref(info))
    if check:
        _check(st, allow=(5,))
    out = info.as_dict(d)
    out["status"] = st
    return out


def read_info(ws: Workspace) -> dict:
    info = Info()
    _check(lib().sync_read_info(ws.ptr, ws.nbytes, ws.n, ws.d, ws.fmt, ctypes.byref(info), _stream()))
    return info.as_dict(ws.d)


def init_spectral(A: StoredMatrix, n: int, d: int, X0: torch.Tensor, ws: Workspace,
                  max_iters: int = 0, tol: float = 0.0, check: bool = True) -> dict:
    """Spectral initialization X0 = sgn(top-d eigenvectors of A) (sync_init_spectral)."""
    _check_x(X0, n * d, d, A.fmt, "X0")
    m = A.c()
    info = Info()
    st = lib().sync_init_spectral(ctypes.byref(m), n, d, X0.data_ptr(), int(max_iters), float(tol),
                                  ws.ptr, ws.nbytes, _stream(), ctypes.byref(info))
    if check:
        _check(st, allow=(5,))
    out = info.as_dict(d)
    out["status"] = st
    return out


METHODS = {"ns_rgs": 0, "polar": 1, "gpm": 2}
STOP_RULES = {"rel_change": 0, "objective": 1}


def solve(A: StoredMatrix, n: int, d: int, X: torch.Tensor, ws: Workspace, mu: float = 0.0,
          ns_steps: int = 3, max_iters: int = 100, tol: float = 0.0, init: bool = True,
          init_iters: int = 60, init_tol: float = 0.0, refine_iters: int = 0,
          A_refine: StoredMatrix | None = None, check_every: int = 16, check: bool = True,
          symmetric: bool = False, method: str = "ns_rgs", stop: str = "rel_change") -> dict:
    """Algorithm 2 end to end (sync_solve).  X receives the result (and holds X0 if init=False).
    symmetric=True runs every iteration as step_symmetric (ws from workspace(..., symmetric=True)).
    method: "ns_rgs", "polar" (exact retraction) or "gpm"; stop: "rel_change" or "objective"
    (the paper's R^t rule), used when tol > 0."""
    _check_x(X, n * d, d, A.fmt, "X")
    m = A.c()
    mref = A_refine.c() if A_refine is not None else None
    opts = _SolveOpts(int(init), int(init_iters), float(init_tol), int(refine_iters),
                      ctypes.pointer(mref) if mref is not None else None, int(check_every), int(symmetric),
                      METHODS[method], STOP_RULES[stop])
    info = Info()
    st = lib().sync_solve(ctypes.byref(m), n, d, float(mu), int(ns_steps), int(max_iters), float(tol),
                          X.data_ptr(), ws.ptr, ws.nbytes, _stream(), ctypes.byref(opts), ctypes.byref(info))
    if check:
        _check(st, allow=(5,))
    out = info.as_dict(d)
    out["status"] = st
    return out


def packed_elems(n: int, d: int) -> int:
    """Elements of the packed upper-block-triangle layout (nsrgs_packed_elems)."""
    return int(lib().nsrgs_packed_elems(int(n), int(d)))


def generate(Z: torch.Tensor, sigma: float, seed: int, fmt: int = F32, zero_diag_blocks: bool = False,
             p: float = 1.0, ld: int | None = None, packed: bool = False) -> torch.Tensor:
    """A = Z Z^T + sigma W on the device (Philox4x32-10 noise); F64 or F32, shape (nd, ld),
    or with packed=True the packed upper block triangle (packed_elems(n, d) values)."""
    if not Z.is_cuda or Z.dtype != torch.float64 or Z.dim() != 2 or not Z.is_contiguous():
        raise ValueError("Z must be a contiguous float64 CUDA tensor (n*d, d)")
    nd, d = Z.shape
    n = nd // d
    if packed:
        A = torch.empty((packed_elems(n, d),), dtype=_xdtype(fmt), device=Z.device)
        ld = PACKED_LD
    else:
        ld = ld or padded_ld(nd)
        A = torch.empty((nd, ld), dtype=_xdtype(fmt), device=Z.device)
        if ld > nd:
            A[:, nd:].zero_()
    _check(lib().nsrgs_generate_measurement(Z.data_ptr(), n, d, float(sigma), int(seed),
                                            int(zero_diag_blocks), float(p), int(fmt), A.data_ptr(),
                                            ld, _stream()))
    return A


def convert(A32: torch.Tensor, fmt: int) -> StoredMatrix:
    """One-time conversion of an FP32 device matrix (nd, ld) into BF16 / BF16_SPLIT / FP8."""
    if not A32.is_cuda or A32.dtype != torch.float32 or A32.dim() != 2 or not A32.is_contiguous():
        raise ValueError("A32 must be a contiguous float32 CUDA tensor (nd, ld)")
    nd, ld = A32.shape
    if fmt in (BF16, BF16_SPLIT):
        data = torch.zeros((nd, ld), dtype=torch.int16, device=A32.device)
        lo = torch.zeros((nd, ld), dtype=torch.int16, device=A32.device) if fmt == BF16_SPLIT else None
        out = StoredMatrix(fmt, data, nd, data_lo=lo)
    elif fmt == FP8_E4M3:
        data = torch.zeros((nd, ld), dtype=torch.uint8, device=A32.device)
        sc = torch.empty((nd,), dtype=torch.float32, device=A32.device)
        out = StoredMatrix(fmt, data, nd, row_scale=sc)
    else:
        raise ValueError(f"cannot convert to format {fmt}")
    m = out.c()
    _check(lib().nsrgs_convert(A32.data_ptr(), nd, ld, ctypes.byref(m), _stream()))
    return out


def convert_packed(A32: torch.Tensor, n: int, d: int, fmt: int) -> StoredMatrix:
    """One-time conversion of a packed FP32 device matrix into packed BF16 / BF16_SPLIT."""
    count = packed_elems(n, d)
    if not A32.is_cuda or A32.dtype != torch.float32 or A32.dim() != 1 or A32.numel() != count:
        raise ValueError(f"A32 must be a float32 CUDA tensor of packed_elems(n, d) = {count} values")
    if fmt not in (BF16, BF16_SPLIT):
        raise ValueError(f"packed conversion targets BF16 or BF16_SPLIT, not format {fmt}")
    data = torch.empty((count,), dtype=torch.int16, device=A32.device)
    lo = torch.empty((count,), dtype=torch.int16, device=A32.device) if fmt == BF16_SPLIT else None
    out = StoredMatrix(fmt, data, n * d, data_lo=lo, packed=True)
    m = out.c()
    _check(lib().nsrgs_convert_packed(A32.data_ptr(), int(n), int(d), ctypes.byref(m), _stream()))
    return out


def stored_packed(A: torch.Tensor, n: int, d: int, fmt: int = F32) -> StoredMatrix:
    """Wrap a packed float32/float64 device matrix (generate(..., packed=True)) as F32/F64
    storage, or convert a packed float32 one into packed BF16 / BF16_SPLIT."""
    if fmt in (F64, F32):
        want = torch.float64 if fmt == F64 else torch.float32
        if A.dtype != want or A.dim() != 1 or A.numel() != packed_elems(n, d):
            raise TypeError(f"format {fmt} needs a packed {want} matrix of packed_elems(n, d) values")
        return StoredMatrix(fmt, A, n * d, packed=True)
    return convert_packed(A, n, d, fmt)


def _batch_args(problems, init=False):
    """C problem array and an aligned workspace for a batch."""
    count = len(problems)
    arr = (_Problem * count)()
    for k, p in enumerate(problems):
        _check_x(p["X"], p["n"] * p["d"], p["d"], p["A"].fmt, f"problems[{k}].X")
        arr[k] = _Problem(p["A"].c(), int(p["n"]), int(p["d"]), float(p.get("mu", 0.0)), p["X"].data_ptr(),
                          int(p.get("iters", 0)), float(p.get("tol", 0.0)))
    nbytes = lib().sync_batch_workspace_bytes(arr, count, int(init))
    if nbytes == 0:
        _check(1)
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=problems[0]["X"].device)
    off = (-buf.data_ptr()) % 256
    return arr, buf, off, nbytes


def solve_batched(problems, ns_steps: int = 3, max_iters: int = 100, init: bool = False, waves: int = 0,
                  order: int = 0, check_every: int = 0, persistent: bool = False, wait_polls: int = 0,
                  ticket_kb: int = 0, check: bool = True):
    """Many problems per launch (sync_solve_batched): one grouped launch per
    iteration, or with persistent=True one launch for the whole budget.

    problems: sequence of dicts with keys A (StoredMatrix), n, d, X (device tensor,
    X^0 on entry unless init, result on return) and optional mu, iters, tol.
    Returns (status, list of per-problem info dicts)."""
    count = len(problems)
    arr, buf, off, nbytes = _batch_args(problems, init)
    opts = _BatchOpts(int(waves), int(order), int(init), int(check_every), int(persistent), int(wait_polls),
                      int(ticket_kb))
    infos = (_ProblemInfo * count)()
    st = lib().sync_solve_batched(arr, count, int(ns_steps), int(max_iters), buf.data_ptr() + off, nbytes,
                                  _stream(), ctypes.byref(opts), infos)
    if check:
        _check(st, allow=(5,))
    out = [{k: getattr(infos[i], k) for k, _ in _ProblemInfo._fields_} for i in range(count)]
    return st, out


class Server:
    """Continuous-batching solve server (nsrgs_server_*), on the current device.

    submit() takes the problem description and the host ground truth Z; the
    result lands in a host float32 array that submit() returns (filled when the
    request's result is posted)."""

    def __init__(self, fmt: int = BF16, pool_bytes: int = 0, max_active: int = 64, iters_per_tick: int = 4,
                 ns_steps: int = 3, waves: int = 0, ingest_workers: int = 0):
        opts = _ServerOpts(int(fmt), int(max_active), int(iters_per_tick), int(ns_steps), int(waves),
                           int(ingest_workers), int(pool_bytes))
        h = ctypes.c_void_p()
        _check(lib().nsrgs_server_create(ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, Z, sigma: float, seed: int, tol: float = 1e-6, max_iters: int = 300):
        import numpy as np
        Z = np.ascontiguousarray(Z, dtype=np.float64)
        nd, d = Z.shape
        out = np.zeros((nd, d), dtype=np.float32)
        req = _Request(nd // d, d, float(sigma), int(seed), Z.ctypes.data, float(tol), int(max_iters),
                       out.ctypes.data)
        rid = ctypes.c_int64()
        _check(lib().nsrgs_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        self._keep[rid.value] = (Z, out)
        return rid.value, out

    def poll(self, max_results: int = 1024) -> list:
        arr = (_Result * max_results)()
        cnt = ctypes.c_int()
        _check(lib().nsrgs_server_poll(self._h, arr, max_results, ctypes.byref(cnt)))
        out = []
        for i in range(cnt.value):
            r = {k: getattr(arr[i], k) for k, _ in _Result._fields_ if k != "pad"}
            self._keep.pop(r["id"], None)
            out.append(r)
        return out

    def wait_idle(self, timeout_s: float = 0.0) -> int:
        return _check(lib().nsrgs_server_wait_idle(self._h, float(timeout_s)), allow=(5,))

    def stats(self) -> dict:
        st = _ServerStats()
        _check(lib().nsrgs_server_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _ServerStats._fields_}

    def clock(self) -> float:
        return lib().nsrgs_server_clock(self._h)

    def close(self) -> None:
        if self._h:
            lib().nsrgs_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def upload(A: "numpy.ndarray", fmt: int = F32, device="cuda") -> StoredMatrix:  # noqa: F821
    """Copy a host matrix (nd x nd, float64) to the device in F64 or F32 with padded ld."""
    import numpy as np
    nd = A.shape[0]
    ld = padded_ld(nd)
    host = np.zeros((nd, ld), dtype=np.float64 if fmt == F64 else np.float32)
    host[:, :nd] = A
    t = torch.from_numpy(host).to(device)
    return StoredMatrix(fmt, t, nd)


__all__.append("upload")
