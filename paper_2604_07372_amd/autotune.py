"""Autotuner front end: measure launch shapes on a real problem, install the
winners in the library's tuning table, and keep the table in a JSON file.

The measuring is done by the library (nsrgs_autotune_step,
nsrgs_autotune_batched: HIP-event or wall-clock timing of the real kernels);
this module only chooses what to install and persists it.
"""
from __future__ import annotations

import ctypes
import json

import torch

from . import (TuneResult, Workspace, _batch_args, _check, _stream, get_tuning, lib, set_tuning,
               workspace)

__all__ = ["tune_step", "tune_batched", "install_step", "save_table", "load_table"]

_RESULT_FIELDS = [k for k, _ in TuneResult._fields_]


def _results(arr, n):
    return [{k: getattr(arr[i], k) for k in _RESULT_FIELDS} for i in range(n)]


def tune_step(A, n: int, d: int, X: torch.Tensor, ws: Workspace | None = None, reps: int = 5,
              install: bool = True, nd_range: tuple[int, int] | None = None) -> list:
    """Time every compiled (blocks_per_panel, unroll) shape and waves in
    {1, 2, 4, 8} (at most 4 for the software-pipelined unroll = 0 shapes) for
    sync_step on this problem; fastest first.  With install,
    the fastest becomes the table entry for (format, d) over nd_range
    (default: half to twice this n*d)."""
    ws = ws if ws is not None else workspace(n, d, A.fmt)
    Xout = torch.empty_like(X)
    res = (TuneResult * 64)()
    cnt = ctypes.c_int(0)
    _check(lib().nsrgs_autotune_step(ctypes.byref(A.c()), int(n), int(d), X.data_ptr(), Xout.data_ptr(),
                                     ws.ptr, ws.nbytes, _stream(), int(reps), res, 64, ctypes.byref(cnt)))
    out = _results(res, min(cnt.value, 64))
    if install and out:
        nd = n * d
        lo, hi = nd_range if nd_range else (nd // 2, 2 * nd)
        install_step(A.fmt, d, lo, hi, out[0])
    return out


def install_step(fmt: int, d: int, nd_min: int, nd_max: int, best: dict) -> None:
    """Put a step shape in the table for (fmt, d, [nd_min, nd_max]), replacing
    entries of the same kind, format and d whose ranges overlap it."""
    keep = [e for e in get_tuning()
            if not (e["kind"] == 0 and e["fmt"] == fmt and e["d"] == d
                    and e["nd_min"] <= nd_max and nd_min <= e["nd_max"])]
    keep.insert(0, {"kind": 0, "fmt": int(fmt), "d": int(d), "nd_min": int(nd_min), "nd_max": int(nd_max),
                    "blocks_per_panel": int(best["blocks_per_panel"]), "unroll": int(best["unroll"]),
                    "waves": int(best["waves"])})
    set_tuning(keep)


def tune_batched(problems, iters: int = 5, ns_steps: int = 3) -> list:
    """Time the batched schedules (grouped / persistent, unit order, waves,
    ticket size) on copies of these problems' iterates; fastest first.  Each
    result converts to solve_batched keyword arguments with batch_options()."""
    copies = [dict(p, X=p["X"].clone()) for p in problems]
    arr, buf, off, nbytes = _batch_args(copies)
    res = (TuneResult * 64)()
    cnt = ctypes.c_int(0)
    _check(lib().nsrgs_autotune_batched(arr, len(copies), int(ns_steps), int(iters), buf.data_ptr() + off,
                                        nbytes, _stream(), res, 64, ctypes.byref(cnt)))
    return _results(res, min(cnt.value, 64))


def batch_options(result: dict) -> dict:
    """solve_batched keyword arguments for one tune_batched result."""
    return {"persistent": bool(result["persistent"]), "order": int(result["order"]),
            "waves": int(result["waves"]), "ticket_kb": int(result["ticket_kb"])}


def save_table(path: str) -> None:
    """Write the library's current tuning table as JSON."""
    with open(path, "w") as f:
        json.dump({"nsrgs_tuning": get_tuning()}, f, indent=1)


def load_table(path: str) -> list:
    """Install a tuning table written by save_table; returns its entries."""
    with open(path) as f:
        entries = json.load(f)["nsrgs_tuning"]
    set_tuning(entries)
    return entries
