"""The autotuner: argument checks and the tuning table's JSON round trip (CPU),
measurements on real problems and use of the installed shapes (GPU)."""
import ctypes
import math

import numpy as np
import pytest
import torch

import paper_2604_07372_amd as P
from paper_2604_07372_amd import autotune
import synth
from oracle import nsrgs as O

from gpu_common import FMT_NAME, device_matrix, host, oracle_matrix, require_gpu, step_tolerance, to_dev


@pytest.fixture
def clean_table():
    saved = P.get_tuning()
    P.set_tuning([])
    yield
    P.set_tuning(saved)


def test_autotune_step_rejects_before_device_use():
    m = P._Matrix(P.F32, 16, None, None, 304)
    res = (P.TuneResult * 4)()
    cnt = ctypes.c_int(0)
    st = P.lib().nsrgs_autotune_step(ctypes.byref(m), 100, 3, 1 << 20, 1 << 24, 256, 1 << 30, None, 0, res, 4,
                                     ctypes.byref(cnt))
    assert st == 1 and "reps" in P.lib().nsrgs_last_error().decode()
    st = P.lib().nsrgs_autotune_step(ctypes.byref(m), 1, 3, 1 << 20, 1 << 24, 256, 1 << 30, None, 5, res, 4,
                                     ctypes.byref(cnt))
    assert st == 1 and "n must be" in P.lib().nsrgs_last_error().decode()


def test_autotune_batched_rejects_before_device_use():
    res = (P.TuneResult * 4)()
    cnt = ctypes.c_int(0)
    assert P.lib().nsrgs_autotune_batched(None, 0, 3, 5, None, 0, None, res, 4, ctypes.byref(cnt)) == 1
    m = P._Matrix(P.F32, 16, None, None, 304)
    arr = (P._Problem * 1)(P._Problem(m, 100, 3, 0.0, 4096, 0, 0.0))
    assert P.lib().nsrgs_autotune_batched(arr, 1, 3, 0, None, 0, None, res, 4, ctypes.byref(cnt)) == 1
    assert "iters" in P.lib().nsrgs_last_error().decode()


def test_install_replaces_overlapping_entries_and_json_round_trip(tmp_path, clean_table):
    autotune.install_step(P.F32, 3, 1000, 4000, {"blocks_per_panel": 4, "unroll": 2, "waves": 4})
    autotune.install_step(P.F32, 3, 100000, 200000, {"blocks_per_panel": 2, "unroll": 1, "waves": 8})
    autotune.install_step(P.F32, 3, 3000, 8000, {"blocks_per_panel": 1, "unroll": 4, "waves": 2})
    table = P.get_tuning()
    ranges = sorted((e["nd_min"], e["nd_max"], e["blocks_per_panel"]) for e in table)
    assert ranges == [(3000, 8000, 1), (100000, 200000, 2)]        # the overlapping one is gone
    path = tmp_path / "tuning.json"
    autotune.save_table(str(path))
    P.set_tuning([])
    assert P.get_tuning() == []
    assert autotune.load_table(str(path)) == table
    assert P.get_tuning() == table


def test_step_variants_cover_every_d():
    """Every d has shapes, a B = 1, U = 1 one for the default, and the batched
    kernel's panel shape as a single-problem shape (the batched result equals
    sync_step's with that shape)."""
    for d in range(1, 17):
        v = P.step_variants(d)
        assert v and all(B >= 1 and U >= 0 for B, U in v)
        assert len(set(v)) == len(v)
        assert (1, 1) in v or d <= 4
        assert (P.batch_rows_per_panel(d) // d, 1) in v
    assert P.step_variants(17) == [] and P.step_variants(0) == []


@pytest.mark.gpu
@pytest.mark.parametrize("fmt", [P.F32, P.BF16], ids=lambda f: FMT_NAME[f])
def test_tune_step_measures_every_shape_and_the_winner_is_used(fmt, clean_table, monkeypatch):
    require_gpu()
    n, d = 700, 3
    Z = synth.haar_blocks(n, d, 77)
    A64 = synth.measurement_matrix(Z, synth.sigma_for(0.2, n, d), 78)
    X = synth.perturbed_start(Z, 0.05, 79)
    Ad = device_matrix(A64, fmt)
    Xd = to_dev(X, torch.float32)
    res = autotune.tune_step(Ad, n, d, Xd, reps=3)
    # waves 1, 2, 4, 8; the software-pipelined shapes (U = 0) launch with at most 4
    assert len(res) == sum(3 if u == 0 else 4 for _, u in P.step_variants(d))
    assert all(r["waves"] <= 4 for r in res if r["unroll"] == 0)
    assert all(r["ms"] > 0 for r in res)
    assert [r["ms"] for r in res] == sorted(r["ms"] for r in res)
    shapes = {(r["blocks_per_panel"], r["unroll"]) for r in res}
    assert shapes == set(P.step_variants(d))
    best = res[0]
    assert P.get_tuning()[0]["blocks_per_panel"] == best["blocks_per_panel"]
    # the tuned launch gives bitwise the result of the same shape forced by hand
    ws = P.workspace(n, d, fmt)
    out_tuned = torch.empty_like(Xd)
    P.step(Ad, n, d, Xd, out_tuned, ws)
    monkeypatch.setenv("NSRGS_STEP_B", str(best["blocks_per_panel"]))
    monkeypatch.setenv("NSRGS_STEP_U", str(best["unroll"]))
    monkeypatch.setenv("NSRGS_STEP_W", str(best["waves"]))
    out_forced = torch.empty_like(Xd)
    P.step(Ad, n, d, Xd, out_forced, ws)
    torch.cuda.synchronize()
    assert torch.equal(out_tuned, out_forced)
    As = oracle_matrix(A64, fmt)
    ref = O.rgs_step(As, host(Xd), d, Ts=3)
    assert np.abs(host(out_tuned) - ref.X).max() <= step_tolerance(As, host(Xd), n, fmt)


@pytest.mark.gpu
def test_tune_batched_ranks_schedules_and_the_winner_matches_grouped():
    require_gpu()
    shapes = [(300, 3), (120, 2), (40, 10), (200, 4), (9, 3)]
    probs = []
    for k, (n, d) in enumerate(shapes):
        Z = synth.haar_blocks(n, d, 300 + k)
        A64 = synth.measurement_matrix(Z, synth.sigma_for(0.2, n, d), 400 + k)
        X0 = synth.perturbed_start(Z, 0.05, 500 + k)
        probs.append({"A": device_matrix(A64, P.F32), "n": n, "d": d, "X": to_dev(X0, torch.float32)})
    X0s = [p["X"].clone() for p in probs]
    res = autotune.tune_batched(probs, iters=3)
    assert len(res) == 24
    assert [r["ms"] for r in res] == sorted(r["ms"] for r in res)
    assert {(r["persistent"], r["order"]) for r in res} == {(0, 0), (0, 1), (1, 0), (1, 1)}
    assert all(torch.equal(p["X"], x) for p, x in zip(probs, X0s))     # tuned on copies
    best = autotune.batch_options(res[0])
    st, _ = P.solve_batched(probs, max_iters=10, **best)
    assert st == 0
    grouped = [dict(p, X=x.clone()) for p, x in zip(probs, X0s)]
    P.solve_batched(grouped, max_iters=10, waves=best["waves"], order=best["order"])
    torch.cuda.synchronize()
    for p, q in zip(probs, grouped):
        assert torch.equal(p["X"], q["X"])
