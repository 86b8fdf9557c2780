"""GPU tests of batched solves: many uneven problems per launch."""
import ctypes
import math

import numpy as np
import pytest
import torch

import paper_2604_07372_amd as P
import synth
from oracle import nsrgs as O

from gpu_common import FMT_NAME, check_stop_iteration, device_matrix, host, oracle_matrix, require_gpu, to_dev, xdtype

# Largest d is 16 (the widest kernel class).
MIX = [(2, 1), (5, 2), (37, 3), (100, 4), (61, 10), (341, 3), (20, 16), (130, 2), (47, 7), (700, 3)]
# The same kind of mix with largest d 10 (the middle kernel class).
MIX10 = [(2, 1), (5, 2), (37, 3), (100, 4), (61, 10), (341, 3), (33, 9), (130, 2), (47, 7), (700, 3)]


def _batch(fmt, shapes, seed=0, c=0.25):
    probs, refs = [], []
    for k, (n, d) in enumerate(shapes):
        Z = synth.haar_blocks(n, d, seed + k)
        A64 = synth.measurement_matrix(Z, synth.sigma_for(c, n, d), seed + 100 + k)
        X0 = O.spectral_init(A64, d)
        probs.append({"A": device_matrix(A64, fmt), "n": n, "d": d, "X": to_dev(X0, xdtype(fmt))})
        refs.append((Z, A64, X0))
    return probs, refs


def _alone(p, iters, monkeypatch, waves):
    """The same problem through sync_solve with the batched launch's panel shape
    (on the streaming kernel, whose arithmetic the batched kernels share: not
    on the matrix cores, which sync_solve picks for F64 from d = 10)."""
    monkeypatch.setenv("NSRGS_WIDE_FROM_D", "99")
    rows = P.batch_rows_per_panel(p["d"])
    monkeypatch.setenv("NSRGS_STEP_B", str(rows // p["d"]))
    monkeypatch.setenv("NSRGS_STEP_U", "1")
    monkeypatch.setenv("NSRGS_STEP_W", str(waves))
    X = p["X0"].clone()
    ws = P.workspace(p["n"], p["d"], p["A"].fmt)
    P.solve(p["A"], p["n"], p["d"], X, ws, max_iters=iters, init=False)
    return X


def test_batch_options_are_checked_on_the_host():
    """CPU: bad schedule options are refused before any device work."""
    m = P._Matrix(P.F32, 16, None, None, 304)
    arr = (P._Problem * 1)(P._Problem(m, 100, 3, 0.0, 4096, 0, 0.0))
    for opts, msg in ((P._BatchOpts(0, 0, 0, 0, 2, 0), "persistent"),
                      (P._BatchOpts(0, 3, 0, 0, 0, 0), "order"),
                      (P._BatchOpts(0, 0, 0, 0, 1, -1), "wait_polls"),
                      (P._BatchOpts(9, 0, 0, 0, 1, 0), "waves")):
        st = P.lib().sync_solve_batched(arr, 1, 3, 10, 256, 1 << 30, None, ctypes.byref(opts), None)
        assert st == 1, msg
        assert msg in P.lib().nsrgs_last_error().decode()


@pytest.mark.gpu
@pytest.mark.parametrize("fmt", [P.F64, P.F32, P.BF16], ids=lambda f: FMT_NAME[f])
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("ticket_kb", [1, 0], ids=["panel_tickets", "merged_tickets"])
def test_persistent_matches_grouped_and_oracle(fmt, order, ticket_kb):
    """One persistent launch gives bitwise the grouped schedule's iterates (the
    same per-panel arithmetic) for every problem of a d <= 16 mix, and the
    oracle's within the format's bar; with one panel per ticket and with the
    default merging (here whole problems per ticket)."""
    require_gpu()
    iters = 30
    probs, refs = _batch(fmt, MIX, seed=20 + 10 * fmt)
    X0s = [p["X"].clone() for p in probs]
    print(f"persistent batch {FMT_NAME[fmt]} order={order} ticket_kb={ticket_kb}", flush=True)
    st, infos = P.solve_batched(probs, max_iters=iters, waves=2, order=order, persistent=True,
                                ticket_kb=ticket_kb)
    assert st == 0
    grouped = [dict(p, X=x.clone()) for p, x in zip(probs, X0s)]
    st2, infos2 = P.solve_batched(grouped, max_iters=iters, waves=2, order=order)
    assert st2 == 0
    torch.cuda.synchronize()
    for p, q, (Z, A64, X0), info, info2 in zip(probs, grouped, refs, infos, infos2):
        n, d = p["n"], p["d"]
        assert info["iters"] == iters == info2["iters"]
        assert torch.equal(p["X"], q["X"]), (n, d)
        assert info["rel_change"] == info2["rel_change"] and info["max_orth_defect"] == info2["max_orth_defect"]
        ref = O.solve(oracle_matrix(A64, fmt), d, Ts=3, T=iters, X0=X0)
        err = O.dist_F(host(p["X"]), ref.X) / math.sqrt(n)
        assert err <= (1e-10 if fmt == P.F64 else 2e-5), (n, d, err)


@pytest.mark.gpu
def test_persistent_budgets_tolerance_and_nonfinite():
    """Per-problem budgets, the relative-change stop and a non-finite problem,
    all decided on the device inside one launch."""
    require_gpu()
    probs, refs = _batch(P.F64, [(60, 3), (80, 2), (40, 4), (50, 3)], seed=7)
    X0 = [host(p["X"]) for p in probs]
    probs[0]["iters"] = 5
    probs[1]["tol"] = 1e-7
    probs[3]["A"].data[5, 40] = float("nan")
    st, infos = P.solve_batched(probs, max_iters=200, persistent=True, check=False)
    assert st == 6                                        # the non-finite problem
    assert infos[0]["iters"] == 5
    ref1 = O.solve(refs[1][1], 2, Ts=3, T=200, stop="rel_change", tol=1e-7, X0=X0[1])
    assert infos[1]["converged"] == 1
    check_stop_iteration(infos[1]["iters"], ref1, 1e-7, slack=1e-6)
    assert infos[2]["iters"] == 200
    assert infos[3]["nonfinite"] == 1 and infos[3]["iters"] == 1
    for k, T in ((0, 5), (2, 200), (1, infos[1]["iters"])):
        ref = O.solve(refs[k][1], probs[k]["d"], Ts=3, T=T, X0=X0[k])
        assert O.dist_F(host(probs[k]["X"]), ref.X) <= 1e-10


@pytest.mark.gpu
def test_persistent_wait_bound_abandons_the_launch_cleanly():
    """With a one-poll bound on every dependency wait (forced from the host),
    the launch gives up instead of waiting, returns NSRGS_ERR_DEVICE, and the
    device is usable afterwards."""
    require_gpu()
    probs, refs = _batch(P.F32, [(400, 3), (300, 3)], seed=13)
    X0s = [p["X"].clone() for p in probs]
    st, infos = P.solve_batched(probs, max_iters=50, persistent=True, wait_polls=1, check=False)
    torch.cuda.synchronize()
    assert st in (0, 4)
    if st == 4:
        assert "polls" in P.lib().nsrgs_last_error().decode()
    again = [dict(p, X=x.clone()) for p, x in zip(probs, X0s)]
    st2, infos2 = P.solve_batched(again, max_iters=50, persistent=True)
    assert st2 == 0 and all(i["iters"] == 50 for i in infos2)


def test_batch_with_too_large_d_is_refused_on_the_host():
    """CPU: d > 16 in a batch is refused before any device work."""
    m = P._Matrix(P.F32, 16, None, None, 352)
    arr = (P._Problem * 2)(P._Problem(m, 20, 17, 0.0, 4096, 0, 0.0), P._Problem(m, 100, 3, 0.0, 4096, 0, 0.0))
    st = P.lib().sync_solve_batched(arr, 2, 3, 10, 256, 1 << 30, None, None, None)
    assert st == 1
    assert "d must be in [1, 16]" in P.lib().nsrgs_last_error().decode()


@pytest.mark.gpu
@pytest.mark.parametrize("fmt", [P.F64, P.F32, P.BF16], ids=lambda f: FMT_NAME[f])
def test_grouped_d16_batch_matches_oracle(fmt, monkeypatch):
    """A batch whose largest d is 16 (the widest kernel class), every problem
    against the oracle and bitwise against its own sync_solve."""
    require_gpu()
    iters = 30
    probs, refs = _batch(fmt, MIX, seed=10 * fmt)
    for p in probs:
        p["X0"] = p["X"].clone()
    print(f"grouped d<=16 batch {FMT_NAME[fmt]}: {len(probs)} problems, {iters} iterations", flush=True)
    st, infos = P.solve_batched(probs, ns_steps=3, max_iters=iters, waves=2)
    assert st == 0
    torch.cuda.synchronize()
    for p, (Z, A64, X0), info in zip(probs, refs, infos):
        n, d = p["n"], p["d"]
        assert info["iters"] == iters
        ref = O.solve(oracle_matrix(A64, fmt), d, Ts=3, T=iters, X0=host(p["X0"]))
        err = O.dist_F(host(p["X"]), ref.X) / math.sqrt(n)
        tol = 1e-10 if fmt == P.F64 else 2e-5
        print(f"  n={n} d={d}: d_F/sqrt(n) vs oracle {err:.2e}", flush=True)
        assert err <= tol, (n, d, err)
        alone = _alone(p, iters, monkeypatch, waves=2)
        assert torch.equal(alone, p["X"]), (n, d)


@pytest.mark.gpu
@pytest.mark.parametrize("fmt", [P.F32, P.BF16, P.F64], ids=lambda f: FMT_NAME[f])
def test_grouped_matches_oracle_and_alone(fmt, monkeypatch):
    require_gpu()
    iters = 30
    probs, refs = _batch(fmt, MIX10, seed=10 * fmt)
    for p in probs:
        p["X0"] = p["X"].clone()
    print(f"grouped batch {FMT_NAME[fmt]}: {len(probs)} problems, {iters} iterations", flush=True)
    st, infos = P.solve_batched(probs, ns_steps=3, max_iters=iters, waves=2)
    assert st == 0
    torch.cuda.synchronize()
    for p, (Z, A64, X0), info in zip(probs, refs, infos):
        n, d = p["n"], p["d"]
        assert info["iters"] == iters
        ref = O.solve(oracle_matrix(A64, fmt), d, Ts=3, T=iters, X0=host(p["X0"]))
        err = O.dist_F(host(p["X"]), ref.X) / math.sqrt(n)
        tol = 1e-10 if fmt == P.F64 else 2e-5
        print(f"  n={n} d={d}: d_F/sqrt(n) vs oracle {err:.2e}", flush=True)
        assert err <= tol, (n, d, err)
        alone = _alone(p, iters, monkeypatch, waves=2)
        assert torch.equal(alone, p["X"]), (n, d)


@pytest.mark.gpu
def test_grouped_orders_and_waves_agree():
    """Unit order and workgroup shape leave every problem's result (nearly) unchanged;
    the order alone changes nothing bitwise."""
    require_gpu()
    base, _ = _batch(P.F32, MIX10, seed=3)
    X0s = [p["X"].clone() for p in base]
    P.solve_batched(base, max_iters=12, waves=1)
    for order in (0, 1):
        for waves in (1, 2, 4):
            probs = [dict(p, X=x.clone()) for p, x in zip(base, X0s)]
            st, _ = P.solve_batched(probs, max_iters=12, order=order, waves=waves)
            assert st == 0
            for p, q in zip(probs, base):
                if waves == 1:
                    assert torch.equal(p["X"], q["X"])
                else:
                    assert (p["X"] - q["X"]).abs().max().item() <= 1e-5


@pytest.mark.gpu
def test_grouped_per_problem_budgets_and_tolerance():
    require_gpu()
    probs, refs = _batch(P.F64, [(60, 3), (80, 2), (40, 4)], seed=7)
    X0 = [host(p["X"]) for p in probs]
    probs[0]["iters"] = 5                  # its own budget
    probs[1]["tol"] = 1e-7                 # stops on the relative-change rule
    st, infos = P.solve_batched(probs, max_iters=200, check_every=4)
    assert st == 0
    assert infos[0]["iters"] == 5
    ref1 = O.solve(refs[1][1], 2, Ts=3, T=200, stop="rel_change", tol=1e-7, X0=X0[1])
    assert infos[1]["converged"] == 1
    check_stop_iteration(infos[1]["iters"], ref1, 1e-7, slack=1e-6)
    assert infos[2]["iters"] == 200
    for k, T in ((0, 5), (2, 200)):
        ref = O.solve(refs[k][1], probs[k]["d"], Ts=3, T=T, X0=X0[k])
        assert O.dist_F(host(probs[k]["X"]), ref.X) <= 1e-10
    ref1x = O.solve(refs[1][1], 2, Ts=3, T=infos[1]["iters"], X0=X0[1])
    assert O.dist_F(host(probs[1]["X"]), ref1x.X) <= 1e-10


@pytest.mark.gpu
def test_grouped_nonfinite_problem_is_isolated():
    require_gpu()
    probs, refs = _batch(P.F32, [(50, 3), (64, 3)], seed=9)
    probs[0]["A"].data[5, 40] = float("nan")
    st, infos = P.solve_batched(probs, max_iters=20, check=False)
    assert st == 6
    assert infos[0]["nonfinite"] == 1 and infos[0]["iters"] == 1
    assert infos[1]["nonfinite"] == 0 and infos[1]["iters"] == 20
    assert torch.isfinite(probs[1]["X"]).all()


@pytest.mark.gpu
def test_grouped_with_spectral_init_matches_single():
    require_gpu()
    probs, refs = _batch(P.F32, [(300, 3), (120, 4)], seed=11)
    for p in probs:
        p["X"].zero_()
    st, infos = P.solve_batched(probs, max_iters=60, init=True)
    assert st == 0
    for p, (Z, A64, X0) in zip(probs, refs):
        ref = O.solve(oracle_matrix(A64, P.F32), p["d"], Ts=3, T=60)
        assert abs(O.alignment_error(host(p["X"]), Z) / O.alignment_error(ref.X, Z) - 1) <= 1e-4
