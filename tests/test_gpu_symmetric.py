"""GPU parity of sync_step_symmetric (the step from the blocks above the block
diagonal only) against the FP64 oracle's full step, through the C ABI."""
import numpy as np
import pytest
import torch

import paper_2604_07372_amd as P
import synth
from oracle import nsrgs as O

from gpu_common import (FMT_NAME, device_matrix, host, oracle_matrix, require_gpu,
                        step_tolerance, to_dev, xdtype)

pytestmark = pytest.mark.gpu

SYM_FMTS = [P.F64, P.F32, P.BF16, P.BF16_SPLIT]
# several strips and chunks with ragged ends, every d the call supports
SHAPES = [(2, 1), (2, 3), (5, 2), (37, 3), (341, 3), (700, 3), (1500, 1), (100, 4), (300, 4),
          (61, 5), (47, 7), (150, 6), (400, 8), (3, 8), (33, 10), (130, 10), (90, 12), (20, 16), (70, 16)]


def _problem(n, d, c=0.3, seed=0, eps=0.05):
    """The generator's A, made exactly symmetric by mirroring its upper
    triangle: the host twin forms Z Z^T with a library product whose last bit
    can differ between (i, j) and (j, i) (the device generator's cannot), and
    the call requires A_ji = A_ij^T exactly."""
    Z = synth.haar_blocks(n, d, seed)
    A64 = synth.measurement_matrix(Z, synth.sigma_for(c, n, d), seed + 1)
    A64 = np.triu(A64) + np.triu(A64, 1).T
    X = synth.perturbed_start(Z, eps, seed + 2)
    return Z, A64, X


def _run(Ad, n, d, Xin, fmt, ws=None):
    ws = ws or P.workspace(n, d, fmt, symmetric=True)
    Xout = torch.empty_like(Xin)
    P.step_symmetric(Ad, n, d, Xin, Xout, ws, mu=0.0, ns_steps=3)
    torch.cuda.synchronize()
    return Xout, ws


@pytest.mark.parametrize("fmt", SYM_FMTS, ids=lambda f: FMT_NAME[f])
@pytest.mark.parametrize("n,d", SHAPES)
def test_symmetric_step_parity(n, d, fmt):
    require_gpu()
    print(f"symmetric step parity n={n} d={d} fmt={FMT_NAME[fmt]}", flush=True)
    if fmt in (P.BF16, P.BF16_SPLIT) and d > 12:
        # refused: the 2-byte tiles spill above d = 12 and lose to sync_step
        assert P.symmetric_workspace_bytes(n, d, fmt) == 0
        return
    Z, A64, X = _problem(n, d, seed=1000 * n + d)
    assert np.array_equal(A64, A64.T)
    Ad = device_matrix(A64, fmt)
    As = oracle_matrix(A64, fmt)
    Xin = to_dev(X, xdtype(fmt))
    Xh = host(Xin)
    Xout, ws = _run(Ad, n, d, Xin, fmt)
    ref = O.rgs_step(As, Xh, d, mu=1.0 / n, Ts=3)
    err = np.abs(host(Xout) - ref.X).max()
    tol = step_tolerance(As, Xh, n, fmt)
    assert err <= tol, (err, tol)
    info = P.read_info(ws)
    assert abs(info["rel_change"] - ref.rel_change) <= 1e-3 * ref.rel_change + 1e-6
    assert abs(info["max_orth_defect"] - ref.max_orth_defect) <= 1e-3 * ref.max_orth_defect + 1e-5
    assert info["nonfinite"] == 0


@pytest.mark.parametrize("W", [1, 2, 4, 8])
@pytest.mark.parametrize("H", [24, 96, 384, 1536])
def test_symmetric_tile_shapes_agree(W, H, monkeypatch):
    """Every strip height and chunk width gives the oracle's step (the strip
    height is rounded to a multiple of the panel and epilogue rows)."""
    require_gpu()
    n, d = 900, 3
    print(f"symmetric tile shape W={W} H={H}", flush=True)
    monkeypatch.setenv("NSRGS_SYM_W", str(W))
    monkeypatch.setenv("NSRGS_SYM_H", str(H))
    Z, A64, X = _problem(n, d, seed=77)
    Ad = device_matrix(A64, P.F32)
    Xin = to_dev(X, torch.float32)
    Xout, _ = _run(Ad, n, d, Xin, P.F32)
    As = oracle_matrix(A64, P.F32)
    ref = O.rgs_step(As, host(Xin), d, mu=1.0 / n, Ts=3)
    assert np.abs(host(Xout) - ref.X).max() <= step_tolerance(As, host(Xin), n, P.F32)


@pytest.mark.parametrize("d", [1, 3, 5, 8, 16])
def test_values_on_and_below_the_block_diagonal_are_never_used(d):
    """NaN in every block on or below the block diagonal, and in the padding
    columns, must not reach the result."""
    require_gpu()
    n = 211
    nd = n * d
    Z, A64, X = _problem(n, d, seed=31 + d)
    Ad = device_matrix(A64, P.F32)
    blk = np.arange(nd) // d
    lower = torch.from_numpy(blk[:, None] >= blk[None, :]).cuda()
    Ad.data[:, :nd][lower] = float("nan")
    Ad.data[:, nd:] = float("nan")
    Xin = to_dev(X, torch.float32)
    Xout, ws = _run(Ad, n, d, Xin, P.F32)
    As = oracle_matrix(A64, P.F32)
    ref = O.rgs_step(As, host(Xin), d, mu=1.0 / n, Ts=3)
    assert np.isfinite(host(Xout)).all()
    assert np.abs(host(Xout) - ref.X).max() <= step_tolerance(As, host(Xin), n, P.F32)
    assert P.read_info(ws)["nonfinite"] == 0


def test_symmetric_step_deterministic_and_close_to_sync_step():
    """Bitwise repeatable; agrees with sync_step to the accumulation rounding."""
    require_gpu()
    n, d = 1200, 3
    Z, A64, X = _problem(n, d, seed=5)
    Ad = device_matrix(A64, P.F32)
    Xin = to_dev(X, torch.float32)
    out1, ws = _run(Ad, n, d, Xin, P.F32)
    out2, _ = _run(Ad, n, d, Xin, P.F32, ws)
    dense = torch.empty_like(Xin)
    P.step(Ad, n, d, Xin, dense, ws)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2)
    As = oracle_matrix(A64, P.F32)
    assert np.abs(host(out1) - host(dense)).max() <= 2 * step_tolerance(As, host(Xin), n, P.F32)


def test_symmetric_step_iterates_like_the_oracle():
    """Twenty iterations from a start near the ground truth (where the
    iteration converges) stay on the oracle's trajectory."""
    require_gpu()
    n, d, T = 500, 4, 20
    Z, A64, X0 = _problem(n, d, seed=9, eps=0.05)
    Ad = device_matrix(A64, P.F32)
    As = oracle_matrix(A64, P.F32)
    Xa = to_dev(X0, torch.float32)
    Xb = torch.empty_like(Xa)
    ws = P.workspace(n, d, P.F32, symmetric=True)
    for _ in range(T):
        P.step_symmetric(Ad, n, d, Xa, Xb, ws)
        Xa, Xb = Xb, Xa
    torch.cuda.synchronize()
    Xr = X0.copy()
    for _ in range(T):
        Xr = O.rgs_step(As, Xr, d, mu=1.0 / n, Ts=3).X
    dF = np.linalg.norm(host(Xa) - Xr) / np.sqrt(n)
    assert dF <= 1e-5, dF


@pytest.mark.parametrize("d,R,U", [(3, 12, 1), (3, 16, 1), (3, 12, 2), (3, 6, 2), (4, 12, 1), (4, 8, 2),
                                   (4, 16, 1)])
@pytest.mark.parametrize("fmt", [P.F32, P.BF16], ids=lambda f: FMT_NAME[f])
def test_symmetric_compiled_panel_shapes(d, R, U, fmt, monkeypatch):
    """Every compiled panel shape (R rows, U vectors per lane per row; chosen
    by NSRGS_SYM_R / NSRGS_SYM_U) gives the oracle's step."""
    require_gpu()
    n = 613
    print(f"symmetric panel shape d={d} R={R} U={U} fmt={FMT_NAME[fmt]}", flush=True)
    monkeypatch.setenv("NSRGS_SYM_R", str(R))
    monkeypatch.setenv("NSRGS_SYM_U", str(U))
    Z, A64, X = _problem(n, d, seed=400 + R + U)
    Ad = device_matrix(A64, fmt)
    As = oracle_matrix(A64, fmt)
    Xin = to_dev(X, torch.float32)
    Xout, _ = _run(Ad, n, d, Xin, fmt)
    ref = O.rgs_step(As, host(Xin), d, mu=1.0 / n, Ts=3)
    assert np.abs(host(Xout) - ref.X).max() <= step_tolerance(As, host(Xin), n, fmt)


@pytest.mark.parametrize("form", ["f32", "bf16+refine", "tol"])
def test_symmetric_solve_matches_full_stream_solve(form):
    """sync_solve with every iteration on the symmetric half-stream lands on the
    full-stream solve's result (same spectral initialization, iterations
    equal up to rounding), for a fixed budget, the BF16 form with FP32
    refinement, and a tolerance stop."""
    require_gpu()
    n, d = 2000, 3
    print(f"symmetric solve {form}", flush=True)
    Z = synth.haar_blocks(n, d, 21)
    A32 = P.generate(torch.from_numpy(Z).cuda(), synth.sigma_for(0.2, n, d), 22, fmt=P.F32)
    Af = P.stored(A32, P.F32)
    Am = P.convert(A32, P.BF16) if form == "bf16+refine" else Af
    kw = dict(refine_iters=10, A_refine=Af) if form == "bf16+refine" else {}
    tol, iters = (1e-6, 300) if form == "tol" else (0.0, 200)
    out = {}
    for sym in (False, True):
        ws = P.workspace(n, d, Am.fmt, symmetric=sym)
        X = torch.empty((n * d, d), dtype=torch.float32, device="cuda")
        info = P.solve(Am, n, d, X, ws, max_iters=iters, tol=tol, symmetric=sym, **kw)
        out[sym] = (host(X), info)
    Xf, inf_f = out[False]
    Xs, inf_s = out[True]
    dF = O.dist_F(Xs, Xf) / np.sqrt(n)
    ef, es = O.alignment_error(Xf, Z), O.alignment_error(Xs, Z)
    print(f"  d_F/sqrt(n) {dF:.2e}, align err {ef:.9f} vs {es:.9f}, iters {inf_f['iters']} vs {inf_s['iters']}",
          flush=True)
    assert dF <= 1e-5
    assert abs(es - ef) <= 1e-6 * ef
    if form == "tol":
        assert inf_s["converged"] == 1 and abs(inf_s["iters"] - inf_f["iters"]) <= 2
    else:
        assert inf_s["iters"] == inf_f["iters"] == iters
