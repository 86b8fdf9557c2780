"""GPU test of sync_step_noalloc (sync_step without a caller workspace): called
through the C ABI, it gives bitwise sync_step's X_out on two calls in a row,
the second on a smaller problem, and refuses a problem beyond its scratch."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2604_07372_amd as P
import synth

from gpu_common import device_matrix, require_gpu, to_dev, xdtype

pytestmark = pytest.mark.gpu


def _case(n, d, seed, fmt):
    Z = synth.haar_blocks(n, d, seed)
    A64 = synth.measurement_matrix(Z, synth.sigma_for(0.2, n, d), seed + 1)
    X = synth.perturbed_start(Z, 0.05, seed + 2)
    return device_matrix(A64, fmt), to_dev(X, xdtype(fmt))


def _noalloc(A, n, d, Xin, Xout, mu=0.0, ns_steps=3):
    m = A.c()
    return P.lib().sync_step_noalloc(ctypes.byref(m), n, d, float(mu), int(ns_steps), Xin.data_ptr(),
                                     Xout.data_ptr(), torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("fmt", [P.F64, P.F32, P.BF16])
def test_noalloc_step_equals_sync_step_twice(fmt):
    require_gpu()
    for (n, d, seed) in ((700, 3, 11), (130, 5, 12)):          # second call: smaller problem
        print(f"noalloc fmt={fmt} n={n} d={d}", flush=True)
        A, Xin = _case(n, d, seed, fmt)
        X_ref = torch.full_like(Xin, float("nan"))
        X_new = torch.full_like(Xin, float("nan"))
        ws = P.workspace(n, d, fmt)
        P.step(A, n, d, Xin, X_ref, ws)
        assert _noalloc(A, n, d, Xin, X_new) == 0, P.lib().nsrgs_last_error().decode()
        torch.cuda.synchronize()
        assert torch.isfinite(X_new).all()
        assert torch.equal(X_new, X_ref), (n, d)


def test_noalloc_refuses_beyond_scratch_and_bad_args():
    require_gpu()
    n, d = 40, 3
    A, Xin = _case(n, d, 13, P.F32)
    Xout = torch.empty_like(Xin)
    # aliasing and ns_steps are checked as for sync_step
    assert _noalloc(A, n, d, Xin, Xin) == 1
    assert _noalloc(A, n, d, Xin, Xout, ns_steps=65) == 1
    # 1.1 million blocks of d = 1 (8-row panels) need more panel records than
    # the scratch holds: refused on the host before any device work (A is never
    # read; the iterates are real buffers of the stated size)
    big_n = 1_100_000
    Xa = torch.zeros(big_n, 1, dtype=torch.float32, device="cuda")
    Xb = torch.zeros_like(Xa)
    m = P._Matrix(P.F32, A.data.data_ptr(), None, None, (big_n + 15) // 16 * 16)
    st = P.lib().sync_step_noalloc(ctypes.byref(m), big_n, 1, 0.0, 3, Xa.data_ptr(), Xb.data_ptr(),
                                   torch.cuda.current_stream().cuda_stream)
    assert st == 3
    assert "scratch" in P.lib().nsrgs_last_error().decode()
    # the array keeps working after a refusal
    X_ref = torch.empty_like(Xin)
    P.step(A, n, d, Xin, X_ref, P.workspace(n, d, P.F32))
    assert _noalloc(A, n, d, Xin, Xout) == 0
    torch.cuda.synchronize()
    assert torch.equal(Xout, X_ref)
