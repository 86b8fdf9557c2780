"""GPU parity of the incomplete observation model (Sec. 4.1) on block-sparse
storage: the generator against its host twin, and sync_step_bsr against the
FP64 oracle's step on the dense masked A with mu = 1/(np)."""
import math

import numpy as np
import pytest
import torch

import paper_2604_07372_amd as P
import synth
from oracle import nsrgs as O

from gpu_common import FMT_NAME, host, oracle_matrix, require_gpu, step_tolerance, to_dev

pytestmark = pytest.mark.gpu


def _masked(n, d, c, seed, p):
    """Noise sigma = c sqrt(p) sqrt(n/d): a block row then sees about the same
    noise-to-signal ratio c at every p (signal ~ n p, noise ~ sigma sqrt(n p d))."""
    Z = synth.haar_blocks(n, d, seed)
    sigma = synth.sigma_for(c * math.sqrt(p), n, d) if p > 0 else synth.sigma_for(c, n, d)
    A64 = synth.measurement_matrix(Z, sigma, seed + 1, p=p)
    return Z, sigma, A64


def _orthogonal_start(Z, eps, seed):
    """Perturbed ground truth with each block replaced by its polar factor.  The
    masked model's step 1/(np) multiplies the orthogonality defect of a start by
    about 1/p (through the (n - 1) X_i term), so, as in the paper, the start
    lies on O(d)^n."""
    X = synth.perturbed_start(Z, eps, seed)
    d = X.shape[1]
    out = np.empty_like(X)
    for i in range(X.shape[0] // d):
        U, _, Vt = np.linalg.svd(X[i * d:(i + 1) * d])
        out[i * d:(i + 1) * d] = U @ Vt
    return out


def _entry_off(k, e, m, d2):
    """Offset of entry e of a row's k-th block from the row's first value: groups
    of 64 blocks, each entry-major over its w = min(64, m - 64 g) blocks."""
    g0 = (k // 64) * 64
    return g0 * d2 + e * min(64, m - g0) + k % 64


def _dense_from_bsr(B: P.BsrMatrix, n, d):
    """Expand the device arrays on the host (test-side reading of the layout)."""
    rp = B.row_ptr.cpu().numpy()
    ci = B.col_idx.cpu().numpy()
    if B.fmt == P.F32:
        vals = B.values.cpu().numpy().astype(np.float64)
    else:
        bits = B.values.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        vals = bits.view(np.float32).astype(np.float64)
    A = np.zeros((n * d, n * d))
    for i in range(n):
        m = rp[i + 1] - rp[i]
        for k in range(m):
            j = ci[rp[i] + k]
            blk = np.array([vals[rp[i] * d * d + _entry_off(k, e, m, d * d)] for e in range(d * d)]).reshape(d, d)
            A[i * d:(i + 1) * d, j * d:(j + 1) * d] = blk
    return A, rp, ci


@pytest.mark.parametrize("p", [0.0, 0.3, 0.5, 1.0])
@pytest.mark.parametrize("d", [1, 3, 5])
def test_bsr_generator_matches_host_twin_and_dense_generator(d, p):
    require_gpu()
    n, seed = 60, 300 + d
    print(f"bsr generator n={n} d={d} p={p}", flush=True)
    Z, sigma, A64 = _masked(n, d, 0.3, seed, p)
    Zd = torch.from_numpy(Z).cuda()
    B = P.generate_bsr(Zd, sigma, seed + 1, p, fmt=P.F32)
    A, rp, ci = _dense_from_bsr(B, n, d)
    blk = np.arange(n * d) // d
    off = blk[:, None] != blk[None, :]
    # the observation pattern is the host twin's, block for block
    obs_host = (np.abs(A64) > 0).reshape(n, d, n, d).any(axis=(1, 3)) & ~np.eye(n, dtype=bool)
    obs_dev = np.zeros((n, n), dtype=bool)
    for i in range(n):
        cols = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0) and not np.any(cols == i)
        obs_dev[i, cols] = True
    assert np.array_equal(obs_dev, obs_host)
    assert B.nnzb == int(obs_host.sum())
    # elements: FP32 rounding of the host twin's FP64 values (the twin's Z Z^T may differ in its last bit)
    ref = np.where(off, A64, 0.0)
    assert np.allclose(A, ref.astype(np.float32).astype(np.float64), rtol=2 ** -22, atol=1e-12)
    # and bitwise the dense device generator's off-diagonal blocks (which takes p in (0, 1])
    if p == 0.0:
        return
    Ad = P.generate(Zd, sigma, seed + 1, fmt=P.F32, p=p)
    dense = Ad[:, :n * d].cpu().numpy().astype(np.float64)
    assert np.array_equal(A, np.where(off, dense, 0.0))


# d <= 6 has two kernels: "sliced" (X of a column slice in LDS; with
# slice_w, slices of that many blocks, so that small n has several) and
# "fused" (one wave per block row, X through the caches); d = 7, 8 run the
# fused one and d > 8 the matrix-core epilogue.
BSR_SHAPES = [(2, 1), (37, 3), (300, 3), (130, 4), (61, 5), (40, 8), (700, 2), (23, 9), (31, 16), (40, 25), (9, 32)]
BSR_PATHS = ([(n, d, path) for n, d in BSR_SHAPES if d <= 6 for path in ("sliced", "fused", "slice_w")]
             + [(n, d, "fused") for n, d in BSR_SHAPES if 6 < d <= 8]
             + [(n, d, "wide") for n, d in BSR_SHAPES if d > 8] + [(1500, 4, "sliced"), (700, 6, "sliced")])


def _bsr_path(path, monkeypatch):
    monkeypatch.setenv("NSRGS_BSR_SLICED", "0" if path == "fused" else "1")
    if path == "slice_w":
        monkeypatch.setenv("NSRGS_BSR_SLICE_W", "7")


@pytest.mark.parametrize("fmt", [P.F32, P.BF16], ids=lambda f: FMT_NAME[f])
@pytest.mark.parametrize("p", [0.05, 0.5, 0.8, 1.0])
@pytest.mark.parametrize("n,d,path", BSR_PATHS)
def test_bsr_step_parity(n, d, path, p, fmt, monkeypatch):
    require_gpu()
    _bsr_path(path, monkeypatch)
    seed = 7000 + 31 * n + d
    print(f"bsr step parity n={n} d={d} {path} p={p} fmt={FMT_NAME[fmt]}", flush=True)
    Z, sigma, A64 = _masked(n, d, 0.3, seed, p)
    B = P.generate_bsr(torch.from_numpy(Z).cuda(), sigma, seed + 1, p, fmt=fmt)
    X = _orthogonal_start(Z, 0.05, seed + 2)
    Xin = to_dev(X, torch.float32)
    Xout = torch.empty_like(Xin)
    ws = P.workspace(n, d, P.F32, bsr=True)
    mu = 1.0 / (n * p) if n * p >= 2 else 1.0 / n     # the paper's 1/(np) where it is a sensible step
    P.step_bsr(B, n, d, Xin, Xout, ws, mu=mu)
    torch.cuda.synchronize()
    As = oracle_matrix(A64, fmt)
    ref = O.rgs_step(As, host(Xin), d, mu=mu, Ts=3)
    err = np.abs(host(Xout) - ref.X).max()
    # a BF16 element can round the other way when the host twin's last FP64 bit differs
    tol = step_tolerance(As, host(Xin), n, fmt) * (4.0 if fmt == P.BF16 else 1.0)
    assert err <= tol, (err, tol)
    info = P.read_info(ws)
    assert abs(info["rel_change"] - ref.rel_change) <= 1e-3 * ref.rel_change + 1e-6
    assert info["nonfinite"] == 0


@pytest.mark.parametrize("path", ["sliced", "fused", "slice_w"])
def test_bsr_step_equals_dense_step_on_the_masked_matrix(path, monkeypatch):
    """The block-sparse step and sync_step on the dense masked A of the same
    generator agree to the accumulation rounding; the step is bitwise
    repeatable."""
    require_gpu()
    _bsr_path(path, monkeypatch)
    n, d, p = 900, 3, 0.5
    Z, sigma, A64 = _masked(n, d, 0.3, 11, p)
    Zd = torch.from_numpy(Z).cuda()
    B = P.generate_bsr(Zd, sigma, 12, p)
    Ad = P.stored(P.generate(Zd, sigma, 12, fmt=P.F32, p=p), P.F32)
    Xin = to_dev(_orthogonal_start(Z, 0.05, 13), torch.float32)
    out_b, out_d = torch.empty_like(Xin), torch.empty_like(Xin)
    ws = P.workspace(n, d, P.F32, bsr=True)
    mu = 1.0 / (n * p)
    P.step_bsr(B, n, d, Xin, out_b, ws, mu=mu)
    P.step(Ad, n, d, Xin, out_d, ws, mu=mu)
    out_b2 = torch.empty_like(Xin)
    P.step_bsr(B, n, d, Xin, out_b2, ws, mu=mu)
    torch.cuda.synchronize()
    assert torch.equal(out_b, out_b2)
    As = oracle_matrix(A64, P.F32)
    assert np.abs(host(out_b) - host(out_d)).max() <= 2 * step_tolerance(As, host(Xin), n, P.F32)


@pytest.mark.parametrize("path", ["sliced", "fused", "slice_w"])
def test_bsr_stored_diagonal_and_out_of_range_blocks_count_nothing(path, monkeypatch):
    """A hand-built block-sparse matrix with a NaN diagonal block and a NaN
    block at an out-of-range column gives the oracle's step without them."""
    require_gpu()
    _bsr_path(path, monkeypatch)
    n, d = 6, 2
    rng = np.random.default_rng(3)
    pairs = [(0, 1), (0, 4), (1, 3), (2, 5), (3, 4)]
    A = np.zeros((n * d, n * d))
    for i, j in pairs:
        b = rng.standard_normal((d, d))
        A[i * d:(i + 1) * d, j * d:(j + 1) * d] = b
        A[j * d:(j + 1) * d, i * d:(i + 1) * d] = b.T
    rows = []
    for i in range(n):
        cols = [j for j in range(n) if np.any(A[i * d:(i + 1) * d, j * d:(j + 1) * d])]
        extra = [i] if i % 2 == 0 else []          # stored diagonal blocks
        bad = [n + 3] if i == 1 else []             # an index outside [0, n)
        rows.append(sorted(cols + extra) + bad)
    rp = np.zeros(n + 1, dtype=np.int64)
    for i, cols in enumerate(rows):
        rp[i + 1] = rp[i] + len(cols)
    ci = np.concatenate([np.array(c, dtype=np.int32) for c in rows])
    vals = np.zeros(rp[-1] * d * d, dtype=np.float32)
    for i, cols in enumerate(rows):
        m = len(cols)
        for k, j in enumerate(cols):
            blk = (np.full((d, d), np.nan) if (j == i or j >= n)
                   else A[i * d:(i + 1) * d, j * d:(j + 1) * d])
            for e in range(d * d):
                vals[rp[i] * d * d + _entry_off(k, e, m, d * d)] = blk.flat[e]
    B = P.BsrMatrix(P.F32, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), torch.from_numpy(vals).cuda(),
                    n, d, int(rp[-1]))
    Z = synth.haar_blocks(n, d, 5)
    Xin = to_dev(synth.perturbed_start(Z, 0.05, 6), torch.float32)
    Xout = torch.empty_like(Xin)
    ws = P.workspace(n, d, P.F32, bsr=True)
    P.step_bsr(B, n, d, Xin, Xout, ws, mu=0.3)
    torch.cuda.synchronize()
    ref = O.rgs_step(A.astype(np.float32).astype(np.float64), host(Xin), d, mu=0.3, Ts=3)
    assert np.isfinite(host(Xout)).all()
    assert np.abs(host(Xout) - ref.X).max() <= 1e-5


@pytest.mark.parametrize("method", ["ns_rgs", "polar"])
def test_bsr_solve_matches_oracle(method):
    """sync_solve_bsr at d = 25 from the oracle's spectral start: 25 iterations
    of the incomplete observation model (p = 0.5, mu = 1/(np)) against the oracle
    on the dense masked matrix of the stored FP32 values."""
    require_gpu()
    n, d, p = 64, 25, 0.5
    Z, sigma, A64 = _masked(n, d, 0.1, 4242, p)
    B = P.generate_bsr(torch.from_numpy(Z).cuda(), sigma, 4243, p, fmt=P.F32)
    As = oracle_matrix(A64, P.F32)
    X0 = O.spectral_init(As, d)
    X = to_dev(X0, torch.float32)
    ws = P.workspace(n, d, P.F32)
    mu = 1.0 / (n * p)
    info = P.solve_bsr(B, n, d, X, ws, mu=mu, ns_steps=3, max_iters=25, init=False, method=method)
    ref = O.solve(As, d, mu=mu, Ts=3, T=25, X0=host(to_dev(X0, torch.float32)),
                  retraction="polar" if method == "polar" else "ns")
    e_g, e_o = O.alignment_error(host(X), Z), O.alignment_error(ref.X, Z)
    dist = O.dist_F(host(X), ref.X) / math.sqrt(n)
    print(f"bsr solve {method}: iters {info['iters']} e {e_g:.8f} vs {e_o:.8f} d_F/sqrt(n) {dist:.2e}", flush=True)
    assert info["iters"] == 25 and info["status"] == 0
    assert abs(e_g - e_o) <= 1e-4 * e_o
    assert dist <= 1e-4 * e_o


def test_bsr_spectral_init_matches_eigh():
    """The initialization with the block-sparse product: the diagonal blocks are
    not stored, so it takes the top-d subspace of A without them, which for the
    paper's model (A_ii = I) is that of A."""
    require_gpu()
    n, d, p = 80, 25, 0.8
    Z, sigma, A64 = _masked(n, d, 0.1, 515, p)
    B = P.generate_bsr(torch.from_numpy(Z).cuda(), sigma, 516, p, fmt=P.F32)
    As = oracle_matrix(A64, P.F32)
    blk = np.arange(n * d) // d
    As_off = np.where(blk[:, None] == blk[None, :], 0.0, As)
    X0_ref = O.spectral_init(As_off, d)
    X = torch.empty((n * d, d), dtype=torch.float32, device="cuda")
    ws = P.workspace(n, d, P.F32)
    info = P.solve_bsr(B, n, d, X, ws, mu=1.0 / (n * p), max_iters=0, init=True, init_iters=200)
    dist = O.dist_F(host(X), X0_ref) / math.sqrt(n)
    print(f"bsr init: residual {info['init_residual']:.2e} d_F/sqrt(n) {dist:.2e}", flush=True)
    assert dist <= 1e-4


def test_bsr_solve_refuses_gpm_on_the_host():
    require_gpu()
    n, d = 10, 3
    Z, sigma, A64 = _masked(n, d, 0.1, 17, 0.5)
    B = P.generate_bsr(torch.from_numpy(Z).cuda(), sigma, 18, 0.5, fmt=P.F32)
    X = torch.zeros((n * d, d), dtype=torch.float32, device="cuda")
    info = P.solve_bsr(B, n, d, X, P.workspace(n, d, P.F32), method="gpm", check=False)
    assert info["status"] == 2


@pytest.mark.parametrize("p", [0.8, 0.5])
def test_table1_masked_rows_on_block_sparse_storage(golden_dir, p):
    """Table 1 (Sec. 4.1), rows p = 0.8 and 0.5, NS-RGS, on block-sparse FP32
    storage: n = 500, d = 25, W_ii = 0 (the diagonal blocks are not stored),
    spectral initialization with the block-sparse product, one Newton-Schulz
    step, mu = 1/(np), stop at R^t < 1e-8 or 100 iterations.  One trial per
    cell against the paper's mean of 10 (2%)."""
    import os
    require_gpu()
    want = {(r[0], r[1]): r[2] for r in np.loadtxt(os.path.join(golden_dir, "table1_masked_relerr.txt"))}
    n, d = 500, 25
    Z = synth.haar_blocks(n, d, 80 + int(10 * p))
    Zd = torch.from_numpy(Z).cuda()
    for sigma in (0.02, 0.1, 0.2):
        B = P.generate_bsr(Zd, sigma, 990 + int(100 * p), p, fmt=P.F32)
        X = torch.empty((n * d, d), dtype=torch.float32, device="cuda")
        ws = P.workspace(n, d, P.F32)
        info = P.solve_bsr(B, n, d, X, ws, mu=1.0 / (n * p), ns_steps=1, max_iters=100, tol=1e-8,
                           init=True, init_iters=300, stop="objective", check=False)
        got = O.rel_err(host(X), Z, form="gram")
        print(f"Table 1 block-sparse p={p} sigma={sigma}: nnzb {B.nnzb} iters {info['iters']} "
              f"Rel.Err {got:.4e} (paper {want[(p, sigma)]:.2e})", flush=True)
        assert info["status"] in (0, 5) and info["nonfinite"] == 0
        assert abs(got / want[(p, sigma)] - 1.0) <= 0.02
        del B, ws
    torch.cuda.empty_cache()


def _bsr_from_rows(A, rows, n, d):
    """Block-sparse FP32 device arrays holding the blocks of A at the given
    (ascending) block columns of each block row, in the grouped value layout."""
    rp = np.zeros(n + 1, dtype=np.int64)
    for i, cols in enumerate(rows):
        rp[i + 1] = rp[i] + len(cols)
    ci = np.concatenate([np.asarray(c, dtype=np.int32) for c in rows] + [np.zeros(0, dtype=np.int32)])
    vals = np.zeros(max(1, int(rp[-1])) * d * d, dtype=np.float32)
    for i, cols in enumerate(rows):
        m = len(cols)
        for k, j in enumerate(cols):
            blk = A[i * d:(i + 1) * d, j * d:(j + 1) * d]
            for e in range(d * d):
                vals[rp[i] * d * d + _entry_off(k, e, m, d * d)] = blk.flat[e]
    return P.BsrMatrix(P.F32, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), torch.from_numpy(vals).cuda(),
                       n, d, int(rp[-1]))


@pytest.mark.parametrize("slice_w", [0, 7, 50])
def test_bsr_sliced_step_on_uneven_rows(slice_w, monkeypatch):
    """Rows whose stored blocks crowd the first or the last tenth of the
    columns, rows of one block, empty rows and nearly full rows: the slice
    bounds (a guess from an even spread of the row's blocks, a gallop away from
    it, a bisection) cut every row where a search of the whole row would, so
    the sliced step is the oracle's step on the dense masked matrix."""
    require_gpu()
    monkeypatch.setenv("NSRGS_BSR_SLICED", "1")
    if slice_w:
        monkeypatch.setenv("NSRGS_BSR_SLICE_W", str(slice_w))
    n, d = 400, 3
    rng = np.random.default_rng(77 + slice_w)
    rows = []
    for i in range(n):
        kind = i % 5
        if kind == 0:
            cols = rng.choice(n // 10, size=int(rng.integers(1, n // 10)), replace=False)
        elif kind == 1:
            cols = n - 1 - rng.choice(n // 10, size=int(rng.integers(1, n // 10)), replace=False)
        elif kind == 2:
            cols = [int(rng.integers(n))]
        elif kind == 3:
            cols = []
        else:
            cols = np.nonzero(rng.random(n) < 0.9)[0]
        rows.append(sorted(set(int(c) for c in cols) - {i}))
    Z = synth.haar_blocks(n, d, 78)
    A64 = synth.measurement_matrix(Z, synth.sigma_for(0.3, n, d), 79)
    mask = np.zeros((n, n), dtype=bool)
    for i, cols in enumerate(rows):
        mask[i, cols] = True
    A = np.where(np.kron(mask, np.ones((d, d), dtype=bool)), A64, 0.0)
    B = _bsr_from_rows(A, rows, n, d)
    Xin = to_dev(_orthogonal_start(Z, 0.05, 80), torch.float32)
    Xout = torch.empty_like(Xin)
    ws = P.workspace(n, d, P.F32, bsr=True)
    P.step_bsr(B, n, d, Xin, Xout, ws, mu=1.0 / n)
    torch.cuda.synchronize()
    As = oracle_matrix(A, P.F32)
    ref = O.rgs_step(As, host(Xin), d, mu=1.0 / n, Ts=3)
    err = np.abs(host(Xout) - ref.X).max()
    tol = step_tolerance(As, host(Xin), n, P.F32)
    print(f"uneven rows slice_w={slice_w}: err {err:.2e} tol {tol:.2e}", flush=True)
    assert err <= tol


@pytest.mark.parametrize("fmt", [P.F32, P.BF16], ids=lambda f: FMT_NAME[f])
@pytest.mark.parametrize("method", ["ns_rgs", "polar"])
@pytest.mark.parametrize("d", [3, 5])
def test_bsr_solve_small_d_on_the_sliced_product(d, method, fmt, monkeypatch):
    """sync_solve_bsr for d <= 6 with the larger workspace runs every product on
    the sliced kernel: 25 iterations from the oracle's spectral start against
    the oracle on the dense masked matrix of the stored values (FP32 or BF16),
    and against the same solve on the chunked product (equal up to the order of
    additions)."""
    require_gpu()
    n, p = 300, 0.5
    print(f"bsr solve sliced d={d} {method} {FMT_NAME[fmt]}", flush=True)
    Z, sigma, A64 = _masked(n, d, 0.2, 600 + d, p)
    B = P.generate_bsr(torch.from_numpy(Z).cuda(), sigma, 601 + d, p, fmt=fmt)
    As = oracle_matrix(A64, fmt)
    X0 = host(to_dev(O.spectral_init(As, d), torch.float32))
    mu = 1.0 / (n * p)
    out = {}
    for path in ("sliced", "chunked"):
        monkeypatch.setenv("NSRGS_BSR_SLICED", "1" if path == "sliced" else "0")
        X = to_dev(X0, torch.float32)
        info = P.solve_bsr(B, n, d, X, P.workspace(n, d, P.F32, bsr=True), mu=mu, ns_steps=3, max_iters=25,
                           init=False, method=method)
        assert info["iters"] == 25 and info["status"] == 0
        out[path] = host(X)
    ref = O.solve(As, d, mu=mu, Ts=3, T=25, X0=X0, retraction="polar" if method == "polar" else "ns")
    e_g, e_o = O.alignment_error(out["sliced"], Z), O.alignment_error(ref.X, Z)
    dist = O.dist_F(out["sliced"], ref.X) / math.sqrt(n)
    print(f"  e {e_g:.8f} vs {e_o:.8f} d_F/sqrt(n) {dist:.2e}", flush=True)
    assert abs(e_g - e_o) <= 1e-4 * e_o
    assert dist <= 1e-4 * e_o
    assert O.dist_F(out["sliced"], out["chunked"]) / math.sqrt(n) <= 1e-5


@pytest.mark.parametrize("d", [3, 6])
def test_bsr_spectral_init_small_d_on_the_sliced_product(d, monkeypatch):
    """The initialization's products on the sliced kernel: the top-d subspace
    of A without its diagonal blocks, as eigh finds it."""
    require_gpu()
    monkeypatch.setenv("NSRGS_BSR_SLICED", "1")
    n, p = 400, 0.8
    Z, sigma, A64 = _masked(n, d, 0.1, 700 + d, p)
    B = P.generate_bsr(torch.from_numpy(Z).cuda(), sigma, 701 + d, p, fmt=P.F32)
    As = oracle_matrix(A64, P.F32)
    blk = np.arange(n * d) // d
    X0_ref = O.spectral_init(np.where(blk[:, None] == blk[None, :], 0.0, As), d)
    X = torch.empty((n * d, d), dtype=torch.float32, device="cuda")
    info = P.solve_bsr(B, n, d, X, P.workspace(n, d, P.F32, bsr=True), mu=1.0 / (n * p), max_iters=0, init=True,
                       init_iters=200)
    dist = O.dist_F(host(X), X0_ref) / math.sqrt(n)
    print(f"bsr init sliced d={d}: residual {info['init_residual']:.2e} d_F/sqrt(n) {dist:.2e}", flush=True)
    assert dist <= 1e-4


def test_bsr_sliced_solve_is_the_sliced_step_repeated(monkeypatch):
    """With the larger workspace, NS-RGS iterations of sync_solve_bsr (d <= 6,
    relative-change rule) are sync_step_bsr's sliced steps on bounds found once:
    bitwise the same iterates, and the stop rule fires at the step whose
    relative change first reaches the tolerance."""
    require_gpu()
    monkeypatch.setenv("NSRGS_BSR_SLICED", "1")
    n, d, p = 500, 3, 0.5
    Z, sigma, A64 = _masked(n, d, 0.2, 909, p)
    B = P.generate_bsr(torch.from_numpy(Z).cuda(), sigma, 910, p, fmt=P.F32)
    X0 = to_dev(_orthogonal_start(Z, 0.05, 911), torch.float32)
    mu = 1.0 / (n * p)
    X = X0.clone()
    info = P.solve_bsr(B, n, d, X, P.workspace(n, d, P.F32, bsr=True), mu=mu, max_iters=12, init=False)
    assert info["iters"] == 12 and info["status"] == 0
    ws = P.workspace(n, d, P.F32, bsr=True)
    Xa, Xb = X0.clone(), torch.empty_like(X0)
    rel = []
    for _ in range(60):
        P.step_bsr(B, n, d, Xa, Xb, ws, mu=mu)
        Xa, Xb = Xb, Xa
        rel.append(P.read_info(ws)["rel_change"])
        if len(rel) == 12:
            assert torch.equal(X, Xa)
    tol = 1e-5
    want = next(k + 1 for k, r in enumerate(rel) if r <= tol)
    X = X0.clone()
    info = P.solve_bsr(B, n, d, X, P.workspace(n, d, P.F32, bsr=True), mu=mu, max_iters=60, tol=tol, init=False,
                       check_every=4)
    print(f"sliced solve stop: iters {info['iters']} (stepping: {want}), rel {info['rel_change']:.2e}", flush=True)
    assert info["converged"] == 1 and info["iters"] == want
    assert info["rel_change"] == rel[want - 1]
