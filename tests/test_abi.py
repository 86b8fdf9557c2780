"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before touching a device (CPU only)."""
import ctypes
import math
import os
import re

import pytest

import paper_2604_07372_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\(", text, flags=re.M):
            name = m.group(1)
            if name not in ("if", "while", "for", "sizeof", "defined"):
                names.append(name)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 10
    L = ctypes.CDLL(P.LIB_PATH)
    for name in names:
        assert hasattr(L, name), name


def test_version_and_status_strings():
    L = P.lib()
    assert L.nsrgs_version() == 100
    for st in range(7):
        assert L.nsrgs_status_string(st)


def _mat(fmt=P.F32, ld=304, data=16):
    return P._Matrix(fmt, data, None, None, ld)


@pytest.mark.parametrize("n,d,msg", [(1, 3, "n must be"), (0, 3, "n must be"), (10, 0, "d must be"),
                                     (10, 33, "d must be")])
def test_step_rejects_bad_sizes(n, d, msg):
    L = P.lib()
    m = _mat()
    st = L.sync_step(ctypes.byref(m), n, d, 0.0, 3, 16, 4096, 256, 1 << 30, None)
    assert st == 1
    assert msg in L.nsrgs_last_error().decode()


def test_step_rejects_bad_matrix_and_buffers():
    L = P.lib()
    n, d = 100, 3
    ws_bytes = L.sync_workspace_bytes(n, d, P.F32)
    cases = [
        (_mat(ld=290), "ld"),                # < nd and not a multiple of 16
        (_mat(ld=308), "multiple of 16"),
        (_mat(data=8), "aligned"),
        (P._Matrix(7, 16, None, None, 304), "format"),
        (P._Matrix(P.BF16_SPLIT, 16, None, None, 304), "data_lo"),
        (P._Matrix(P.FP8_E4M3, 16, None, None, 304), "row_scale"),
    ]
    for m, msg in cases:
        st = L.sync_step(ctypes.byref(m), n, d, 0.0, 3, 4096, 1 << 20, 256, ws_bytes, None)
        assert st == 1, msg
        assert msg in L.nsrgs_last_error().decode()
    m = _mat()
    # aliasing input/output
    st = L.sync_step(ctypes.byref(m), n, d, 0.0, 3, 4096, 4096 + 64, 256, ws_bytes, None)
    assert st == 1 and "overlap" in L.nsrgs_last_error().decode()
    # workspace too small (the streaming-kernel calls need only the part before
    # the matrix-core region; the exact-polar step needs all of it)
    st = L.sync_step(ctypes.byref(m), n, d, 0.0, 3, 4096, 1 << 20, 256, 4096, None)
    assert st == 3
    st = L.sync_step_polar(ctypes.byref(m), n, d, 0.0, 4096, 1 << 20, 256, ws_bytes - 1, None)
    assert st == 3
    # ns_steps out of range, non-finite mu
    assert L.sync_step(ctypes.byref(m), n, d, 0.0, 65, 4096, 1 << 20, 256, ws_bytes, None) == 1
    assert L.sync_step(ctypes.byref(m), n, d, float("nan"), 3, 4096, 1 << 20, 256, ws_bytes, None) == 1


def test_workspace_size_scales_and_rejects():
    L = P.lib()
    assert L.sync_workspace_bytes(1, 3, P.F32) == 0
    assert L.sync_workspace_bytes(10, 33, P.F32) == 0
    assert L.sync_workspace_bytes(10, 17, P.BF16) == 0
    assert L.sync_workspace_bytes(10, 3, 9) == 0
    small = L.sync_workspace_bytes(100, 3, P.F32)
    big = L.sync_workspace_bytes(20000, 3, P.F32)
    bigger = L.sync_workspace_bytes(40000, 3, P.F32)
    f64 = L.sync_workspace_bytes(100, 3, P.F64)
    assert 0 < small < big < bigger and f64 > small
    # the workspace grows linearly in n d (iterates, per-block records, partial
    # products of at most a few column chunks): no nd x nd scratch
    nd = 60000
    assert big < 0.01 * nd * nd * 4
    assert bigger < 2.2 * big


def test_solve_and_init_reject_before_device_use():
    L = P.lib()
    m = _mat()
    info = P.Info()
    assert L.sync_solve(ctypes.byref(m), 1, 3, 0.0, 3, 10, 0.0, 4096, 256, 1 << 30, None, None,
                        ctypes.byref(info)) == 1
    assert L.sync_solve(ctypes.byref(m), 100, 3, 0.0, 3, -1, 0.0, 4096, 256, 1 << 30, None, None,
                        ctypes.byref(info)) == 1
    assert L.sync_init_spectral(ctypes.byref(m), 100, 3, None, 0, 0.0, 256, 1 << 30, None,
                                ctypes.byref(info)) == 1
    assert L.nsrgs_generate_measurement(None, 100, 3, 1.0, 0, 0, 1.0, P.F32, 16, 304, None) == 1
    assert L.nsrgs_generate_measurement(16, 100, 3, 1.0, 0, 0, 1.0, P.BF16, 16, 304, None) == 1
    out = P._Matrix(P.F32, 16, None, None, 304)
    assert L.nsrgs_convert(16, 300, 304, ctypes.byref(out), None) == 1
    # symmetric solves: flag values, FP8, and a workspace sized for sync_step only
    ws_sym = L.sync_step_symmetric_workspace_bytes(100, 3, P.F32)
    for flag, mat, ws, want in [(2, m, ws_sym, 1),
                                (1, P._Matrix(P.FP8_E4M3, 16, None, 32, 304), ws_sym, 2),
                                (1, m, L.sync_workspace_bytes(100, 3, P.F32), 3)]:
        o = P._SolveOpts(0, 60, 0.0, 0, None, 16, flag)
        assert L.sync_solve(ctypes.byref(mat), 100, 3, 0.0, 3, 10, 0.0, 4096, 256, ws, None, ctypes.byref(o),
                            ctypes.byref(info)) == want, (flag, want)


def test_symmetric_step_workspace_and_refusals():
    """sync_step_symmetric: workspace sizes from the tile shape (the partial sums
    grow like (n d)^2 d / H), and every refusal happens on the host."""
    L = P.lib()
    assert L.sync_step_symmetric_workspace_bytes(100, 17, P.F32) == 0         # d <= 16
    assert L.sync_step_symmetric_workspace_bytes(100, 16, P.F32) > 0
    assert L.sync_step_symmetric_workspace_bytes(100, 3, P.FP8_E4M3) == 0     # not symmetric storage
    assert L.sync_step_symmetric_workspace_bytes(100, 13, P.BF16) == 0        # 2-byte formats: d <= 12
    assert L.sync_step_symmetric_workspace_bytes(100, 12, P.BF16_SPLIT) > 0
    assert L.sync_step_symmetric_workspace_bytes(100, 13, P.F32) > 0
    st = L.sync_step_symmetric(ctypes.byref(_mat(P.BF16, ld=1312)), 100, 13, 0.0, 3, 4096, 1 << 20, 256, 1 << 30, None)
    assert st == 2 and "2-byte" in L.nsrgs_last_error().decode()
    assert L.sync_step_symmetric_workspace_bytes(1, 3, P.F32) == 0
    n, d = 20000, 3
    base = L.sync_workspace_bytes(n, d, P.F32)
    sym = L.sync_step_symmetric_workspace_bytes(n, d, P.F32)
    nd = n * d
    # sized for the FP32-accumulating formats' default shapes: FP32 strips of
    # 1344 rows (the tallest whose per-wave row sums fit 64 KiB of LDS) and
    # chunks of 1024 columns, BF16 strips of 768 rows and chunks of 2048
    rows_sums = max(math.ceil(nd / 1024), math.ceil(nd / 2048)) * nd * d * 4
    col_sums = max(math.ceil(nd / 1344), math.ceil(nd / 768)) * nd * d * 4
    parts = rows_sums + col_sums
    assert L.sync_step_symmetric_workspace_bytes(n, d, P.BF16) == sym
    assert parts <= sym - base <= parts + 1024
    assert sym - base < 0.02 * nd * nd * 4        # small next to the A it replaces reading
    m = _mat()
    ws_bytes = L.sync_step_symmetric_workspace_bytes(100, 3, P.F32)
    # FP8 is refused as unsupported, after the common checks
    f8 = P._Matrix(P.FP8_E4M3, 16, None, 32, 304)
    st = L.sync_step_symmetric(ctypes.byref(f8), 100, 3, 0.0, 3, 4096, 1 << 20, 256, ws_bytes, None)
    assert st == 2 and "FP8" in L.nsrgs_last_error().decode()
    # d > 16 is refused by the common checks; the sync_step workspace alone is too small
    st = L.sync_step_symmetric(ctypes.byref(m), 30, 17, 0.0, 3, 4096, 1 << 20, 256, 1 << 30, None)
    assert st == 1
    st = L.sync_step_symmetric(ctypes.byref(m), 100, 3, 0.0, 3, 4096, 1 << 20, 256,
                               L.sync_workspace_bytes(100, 3, P.F32), None)
    assert st == 3 and "sync_step_symmetric" in L.nsrgs_last_error().decode()
    # the common checks (aliasing, mu)
    assert L.sync_step_symmetric(ctypes.byref(m), 100, 3, 0.0, 3, 4096, 4096 + 64, 256, ws_bytes, None) == 1
    assert L.sync_step_symmetric(ctypes.byref(m), 100, 3, float("inf"), 3, 4096, 1 << 20, 256, ws_bytes,
                                 None) == 1


def test_block_sparse_entry_points_reject_on_the_host():
    L = P.lib()
    b = P._Bsr(P.F32, 0, 256, 512, 1024)
    ws = L.sync_workspace_bytes(100, 3, P.F32)
    # d > 32, format, NULL arrays, overlap, small workspace, mu
    assert L.sync_step_bsr(ctypes.byref(b), 100, 33, 0.0, 3, 4096, 1 << 20, 256, 1 << 30, None) == 2
    # 8 < d <= 32 runs through the matrix-core epilogue and needs its whole workspace
    assert L.sync_step_bsr(ctypes.byref(b), 100, 9, 0.0, 3, 4096, 1 << 20, 256,
                           L.sync_workspace_bytes(100, 9, P.F32) - 256, None) == 3
    f64 = P._Bsr(P.F64, 0, 256, 512, 1024)
    assert L.sync_step_bsr(ctypes.byref(f64), 100, 3, 0.0, 3, 4096, 1 << 20, 256, ws, None) == 2
    null = P._Bsr(P.F32, 0, 256, None, 1024)
    assert L.sync_step_bsr(ctypes.byref(null), 100, 3, 0.0, 3, 4096, 1 << 20, 256, ws, None) == 1
    assert L.sync_step_bsr(ctypes.byref(b), 100, 3, 0.0, 3, 4096, 4096 + 64, 256, ws, None) == 1
    assert L.sync_step_bsr(ctypes.byref(b), 100, 3, 0.0, 3, 4096, 1 << 20, 256, 4096, None) == 3
    assert L.sync_step_bsr(ctypes.byref(b), 100, 3, float("nan"), 3, 4096, 1 << 20, 256, ws, None) == 1
    nnzb = ctypes.c_int64(0)
    assert L.nsrgs_bsr_count(16, 100, 3, 1.5, 0, 256, 512, ctypes.byref(nnzb), None) == 1      # p > 1
    assert L.nsrgs_bsr_count(None, 100, 3, 0.5, 0, 256, 512, ctypes.byref(nnzb), None) == 1
    assert L.nsrgs_bsr_fill(16, 100, 3, 1.0, 0.5, 0, ctypes.byref(f64), None) == 2
    assert L.nsrgs_bsr_fill(16, 100, 3, float("inf"), 0.5, 0, ctypes.byref(b), None) == 1


@pytest.mark.parametrize("n,d", [(2, 1), (100, 3), (20000, 3), (7000, 4), (513, 6), (100, 7), (40, 25)])
def test_block_sparse_workspace_holds_the_slice_region(n, d):
    """sync_step_bsr_workspace_bytes: the whole sync_workspace_bytes region, and
    for d <= 6 after it the sliced product's (S + 1) n int32 slice bounds and
    S n d^2 FP32 partial sums, S = ceil(n / W) slices of W = 128 KiB / (4 ceil4(d^2))
    block columns (X_j padded to whole float4s in LDS), each part 256-byte aligned."""
    L = P.lib()
    full = L.sync_workspace_bytes(n, d, P.F32)
    got = L.sync_step_bsr_workspace_bytes(n, d)
    if d > 6:
        assert got == full
        return
    a256 = lambda v: (v + 255) // 256 * 256
    W = 131072 // (4 * ((d * d + 3) // 4 * 4))
    S = (n + W - 1) // W
    assert full % 256 == 0
    assert got == full + a256((S + 1) * n * 4) + a256(S * n * d * d * 4)


def test_wide_block_sizes_need_f64_or_f32():
    """16 < d <= 32 runs on the matrix-core path, F64 and F32 storage only; the
    exact-polar and GPM steps likewise (checked before any device work)."""
    L = P.lib()
    m = _mat(P.BF16, ld=352)
    st = L.sync_step(ctypes.byref(m), 20, 17, 0.0, 3, 16, 4096, 256, 1 << 30, None)
    assert st == 2 and "F64 or F32" in L.nsrgs_last_error().decode()
    st = L.sync_step_gpm(ctypes.byref(m), 20, 3, 16, 4096, 256, 1 << 30, None)
    assert st == 2
    assert L.sync_workspace_bytes(20, 17, P.BF16) == 0
    assert L.sync_workspace_bytes(20, 25, P.F64) > L.sync_workspace_bytes(20, 16, P.F64) > 0
    assert L.sync_workspace_bytes(20, 33, P.F64) == 0
    # the no-allocation step keeps the narrow path's limit
    m32 = _mat(P.F32, ld=352)
    st = L.sync_step_noalloc(ctypes.byref(m32), 20, 17, 0.0, 3, 16, 4096, None)
    assert st == 1 and "d must be" in L.nsrgs_last_error().decode()


def test_solve_rejects_unknown_method_and_stop_rule():
    L = P.lib()
    m = _mat(P.F64, ld=304)
    for method, stop, msg in ((3, 0, "method"), (0, 2, "stop rule")):
        o = P._SolveOpts(0, 60, 0.0, 0, None, 16, 0, method, stop)
        st = L.sync_solve(ctypes.byref(m), 100, 3, 0.0, 3, 10, 0.0, 4096, 256, 1 << 30, None,
                          ctypes.byref(o), None)
        assert st == 1 and msg in L.nsrgs_last_error().decode()
    o = P._SolveOpts(0, 60, 0.0, 0, None, 16, 1, 1, 0)             # symmetric + exact polar
    st = L.sync_solve(ctypes.byref(m), 100, 3, 0.0, 3, 10, 0.0, 4096, 256, 1 << 30, None, ctypes.byref(o), None)
    assert st == 2


def _packed_count(n, d):
    """Elements of the packed upper-block-triangle layout, summed row by row
    from its definition: row r of block i = r // d keeps columns
    [64 floor(i d / 64), ndp), ndp = n d rounded up to 64."""
    import numpy as np
    nd = n * d
    ndp = -(-nd // 64) * 64
    i = np.arange(nd, dtype=np.int64) // d
    return int(np.sum(ndp - 64 * ((i * d) // 64)))


@pytest.mark.parametrize("n,d", [(1, 1), (2, 1), (2, 3), (5, 2), (17, 16), (37, 3), (100, 7), (211, 5),
                                 (300, 12), (1000, 16), (20000, 3), (9, 32)])
def test_packed_element_count(n, d):
    assert P.lib().nsrgs_packed_elems(n, d) == _packed_count(n, d)


def test_packed_footprint_is_half_of_the_full_layout():
    n, d = 20000, 3
    full = n * d * P.padded_ld(n * d) * 4
    packed = P.lib().nsrgs_packed_elems(n, d) * 4
    assert packed <= 7.22e9 and full >= 14.4e9
    assert abs(packed / full - 0.5) < 0.002
    for bad in [(0, 3), (10, 0), (10, 33), (1 << 20, 2048)]:
        assert P.lib().nsrgs_packed_elems(*bad) == 0


def test_packed_storage_is_refused_where_it_is_not_read():
    """Only the symmetric step, symmetric solves and the initialization read
    the packed layout; every other call refuses it on the host."""
    L = P.lib()
    n, d = 100, 3
    pk = P._Matrix(P.F32, 16, None, None, P.PACKED_LD)
    ws = L.sync_step_symmetric_workspace_bytes(n, d, P.F32)
    info = P.Info()
    assert L.sync_step(ctypes.byref(pk), n, d, 0.0, 3, 4096, 1 << 20, 256, ws, None) == 2
    assert "packed" in L.nsrgs_last_error().decode()
    assert L.sync_step_polar(ctypes.byref(pk), n, d, 0.0, 4096, 1 << 20, 256, 1 << 30, None) == 2
    assert L.sync_step_gpm(ctypes.byref(pk), n, d, 4096, 1 << 20, 256, 1 << 30, None) == 2
    assert L.sync_step_noalloc(ctypes.byref(pk), n, d, 0.0, 3, 4096, 1 << 20, None) == 2
    # a solve that is not symmetric
    o = P._SolveOpts(0, 60, 0.0, 0, None, 16, 0)
    assert L.sync_solve(ctypes.byref(pk), n, d, 0.0, 3, 10, 0.0, 4096, 256, ws, None, ctypes.byref(o),
                        ctypes.byref(info)) == 2
    # symmetric: the format must be stored symmetrically, the workspace sized for the tiles
    f8 = P._Matrix(P.FP8_E4M3, 16, None, 32, P.PACKED_LD)
    assert L.sync_step_symmetric(ctypes.byref(f8), n, d, 0.0, 3, 4096, 1 << 20, 256, ws, None) == 2
    assert L.sync_step_symmetric(ctypes.byref(pk), n, d, 0.0, 3, 4096, 1 << 20, 256,
                                 L.sync_workspace_bytes(n, d, P.F32), None) == 3
    # the initialization on packed storage needs the symmetric workspace and d <= 16
    assert L.sync_init_spectral(ctypes.byref(pk), n, d, 4096, 0, 0.0, 256, L.sync_workspace_bytes(n, d, P.F32),
                                None, ctypes.byref(info)) == 3
    assert L.sync_init_spectral(ctypes.byref(pk), 30, 17, 4096, 0, 0.0, 256, 1 << 30, None,
                                ctypes.byref(info)) == 2
    # packed conversion: BF16 / BF16_SPLIT only, out must be packed
    out = P._Matrix(P.BF16, 16, None, None, P.PACKED_LD)
    out8 = P._Matrix(P.FP8_E4M3, 16, None, 32, P.PACKED_LD)
    assert L.nsrgs_convert_packed(16, n, d, ctypes.byref(out8), None) == 2
    assert L.nsrgs_convert_packed(16, n, d, ctypes.byref(_mat(P.BF16)), None) == 1
    assert L.nsrgs_convert_packed(16, 0, d, ctypes.byref(out), None) == 1
    assert L.nsrgs_convert_packed(None, n, d, ctypes.byref(out), None) == 1
    # the generator writes packed storage for d <= 32 only
    assert L.nsrgs_generate_measurement(16, n, 33, 1.0, 0, 0, 1.0, P.F32, 16, P.PACKED_LD, None) == 1


def test_stiefel_entry_points_reject_on_the_host():
    L = P.lib()
    n, d, p = 100, 3, 5
    ws = L.sync_stiefel_workspace_bytes(n, d, p, P.F32)
    assert ws >= L.sync_workspace_bytes(n, d, P.F32) + n * d * p * 4
    assert L.sync_stiefel_workspace_bytes(n, 4, 3, P.F32) == 0        # p < d
    assert L.sync_stiefel_workspace_bytes(n, 3, 33, P.F32) == 0       # p > 32
    assert L.sync_stiefel_workspace_bytes(n, 3, 5, P.BF16) == 0       # F64 / F32 only
    assert L.sync_stiefel_workspace_bytes(1, 3, 5, P.F32) == 0
    m = _mat()
    info = P.Info()
    big = 1 << 30
    assert L.sync_step_stiefel(ctypes.byref(m), n, 4, 3, 0.0, 3, 4096, 1 << 20, 256, big, None) == 1
    assert L.sync_step_stiefel(ctypes.byref(_mat(P.BF16)), n, d, p, 0.0, 3, 4096, 1 << 20, 256, big, None) == 2
    assert L.sync_step_stiefel(ctypes.byref(m), n, d, p, 0.0, 3, 4096, 1 << 20, 256, ws - 256, None) == 3
    assert L.sync_step_stiefel(ctypes.byref(m), n, d, p, 0.0, 3, 4096, 4096 + 64, 256, ws, None) == 1   # overlap
    assert L.sync_step_stiefel(ctypes.byref(m), n, d, p, float("nan"), 3, 4096, 1 << 20, 256, ws, None) == 1
    pk = P._Matrix(P.F32, 16, None, None, P.PACKED_LD)
    assert L.sync_step_stiefel(ctypes.byref(pk), n, d, p, 0.0, 3, 4096, 1 << 20, 256, ws, None) == 2
    assert L.sync_solve_stiefel(ctypes.byref(m), n, d, p, 0.0, 3, -1, 0.0, 4096, 256, ws, None,
                                ctypes.byref(info)) == 1
    assert L.sync_solve_stiefel(ctypes.byref(m), n, d, p, 0.0, 3, 10, 0.0, None, 256, ws, None,
                                ctypes.byref(info)) == 1
    assert L.sync_stiefel_round(4096, n, d, p, P.F32, 4096, 256, ws, None) == 1            # overlap
    assert L.sync_stiefel_round(4096, n, d, p, P.FP8_E4M3, 1 << 20, 256, big, None) == 2
    assert L.sync_stiefel_round(4096, n, d, p, P.F32, 1 << 20, 256, 1024, None) == 3
