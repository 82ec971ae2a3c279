"""GPU parity of the two-phase product against the oracle (through the C ABI).

Structure (row_ptr, col_idx) must be bit-exact; values within
|c - c_ref| <= 1e-12 * sum|a||b| (the oracle's error scale), and -- because
the kernels add the terms of each entry in ascending k with rounded products,
as the oracle does -- also bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

mls = pytest.importorskip("paper_1804_00695_amd")
TOL = 1e-12


@pytest.fixture(autouse=True)
def _reset_options():
    yield
    mls.set_option(mls._abi.OPT_FORCE_SPILL, 0)
    mls.set_option(mls._abi.OPT_GROUP_SIZE, 0)
    mls.set_option(mls._abi.OPT_VALIDATE, 1)
    mls.set_option(mls._abi.OPT_WIDE_TABLE, 0)
    mls.set_option(mls._abi.OPT_FORCE_CLASS, -1)


def gpu_product(A, B):
    dA, dB = mls.DeviceCsr.from_host(A), mls.DeviceCsr.from_host(B)
    C = mls.spgemm(dA, dB)
    torch.cuda.synchronize()
    mls.check_errors()
    return C.numpy()


def check(A, B, bitwise=True):
    rp, ci, v = gpu_product(A, B)
    R, cabs = oracle.spgemm(A, B)
    assert np.array_equal(rp, R.row_ptr), "row_ptr differs"
    assert np.array_equal(ci, R.col_idx), "col_idx differs"
    if R.values is not None:
        err = np.abs(v - R.values)
        assert np.all(err <= TOL * cabs), float(np.max(err - TOL * cabs))
        if bitwise:
            assert np.array_equal(v, R.values)
    return R


def test_laplace2d_64_square():
    A = synth.laplace2d_5pt(64)
    R = check(A, A)
    assert R.nnz == 51972


@pytest.mark.parametrize("n,amp", [(2, 0.0), (5, 0.0), (12, 0.0), (12, 0.1), (21, 0.1)])
def test_stencil27_square(n, amp):
    A = synth.stencil27_3d(n, amp=amp, seed=2)
    R = check(A, A)
    assert R.nnz == (5 * n - 6) ** 3


@pytest.mark.parametrize("shape", [(3000, 2000, 2500, 5.0, 7.0), (1000, 1000, 1000, 8.0, 8.0),
                                   (777, 4099, 33, 3.0, 2.0), (1, 500, 300, 40.0, 9.0)])
def test_poisson_rect(shape):
    m, k, n, la, lb = shape
    A = synth.poisson_csr(m, k, la, seed=m + 1)
    B = synth.poisson_csr(k, n, lb, seed=k + 2)
    check(A, B)


def test_empty_rows_and_matrices():
    A = synth.random_csr(300, 200, 0.05, 3, empty_rows=0.5)
    B = synth.random_csr(200, 150, 0.05, 4, empty_rows=0.5)
    check(A, B)
    Z = synth.Csr(50, 40, np.zeros(51, np.int32), np.zeros(0, np.int32), np.zeros(0))
    W = synth.poisson_csr(40, 60, 3.0, 5)
    check(Z, W)
    check(synth.poisson_csr(30, 50, 3.0, 6), synth.Csr(50, 70, np.zeros(51, np.int32), np.zeros(0, np.int32), np.zeros(0)))


def wide_rows(m, k, per_row, seed):
    g = synth.rng(seed)
    rows = [np.sort(g.choice(k, per_row, replace=False)) for _ in range(m)]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    return synth.Csr(m, k, rp, np.concatenate(rows).astype(np.int32), g.standard_normal(int(rp[-1])))


@pytest.mark.parametrize("per_row", [30, 120, 400, 1500])
def test_large_rows_all_classes(per_row):
    # nnz(C_i) ~ per_row * 8 spans the LDS classes and the global spill path
    A = wide_rows(64, 6000, per_row, per_row)
    B = synth.poisson_csr(6000, 20000, 8.0, 99)
    check(A, B)


@pytest.mark.parametrize("G", [8, 16, 32, 64])
def test_forced_group_sizes(G):
    mls.set_option(mls._abi.OPT_GROUP_SIZE, G)
    check(synth.stencil27_3d(9, amp=0.1), synth.stencil27_3d(9, amp=0.1, seed=3))
    check(synth.poisson_csr(500, 400, 6.0, 7), synth.poisson_csr(400, 450, 12.0, 8))


def test_forced_spill_identical():
    A = synth.stencil27_3d(8, amp=0.1)
    mls.set_option(mls._abi.OPT_FORCE_SPILL, 1)
    check(A, A)
    check(synth.poisson_csr(300, 300, 5.0, 9), synth.poisson_csr(300, 400, 5.0, 10))


def test_class_boundaries():
    # rows of C with exactly the sizes where the LDS classes change (32/33,
    # 128/129, 512/513, 1024/1025, 2048/2049 outputs; the count bound equals
    # the row length here, so 128/129, 256/257, 512/513, 2048/2049 and
    # 8192/8193 for the count classes)
    lengths = [1, 31, 32, 33, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1024, 1025, 2047, 2048, 2049,
               4096, 8192, 8193, 9000]
    n = 20000
    g = synth.rng(17)
    rows = [np.sort(g.choice(n, L, replace=False)) for L in lengths]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    A = synth.Csr(len(rows), n, rp, np.concatenate(rows).astype(np.int32), g.standard_normal(int(rp[-1])))
    # B: row k holds the single column 32 * (k % 625) + k // 625 (a permutation), so every B row is one
    # word and C's row i has exactly as many columns as A's row i
    cols = (32 * (np.arange(n) % 625) + np.arange(n) // 625).astype(np.int32)
    B = synth.Csr(n, n, np.arange(n + 1, dtype=np.int32), cols, g.standard_normal(n))
    R = check(A, B)
    assert np.array_equal(np.diff(R.row_ptr), lengths)


def test_wide_table_identical():
    # the 8-byte (column, position) slots, which products with many columns use
    mls.set_option(mls._abi.OPT_WIDE_TABLE, 1)
    A = synth.stencil27_3d(9, amp=0.1)
    check(A, A)
    check(wide_rows(64, 6000, 120, 5), synth.poisson_csr(6000, 20000, 8.0, 99))
    check(synth.poisson_csr(500, 400, 6.0, 7), synth.poisson_csr(400, 450, 12.0, 8))


def with_last_column(B):
    """B with column ncols-1 present in every row (the largest key a table holds)."""
    rows, vals = [], []
    for k in range(B.nrows):
        c = B.col_idx[B.row_ptr[k]:B.row_ptr[k + 1]]
        v = B.values[B.row_ptr[k]:B.row_ptr[k + 1]]
        if len(c) == 0 or c[-1] != B.ncols - 1:
            c = np.append(c, B.ncols - 1)
            v = np.append(v, 0.5 + k % 7)
        rows.append(c)
        vals.append(v)
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    return synth.Csr(B.nrows, B.ncols, rp, np.concatenate(rows).astype(np.int32), np.concatenate(vals))


@pytest.mark.parametrize("ncols", [(1 << 21) - 1, 1 << 21, (1 << 23) - 1, 1 << 23, (1 << 25) - 1, 1 << 25])
def test_packed_table_column_limits(ncols):
    # row sizes in all four LDS classes; the packed slots hold column indices
    # below 2^21 - 1, 2^23 - 1, 2^25 - 1 and 2^27 - 1 for the classes of 4096,
    # 1024, 256 and 64 slots, and the wide slots take over from there
    B = with_last_column(synth.poisson_csr(3000, ncols, 6.0, 31))
    for per_row, seed in ((3, 4), (10, 1), (60, 2), (200, 3)):
        check(wide_rows(24, 3000, per_row, seed), B)


def test_row_work_and_compress():
    A = synth.poisson_csr(2000, 1500, 6.0, 21)
    B = synth.poisson_csr(1500, 3000, 9.0, 22)
    dA, dB = mls.DeviceCsr.from_host(A), mls.DeviceCsr.from_host(B)
    w, tot = mls.row_work(dA, dB)
    ref = oracle.row_work(A, B)
    assert np.array_equal(w.cpu().numpy(), ref) and tot == int(ref.sum())
    words, count = mls.compress(dB)
    words = words.cpu().numpy().view(np.uint32)
    count = count.cpu().numpy()
    rp, sets, masks = oracle.compress(B)
    assert np.array_equal(count, np.diff(rp))
    for k in range(B.nrows):
        s = int(B.row_ptr[k])
        got = words[2 * s: 2 * (s + count[k])]
        assert np.array_equal(got[0::2], sets[rp[k]:rp[k + 1]].view(np.uint32))
        assert np.array_equal(got[1::2], masks[rp[k]:rp[k + 1]])


def test_compress_long_rows():
    # rows longer than 64 entries take the wave-cooperative path: dense runs
    # (words spanning the 64-entry steps), sparse rows, and lengths around 64
    g = synth.rng(13)
    rows = [np.arange(17, 217), np.sort(g.choice(5000, 300, replace=False)), np.arange(64), np.arange(30, 95),
            np.array([4999]), np.sort(g.choice(5000, 63, replace=False)), np.arange(0, 5000, 7)[:400],
            np.array([], dtype=np.int64), np.sort(g.choice(5000, 129, replace=False))]
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    B = synth.Csr(len(rows), 5000, rp, np.concatenate(rows).astype(np.int32), None)
    dB = mls.DeviceCsr.from_host(B)
    words, count = mls.compress(dB)
    words = words.cpu().numpy().view(np.uint32)
    count = count.cpu().numpy()
    crp, sets, masks = oracle.compress(B)
    assert np.array_equal(count, np.diff(crp))
    for k in range(B.nrows):
        s0 = int(B.row_ptr[k])
        got = words[2 * s0: 2 * (s0 + count[k])]
        assert np.array_equal(got[0::2], sets[crp[k]:crp[k + 1]].view(np.uint32)), k
        assert np.array_equal(got[1::2], masks[crp[k]:crp[k + 1]]), k


@pytest.mark.parametrize("bad", ["unsorted", "duplicate", "out_of_range", "decreasing"])
def test_device_validation(bad):
    B = synth.poisson_csr(20, 30, 4.0, 1)
    A = synth.poisson_csr(10, 20, 4.0, 2)
    rp, ci = A.row_ptr.copy(), A.col_idx.copy()
    r = int(np.argmax(np.diff(rp) >= 2))
    s = int(rp[r])
    if bad == "unsorted":
        ci[s], ci[s + 1] = ci[s + 1], ci[s]
    elif bad == "duplicate":
        ci[s + 1] = ci[s]
    elif bad == "out_of_range":
        ci[s] = 25
    else:
        r = int(np.argmax(rp[1:-1] >= 1)) + 1     # a row r >= 1 with row_ptr[r] >= 1
        rp[r + 1] = rp[r] - 1                     # still inside [0, nnz]
    Abad = synth.Csr(A.nrows, A.ncols, rp, ci, A.values)
    with pytest.raises(mls.SpgemmError, match="BAD_CSR"):
        mls.symbolic(mls.DeviceCsr.from_host(Abad), mls.DeviceCsr.from_host(B))


@pytest.mark.parametrize("side", ["A", "B"])
@pytest.mark.parametrize("length,pos", [(200, 0), (200, 63), (200, 64), (200, 130), (200, 199),
                                        (20, 0), (20, 10), (20, 19)])
@pytest.mark.parametrize("bad", ["unsorted", "duplicate", "out_of_range"])
def test_device_validation_long_rows(side, length, pos, bad):
    # rows of more than 16 entries take the wave-cooperative check; the planted
    # error sits at chunk starts, chunk ends and the row's last entry
    M = wide_rows(40, 500, length, 7)
    rp, ci = M.row_ptr.copy(), M.col_idx.copy()
    s = int(rp[17])
    q = s + pos
    last = length - 1
    if bad == "unsorted":
        a, b2 = (q, q + 1) if pos < last else (q - 1, q)
        ci[a], ci[b2] = ci[b2], ci[a]
    elif bad == "duplicate":
        if pos < last:
            ci[q + 1] = ci[q]
        else:
            ci[q] = ci[q - 1]
    else:
        ci[q] = 500 if pos == last else -3
    Mbad = synth.Csr(M.nrows, M.ncols, rp, ci, M.values)
    if side == "A":
        X, Y = Mbad, synth.poisson_csr(500, 30, 4.0, 1)
    else:
        X, Y = synth.poisson_csr(30, 40, 4.0, 2), Mbad
    with pytest.raises(mls.SpgemmError, match="BAD_CSR"):
        mls.symbolic(mls.DeviceCsr.from_host(X), mls.DeviceCsr.from_host(Y))


def test_dimension_mismatch():
    A = synth.poisson_csr(10, 20, 4.0, 2)
    B = synth.poisson_csr(21, 30, 4.0, 1)
    with pytest.raises(mls.SpgemmError, match="DIM_MISMATCH"):
        mls.symbolic(mls.DeviceCsr.from_host(A), mls.DeviceCsr.from_host(B))


def test_numeric_detects_missing_structure():
    A = synth.poisson_csr(100, 80, 4.0, 31)
    B = synth.poisson_csr(80, 90, 4.0, 32)
    R, _ = oracle.spgemm(A, B)
    # drop the last entry of the first non-empty row
    r = int(np.argmax(np.diff(R.row_ptr) > 0))
    keep = np.ones(R.nnz, bool)
    keep[int(R.row_ptr[r + 1]) - 1] = False
    rp = R.row_ptr.copy()
    rp[r + 1:] -= 1
    C = synth.Csr(R.nrows, R.ncols, rp, R.col_idx[keep], np.zeros(int(keep.sum())))
    dA, dB, dC = mls.DeviceCsr.from_host(A), mls.DeviceCsr.from_host(B), mls.DeviceCsr.from_host(C)
    ws = mls.Workspace()
    mls.numeric(dA, dB, dC, ws)
    with pytest.raises(mls.SpgemmError, match="STRUCTURE"):
        mls.check_errors(ws)


def test_deterministic_repeat():
    A = synth.stencil27_3d(14, amp=0.1)
    r1 = gpu_product(A, A)
    r2 = gpu_product(A, A)
    for x, y in zip(r1, r2):
        assert np.array_equal(x, y)


def raw_symbolic(A, B, ws_bytes_fn=lambda full, minimal: full, separate_fill_ws=False, fill_twice=False):
    """Count and fill through the ABI with chosen workspaces."""
    import ctypes
    dA, dB = mls.DeviceCsr.from_host(A), mls.DeviceCsr.from_host(B)
    full = mls.workspace_size(dA, dB)
    nb = ws_bytes_fn(full, None)
    w1 = mls.Workspace()
    w2 = mls.Workspace()
    p1 = w1.get(nb)
    crp = torch.empty(A.nrows + 1, dtype=torch.int32, device="cuda")
    nnz = ctypes.c_int64(0)
    ha, hb = dA.handle(), dB.handle()
    s = mls.stream_handle()
    mls.check(mls.lib.spgemm_symbolic(ctypes.byref(ha), ctypes.byref(hb), crp.data_ptr(), None, ctypes.byref(nnz),
                                      p1, nb, s), "count")
    cci = torch.full((max(nnz.value, 1),), -7, dtype=torch.int32, device="cuda")
    p2 = w2.get(nb) if separate_fill_ws else p1
    for _ in range(2 if fill_twice else 1):
        mls.check(mls.lib.spgemm_symbolic(ctypes.byref(ha), ctypes.byref(hb), crp.data_ptr(), cci.data_ptr(), None,
                                          p2, nb, s), "fill")
    torch.cuda.synchronize()
    mls.check(mls.lib.spgemm_check_errors(p2, nb, s), "errors")
    return crp.cpu().numpy(), cci[:nnz.value].cpu().numpy()


@pytest.mark.parametrize("mode", ["scratch", "separate_ws", "no_scratch_room", "fill_twice"])
def test_symbolic_fill_paths(mode):
    A = synth.stencil27_3d(9, amp=0.1)
    B = wide_rows(729, 20000, 60, 5)        # rows of C with > 64 words overflow the scratch
    # rows with 0 or 1 entries of A fit the scratch, longer ones overflow it
    for X, Y in ((A, A), (synth.poisson_csr(400, 729, 1.5, 3), B)):
        R, _ = oracle.spgemm(X, Y, with_abs=False)
        kw = {}
        if mode == "separate_ws":
            kw["separate_fill_ws"] = True
        elif mode == "no_scratch_room":
            # one byte short of the full size: above the minimum, without the scratch
            kw["ws_bytes_fn"] = lambda full, _: full - 1
        elif mode == "fill_twice":
            kw["fill_twice"] = True
        rp, ci = raw_symbolic(X, Y, **kw)
        assert np.array_equal(rp, R.row_ptr) and np.array_equal(ci, R.col_idx)


def test_spill_column_windows():
    # rows of C with ~12k entries spread over 3M columns: the spill bitmap
    # covers the columns in several windows, each entry's words narrowed to
    # the window; also a batch row of C whose columns are all in the last window
    A = wide_rows(6, 5000, 3000, 31)
    B = synth.poisson_csr(5000, 3_000_000, 4.0, 32)
    check(A, B)
    g = synth.rng(33)
    rp = np.arange(0, 4 * 5001, 4, dtype=np.int32)
    ci = np.sort(g.integers(2_990_000, 3_000_000, (5000, 4)), axis=1).astype(np.int32)
    ci[:, 1:] += np.cumsum(ci[:, 1:] == ci[:, :-1], axis=1).astype(np.int32)   # keep each row strictly rising
    B2 = synth.Csr(5000, 3_000_010, rp, ci.ravel(), g.standard_normal(ci.size))
    check(A, B2)


def test_rmat_power_law_spill():
    # A*A for a power-law graph (R-MAT scale 13): ~1300 rows of C hold more
    # than 2048 entries (up to ~5400, three spill windows), long rows of B
    # (hubs) are narrowed to each window by binary search
    G = synth.rmat_graph(13, 8, seed=5)
    A = synth.Csr(G.nrows, G.ncols, G.row_ptr, G.col_idx, synth.normal_values(len(G.col_idx), 8))
    R = check(A, A)
    assert np.diff(R.row_ptr).max() > 4096


def test_many_long_rows_in_one_block():
    # 100 rows of 600 entries in one binning block: 64 are sized by the whole
    # workgroup, the rest in place; sizes feed both the bins and row_work
    A = wide_rows(100, 5000, 600, 41)
    B = synth.poisson_csr(5000, 9000, 3.0, 42)
    check(A, B)
    w, madds = mls.row_work(mls.DeviceCsr.from_host(A), mls.DeviceCsr.from_host(B))
    per_entry = np.diff(B.row_ptr)[A.col_idx]
    ref = np.add.reduceat(per_entry, A.row_ptr[:-1]).astype(np.int64)
    assert np.array_equal(w.cpu().numpy(), ref) and madds == int(ref.sum())


@pytest.mark.parametrize("side", ["A", "B"])
@pytest.mark.parametrize("length", [5, 16, 17, 32, 33])
@pytest.mark.parametrize("row", [16, 17, 19])
@pytest.mark.parametrize("where", ["first", "last"])
def test_device_validation_group_rows(side, length, row, where):
    # rows of 5-16 (17-32) entries are checked and compressed four (two) at a
    # time, 16 (32) lanes each, so rows 16-19 (16-17) share a step; a 33-entry
    # row takes the wave
    M = wide_rows(40, 500, length, 9)
    # the compressed words of these rows first, against the oracle
    if side == "B":
        words, count = mls.compress(mls.DeviceCsr.from_host(M))
        crp, sets, masks = oracle.compress(M)
        assert np.array_equal(count.cpu().numpy(), np.diff(crp))
    rp, ci = M.row_ptr.copy(), M.col_idx.copy()
    s = int(rp[row])
    if where == "first":
        ci[s] = ci[s + 1]                        # duplicate at the row's start
    else:
        ci[s + length - 1] = 500                 # out of range at its end
    Mbad = synth.Csr(M.nrows, M.ncols, rp, ci, M.values)
    if side == "A":
        X, Y = Mbad, synth.poisson_csr(500, 30, 4.0, 1)
    else:
        X, Y = synth.poisson_csr(30, 40, 4.0, 2), Mbad
    with pytest.raises(mls.SpgemmError, match="BAD_CSR"):
        mls.symbolic(mls.DeviceCsr.from_host(X), mls.DeviceCsr.from_host(Y))


@pytest.mark.parametrize("cls", [0, 1, 2, 3, 4])
def test_forced_class(cls):
    # every row moves up to LDS class `cls` (count, fill and numeric): each
    # class kernel then sees short rows, long rows and rows with no work
    mls.set_option(mls._abi.OPT_FORCE_CLASS, cls)
    check(synth.stencil27_3d(7, amp=0.1), synth.stencil27_3d(7, amp=0.1, seed=3))
    check(synth.poisson_csr(700, 500, 6.0, 7), synth.poisson_csr(500, 650, 9.0, 8))
    A = synth.random_csr(200, 150, 0.05, 3, empty_rows=0.5)
    B = synth.random_csr(150, 120, 0.05, 4, empty_rows=0.5)
    check(A, B)
    check(wide_rows(24, 3000, 120, 11), synth.poisson_csr(3000, 9000, 8.0, 12))


def colliding_columns(count, bits, target, ncols):
    """Columns whose multiplicative hash (the LDS tables' key -> slot map,
    column * 0x9E3779B1 mod 2^32, top bits) has the given top `bits` bits:
    they all share one home bucket, so inserts and lookups run through the
    probing past full buckets."""
    j = np.arange(ncols, dtype=np.uint64)
    top = ((j * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)) >> np.uint64(32 - bits)
    cols = np.nonzero(top == target)[0]
    assert len(cols) >= count
    return cols[:count].astype(np.int32)


def colliding_instance(per_row, bits, seed):
    g = synth.rng(seed)
    ncols = 1 << 16
    fam = colliding_columns(3 * per_row, bits, 5, ncols)
    kb = 48
    rows = [np.sort(g.choice(fam, per_row, replace=False)) for _ in range(kb)]
    brp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    B = synth.Csr(kb, ncols, brp, np.concatenate(rows).astype(np.int32), synth.normal_values(int(brp[-1]), seed + 1))
    m = 40
    arows = [np.sort(g.choice(kb, 3, replace=False)) for _ in range(m)]
    arp = np.arange(0, 3 * m + 1, 3, dtype=np.int32)
    A = synth.Csr(m, kb, arp, np.concatenate(arows).astype(np.int32), synth.normal_values(3 * m, seed + 2))
    return A, B


@pytest.mark.parametrize("group", [0, 8, 16, 32, 64])
@pytest.mark.parametrize("per_row,bits", [(20, 7), (40, 8)])
@pytest.mark.parametrize("wide", [0, 1])
def test_hash_bucket_overflow(group, per_row, bits, wide):
    # rows of C of 40-120 columns, all with one home bucket in their table
    # (2- and 4-slot buckets alike): bit-exact values, and the adjoint too
    A, B = colliding_instance(per_row, bits, 31 + per_row)
    mls.set_option(mls._abi.OPT_GROUP_SIZE, group)
    mls.set_option(mls._abi.OPT_WIDE_TABLE, wide)
    R = check(A, B)
    W = synth.Csr(R.nrows, R.ncols, R.row_ptr, R.col_idx, synth.normal_values(R.nnz, 7))
    dA, dB = mls.backward(mls.DeviceCsr.from_host(A), mls.DeviceCsr.from_host(B), mls.DeviceCsr.from_host(W))
    torch.cuda.synchronize()
    rA, rB, aA, aB = oracle.backward(A, B, W)
    assert np.all(np.abs(dA.cpu().numpy() - rA) <= 1e-10 * aA + 1e-300)
    assert np.all(np.abs(dB.cpu().numpy() - rB) <= 1e-10 * aB + 1e-300)
