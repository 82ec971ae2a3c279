"""Host-side argument checks that run before any library call or kernel
launch: the Python binding refuses arrays of the wrong dtype, memory kind,
length or layout (ValueError), and the chunked executor refuses operands that
differ from the ones its plan was cut for (no GPU needed: both fail before
any HIP call)."""
import ctypes

import numpy as np
import pytest
import torch

import synth

mls = pytest.importorskip("paper_1804_00695_amd")


def cpu_csr(M, cls):
    return cls(M.nrows, M.ncols, torch.from_numpy(M.row_ptr.astype(np.int32)),
               torch.from_numpy(M.col_idx.astype(np.int32)), torch.from_numpy(M.values.astype(np.float64)))


def test_device_csr_rejects_host_tensors():
    M = synth.poisson_csr(20, 30, 3.0, 1)
    with pytest.raises(ValueError, match="GPU tensor"):
        cpu_csr(M, mls.DeviceCsr).handle()


@pytest.mark.parametrize("bad", ["dtype_rp", "dtype_ci", "dtype_v", "short_v", "short_rp", "strided"])
def test_array_checks(bad):
    M = synth.poisson_csr(20, 30, 3.0, 2)
    rp = torch.from_numpy(M.row_ptr.astype(np.int32))
    ci = torch.from_numpy(M.col_idx.astype(np.int32))
    v = torch.from_numpy(M.values)
    if bad == "dtype_rp":
        rp = rp.long()
    elif bad == "dtype_ci":
        ci = ci.long()
    elif bad == "dtype_v":
        v = v.float()
    elif bad == "short_v":
        v = v[:-1]
    elif bad == "short_rp":
        rp = rp[:-1]
    else:
        v = torch.stack([v, v], 1)[:, 0]
    with pytest.raises(ValueError):
        mls._check_csr(mls.DeviceCsr(M.nrows, M.ncols, rp, ci, v), "cpu_test")


def test_host_csr_requires_pinned_memory():
    M = synth.poisson_csr(20, 30, 3.0, 3)
    with pytest.raises(ValueError, match="pinned"):
        cpu_csr(M, mls.HostCsr).handle()


def test_autograd_forward_checks_values():
    M = synth.poisson_csr(20, 30, 3.0, 4)
    D = cpu_csr(M, mls.DeviceCsr)
    with pytest.raises(ValueError):
        mls.SpGEMMFn.apply(torch.zeros(M.nnz, dtype=torch.float32), torch.zeros(M.nnz, dtype=torch.float64),
                           D, D, D)
    with pytest.raises(ValueError, match="GPU tensor"):
        mls.SpGEMMFn.apply(torch.zeros(M.nnz, dtype=torch.float64), torch.zeros(M.nnz, dtype=torch.float64),
                           D, D, D)


def _host_handle(rp, ci, v, nrows, ncols):
    return mls.CsrT(nrows, ncols, len(ci), rp.ctypes.data, ci.ctypes.data, v.ctypes.data)


def test_chunked_rejects_operands_unlike_the_plan():
    A = synth.poisson_csr(400, 300, 5.0, 5)
    B = synth.poisson_csr(300, 350, 5.0, 6)
    import oracle
    R, _ = oracle.spgemm(A, B, with_abs=False)
    plan = mls.chunked_plan(A.row_ptr, B.row_ptr, B.ncols, R.row_ptr, 2_000_000, nbuf=2, min_parts=3)
    nb = plan.info["ws_bytes"]
    keep = []

    def h(M, rp=None):
        rp = np.ascontiguousarray(M.row_ptr if rp is None else rp, dtype=np.int32)
        ci = np.ascontiguousarray(M.col_idx, dtype=np.int32)
        v = np.ascontiguousarray(M.values if M.values is not None else np.zeros(len(ci)), dtype=np.float64)
        keep.append((rp, ci, v))
        return _host_handle(rp, ci, v, M.nrows, M.ncols)

    fake_ws = ctypes.c_void_p(1 << 20)   # never dereferenced: the calls fail first

    def run(a, b, c):
        return mls.lib.spgemm_numeric_chunked(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), plan._h, fake_ws,
                                              nb, None, None, None)

    # a different entry count of B
    B2 = synth.poisson_csr(300, 350, 6.0, 7)
    assert run(h(A), h(B2), h(R)) == 3
    # same entry count, all of A's entries moved into its first row: the
    # first A/C part no longer fits its buffer
    rp = np.full(A.nrows + 1, A.nnz, dtype=np.int32)
    rp[0] = 0
    assert run(h(A, rp), h(B), h(R)) == 3
    # decreasing row pointers
    rp = A.row_ptr.astype(np.int32).copy()
    rp[5], rp[6] = rp[6], rp[5] - 1
    assert run(h(A, rp), h(B), h(R)) in (2, 3)
