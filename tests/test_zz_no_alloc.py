"""The allocation-free numeric entry point (spgemm_numeric_noalloc) against
the workspace entry point (spgemm_numeric) and the oracle, through the C ABI.

Two calls in a row share the device's fixed scratch array, the second on a
smaller product, so whatever the first call left there must not leak into the
second; a third call runs every row through the spill windows (which use the
array's per-row prefix region). Values must equal spgemm_numeric's and the
oracle's bit for bit (both add every entry's terms in ascending k with rounded
products). The size limit is checked on the host before any HIP call."""
import ctypes

import numpy as np
import pytest

import synth
from paper_1804_00695_amd import _abi

WORKSPACE_TOO_SMALL = 5


def test_rejects_a_too_large_product_before_any_hip_call():
    lib = _abi.load()
    n = 5_000_000     # 17 bytes per row of A exceed the 64 MiB array
    rp = np.zeros(n + 1, dtype=np.int32)
    h = _abi.CsrT(n, n, 0, rp.ctypes.data, None, None)
    c = _abi.CsrT(n, n, 0, rp.ctypes.data, None, None)
    st = lib.spgemm_numeric_noalloc(ctypes.byref(h), ctypes.byref(h), ctypes.byref(c), None)
    assert st == WORKSPACE_TOO_SMALL


def test_fits_the_headline_rows():
    """The 27-point stencil on 128^3 (2,097,152 rows) is within the limit: the
    check passes, and with no GPU the call then fails at its first HIP call."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-only check")
    lib = _abi.load()
    n = 128 ** 3
    rp = np.zeros(n + 1, dtype=np.int32)
    h = _abi.CsrT(n, n, 0, rp.ctypes.data, None, None)
    st = lib.spgemm_numeric_noalloc(ctypes.byref(h), ctypes.byref(h), ctypes.byref(h), None)
    assert st != WORKSPACE_TOO_SMALL


@pytest.mark.gpu
def test_noalloc_matches_workspace_entry_point_twice():
    import torch

    import oracle
    import paper_1804_00695_amd as mls

    cases = [
        ("stencil27 22^3 x Poisson(6)", synth.stencil27_3d(22, amp=0.1, seed=2), None),
        ("Poisson(5) 3000x2000 x Poisson(7) 2000x2500", synth.poisson_csr(3000, 2000, 5.0, seed=21),
         synth.poisson_csr(2000, 2500, 7.0, seed=22)),
    ]
    A0 = cases[0][1]
    cases[0] = (cases[0][0], A0, synth.poisson_csr(A0.ncols, 900, 6.0, seed=23))
    try:
        for it, (name, A, B) in enumerate(cases + [("forced spill, " + cases[1][0], cases[1][1], cases[1][2])]):
            print(f"noalloc call {it}: {name}", flush=True)
            spill = it == 2
            mls.set_option(_abi.OPT_FORCE_SPILL, 1 if spill else 0)
            dA, dB = mls.DeviceCsr.from_host(A), mls.DeviceCsr.from_host(B)
            C = mls.symbolic(dA, dB)
            ref = mls.numeric(dA, dB, C).values.clone()
            torch.cuda.synchronize()
            mls.check_errors()
            C.values.fill_(float("nan"))
            mls.numeric_noalloc(dA, dB, C)
            torch.cuda.synchronize()
            got = C.values.cpu().numpy()
            assert np.array_equal(got.view(np.int64), ref.cpu().numpy().view(np.int64)), name
            R, _ = oracle.spgemm(A, B)
            rp, ci, _ = C.numpy()
            assert np.array_equal(rp, R.row_ptr) and np.array_equal(ci, R.col_idx), name
            assert np.array_equal(got, R.values), name
    finally:
        mls.set_option(_abi.OPT_FORCE_SPILL, 0)
