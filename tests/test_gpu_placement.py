"""Data placement (Sec. 3.3, Table "gpudp") on the GPU: the numeric phase with
A, B or C (or all three) left in pinned host memory and accessed in place by
the kernels must give the oracle's values bit for bit, as the all-in-HBM run
does (same kernels, same summation order). Inputs: small instances of the
four multigrid stand-ins, R x A and A x P. Also: memory the device cannot
reach (pageable host memory) is refused before anything runs."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from synth import multigrid as mg

pytestmark = pytest.mark.gpu

mls = pytest.importorskip("paper_1804_00695_amd")

PLACEMENTS = {"HBM": (0, 0, 0), "A_Pin": (1, 0, 0), "B_Pin": (0, 1, 0), "C_Pin": (0, 0, 1), "HostPin": (1, 1, 1)}


def device(M):
    return mls.DeviceCsr.from_host(M)


def pinned(M, values=True):
    return mls.HostCsr.from_host(M, values=values)


@pytest.fixture(scope="module")
def products():
    out = {}
    for name, n in (("laplace3d", 10), ("bigstar2d", 30), ("brick3d", 9), ("elasticity3d", 6)):
        A, P, R = (M.to_csr() for M in mg.problem(name, n))
        out[(name, "RxA")] = (R, A)
        out[(name, "AxP")] = (A, P)
    return out


@pytest.mark.parametrize("name", list(mg.PROBLEMS))
@pytest.mark.parametrize("prod", ["RxA", "AxP"])
def test_placements_match_oracle(products, name, prod):
    L, Rt = products[(name, prod)]
    ref, _ = oracle.spgemm(L, Rt)
    for label, (pa, pb, pc) in PLACEMENTS.items():
        print(f"placement {name} {prod} {label}", flush=True)
        dA = pinned(L) if pa else device(L)
        dB = pinned(Rt) if pb else device(Rt)
        Cs = synth.Csr(ref.nrows, ref.ncols, ref.row_ptr, ref.col_idx, np.full(ref.nnz, np.nan))
        dC = pinned(Cs) if pc else device(Cs)
        bits = mls.numeric_placed(dA, dB, dC)
        torch.cuda.synchronize()
        mls.check_errors()
        assert bits == pa | (pb << 1) | (pc << 2), (label, bits)
        v = dC.values.cpu().numpy() if not pc else dC.values.numpy()
        assert np.array_equal(v, ref.values), (name, prod, label)


def test_pageable_and_host_workspace_refused():
    A = synth.poisson_csr(100, 80, 3.0, 1)
    B = synth.poisson_csr(80, 60, 3.0, 2)
    ref, _ = oracle.spgemm(A, B)
    dA, dB = device(A), device(B)
    dC = device(synth.Csr(ref.nrows, ref.ncols, ref.row_ptr, ref.col_idx, np.zeros(ref.nnz)))
    lib = mls.lib
    nb = ctypes.c_size_t(0)
    ha, hb, hc = dA.handle(), dB.handle(), dC.handle()
    mls.check(lib.spgemm_workspace_size(ctypes.byref(ha), ctypes.byref(hb), ctypes.byref(nb)))
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    wp = (ws.data_ptr() + 255) & ~255
    s = mls.stream_handle()
    # pageable host memory (numpy) as A's values
    pageable = np.ascontiguousarray(A.values)
    hbad = mls.CsrT(A.nrows, A.ncols, A.nnz, ha.row_ptr, ha.col_idx, pageable.ctypes.data)
    bits = ctypes.c_uint32(0)
    st = lib.spgemm_numeric_placed(ctypes.byref(hbad), ctypes.byref(hb), ctypes.byref(hc), ctypes.byref(bits),
                                   wp, nb.value, s)
    assert st == 1
    # a pinned host workspace
    wh = torch.empty(nb.value + 256, dtype=torch.uint8, pin_memory=True)
    st = lib.spgemm_numeric_placed(ctypes.byref(ha), ctypes.byref(hb), ctypes.byref(hc), ctypes.byref(bits),
                                   (wh.data_ptr() + 255) & ~255, nb.value, s)
    assert st == 1
    # and the valid call still works afterwards
    st = lib.spgemm_numeric_placed(ctypes.byref(ha), ctypes.byref(hb), ctypes.byref(hc), ctypes.byref(bits),
                                   wp, nb.value, s)
    assert st == 0 and bits.value == 0
    torch.cuda.synchronize()
    assert np.array_equal(dC.values.cpu().numpy(), ref.values)
