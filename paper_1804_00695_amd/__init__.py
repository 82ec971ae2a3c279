"""MI355X (gfx950) two-phase SpGEMM with HBM / pinned-host chunking.

Thin Python layer over the C ABI in include/mlspgemm.h: it allocates device
memory and workspaces with PyTorch, passes raw pointers and the current HIP
stream, and maps status codes to exceptions. Every step of the computation
runs in the HIP library (libmlspgemm.so); there is no CPU fallback -- if the
library is missing, importing this package raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _abi
from ._abi import CsrT, SpgemmError, check

lib = _abi.load()

__all__ = ["DeviceCsr", "HostCsr", "lib", "SpgemmError", "Workspace", "set_option", "get_option",
           "row_work", "compress", "symbolic", "numeric", "spgemm", "stream_handle"]


def stream_handle(stream: Optional[torch.cuda.Stream] = None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def set_option(opt: int, value: int):
    check(lib.spgemm_set_option(opt, value), "spgemm_set_option")


def get_option(opt: int) -> int:
    return lib.spgemm_get_option(opt)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None or t.numel() == 0 else t.data_ptr()


def _check_array(t, name: str, dtype, numel: int, where: str):
    """The array the kernels will read or write: right dtype, memory kind and
    length, contiguous. `where` is "cuda" (device memory) or "pinned" (page-
    locked host memory). Raises ValueError before any library call."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if where == "cuda" and t.device.type != "cuda":
        raise ValueError(f"{name}: on {t.device}, expected a GPU tensor")
    if where == "pinned" and (t.device.type != "cpu" or (t.numel() > 0 and not t.is_pinned())):
        raise ValueError(f"{name}: expected pinned host memory (torch pin_memory)")
    if not t.is_contiguous():
        raise ValueError(f"{name}: not contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")


def _check_csr(M, where: str, need_values: bool = False):
    if M.nrows < 0 or M.ncols < 0:
        raise ValueError(f"negative shape {M.nrows} x {M.ncols}")
    _check_array(M.row_ptr, "row_ptr", torch.int32, M.nrows + 1, where)
    nnz = int(M.col_idx.numel()) if isinstance(M.col_idx, torch.Tensor) else -1
    _check_array(M.col_idx, "col_idx", torch.int32, nnz, where)
    if M.values is not None:
        _check_array(M.values, "values", torch.float64, nnz, where)
    elif need_values and nnz > 0:
        raise ValueError("values are required here")
    if where == "cuda" and M.row_ptr.device != M.col_idx.device:
        raise ValueError("row_ptr and col_idx on different devices")


@dataclass
class DeviceCsr:
    """CSR matrix in device memory (int32 indices, fp64 values or None)."""
    nrows: int
    ncols: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    values: Optional[torch.Tensor]

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    def __setattr__(self, name, value):
        # any change of a field drops the checked handle
        object.__setattr__(self, name, value)
        if name != "_handle":
            object.__setattr__(self, "_handle", None)

    def handle(self) -> CsrT:
        """C handle; checks dtypes, device, contiguity and lengths the first
        time (and again after a field is reassigned). Tensors resized in place
        after that are not seen: build a new DeviceCsr instead."""
        h = self.__dict__.get("_handle")
        if h is None:
            _check_csr(self, "cuda")
            h = CsrT(self.nrows, self.ncols, self.nnz, _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.values))
            object.__setattr__(self, "_handle", h)
        return h

    @classmethod
    def from_host(cls, M, device="cuda", values: bool = True) -> "DeviceCsr":
        """From any object with nrows, ncols, row_ptr, col_idx, values (numpy)."""
        rp = torch.from_numpy(np.ascontiguousarray(M.row_ptr, dtype=np.int32)).to(device)
        ci = torch.from_numpy(np.ascontiguousarray(M.col_idx, dtype=np.int32)).to(device)
        v = None
        if values and getattr(M, "values", None) is not None:
            v = torch.from_numpy(np.ascontiguousarray(M.values, dtype=np.float64)).to(device)
        return cls(int(M.nrows), int(M.ncols), rp, ci, v)

    def numpy(self):
        v = None if self.values is None else self.values.cpu().numpy()
        return self.row_ptr.cpu().numpy(), self.col_idx.cpu().numpy(), v


@dataclass
class HostCsr:
    """CSR matrix in pinned host memory (the slow tier of the chunked path)."""
    nrows: int
    ncols: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    values: Optional[torch.Tensor]

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    def handle(self) -> CsrT:
        """C handle; checks dtypes, pinning, contiguity and lengths first."""
        _check_csr(self, "pinned")
        return CsrT(self.nrows, self.ncols, self.nnz, _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.values))

    @classmethod
    def from_host(cls, M, values: bool = True) -> "HostCsr":
        def pin(a, dt):
            t = torch.empty(len(a), dtype=dt, pin_memory=True)
            t.copy_(torch.from_numpy(np.ascontiguousarray(a)))
            return t
        rp = pin(np.asarray(M.row_ptr, dtype=np.int32), torch.int32)
        ci = pin(np.asarray(M.col_idx, dtype=np.int32), torch.int32)
        v = None
        if values and getattr(M, "values", None) is not None:
            v = pin(np.asarray(M.values, dtype=np.float64), torch.float64)
        return cls(int(M.nrows), int(M.ncols), rp, ci, v)


class Workspace:
    """A 256-byte aligned device scratch buffer, grown on demand."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None
        self.nbytes = 0

    def get(self, nbytes: int) -> int:
        if self.buf is None or self.nbytes < nbytes:
            self.buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=self.device)
            self.nbytes = int(nbytes)
        p = self.buf.data_ptr()
        return (p + 255) & ~255


_default_ws = {}


def _ws(ws: Optional[Workspace], device) -> Workspace:
    if ws is not None:
        return ws
    d = torch.device(device)
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    key = str(d)
    if key not in _default_ws:
        _default_ws[key] = Workspace(device)
    return _default_ws[key]


def workspace_size(A: DeviceCsr, B: DeviceCsr) -> int:
    n = ctypes.c_size_t(0)
    check(lib.spgemm_workspace_size(ctypes.byref(A.handle()), ctypes.byref(B.handle()), ctypes.byref(n)),
          "spgemm_workspace_size")
    return n.value


def row_work(A: DeviceCsr, B: DeviceCsr, ws: Optional[Workspace] = None):
    """Per-row multiply-add counts (int32 tensor) and their int64 total."""
    dev = A.row_ptr.device
    w = _ws(ws, dev)
    nb = workspace_size(A, B)
    out = torch.empty(max(A.nrows, 1), dtype=torch.int32, device=dev)
    tot = ctypes.c_int64(0)
    check(lib.spgemm_row_work(ctypes.byref(A.handle()), ctypes.byref(B.handle()), out.data_ptr(),
                              ctypes.byref(tot), w.get(nb), nb, stream_handle()), "spgemm_row_work")
    return out[:A.nrows], tot.value


def compress(B: DeviceCsr):
    """Compressed rows of B: (words uint32 [2*nnz] as int32 tensor, count int32 [nrows])."""
    dev = B.row_ptr.device
    words = torch.empty(max(2 * B.nnz, 2), dtype=torch.int32, device=dev)
    count = torch.empty(max(B.nrows, 1), dtype=torch.int32, device=dev)
    check(lib.spgemm_compress(ctypes.byref(B.handle()), words.data_ptr(), count.data_ptr(), None, 0,
                              stream_handle()), "spgemm_compress")
    return words[:2 * B.nnz], count[:B.nrows]


def symbolic(A: DeviceCsr, B: DeviceCsr, ws: Optional[Workspace] = None, with_values: bool = True) -> DeviceCsr:
    """Symbolic phase: structure of C = A*B (count pass, allocation, fill pass)."""
    dev = A.row_ptr.device
    w = _ws(ws, dev)
    nb = workspace_size(A, B)
    p = w.get(nb)
    crp = torch.empty(A.nrows + 1, dtype=torch.int32, device=dev)
    nnz = ctypes.c_int64(0)
    ha, hb = A.handle(), B.handle()
    s = stream_handle()
    check(lib.spgemm_symbolic(ctypes.byref(ha), ctypes.byref(hb), crp.data_ptr(), None, ctypes.byref(nnz), p, nb, s),
          "spgemm_symbolic(count)")
    cci = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)
    check(lib.spgemm_symbolic(ctypes.byref(ha), ctypes.byref(hb), crp.data_ptr(), cci.data_ptr(), None, p, nb, s),
          "spgemm_symbolic(fill)")
    vals = torch.empty(max(nnz.value, 1), dtype=torch.float64, device=dev) if with_values else None
    return DeviceCsr(A.nrows, B.ncols, crp, cci[:nnz.value], None if vals is None else vals[:nnz.value])


def symbolic_chunked(A, B, budget: int, ws: Optional[Workspace] = None, device="cuda"):
    """Structure of C = A*B under an HBM budget (bytes of device workspace):
    A and B are host CSR (numpy arrays: row_ptr, col_idx); returns host
    (row_ptr, col_idx) of C. B's compressed pattern stays in HBM while row
    parts of A stream through."""
    def host(M):
        rp = np.ascontiguousarray(M.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(M.col_idx, dtype=np.int32)
        return CsrT(int(M.nrows), int(M.ncols), int(rp[-1]), rp.ctypes.data, ci.ctypes.data if ci.size else None,
                    None), (rp, ci)
    ha, keep_a = host(A)
    hb, keep_b = host(B)
    w = _ws(ws, device)
    p = w.get(int(budget))
    s = stream_handle()
    crp = np.zeros(int(A.nrows) + 1, dtype=np.int32)
    nnz = ctypes.c_int64(0)
    check(lib.spgemm_symbolic_chunked(ctypes.byref(ha), ctypes.byref(hb), crp.ctypes.data, None, ctypes.byref(nnz),
                                      p, int(budget), s), "spgemm_symbolic_chunked(count)")
    cci = np.zeros(max(nnz.value, 1), dtype=np.int32)
    check(lib.spgemm_symbolic_chunked(ctypes.byref(ha), ctypes.byref(hb), crp.ctypes.data, cci.ctypes.data, None,
                                      p, int(budget), s), "spgemm_symbolic_chunked(fill)")
    return crp, cci[:nnz.value]


def numeric(A: DeviceCsr, B: DeviceCsr, C: DeviceCsr, ws: Optional[Workspace] = None) -> DeviceCsr:
    """Numeric phase: fills C.values on C's structure."""
    dev = A.row_ptr.device
    w = _ws(ws, dev)
    nb = workspace_size(A, B)
    if C.values is None:
        C.values = torch.empty(C.nnz, dtype=torch.float64, device=dev)
    check(lib.spgemm_numeric(ctypes.byref(A.handle()), ctypes.byref(B.handle()), ctypes.byref(C.handle()),
                             w.get(nb), nb, stream_handle()), "spgemm_numeric")
    return C


def numeric_placed(A, B, C, ws: Optional[Workspace] = None, device="cuda") -> int:
    """Numeric phase with each of A, B, C either a DeviceCsr (HBM) or a HostCsr
    (pinned host memory read and written in place by the kernels, no copy).
    C.values must be allocated where C lives. Returns the placement bits the
    library found (1 = A, 2 = B, 4 = C in host memory)."""
    if C.values is None:
        raise ValueError("numeric_placed writes into C.values, which must be allocated")
    if A.values is None or B.values is None:
        raise ValueError("numeric_placed needs the values of A and B")
    w = _ws(ws, device)
    sizes = ctypes.c_size_t(0)
    ha, hb, hc = A.handle(), B.handle(), C.handle()
    # the workspace depends on shapes and entry counts only
    check(lib.spgemm_workspace_size(ctypes.byref(ha), ctypes.byref(hb), ctypes.byref(sizes)), "spgemm_workspace_size")
    bits = ctypes.c_uint32(0)
    check(lib.spgemm_numeric_placed(ctypes.byref(ha), ctypes.byref(hb), ctypes.byref(hc), ctypes.byref(bits),
                                    w.get(sizes.value), sizes.value, stream_handle()), "spgemm_numeric_placed")
    return bits.value


def numeric_noalloc(A: DeviceCsr, B: DeviceCsr, C: DeviceCsr) -> DeviceCsr:
    """Numeric phase without a workspace: the library's fixed device scratch
    array (for callers that cannot allocate). C.values must be allocated."""
    if C.values is None:
        raise ValueError("numeric_noalloc writes into C.values, which must be allocated")
    check(lib.spgemm_numeric_noalloc(ctypes.byref(A.handle()), ctypes.byref(B.handle()), ctypes.byref(C.handle()),
                                     stream_handle()), "spgemm_numeric_noalloc")
    return C


def check_errors(ws: Optional[Workspace] = None, device="cuda"):
    w = _ws(ws, device)
    check(lib.spgemm_check_errors(w.get(0), w.nbytes, stream_handle()), "spgemm_check_errors")


def spgemm(A: DeviceCsr, B: DeviceCsr, ws: Optional[Workspace] = None) -> DeviceCsr:
    """C = A*B, both phases."""
    C = symbolic(A, B, ws)
    return numeric(A, B, C, ws)


# ---------------------------------------------------------------------------
# chunked execution (host pinned A, B, C; HBM budget)

class Plan:
    """Alg. "chunker" decision for one product (owns the C plan object)."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep
        self._destroy = lib.spgemm_plan_destroy   # still bound at interpreter exit

    def __del__(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None

    @property
    def info(self) -> dict:
        inf = _abi.PlanInfo()
        check(lib.spgemm_plan_info_get(self._h, ctypes.byref(inf)), "spgemm_plan_info_get")
        return {f: getattr(inf, f) for f, _ in _abi.PlanInfo._fields_}

    def parts(self, which: int):
        n = self.info["n_ac_parts" if which == 0 else "n_b_parts"]
        arr = np.zeros(2 * max(n, 1), dtype=np.int32)
        check(lib.spgemm_plan_parts(self._h, which, arr.ctypes.data, n), "spgemm_plan_parts")
        return [(int(arr[2 * i]), int(arr[2 * i + 1])) for i in range(n)]

    def steps(self):
        n = self.info["n_steps"]
        arr = (_abi.PlanStep * max(n, 1))()
        check(lib.spgemm_plan_steps(self._h, arr, n), "spgemm_plan_steps")
        return [(s.kind, s.matrix, s.part, s.row_begin, s.row_end, int(s.bytes), s.slot) for s in arr[:n]]


def chunked_plan(a_row_ptr, b_row_ptr, ncols_b: int, c_row_ptr, budget: int, nbuf: int = 2,
                 min_parts: int = 1, knl: bool = False) -> Plan:
    """Partition A/C and B into row parts for an HBM budget (host only, no GPU).
    knl=True: Alg. "chunkknl" (only B is cut; A and C are used in place)."""
    arp = np.ascontiguousarray(a_row_ptr, dtype=np.int32)
    brp = np.ascontiguousarray(b_row_ptr, dtype=np.int32)
    crp = np.ascontiguousarray(c_row_ptr, dtype=np.int32)
    nA, nB = len(arp) - 1, len(brp) - 1
    ha = CsrT(nA, nB, int(arp[-1]), arp.ctypes.data, None, None)
    hb = CsrT(nB, ncols_b, int(brp[-1]), brp.ctypes.data, None, None)
    out = ctypes.c_void_p(0)
    fn = lib.spgemm_chunked_plan_knl if knl else lib.spgemm_chunked_plan
    check(fn(ctypes.byref(ha), ctypes.byref(hb), crp.ctypes.data, int(budget), nbuf, min_parts, ctypes.byref(out)),
          "spgemm_chunked_plan_knl" if knl else "spgemm_chunked_plan")
    return Plan(out.value, (arp, brp, crp))


class ChunkStreams:
    """Compute, host-to-device and device-to-host streams (default priority)."""

    def __init__(self, device="cuda"):
        self.compute = torch.cuda.current_stream(device)
        self.h2d = torch.cuda.Stream(device)
        self.d2h = torch.cuda.Stream(device)


def numeric_chunked(A, B, C, plan: Plan, ws: Optional[Workspace] = None,
                    streams: Optional[ChunkStreams] = None, device="cuda"):
    """Chunked numeric phase: C.values = A*B on C's structure. B (and, for
    Algs. chunk1 / chunk2, A and C) must be HostCsr in pinned host memory;
    under a chunkknl plan A and C are used in place and may be HostCsr or
    DeviceCsr."""
    w = _ws(ws, device)
    nb = plan.info["ws_bytes"]
    st = streams or ChunkStreams(device)
    if not isinstance(B, HostCsr):
        raise ValueError("B must be a HostCsr (pinned host memory)")
    if plan.info["algo"] != 3 and not (isinstance(A, HostCsr) and isinstance(C, HostCsr)):
        raise ValueError("Algs. chunk1 / chunk2 copy A and C from pinned host memory: pass HostCsr")
    check(lib.spgemm_numeric_chunked(ctypes.byref(A.handle()), ctypes.byref(B.handle()), ctypes.byref(C.handle()),
                                     plan._h, w.get(nb), nb, st.compute.cuda_stream, st.h2d.cuda_stream,
                                     st.d2h.cuda_stream), "spgemm_numeric_chunked")
    return C


def chunked_trace(A, B, C, plan: Plan):
    """The operations spgemm_numeric_chunked would queue (recorded, not run;
    no GPU needed). A, B, C: host CSR with numpy arrays (C's values array is
    only used as the base of its host byte ranges). Returns a list of
    (op, kind, stream, event, space, write, lo, hi) tuples."""
    keep = []

    def host(M, values=True):
        rp = np.ascontiguousarray(M.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(M.col_idx, dtype=np.int32)
        v = np.ascontiguousarray(M.values if M.values is not None else np.zeros(len(ci)), dtype=np.float64)
        keep.append((rp, ci, v))
        return CsrT(int(M.nrows), int(M.ncols), int(rp[-1]), rp.ctypes.data, ci.ctypes.data if ci.size else None,
                    v.ctypes.data if v.size else None)
    ha, hb, hc = host(A), host(B), host(C)
    n = ctypes.c_int64(0)
    check(lib.spgemm_numeric_chunked_trace(ctypes.byref(ha), ctypes.byref(hb), ctypes.byref(hc), plan._h, None, 0,
                                           ctypes.byref(n)), "spgemm_numeric_chunked_trace")
    arr = (_abi.TraceEntry * max(n.value, 1))()
    check(lib.spgemm_numeric_chunked_trace(ctypes.byref(ha), ctypes.byref(hb), ctypes.byref(hc), plan._h, arr,
                                           n.value, ctypes.byref(n)), "spgemm_numeric_chunked_trace")
    return [(t.op, t.kind, t.stream, t.event, t.space, t.write, t.lo, t.hi) for t in arr[:n.value]]


# ---------------------------------------------------------------------------
# triangle counting

def tc_lower(G):
    """Host preprocessing: (perm, L) with L the strict lower triangle of G after
    the descending-degree relabelling (ties by ascending id); numpy arrays."""
    rp = np.ascontiguousarray(G.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(G.col_idx, dtype=np.int32)
    n = int(G.nrows)
    h = CsrT(n, n, int(rp[-1]), rp.ctypes.data, ci.ctypes.data if ci.size else None, None)
    perm = np.empty(max(n, 1), dtype=np.int32)
    lrp = np.empty(n + 1, dtype=np.int32)
    lci = np.empty(max(int(rp[-1]) // 2, 1), dtype=np.int32)
    nnz = ctypes.c_int64(0)
    check(lib.spgemm_tc_lower(ctypes.byref(h), perm.ctypes.data, lrp.ctypes.data, lci.ctypes.data, ctypes.byref(nnz)),
          "spgemm_tc_lower")
    return perm[:n], (n, lrp, lci[:nnz.value].copy())


def triangle_count(L: DeviceCsr, ws: Optional[Workspace] = None):
    """Masked product (L * compressed(L)) o L: per-row int64 counts and the total."""
    dev = L.row_ptr.device
    w = _ws(ws, dev)
    h = L.handle()
    n = ctypes.c_size_t(0)
    check(lib.spgemm_tc_workspace_size(ctypes.byref(h), ctypes.byref(n)), "spgemm_tc_workspace_size")
    counts = torch.empty(max(L.nrows, 1), dtype=torch.int64, device=dev)
    tot = ctypes.c_int64(0)
    check(lib.spgemm_tc(ctypes.byref(h), counts.data_ptr(), ctypes.byref(tot), w.get(n.value), n.value,
                        stream_handle()), "spgemm_tc")
    return counts[:L.nrows], tot.value


# ---------------------------------------------------------------------------
# adjoint (backward) and its unfused per-call counterpart

def backward_workspace_size(A: DeviceCsr, B: DeviceCsr, W: DeviceCsr, deterministic: bool = False) -> int:
    n = ctypes.c_size_t(0)
    check(lib.spgemm_backward_workspace_size(ctypes.byref(A.handle()), ctypes.byref(B.handle()),
                                             ctypes.byref(W.handle()), int(deterministic), ctypes.byref(n)),
          "spgemm_backward_workspace_size")
    return n.value


def backward(A: DeviceCsr, B: DeviceCsr, W: DeviceCsr, need_a: bool = True, need_b: bool = True,
             ws: Optional[Workspace] = None, deterministic: bool = False, check_structure: bool = True):
    """Fused adjoint of sum(W o (A*B)): (dA values on pat(A), dB values on pat(B)).

    deterministic: dB by a gather over the transpose of A (each entry's terms in
    ascending row order, repeatable bit for bit) instead of device atomics.
    check_structure: read the device error word back afterwards (one 4-byte
    copy and a stream synchronisation) and raise when W misses a column of
    A*B."""
    dev = A.row_ptr.device
    w = _ws(ws, dev)
    ha, hb, hw = A.handle(), B.handle(), W.handle()
    if A.values is None or B.values is None or W.values is None:
        raise ValueError("backward needs the values of A, B and W")
    nb = backward_workspace_size(A, B, W, deterministic)
    dA = torch.empty(max(A.nnz, 1), dtype=torch.float64, device=dev) if need_a else None
    dB = torch.empty(max(B.nnz, 1), dtype=torch.float64, device=dev) if need_b else None
    p = w.get(nb)
    check(lib.spgemm_backward(ctypes.byref(ha), ctypes.byref(hb), ctypes.byref(hw), _ptr(dA), _ptr(dB),
                              int(deterministic), p, nb, stream_handle()), "spgemm_backward")
    if check_structure:
        check(lib.spgemm_check_errors(p, nb, stream_handle()), "spgemm_backward")
    return (None if dA is None else dA[:A.nnz]), (None if dB is None else dB[:B.nnz])


def transpose(M: DeviceCsr, ws: Optional[Workspace] = None) -> DeviceCsr:
    dev = M.row_ptr.device
    w = _ws(ws, dev)
    n = ctypes.c_size_t(0)
    hm = M.handle()
    check(lib.spgemm_transpose_workspace_size(ctypes.byref(hm), ctypes.byref(n)), "spgemm_transpose_workspace_size")
    T = DeviceCsr(M.ncols, M.nrows, torch.empty(M.ncols + 1, dtype=torch.int32, device=dev),
                  torch.empty(M.nnz, dtype=torch.int32, device=dev),
                  None if M.values is None else torch.empty(M.nnz, dtype=torch.float64, device=dev))
    check(lib.spgemm_transpose(ctypes.byref(hm), ctypes.byref(T.handle()), w.get(n.value), n.value, stream_handle()),
          "spgemm_transpose")
    return T


def mask_gather(X: DeviceCsr, P: DeviceCsr) -> torch.Tensor:
    """Values of X at the entries of pattern P (0 where X has none)."""
    out = torch.empty(max(P.nnz, 1), dtype=torch.float64, device=X.row_ptr.device)
    check(lib.spgemm_mask_gather(ctypes.byref(X.handle()), ctypes.byref(P.handle()), out.data_ptr(), stream_handle()),
          "spgemm_mask_gather")
    return out[:P.nnz]


def backward_unfused(A: DeviceCsr, B: DeviceCsr, W: DeviceCsr, ws: Optional[Workspace] = None):
    """The plain per-call adjoint: dA = (W B^T) o pat(A), dB = (A^T W) o pat(B),
    each through a transpose, a full two-phase product and a masked gather."""
    Bt = transpose(B, ws)
    dA = mask_gather(spgemm(W, Bt, ws), A)
    At = transpose(A, ws)
    dB = mask_gather(spgemm(At, W, ws), B)
    return dA, dB


class SpGEMMFn(torch.autograd.Function):
    """c_values = values of A*B on a fixed structure; differentiable in the
    values of A and B (structures are constants). Both directions read the
    library's device error word back, so a structure of C that misses a
    column A*B reaches raises instead of giving wrong values."""

    @staticmethod
    def forward(ctx, a_values, b_values, A, B, C):
        _check_array(a_values, "a_values", torch.float64, A.nnz, "cuda")
        _check_array(b_values, "b_values", torch.float64, B.nnz, "cuda")
        av, bv = a_values.detach(), b_values.detach()
        A2 = DeviceCsr(A.nrows, A.ncols, A.row_ptr, A.col_idx, av)
        B2 = DeviceCsr(B.nrows, B.ncols, B.row_ptr, B.col_idx, bv)
        C2 = DeviceCsr(C.nrows, C.ncols, C.row_ptr, C.col_idx,
                       torch.empty(C.nnz, dtype=torch.float64, device=a_values.device))
        ws = _ws(None, a_values.device)
        numeric(A2, B2, C2, ws)
        check_errors(ws, a_values.device)
        # saved through autograd, so an in-place change of the inputs after
        # the forward pass is detected instead of silently changing dB / dA
        ctx.save_for_backward(a_values, b_values)
        ctx.shapes = (A, B, C)
        return C2.values

    @staticmethod
    def backward(ctx, grad_c):
        a_values, b_values = ctx.saved_tensors
        A, B, C = ctx.shapes
        A2 = DeviceCsr(A.nrows, A.ncols, A.row_ptr, A.col_idx, a_values.detach())
        B2 = DeviceCsr(B.nrows, B.ncols, B.row_ptr, B.col_idx, b_values.detach())
        W = DeviceCsr(C.nrows, C.ncols, C.row_ptr, C.col_idx, grad_c.contiguous())
        dA, dB = backward(A2, B2, W, need_a=ctx.needs_input_grad[0], need_b=ctx.needs_input_grad[1])
        return dA, dB, None, None, None


def spgemm_autograd(A: DeviceCsr, a_values: torch.Tensor, B: DeviceCsr, b_values: torch.Tensor):
    """Differentiable C = A*B: returns (C structure as DeviceCsr, c_values with grad_fn)."""
    C = symbolic(DeviceCsr(A.nrows, A.ncols, A.row_ptr, A.col_idx, None),
                 DeviceCsr(B.nrows, B.ncols, B.row_ptr, B.col_idx, None), with_values=False)
    cv = SpGEMMFn.apply(a_values, b_values, A, B, C)
    return C, cv


# ---------------------------------------------------------------------------
# batches of independent products

def _handles(mats):
    arr = (CsrT * len(mats))()
    for i, m in enumerate(mats):
        arr[i] = m.handle()
    return arr


def batch_workspace_size(As, Bs, ha=None, hb=None) -> int:
    n = ctypes.c_size_t(0)
    check(lib.spgemm_batch_workspace_size(len(As), _handles(As) if ha is None else ha,
                                          _handles(Bs) if hb is None else hb, ctypes.byref(n)),
          "spgemm_batch_workspace_size")
    return n.value


def _pooled(sizes, dtype, dev, align=64):
    """One allocation holding arrays of the given sizes, each starting at a
    multiple of `align` elements: (buffer, element offsets, exact-size views)."""
    padded = [(z + align - 1) // align * align for z in sizes]
    offs = np.concatenate([[0], np.cumsum(padded)]).astype(np.int64)
    buf = torch.empty(max(int(offs[-1]), 1), dtype=dtype, device=dev)
    parts = []
    for z, pz in zip(sizes, padded):
        parts += [z, pz - z]
    tail = buf.numel() - int(offs[-1])
    views = torch.split(buf, parts + ([tail] if tail else []))[0:2 * len(sizes):2]
    return buf, offs, views


def batch_symbolic(As, Bs, ws: Optional[Workspace] = None, with_values: bool = True):
    """Structures of all C_t = A_t * B_t: one count pass (one readback), one fill pass.
    The outputs' arrays are views into one allocation per array kind."""
    dev = As[0].row_ptr.device
    w = _ws(ws, dev)
    ha, hb = _handles(As), _handles(Bs)
    nb = batch_workspace_size(As, Bs, ha, hb)
    p = w.get(nb)
    nt = len(As)
    rp_buf, rp_off, rps = _pooled([a.nrows + 1 for a in As], torch.int32, dev)
    rp0 = rp_buf.data_ptr()
    hc = (CsrT * nt)()
    for t in range(nt):
        q = rp0 + 4 * int(rp_off[t])
        hc[t] = CsrT(As[t].nrows, Bs[t].ncols, 0, q, q, None)
    nnz = (ctypes.c_int64 * nt)()
    check(lib.spgemm_batch_symbolic(nt, ha, hb, hc, 0, nnz, p, nb, stream_handle()),
          "spgemm_batch_symbolic(count)")
    zs = [int(z) for z in nnz]
    ci_buf, ci_off, cis = _pooled(zs, torch.int32, dev)
    vs = [None] * nt
    v0 = 0
    if with_values:
        v_buf, _, vs = _pooled(zs, torch.float64, dev)
        v0 = v_buf.data_ptr()
    c0 = ci_buf.data_ptr()
    for t in range(nt):
        hc[t].nnz = zs[t]
        hc[t].col_idx = c0 + 4 * int(ci_off[t])
        hc[t].values = (v0 + 8 * int(ci_off[t])) if with_values else None
    check(lib.spgemm_batch_symbolic(nt, ha, hb, hc, 1, None, p, nb, stream_handle()),
          "spgemm_batch_symbolic(fill)")
    return [DeviceCsr(a.nrows, b.ncols, rps[t], cis[t], vs[t]) for t, (a, b) in enumerate(zip(As, Bs))]


def batch_numeric(As, Bs, Cs, ws: Optional[Workspace] = None):
    dev = As[0].row_ptr.device
    w = _ws(ws, dev)
    ha, hb = _handles(As), _handles(Bs)
    nb = batch_workspace_size(As, Bs, ha, hb)
    check(lib.spgemm_batch_numeric(len(As), ha, hb, _handles(Cs), w.get(nb), nb, stream_handle()),
          "spgemm_batch_numeric")
    return Cs


class BatchPlan:
    """Reusable numeric plan over a batch with fixed structure (HIP graph replay).

    Owns its own workspace: the binning lives there between runs."""

    def __init__(self, As, Bs, Cs, group_size: int = 0, use_graph: bool = True, tune_cache: Optional[str] = None):
        dev = As[0].row_ptr.device
        self.ws = Workspace(dev)
        self._destroy = lib.spgemm_batch_plan_destroy   # still bound at interpreter exit
        nb = batch_workspace_size(As, Bs)
        self._keep = (As, Bs, Cs, _handles(As), _handles(Bs), _handles(Cs))
        out = ctypes.c_void_p(0)
        path = None if tune_cache is None else str(tune_cache).encode()
        check(lib.spgemm_batch_plan_create(len(As), self._keep[3], self._keep[4], self._keep[5], group_size,
                                           1 if use_graph else 0, path, self.ws.get(nb), nb, stream_handle(),
                                           ctypes.byref(out)), "spgemm_batch_plan_create")
        self._h = out.value

    @property
    def group_size(self) -> int:
        return lib.spgemm_batch_plan_group_size(self._h)

    @property
    def schedule(self):
        """(lanes per row of the first LDS class, of the second, row-bin floor)."""
        g1, g2, fl = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        check(lib.spgemm_batch_plan_schedule(self._h, ctypes.byref(g1), ctypes.byref(g2), ctypes.byref(fl)),
              "spgemm_batch_plan_schedule")
        return g1.value, g2.value, fl.value

    def run(self):
        check(lib.spgemm_batch_plan_run(self._h, stream_handle()), "spgemm_batch_plan_run")

    def __del__(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None
