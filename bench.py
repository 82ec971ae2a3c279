"""Benchmark of the two-phase SpGEMM hot path on one MI355X.

Headline workload: C = A*A with A the 27-point stencil on a 128^3 grid
(2,097,152 rows, 55,742,968 entries), fp64 values: diagonal 26, off-diagonals
-(1 + U(-0.1, 0.1)) (seed 2), int32 CSR indices. One step is one pass of the
whole plain path in HBM: symbolic count (validation, binning, column
compression, LDS hash union, scan, nnz readback), symbolic fill (sorted
columns) and numeric (ordered LDS hash accumulation). Inputs are resident in
HBM before timing; output buffers are reused between steps. The timed steps
run with no instrumentation; kernel times come from a separate pass with the
library's per-launch event pairs on.

Printed as one JSON line. ``value`` = 2 * multiply-adds / time per step
(GFLOP/s). ``roofline`` covers the dominant kernel, the numeric LDS kernel of
the class holding the rows. Its ``achieved`` rate is the algorithmic byte
model of the numeric phase over that kernel's average duration: A streamed,
the two row pointers of B_k and the entries of B_k gathered for every entry of
A (12 bytes per multiply-add, counted whether the gather hits a cache or HBM),
C's structure read and its values written. Beside it: the compulsory bytes
(A, B and C each touched once) and, from the committed rocprofv3 counter
summary when it was taken on the current kernel source, the HBM traffic the
counters measured (``traffic``) and its rate as a fraction of peak.

``parity`` compares every configuration's outputs with the CPU oracle on the
same inputs, after the timed region: structure and values bit for bit where
the method fixes the order of the sums, within the stated tolerance where it
does not (the atomic adjoint). ``cpu_baseline`` times the oracle on the whole
headline product (the same run that the parity check uses).

The other parts of the metric are measured too (``extras``), unless --quick:
  tc       : triangle counting on R-MAT scale 22 (edge factor 16, seed 3);
  chunked  : the numeric phase with A, B, C in pinned host memory under HBM
             budgets of 8 GB, 2 GB, 512 MB and 256 MB, pipelined (2, 3, 4
             buffers), in the paper's single-buffered mode, and under
             Alg. chunkknl (only B copied; A and C used in place, in pinned
             host memory or in HBM), end to end including copies;
  batched  : 256 Galerkin products Ac = P^T (A P) on 7-point Laplacians
             (n ~ U{16..64}, seed 4): batched two-stage pipeline and numeric
             graph replay against 256 separate calls per stage;
  backward : 1M x 1M random CSR, Poisson(8) rows (seeds 5, 6; W seed 7):
             forward numeric, fused adjoint, deterministic adjoint, and the
             unfused per-call adjoint;
  power_law: C = A*A and its adjoint on R-MAT scale 16 (spill paths).
--workload NAME runs one of them alone (for profiling).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
                       [--workload all|spgemm|tc|chunked|batched|backward|power_law]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "num_lds_stencil27_128_traffic.txt")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def csr_bytes(nrows, nnz):
    return 4 * (nrows + 1) + 12 * nnz


def numeric_model_bytes(nrows_a, nnz_a, madds, nnz_c):
    """Byte model of the numeric phase: A streamed, the two row pointers of
    B_k gathered per entry of A, 12 bytes per multiply-add of gathered B, C's
    structure read and its values written."""
    return csr_bytes(nrows_a, nnz_a) + 8 * nnz_a + 12 * madds + csr_bytes(nrows_a, nnz_c)


def frac(nbytes, ms):
    return round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if ms > 0 else None


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("k_numeric.hip", "common.h", "postab.h"):
        with open(os.path.join(ROOT, "paper_1804_00695_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic():
    """HBM bytes per launch of the numeric kernel from the committed counter
    summary, if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    kv = {}
    for line in open(TRAFFIC_SUMMARY):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return int(float(kv["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def profile_table(mls):
    n = mls.lib.spgemm_profile_read(None, 0)
    arr = (mls._abi.ProfileEntry * max(n, 1))()
    n = mls.lib.spgemm_profile_read(arr, n)
    return {arr[i].name.decode(): (arr[i].calls, arr[i].total_ms) for i in range(n)}


def profiled(torch, mls, fn, reps):
    """Per-kernel (calls, total ms) over `reps` calls of fn with the library's
    per-launch event pairs on (a separate pass from the timed ones)."""
    torch.cuda.synchronize()
    mls.lib.spgemm_profile_reset()
    mls.set_option(mls._abi.OPT_PROFILE, 1)
    try:
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
    finally:
        mls.set_option(mls._abi.OPT_PROFILE, 0)
    return profile_table(mls)


def kernels_ms(prof, reps, prefixes):
    """Summed kernel time per call of the kernels whose names start with one
    of the prefixes."""
    return sum(t for k, (c, t) in prof.items() if k.startswith(prefixes)) / reps


def kernel_dict(prof, reps):
    return {k: {"calls_per_rep": round(c / reps, 2), "avg_ms": round(t / c, 4)} for k, (c, t) in sorted(prof.items())}


def timed(torch, fn, reps, pre=None):
    """Median and best of per-repetition times (ms), each bracketed by syncs;
    `pre` (untimed) runs before every repetition."""
    out = []
    for _ in range(reps):
        if pre is not None:
            pre()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(out)), float(np.min(out))


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_threads():
    return min(16, os.cpu_count() or 1)


class Flush:
    """Writes a 512 MB buffer so that the next repetition does not find its
    inputs in the last-level cache (MALL)."""

    def __init__(self, torch):
        self.buf = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        self.k = 0

    def __call__(self):
        self.k = (self.k + 1) & 0xff
        self.buf.fill_(self.k)


def same_bits(x, y):
    x, y = np.asarray(x), np.asarray(y)
    if x.shape != y.shape or x.dtype != y.dtype:
        return False
    if x.dtype == np.float64:
        return bool(np.array_equal(x.view(np.int64), y.view(np.int64)))
    return bool(np.array_equal(x, y))


def within(x, ref, scale, tol):
    return bool(np.all(np.abs(np.asarray(x) - ref) <= tol * scale + 1e-300))


def pcie_peak(torch):
    """Pinned host <-> HBM copy rates (GB/s): each direction alone, then both at
    once on two streams (1 GiB each)."""
    nbytes = 1 << 30
    h_src = torch.empty(nbytes, dtype=torch.uint8).pin_memory()
    h_dst = torch.empty(nbytes, dtype=torch.uint8).pin_memory()
    d_a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    d_b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def h2d():
        with torch.cuda.stream(s1):
            d_a.copy_(h_src, non_blocking=True)
        s1.synchronize()

    def d2h():
        with torch.cuda.stream(s2):
            h_dst.copy_(d_b, non_blocking=True)
        s2.synchronize()

    def both():
        with torch.cuda.stream(s1):
            d_a.copy_(h_src, non_blocking=True)
        with torch.cuda.stream(s2):
            h_dst.copy_(d_b, non_blocking=True)
        s1.synchronize()
        s2.synchronize()

    h2d(); d2h()
    t_h, _ = timed(torch, h2d, 3)
    t_d, _ = timed(torch, d2h, 3)
    t_b, _ = timed(torch, both, 3)
    del h_src, h_dst, d_a, d_b
    return {"h2d_GBs": round(nbytes / (t_h * 1e-3) / 1e9, 1), "d2h_GBs": round(nbytes / (t_d * 1e-3) / 1e9, 1),
            "duplex_GBs": round(2 * nbytes / (t_b * 1e-3) / 1e9, 1)}


# ---------------------------------------------------------------------------
# headline: the plain two-phase path on the 27-point stencil square

def bench_headline(torch, mls, synth, args, keep_host, parity):
    n = args.n
    log(f"generating 27-point stencil {n}^3")
    A = synth.stencil27_3d(n, amp=0.1, seed=2)
    madds = (9 * (n - 2) + 8) ** 3
    nnzC = (5 * n - 6) ** 3
    dA = mls.DeviceCsr.from_host(A)
    lib = mls.lib
    hA = dA.handle()
    wsz = mls.workspace_size(dA, dA)
    ws_t = torch.empty(wsz + 256, dtype=torch.uint8, device="cuda")
    ws = (ws_t.data_ptr() + 255) & ~255
    crp = torch.empty(A.nrows + 1, dtype=torch.int32, device="cuda")
    cci = torch.empty(nnzC, dtype=torch.int32, device="cuda")
    cval = torch.empty(nnzC, dtype=torch.float64, device="cuda")
    sh = torch.cuda.current_stream().cuda_stream
    nnz_out = ctypes.c_int64(0)
    hC = mls.CsrT(A.nrows, A.ncols, nnzC, crp.data_ptr(), cci.data_ptr(), cval.data_ptr())

    def step():
        mls.check(lib.spgemm_symbolic(ctypes.byref(hA), ctypes.byref(hA), crp.data_ptr(), None,
                                      ctypes.byref(nnz_out), ws, wsz, sh), "symbolic count")
        if nnz_out.value != nnzC:
            raise RuntimeError(f"nnz(C) {nnz_out.value} != closed form {nnzC}")
        mls.check(lib.spgemm_symbolic(ctypes.byref(hA), ctypes.byref(hA), crp.data_ptr(), cci.data_ptr(),
                                      None, ws, wsz, sh), "symbolic fill")
        mls.check(lib.spgemm_numeric(ctypes.byref(hA), ctypes.byref(hA), ctypes.byref(hC), ws, wsz, sh), "numeric")

    def numeric():
        mls.check(lib.spgemm_numeric(ctypes.byref(hA), ctypes.byref(hA), ctypes.byref(hC), ws, wsz, sh), "numeric")

    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    mls.check(lib.spgemm_check_errors(ws, wsz, sh), "errors")

    # timed region: K steps, no instrumentation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    mls.check(lib.spgemm_check_errors(ws, wsz, sh), "errors")

    # kernel times: a separate pass with the per-launch event pairs on
    preps = max(3, min(args.steps, 10))
    prof = profiled(torch, mls, step, preps)

    # numeric phase alone, with the MALL flushed before every repetition
    flush = Flush(torch)
    ms_numeric, best_numeric = timed(torch, numeric, max(args.steps, 5), pre=flush)
    del flush

    num_kernels = {k: v for k, v in prof.items() if k.startswith("num_")}
    dom_name, (dom_calls, dom_total) = max(num_kernels.items(), key=lambda kv: kv[1][1])
    dom_ms = dom_total / dom_calls
    model = numeric_model_bytes(A.nrows, A.nnz, madds, nnzC)
    compulsory = csr_bytes(A.nrows, A.nnz) * 2 + csr_bytes(A.nrows, nnzC)
    achieved = model / (dom_ms * 1e-3) / 1e9
    traffic = committed_traffic() if n == 128 else None
    sym_ms = kernels_ms(prof, preps, ("sym_",))
    num_ms = kernels_ms(prof, preps, ("num_",))
    step_kernels_ms = kernels_ms(prof, preps, ("",))

    result = {
        "metric": "SpGEMM GFLOP/s (2 flops per multiply-add), two-phase C=A*A, all in HBM",
        "value": round(2.0 * madds / (ms_step * 1e-3) / 1e9, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"27-point stencil {n}^3, C=A*A, fp64 values, int32 CSR", "rows": A.nrows,
                   "nnz_A": A.nnz, "nnz_C": nnzC, "multiply_adds": madds, "parallelism": "none (1 GPU)"},
        "numeric_ms": round(ms_numeric, 4),
        "numeric_gflops": round(2.0 * madds / (ms_numeric * 1e-3) / 1e9, 2),
        "numeric_best_ms": round(best_numeric, 4),
        "kernels_per_step_ms": {"all": round(step_kernels_ms, 4), "symbolic": round(sym_ms, 4),
                                "numeric": round(num_ms, 4)},
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "bytes_model": "A + 8 B per entry of A (row pointers of B_k) + 12 B per multiply-add "
                                    "(gathered B, cache hits included) + C structure read + C values written",
                     "kernel_avg_ms": round(dom_ms, 4), "algorithmic_bytes": model,
                     "compulsory_bytes": compulsory, "compulsory_frac": frac(compulsory, dom_ms),
                     "traffic_frac": frac(traffic, dom_ms) if traffic else None,
                     "numeric_phase_kernels_ms": round(num_ms, 4),
                     "numeric_phase_traffic_frac": frac(traffic, num_ms) if traffic else None,
                     "note": ("model rate above the HBM peak: L2 and MALL reuse serve the gathered rows of B; "
                              "traffic_frac is the counter-measured HBM-side fraction")
                     if achieved > HBM_PEAK_GBS else None},
        "kernels": kernel_dict(prof, preps),
    }
    host = None
    if keep_host or parity:
        host = (crp.cpu().numpy(), cci.cpu().numpy(), cval.cpu().numpy())
    if parity:
        log("parity + cpu baseline (oracle, whole product)")
        result["cpu_baseline"], par = headline_oracle(A, madds, *host)
        result["parity"] = {"cfg2_stencil128": par}
    del ws_t, cci, cval, crp
    torch.cuda.empty_cache()
    return result, A, host, ms_numeric


def headline_oracle(A, madds, rp, ci, v):
    """The oracle on the whole product: timed (cpu_baseline) and compared with
    the GPU's C bit for bit (row_ptr, col_idx, values; the tolerance
    |c - c_ref| <= 1e-12 sum|a||b| is checked where the bits differ)."""
    import oracle
    threads = oracle_threads()
    best, R = None, None
    for _ in range(2):
        R = None
        t0 = time.perf_counter()
        R, _ = oracle.spgemm(A, A, nthreads=threads, with_abs=False)
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    rows1 = np.arange(0, A.nrows, 16, dtype=np.int32)
    t0 = time.perf_counter()
    oracle.spgemm(A, A, rows=rows1, nthreads=1, with_abs=False)
    dt1 = time.perf_counter() - t0
    w = np.diff(A.row_ptr.astype(np.int64))[A.col_idx]
    arow = np.repeat(np.arange(A.nrows), np.diff(A.row_ptr.astype(np.int64)))
    madds1 = int(np.bincount(arow, weights=w, minlength=A.nrows)[rows1].sum())
    cpu = {"value": round(2.0 * madds / best / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
           "sample": f"the whole product ({A.nrows} rows, {madds} multiply-adds), dense-accumulator oracle in C "
                     f"with OpenMP, best of 2 runs: {best:.2f} s",
           "single_thread_value": round(2.0 * madds1 / dt1 / 1e9, 3),
           "single_thread_sample": f"rows 0::16 ({len(rows1)} rows, {madds1} multiply-adds), 1 thread, {dt1:.2f} s",
           "host_cpus": os.cpu_count(), "host_cpu_model": host_cpu_model()}
    par = {"row_ptr": same_bits(rp, R.row_ptr), "col_idx": same_bits(ci, R.col_idx),
           "values_bitwise": same_bits(v, R.values)}
    if par["row_ptr"] and par["col_idx"] and not par["values_bitwise"]:
        R2, cabs = oracle.spgemm(A, A, nthreads=threads, with_abs=True)
        par["values_within_1e-12"] = within(v, R2.values, cabs, 1e-12)
    par["ok"] = par["row_ptr"] and par["col_idx"] and (par["values_bitwise"] or par.get("values_within_1e-12", False))
    return cpu, par


# ---------------------------------------------------------------------------
# chunked (pinned host A, B, C; HBM budget)

def bench_chunked(torch, mls, synth, A, host_c, ms_numeric_hbm):
    """Chunked numeric phase, end to end (copies included), for several budgets:
    Algs. chunk1 / chunk2 pipelined with 2, 3 and 4 inner buffers and in the
    paper's single-buffered mode, and Alg. chunkknl (only B's parts copied)
    with A and C in pinned host memory (used in place) or in HBM; each result
    compared bit for bit with the in-HBM C."""
    C_rp, C_ci, C_v = host_c
    Ah = mls.HostCsr.from_host(A)
    nnzC = len(C_ci)
    Ch = mls.HostCsr(A.nrows, A.ncols, torch.from_numpy(C_rp).pin_memory(),
                     torch.from_numpy(C_ci).pin_memory(), torch.empty(nnzC, dtype=torch.float64).pin_memory())
    Ad = mls.DeviceCsr.from_host(A)
    Cd = mls.DeviceCsr(A.nrows, A.ncols, torch.from_numpy(C_rp).cuda(), torch.from_numpy(C_ci).cuda(),
                       torch.empty(nnzC, dtype=torch.float64, device="cuda"))
    streams = mls.ChunkStreams()
    ws = mls.Workspace()
    peak = pcie_peak(torch)
    out = {"pcie_peak": peak}
    log(f"pcie peak: {peak}")
    ok = True
    modes = (("pipelined", 2, 4, None), ("nbuf3", 3, 4, None), ("nbuf4", 4, 4, None), ("paper", 1, 1, None),
             ("knl_AC_pinned", 2, 2, "pinned"), ("knl_AC_hbm", 2, 2, "hbm"))
    for label, budget in (("8GB", 8 << 30), ("2GB", 2 << 30), ("512MB", 512 << 20), ("256MB", 256 << 20)):
        for mode, nbuf, min_parts, knl in modes:
            plan = mls.chunked_plan(A.row_ptr, A.row_ptr, A.ncols, C_rp, budget, nbuf=nbuf, min_parts=min_parts,
                                    knl=knl is not None)
            a, c = (Ad, Cd) if knl == "hbm" else (Ah, Ch)
            c.values.fill_(float("nan"))
            med, best = timed(torch, lambda: mls.numeric_chunked(a, Ah, c, plan, ws, streams), 3)
            info = plan.info   # after a run: holds the bytes the last run issued
            moved = info["issued_h2d"] + info["issued_d2h"]
            got = c.values.cpu().numpy() if knl == "hbm" else c.values.numpy()
            bit = same_bits(got, C_v)
            ok = ok and bit
            key = label if mode == "pipelined" else f"{label}_{mode}"
            out[key] = {"ms": round(med, 2), "best_ms": round(best, 2),
                        "slowdown_vs_hbm": round(med / ms_numeric_hbm, 2), "mode": mode, "nbuf": nbuf,
                        "min_parts": min_parts, "algo": {1: "chunk1", 2: "chunk2", 3: "chunkknl"}[info["algo"]],
                        "branch": info["branch"], "parts_ac": info["n_ac_parts"], "parts_b": info["n_b_parts"],
                        "h2d_GB": round(info["h2d_bytes"] / 1e9, 3), "d2h_GB": round(info["d2h_bytes"] / 1e9, 3),
                        "issued_equals_plan": info["issued_h2d"] == info["h2d_bytes"] and
                        info["issued_d2h"] == info["d2h_bytes"],
                        "pcie_GBs": round(moved / (med * 1e-3) / 1e9, 1),
                        "link_frac_of_duplex_peak": round(moved / (med * 1e-3) / 1e9 / peak["duplex_GBs"], 3),
                        "bitwise_vs_in_hbm": bit}
            if knl == "pinned":
                out[key]["zero_copy_GB"] = round(info["zero_copy_bytes"] / 1e9, 3)
            log(f"chunked {key}: {out[key]}")
            del plan
    return out, ok


# ---------------------------------------------------------------------------
# batched Galerkin products

def bench_batched(torch, mls, synth, with_parity):
    sizes = synth.amg_batch_sizes(256, 16, 64, seed=4)
    cache, host = {}, {}
    for n in sorted(set(int(x) for x in sizes)):
        A, P, R = synth.amg_instance(n)
        host[n] = (A, P, R)
        cache[n] = tuple(mls.DeviceCsr.from_host(M) for M in (A, P, R))
    As = [cache[int(n)][0] for n in sizes]
    Ps = [cache[int(n)][1] for n in sizes]
    Rs = [cache[int(n)][2] for n in sizes]
    ws = mls.Workspace()

    def per_call():
        for a, p, r in zip(As, Ps, Rs):
            ap = mls.spgemm(a, p, ws)
            mls.spgemm(r, ap, ws)

    def batched():
        APs = mls.batch_symbolic(As, Ps, ws)
        mls.batch_numeric(As, Ps, APs, ws)
        Acs = mls.batch_symbolic(Rs, APs, ws)
        mls.batch_numeric(Rs, APs, Acs, ws)
        return APs, Acs

    log("batched: inputs ready; per-call path")
    per_call()
    t_call, _ = timed(torch, per_call, 3)
    log("batched: per-call timed")
    APs, Acs = batched()
    t_batch, _ = timed(torch, batched, 3)
    # the stages one at a time
    t_sym1, _ = timed(torch, lambda: mls.batch_symbolic(As, Ps, ws), 3)
    t_num1, _ = timed(torch, lambda: mls.batch_numeric(As, Ps, APs, ws), 3)
    t_sym2, _ = timed(torch, lambda: mls.batch_symbolic(Rs, APs, ws), 3)
    t_num2, _ = timed(torch, lambda: mls.batch_numeric(Rs, APs, Acs, ws), 3)
    plan1 = mls.BatchPlan(As, Ps, APs)
    plan2 = mls.BatchPlan(Rs, APs, Acs)

    def replay():
        plan1.run()
        plan2.run()

    log("batched: stages timed; graph replay next")
    replay()
    t_replay, _ = timed(torch, replay, 5)
    t_rep1, _ = timed(torch, plan1.run, 5)
    t_rep2, _ = timed(torch, plan2.run, 5)

    def numeric_per_call():
        for a, p, r, ap, ac in zip(As, Ps, Rs, APs, Acs):
            mls.numeric(a, p, ap, ws)
            mls.numeric(r, ap, ac, ws)

    numeric_per_call()
    t_num_call, _ = timed(torch, numeric_per_call, 3)
    prof_rep = profiled(torch, mls, lambda: (mls.batch_numeric(As, Ps, APs, ws), mls.batch_numeric(Rs, APs, Acs, ws)),
                        3)
    prof_sym = profiled(torch, mls, lambda: (mls.batch_symbolic(As, Ps, ws), mls.batch_symbolic(Rs, APs, ws)), 3)
    replay()   # the outputs checked below are the graph's
    torch.cuda.synchronize()

    # multiply-adds and model bytes per distinct size, counted once per instance
    per_n = {}
    for n in set(int(x) for x in sizes):
        a, p, r = cache[n]
        _, w1 = mls.row_work(a, p, ws)
        ap = mls.spgemm(a, p, ws)
        _, w2 = mls.row_work(r, ap, ws)
        m1 = numeric_model_bytes(a.nrows, a.nnz, w1, ap.nnz)
        ac_nnz = int(mls.symbolic(r, ap, ws, with_values=False).nnz)
        m2 = numeric_model_bytes(r.nrows, r.nnz, w2, ac_nnz)
        per_n[n] = (w1 + w2, m1, m2)
    madds = sum(per_n[int(n)][0] for n in sizes)
    model1 = sum(per_n[int(n)][1] for n in sizes)
    model2 = sum(per_n[int(n)][2] for n in sizes)
    num_kernels_ms = kernels_ms(prof_rep, 3, ("num_",))
    res = {"instances": 256, "multiply_adds": int(madds),
           "per_call_ms": round(t_call, 2), "batched_ms": round(t_batch, 2),
           "speedup_batched_vs_per_call": round(t_call / t_batch, 2),
           "stage_ms": {"symbolic_AP": round(t_sym1, 3), "numeric_AP": round(t_num1, 3),
                        "symbolic_Ac": round(t_sym2, 3), "numeric_Ac": round(t_num2, 3),
                        "replay_AP": round(t_rep1, 3), "replay_Ac": round(t_rep2, 3)},
           "numeric_per_call_ms": round(t_num_call, 2), "numeric_graph_replay_ms": round(t_replay, 3),
           "speedup_replay_vs_numeric_per_call": round(t_num_call / t_replay, 2),
           "autotuned_schedule_g1_g2_floor": [plan1.schedule, plan2.schedule],
           "replay_gflops": round(2.0 * madds / (t_replay * 1e-3) / 1e9, 1),
           "roofline": {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "bytes_model": "numeric byte model summed over the 512 products",
                        "model_bytes": int(model1 + model2), "model_bytes_AP": int(model1),
                        "model_bytes_Ac": int(model2),
                        "replay_ms": round(t_replay, 3), "frac_replay": frac(model1 + model2, t_replay),
                        "frac_replay_AP": frac(model1, t_rep1), "frac_replay_Ac": frac(model2, t_rep2),
                        "numeric_kernels_ms": round(num_kernels_ms, 3),
                        "frac_numeric_kernels": frac(model1 + model2, num_kernels_ms)},
           "kernels_numeric_stages": kernel_dict(prof_rep, 3),
           "symbolic_stages_kernels_ms": round(kernels_ms(prof_sym, 3, ("",)), 3),
           "kernels_symbolic_stages": kernel_dict(prof_sym, 3)}
    ok = None
    if with_parity:
        import oracle
        ref = {}
        for n, (A, P, R) in host.items():
            AP, _ = oracle.spgemm(A, P, nthreads=oracle_threads(), with_abs=False)
            Ac, _ = oracle.spgemm(R, AP, nthreads=oracle_threads(), with_abs=False)
            ref[n] = (AP, Ac)
        ok = True
        for t, n in enumerate(sizes):
            AP, Ac = ref[int(n)]
            for G, Rf in ((APs[t], AP), (Acs[t], Ac)):
                rp, ci, v = G.numpy()
                ok = ok and same_bits(rp, Rf.row_ptr) and same_bits(ci, Rf.col_idx) and same_bits(v, Rf.values)
        res["parity_all_512_products_bitwise"] = ok
    log(f"batched: {res}")
    return res, ok


# ---------------------------------------------------------------------------
# backward (adjoint)

def bench_backward(torch, mls, synth, with_parity):
    n = 1_000_000
    A = synth.poisson_csr(n, n, 8.0, 5)
    B = synth.poisson_csr(n, n, 8.0, 6)
    dA, dB = mls.DeviceCsr.from_host(A), mls.DeviceCsr.from_host(B)
    ws = mls.Workspace()
    C = mls.symbolic(dA, dB, ws)
    torch.cuda.synchronize()
    Wv = synth.normal_values(C.nnz, 7)
    W = mls.DeviceCsr(C.nrows, C.ncols, C.row_ptr, C.col_idx, torch.from_numpy(Wv).cuda())
    _, madds = mls.row_work(dA, dB, ws)
    log("backward: inputs ready")
    fwd = lambda: mls.numeric(dA, dB, C, ws)
    bwd = lambda: mls.backward(dA, dB, W, ws=ws, check_structure=False)
    det = lambda: mls.backward(dA, dB, W, ws=ws, deterministic=True, check_structure=False)
    unf = lambda: mls.backward_unfused(dA, dB, W, ws)
    fwd(); bwd(); det()
    # B (about 100 MB) fits in the MALL: flush between repetitions
    flush = Flush(torch)
    t_f, _ = timed(torch, fwd, 5, pre=flush)
    t_b, _ = timed(torch, bwd, 5, pre=flush)
    t_d, _ = timed(torch, det, 5, pre=flush)
    t_f_warm, _ = timed(torch, fwd, 5)
    t_b_warm, _ = timed(torch, bwd, 5)
    log("backward: fused timed; unfused per-call path next")
    unf()
    t_u, _ = timed(torch, unf, 2, pre=flush)
    prof_f = profiled(torch, mls, lambda: (flush(), fwd()), 5)
    prof_b = profiled(torch, mls, lambda: (flush(), bwd()), 5)
    prof_d = profiled(torch, mls, lambda: (flush(), det()), 3)
    del flush
    nnzC = C.nnz
    fwd_model = numeric_model_bytes(A.nrows, A.nnz, madds, nnzC)
    # fused adjoint: A and W streamed, B's row pointers and entries gathered
    # per multiply-add as in the forward, dA and dB written once
    bwd_model = csr_bytes(A.nrows, A.nnz) + csr_bytes(C.nrows, nnzC) + 8 * A.nnz + 12 * madds + 8 * A.nnz + 8 * B.nnz
    fk = kernels_ms(prof_f, 5, ("num_", "bin", "scatter"))
    fk_num = kernels_ms(prof_f, 5, ("num_",))
    bk = kernels_ms(prof_b, 5, ("bwd", "bin", "scatter"))
    bk_main = kernels_ms(prof_b, 5, ("bwd",))
    res = {"rows": n, "nnz_A": A.nnz, "nnz_B": B.nnz, "nnz_C": nnzC, "multiply_adds": int(madds),
           "forward_ms": round(t_f, 3), "fused_backward_ms": round(t_b, 3),
           "deterministic_backward_ms": round(t_d, 3),
           "fwd_plus_bwd_over_fwd": round((t_f + t_b) / t_f, 2),
           "forward_warm_ms": round(t_f_warm, 3), "fused_backward_warm_ms": round(t_b_warm, 3),
           "unfused_per_call_backward_ms": round(t_u, 2),
           "speedup_fused_vs_unfused": round(t_u / t_b, 1),
           "roofline": {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "forward_model_bytes": fwd_model, "backward_model_bytes": bwd_model,
                        "forward_kernels_ms": round(fk, 4), "forward_numeric_kernels_ms": round(fk_num, 4),
                        "frac_forward_kernels": frac(fwd_model, fk),
                        "frac_forward_numeric_kernels": frac(fwd_model, fk_num),
                        "frac_forward_call": frac(fwd_model, t_f),
                        "backward_kernels_ms": round(bk, 4), "backward_adjoint_kernels_ms": round(bk_main, 4),
                        "frac_backward_kernels": frac(bwd_model, bk),
                        "frac_backward_adjoint_kernels": frac(bwd_model, bk_main),
                        "frac_backward_call": frac(bwd_model, t_b)},
           "kernels_forward": kernel_dict(prof_f, 5), "kernels_backward": kernel_dict(prof_b, 5),
           "kernels_deterministic": kernel_dict(prof_d, 3)}
    ok = None
    if with_parity:
        import oracle
        fwd(); torch.cuda.synchronize()
        R, _ = oracle.spgemm(A, B, nthreads=oracle_threads(), with_abs=False)
        rp, ci, v = C.numpy()
        f_ok = same_bits(rp, R.row_ptr) and same_bits(ci, R.col_idx) and same_bits(v, R.values)
        Wh = synth.Csr(C.nrows, C.ncols, rp, ci, Wv)
        rA, rB, aA, aB = oracle.backward(A, B, Wh)
        gA, gB = mls.backward(dA, dB, W, ws=ws)
        b_ok = within(gA.cpu().numpy(), rA, aA, 1e-10) and within(gB.cpu().numpy(), rB, aB, 1e-10)
        hA, hB = mls.backward(dA, dB, W, ws=ws, deterministic=True)
        d_ok = same_bits(hA.cpu().numpy(), rA) and same_bits(hB.cpu().numpy(), rB)
        res["parity"] = {"forward_bitwise": f_ok, "fused_within_1e-10": b_ok, "deterministic_bitwise": d_ok}
        ok = f_ok and b_ok and d_ok
    log(f"backward: {res}")
    return res, ok


# ---------------------------------------------------------------------------
# power-law product (spill paths)

def bench_power_law(torch, mls, synth, with_parity):
    """C = A*A and its adjoint for a power-law matrix (R-MAT scale 16, edge
    factor 8, seed 5, symmetric, N(0,1) values): most multiply-adds fall in
    rows of C past the LDS classes, i.e. on the spill paths."""
    G = synth.rmat_graph(16, 8, seed=5)
    A = synth.Csr(G.nrows, G.ncols, G.row_ptr, G.col_idx, synth.normal_values(len(G.col_idx), 8))
    dA = mls.DeviceCsr.from_host(A)
    ws = mls.Workspace()
    C = mls.symbolic(dA, dA, ws)
    torch.cuda.synchronize()
    _, madds = mls.row_work(dA, dA, ws)
    lens = torch.diff(C.row_ptr.long())
    spill_rows = int((lens > 2048).sum().item())
    W = mls.DeviceCsr(C.nrows, C.ncols, C.row_ptr, C.col_idx,
                      torch.from_numpy(synth.normal_values(C.nnz, 9)).cuda())
    t_s, _ = timed(torch, lambda: mls.symbolic(dA, dA, ws), 3)
    t_n, _ = timed(torch, lambda: mls.numeric(dA, dA, C, ws), 3)
    t_b, _ = timed(torch, lambda: mls.backward(dA, dA, W, ws=ws, check_structure=False), 3)
    res = {"workload": "R-MAT scale 16, edge factor 8, seed 5, C = A*A", "rows": A.nrows, "nnz_A": A.nnz,
           "nnz_C": int(C.nnz), "multiply_adds": int(madds), "rows_of_C_past_LDS_classes": spill_rows,
           "symbolic_ms": round(t_s, 3), "numeric_ms": round(t_n, 3), "backward_ms": round(t_b, 3),
           "numeric_gflops": round(2 * madds / (t_n * 1e-3) / 1e9, 1),
           "numeric_frac_model": frac(numeric_model_bytes(A.nrows, A.nnz, madds, int(C.nnz)), t_n)}
    ok = None
    if with_parity:
        import oracle
        mls.numeric(dA, dA, C, ws)
        torch.cuda.synchronize()
        R, _ = oracle.spgemm(A, A, nthreads=oracle_threads(), with_abs=False)
        rp, ci, v = C.numpy()
        ok = same_bits(rp, R.row_ptr) and same_bits(ci, R.col_idx) and same_bits(v, R.values)
        res["parity_bitwise"] = ok
    log(f"power law: {res}")
    return res, ok


# ---------------------------------------------------------------------------
# multigrid stand-ins: data placement (Table "gpudp") and chunk sweeps

MG_NAMES = ("laplace3d", "bigstar2d", "brick3d", "elasticity3d")
PLACEMENTS = (("A_Pin", (1, 0, 0)), ("B_Pin", (0, 1, 0)), ("C_Pin", (0, 0, 1)), ("HostPin", (1, 1, 1)))


def mg_build(mls, name, gb):
    """(grid edge, A, P, R) of a multigrid stand-in with A of about `gb` GB,
    generated on the GPU (positional values: the same matrix on any device)."""
    from synth import multigrid as mg
    n = mg.grid_for_bytes(name, gb * 1e9)
    A, P, R = mg.problem(name, n, device="cuda")
    dev = lambda M: mls.DeviceCsr(M.nrows, M.ncols, M.row_ptr, M.col_idx, M.values)
    return n, dev(A), dev(P), dev(R)


def pinned_copy(torch, mls, D, values=True):
    def pin(t):
        h = torch.empty(t.numel(), dtype=t.dtype, pin_memory=True)
        h.copy_(t)
        return h
    v = pin(D.values) if (values and D.values is not None) else None
    return mls.HostCsr(D.nrows, D.ncols, pin(D.row_ptr), pin(D.col_idx), v)


def host_cache_release(torch):
    """Hand the pinned blocks torch caches back to the system."""
    fn = getattr(torch._C, "_host_emptyCache", None)
    if fn is not None:
        fn()


def dcsr_bytes(M):
    return csr_bytes(M.nrows, M.nnz)


def host_numpy(M):
    import synth
    v = None if M.values is None else M.values.cpu().numpy()
    return synth.Csr(M.nrows, M.ncols, M.row_ptr.cpu().numpy(), M.col_idx.cpu().numpy(), v)


def bench_placement(torch, mls, gb, with_parity, names=MG_NAMES):
    """Table "gpudp" on MI355X: the numeric phase of R x A and A x P with all of
    A, B, C in HBM, then with one of them (or all three) in pinned host memory
    read and written in place by the kernels. Every placement's C is compared
    bit for bit with the all-in-HBM C, and that one with the oracle."""
    ws = mls.Workspace()
    flush = Flush(torch)
    rows, ok = [], True
    for name in names:
        log(f"placement: {name} ({gb} GB A)")
        n, A, P, R = mg_build(mls, name, gb)
        for prod, (L, Rt) in (("RxA", (R, A)), ("AxP", (A, P))):
            C = mls.symbolic(L, Rt, ws)
            _, madds = mls.row_work(L, Rt, ws)
            hbm = lambda: mls.numeric(L, Rt, C, ws)
            hbm()
            t_hbm, b_hbm = timed(torch, hbm, 5, pre=flush)
            ref = C.values.cpu().numpy()
            gfl = lambda ms: round(2.0 * madds / (ms * 1e-3) / 1e9, 2)
            entry = {"problem": name, "product": prod, "grid": n, "multiply_adds": int(madds),
                     "GB": {"A": round(dcsr_bytes(L) / 1e9, 3), "B": round(dcsr_bytes(Rt) / 1e9, 3),
                            "C": round(dcsr_bytes(C) / 1e9, 3)},
                     "GFLOPs": {"HBM": gfl(t_hbm)}, "ms": {"HBM": round(t_hbm, 3)}, "bitwise_vs_HBM": {}}
            hL, hR = pinned_copy(torch, mls, L), pinned_copy(torch, mls, Rt)
            hC = pinned_copy(torch, mls, C)
            for label, (pa, pb, pc) in PLACEMENTS:
                a, b = (hL if pa else L), (hR if pb else Rt)
                c = hC if pc else C
                c.values.fill_(float("nan"))
                fn = lambda: mls.numeric_placed(a, b, c, ws)
                fn()
                t, _ = timed(torch, fn, 2, pre=flush)
                got = c.values.numpy() if pc else c.values.cpu().numpy()
                bit = same_bits(got, ref)
                ok = ok and bit
                entry["GFLOPs"][label] = gfl(t)
                entry["ms"][label] = round(t, 3)
                entry["bitwise_vs_HBM"][label] = bit
            entry["slowdown_vs_HBM"] = {k: round(entry["ms"][k] / entry["ms"]["HBM"], 2) for k, _ in PLACEMENTS}
            if with_parity:
                import oracle
                Rf, _ = oracle.spgemm(host_numpy(L), host_numpy(Rt), nthreads=oracle_threads(), with_abs=False)
                rp, ci = C.row_ptr.cpu().numpy(), C.col_idx.cpu().numpy()
                par = same_bits(rp, Rf.row_ptr) and same_bits(ci, Rf.col_idx) and same_bits(ref, Rf.values)
                entry["oracle_bitwise"] = par
                ok = ok and par
            log(f"placement {name} {prod}: {entry}")
            rows.append(entry)
            del hL, hR, hC, C
        del A, P, R
        torch.cuda.empty_cache()
        host_cache_release(torch)
    return {"gb_of_A": gb, "products": rows}, ok


def bench_mg_sweep(torch, mls, sizes, budgets_gb=(8, 16), names=MG_NAMES, hostpin_max_gb=4.0, reps=2):
    """Figs. "expgpuap" / "expgpura" on MI355X: R x A and A x P on the four
    stand-ins as A grows, all in HBM, all in pinned host memory (zero copy,
    up to hostpin_max_gb), and chunked under HBM budgets of 8 and 16 GB
    (Chunk8, Chunk16; pipelined plan executed, the paper-mode plan reported
    beside it). Every chunked C is compared bit for bit with the in-HBM C."""
    ws = mls.Workspace()
    streams = mls.ChunkStreams()
    flush = Flush(torch)
    rows, ok = [], True
    for name in names:
        for gb in sizes:
            log(f"sweep: {name} {gb} GB")
            n, A, P, R = mg_build(mls, name, gb)
            for prod, (L, Rt) in (("RxA", (R, A)), ("AxP", (A, P))):
                C = mls.symbolic(L, Rt, ws)
                _, madds = mls.row_work(L, Rt, ws)
                hbm = lambda: mls.numeric(L, Rt, C, ws)
                hbm()
                t_hbm, _ = timed(torch, hbm, 3, pre=flush)
                ref = C.values.cpu().numpy()
                gfl = lambda ms: round(2.0 * madds / (ms * 1e-3) / 1e9, 2)
                sA, sB, sC = dcsr_bytes(L), dcsr_bytes(Rt), dcsr_bytes(C)
                entry = {"problem": name, "product": prod, "gb_of_A_target": gb, "grid": n,
                         "GB": {"A": round(sA / 1e9, 3), "B": round(sB / 1e9, 3), "C": round(sC / 1e9, 3)},
                         "multiply_adds": int(madds), "HBM": {"ms": round(t_hbm, 3), "GFLOPs": gfl(t_hbm)}}
                hL, hR, hC = (pinned_copy(torch, mls, M) for M in (L, Rt, C))
                arp, brp, crp = (M.row_ptr.numpy() for M in (hL, hR, hC))
                if gb <= hostpin_max_gb:
                    hC.values.fill_(float("nan"))
                    fn = lambda: mls.numeric_placed(hL, hR, hC, ws)
                    t_pin, _ = timed(torch, fn, 1, pre=flush)
                    bit = same_bits(hC.values.numpy(), ref)
                    ok = ok and bit
                    entry["HostPin"] = {"ms": round(t_pin, 2), "GFLOPs": gfl(t_pin), "bitwise_vs_HBM": bit}
                for bgb in budgets_gb:
                    budget = int(bgb) << 30
                    key = f"Chunk{bgb}"
                    try:
                        paper = mls.chunked_plan(arp, brp, Rt.ncols, crp, budget, nbuf=1, min_parts=1).info
                        plan = mls.chunked_plan(arp, brp, Rt.ncols, crp, budget, nbuf=2, min_parts=4)
                    except mls.SpgemmError as e:
                        entry[key] = {"error": str(e)}
                        continue
                    hC.values.fill_(float("nan"))
                    fn = lambda: mls.numeric_chunked(hL, hR, hC, plan, ws, streams)
                    t, best = timed(torch, fn, reps)
                    info = plan.info
                    bit = same_bits(hC.values.numpy(), ref)
                    ok = ok and bit
                    moved = info["issued_h2d"] + info["issued_d2h"]
                    # A, B and C's structure in once, C's values out once (plus the
                    # duplicated boundary row pointer of each part)
                    compulsory = sA + sB + sC
                    res = {"ms": round(t, 2), "best_ms": round(best, 2), "GFLOPs": gfl(t),
                           "slowdown_vs_HBM": round(t / t_hbm, 2), "algo": f"chunk{info['algo']}",
                           "branch": info["branch"], "parts_ac": info["n_ac_parts"], "parts_b": info["n_b_parts"],
                           "copied_GB": round(moved / 1e9, 3), "link_GBs": round(moved / (t * 1e-3) / 1e9, 1),
                           "bitwise_vs_HBM": bit,
                           "paper_mode_plan": {"algo": f"chunk{paper['algo']}", "branch": paper["branch"],
                                               "parts_ac": paper["n_ac_parts"], "parts_b": paper["n_b_parts"],
                                               "copied_GB": round((paper["h2d_bytes"] + paper["d2h_bytes"]) / 1e9, 3),
                                               "optimal_copy": paper["h2d_bytes"] + paper["d2h_bytes"] - compulsory
                                               <= 8 * (paper["n_ac_parts"] + paper["n_b_parts"]),
                                               "whole_problem_fits": paper["n_ac_parts"] == 1 and paper["n_b_parts"] == 1}}
                    if "HostPin" in entry:
                        res["speedup_vs_HostPin"] = round(entry["HostPin"]["ms"] / t, 2)
                    entry[key] = res
                    del plan
                log(f"sweep {name} {gb} {prod}: {entry}")
                rows.append(entry)
                del hL, hR, hC, C
                host_cache_release(torch)
            del A, P, R
            torch.cuda.empty_cache()
            host_cache_release(torch)
    return {"sizes_gb": list(sizes), "budgets_gb": list(budgets_gb), "runs": rows}, ok


def bench_density(torch, mls, with_parity, n=24, deltas=(1, 4, 16, 64, 256)):
    """Table "expdensity" on MI355X: the elasticity stand-in's R and A times a
    random right-hand side with delta entries per row (as many columns as P),
    numeric phase with everything in HBM, with the right-hand side in pinned
    host memory (B_Pin, read in place), and with all three in pinned host
    memory (HostPin, the analog of the paper's all-in-DDR runs). Every
    placement's C is compared bit for bit with the in-HBM C, and that one with
    the oracle."""
    from synth import multigrid as mg
    ws = mls.Workspace()
    flush = Flush(torch)
    A, P, R = mg.problem("elasticity3d", n, device="cuda")
    dev = lambda M: mls.DeviceCsr(M.nrows, M.ncols, M.row_ptr, M.col_idx, M.values)
    A, R = dev(A), dev(R)
    rows, ok = [], True
    for delta in deltas:
        rhs = dev(mg.random_rhs(A.ncols, P.ncols, delta, seed=100 + delta, device="cuda"))
        for name, L in (("R x RHS", R), ("A x RHS", A)):
            C = mls.symbolic(L, rhs, ws)
            _, madds = mls.row_work(L, rhs, ws)
            hbm = lambda: mls.numeric(L, rhs, C, ws)
            hbm()
            t_hbm, _ = timed(torch, hbm, 5, pre=flush)
            ref = C.values.cpu().numpy()
            gfl = lambda ms: round(2.0 * madds / (ms * 1e-3) / 1e9, 2)
            hL, hB, hC = (pinned_copy(torch, mls, M) for M in (L, rhs, C))
            entry = {"product": name, "delta": delta, "multiply_adds": int(madds), "nnz_C": int(C.nnz),
                     "GFLOPs": {"HBM": gfl(t_hbm)}, "ms": {"HBM": round(t_hbm, 3)}, "bitwise_vs_HBM": {}}
            for label, (a, b, c) in (("B_Pin", (L, hB, C)), ("HostPin", (hL, hB, hC))):
                c.values.fill_(float("nan"))
                fn = lambda: mls.numeric_placed(a, b, c, ws)
                fn()
                t, _ = timed(torch, fn, 3, pre=flush)
                got = c.values.numpy() if c is hC else c.values.cpu().numpy()
                bit = same_bits(got, ref)
                ok = ok and bit
                entry["GFLOPs"][label] = gfl(t)
                entry["ms"][label] = round(t, 3)
                entry["bitwise_vs_HBM"][label] = bit
            if with_parity:
                import oracle
                Rf, _ = oracle.spgemm(host_numpy(L), host_numpy(rhs), nthreads=oracle_threads(), with_abs=False)
                par = same_bits(C.row_ptr.cpu().numpy(), Rf.row_ptr) and \
                    same_bits(C.col_idx.cpu().numpy(), Rf.col_idx) and same_bits(ref, Rf.values)
                entry["oracle_bitwise"] = par
                ok = ok and par
            log(f"density {name} delta={delta}: {entry}")
            rows.append(entry)
            del hL, hB, hC, C
        del rhs
        torch.cuda.empty_cache()
        host_cache_release(torch)
    return {"problem": f"elasticity3d on {n}^3 nodes ({A.nrows} rows), RHS {A.ncols} x {P.ncols}",
            "products": rows}, ok


# ---------------------------------------------------------------------------
# triangle counting

def tc_word_model(n, lrp, lci):
    """Compressed-word accounting of (L * comp(L)) o L from L's structure:
    words of each row (distinct col >> 5), the word operations (for every
    entry (i, k) of L, the words of row k), and the model bytes (L streamed,
    row i's own words, 8 bytes per gathered word, 8 bytes per row written)."""
    sets = lci.astype(np.int64) >> 5
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(lrp))
    new_word = np.ones(len(lci), dtype=bool)
    if len(lci):
        new_word[1:] = (sets[1:] != sets[:-1]) | (rows[1:] != rows[:-1])
    words = np.bincount(rows[new_word], minlength=n).astype(np.int64)
    wordops = int(words[lci].sum())
    uncompressed = int(np.diff(lrp).astype(np.int64)[lci].sum())
    model = 4 * (n + 1) + 4 * len(lci) + 8 * int(words.sum()) + 8 * wordops + 8 * n
    return words, wordops, uncompressed, model


def bench_tc(torch, mls, synth, scale, with_parity):
    log(f"generating R-MAT scale {scale}")
    G = synth.rmat_graph(scale, 16, seed=3)
    t0 = time.perf_counter()
    perm, (n, lrp, lci) = mls.tc_lower(G)
    t_pre = time.perf_counter() - t0
    del G
    L = mls.DeviceCsr.from_host(synth.Csr(n, n, lrp, lci, None))
    ws = mls.Workspace()
    mls.triangle_count(L, ws)
    med, best = timed(torch, lambda: mls.triangle_count(L, ws), 5)
    prof = profiled(torch, mls, lambda: mls.triangle_count(L, ws), 3)
    counts, total = mls.triangle_count(L, ws)
    words, wordops, unc, model = tc_word_model(n, np.asarray(lrp), np.asarray(lci))
    lds = {k: v for k, v in prof.items() if k.startswith("tc_lds")}
    dom_name = max(lds.items(), key=lambda kv: kv[1][1])[0] if lds else None
    tc_ms = kernels_ms(prof, 3, ("tc_",))
    all_ms = kernels_ms(prof, 3, ("",))
    res = {"metric": "triangle counting time (masked L*compressed(L)), R-MAT", "ms": round(med, 3),
           "best_ms": round(best, 3), "triangles": int(total),
           "config": {"workload": f"R-MAT scale {scale}, edge factor 16, a=.57 b=.19 c=.19 d=.05, seed 3",
                      "vertices": n, "edges": int(len(lci)), "words_L": int(words.sum()),
                      "word_ops": wordops, "uncompressed_ops": unc},
           "word_ops_per_s": round(wordops / (med * 1e-3), 1),
           "roofline": {"bound": "hbm", "kernels": "tc_*", "achieved": round(model / (tc_ms * 1e-3) / 1e9, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": frac(model, tc_ms), "model_bytes": model,
                        "bytes_model": "L streamed + own words + 8 B per gathered word + 8 B per row written",
                        "kernels_ms": round(tc_ms, 4), "all_kernels_ms": round(all_ms, 4),
                        "frac_call": frac(model, med), "dominant": dom_name},
           "kernels": kernel_dict(prof, 3), "host_preprocessing_s": round(t_pre, 2), "dtype": "int64"}
    ok = None
    if with_parity:
        import oracle
        threads = oracle_threads()
        Lh = synth.Csr(n, n, lrp, lci, None)
        t0 = time.perf_counter()
        rc, rt = oracle.tc_count(Lh, nthreads=threads)
        dt = time.perf_counter() - t0
        ok = bool(rt == total and same_bits(counts.cpu().numpy(), rc))
        res["parity_counts_bitwise"] = ok
        res["cpu_baseline"] = {"value": round(dt * 1e3, 1), "unit": "ms", "cores": threads, "kind": "oracle",
                               "sample": f"the whole graph ({n} rows of L), flag-stamping oracle in C with "
                                         f"OpenMP, {dt:.2f} s (the run the parity check uses)"}
    log(f"tc: {res}")
    return res, ok


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128, help="grid edge (128 = the headline workload)")
    ap.add_argument("--quick", action="store_true", help="headline only: no extras, no parity, no CPU baseline")
    ap.add_argument("--no-parity", action="store_true", help="skip the oracle comparisons")
    ap.add_argument("--workload", default="all",
                    choices=["all", "spgemm", "tc", "chunked", "batched", "backward", "power_law", "placement",
                             "mg_sweep", "density"])
    ap.add_argument("--mg-gb", type=float, default=1.0, help="size of A (GB) in the placement study")
    ap.add_argument("--mg-sizes", default="1,2,4,8,16", help="sizes of A (GB) in the multigrid chunk sweep")
    ap.add_argument("--mg-problems", default=",".join(MG_NAMES))
    ap.add_argument("--hostpin-max-gb", type=float, default=4.0)
    ap.add_argument("--tc-scale", type=int, default=22)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (anchors HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(the row-partitioned multi-GPU design is described, not built)"}))
        sys.exit(2)

    import torch
    import synth
    import paper_1804_00695_amd as mls

    torch.cuda.set_device(0)
    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    parity = not (args.quick or args.no_parity)
    single = {"tc": lambda: bench_tc(torch, mls, synth, args.tc_scale, parity),
              "batched": lambda: bench_batched(torch, mls, synth, parity),
              "backward": lambda: bench_backward(torch, mls, synth, parity),
              "power_law": lambda: bench_power_law(torch, mls, synth, parity),
              "placement": lambda: bench_placement(torch, mls, args.mg_gb, parity,
                                                   tuple(args.mg_problems.split(","))),
              "density": lambda: bench_density(torch, mls, parity),
              "mg_sweep": lambda: bench_mg_sweep(torch, mls, [float(x) for x in args.mg_sizes.split(",")],
                                                 names=tuple(args.mg_problems.split(",")),
                                                 hostpin_max_gb=args.hostpin_max_gb)}
    if args.workload in single:
        res, ok = single[args.workload]()
        res["parity_ok"] = ok
        print(json.dumps(res), flush=True)
        return

    keep_host = args.workload == "chunked" or (args.workload == "all" and not args.quick)
    result, A, host_c, ms_numeric = bench_headline(torch, mls, synth, args, keep_host,
                                                   parity and args.workload != "chunked")
    if args.workload == "chunked":
        res, ok = bench_chunked(torch, mls, synth, A, host_c, ms_numeric)
        res["parity_ok"] = ok
        print(json.dumps(res), flush=True)
        return
    if args.workload == "all" and not args.quick:
        extras = {}
        par = result.setdefault("parity", {})
        steps = [("chunked", lambda: bench_chunked(torch, mls, synth, A, host_c, ms_numeric)),
                 ("tc", single["tc"]), ("batched", single["batched"]), ("backward", single["backward"]),
                 ("power_law", single["power_law"])]
        for name, fn in steps:
            log(name)
            try:
                extras[name], ok = fn()
                if parity:
                    par[name] = ok
            except Exception as e:  # report, keep the line
                extras[name] = {"error": repr(e)}
                if parity:
                    par[name] = False
            if name == "chunked":
                host_c = None
            torch.cuda.empty_cache()
        result["extras"] = extras
        if parity:
            par["all_ok"] = all(bool(v["ok"] if isinstance(v, dict) else v) for v in par.values())
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
