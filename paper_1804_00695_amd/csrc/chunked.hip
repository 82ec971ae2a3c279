// chunked.hip -- executor of the chunking algorithms (Sec. 3.3.1, Algs.
// "chunk1" and "chunk2"; Sec. 3.2.2, Alg. "chunkknl"): A, B and C live in
// pinned host memory (the slow tier); row parts are copied into part buffers
// carved from the workspace (the fast tier, HBM), multiplied by the
// row-range fused multiply-add kernel (C_r += A_r[:, P_b] * B_b, Sec. 3.2.2)
// and copied back. Under chunkknl only B's parts are copied; the kernels use
// A and C where they are, through the device mapping of the host memory.
//
// Copies host->device go on s_h2d, device->host on s_d2h and kernels on
// s_compute; events order them:
//   - a part buffer is overwritten only after the kernel (and, for C, the
//     copy back) that used its previous contents has finished;
//   - a kernel starts after the copies of its A/C part and B part;
//   - C's partial values are copied back in (Alg. chunk2, second B part on)
//     only after every earlier copy back has finished.
// With nbuf_inner = 2..4 the inner-loop matrix rotates through that many
// buffers, so its next copies overlap the current kernel. The row binning of
// each A/C part (which depends only on the row sizes of C) is computed by the
// part's first kernel step into its own slice of the per-row arrays and kept
// for the part's later steps. Every B part is visited in ascending order and
// each kernel adds its terms in ascending k, so the result is bit-identical
// to spgemm_numeric.
#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/mlspgemm.h"
#include "common.h"
#include "internal.h"
#include "launch.h"
#include "plan.h"
#include "profile.h"

using namespace mls;

namespace {

constexpr size_t kRegionSlack = 2048;

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct AcBuf {
    char *base = nullptr;
    int32_t r0 = 0, r1 = 0;
    int32_t *arp = nullptr, *aci = nullptr, *crp = nullptr, *cci = nullptr;
    double *aval = nullptr, *cval = nullptr;
    int64_t nnz_c = 0;
};

struct BBuf {
    char *base = nullptr;
    int32_t r0 = 0, r1 = 0;
    int32_t *brp = nullptr, *bci = nullptr;
    double *bval = nullptr;
};

// Records, instead of queueing, what a chunked run would queue: every copy,
// fill and kernel with the byte ranges it reads and writes, and every event
// record and wait, with the stream each goes to (test support; nothing is
// touched but the host row pointers).
enum { kTrH2D = 0, kTrD2H = 1, kTrKernel = 2, kTrFill = 3, kTrRecord = 4, kTrWait = 5 };
enum { kSpaceWs = 0, kSpaceHostCVal = 1 };

struct Tracer {
    std::vector<spgemm_trace_entry> v;
    const char *ws = nullptr;
    const double *host_cval = nullptr;
    hipStream_t sc = nullptr, sh = nullptr, sd = nullptr;
    int op = 0;
    int sid(hipStream_t s) const { return s == sc ? 0 : (s == sh ? 1 : 2); }
    void begin() { ++op; }
    void access(int kind, hipStream_t s, int space, int write, int64_t lo, int64_t hi)
    {
        spgemm_trace_entry t;
        t.op = op; t.kind = kind; t.stream = sid(s); t.event = -1; t.space = space; t.write = write;
        t.lo = lo; t.hi = hi;
        v.push_back(t);
    }
    void ws_range(int kind, hipStream_t s, int write, const void *p, size_t bytes)
    {
        const int64_t lo = (const char *)p - ws;
        access(kind, s, kSpaceWs, write, lo, lo + (int64_t)bytes);
    }
    void event(int kind, hipStream_t s, int id)
    {
        begin();
        spgemm_trace_entry t;
        t.op = op; t.kind = kind; t.stream = sid(s); t.event = id; t.space = -1; t.write = 0; t.lo = t.hi = 0;
        v.push_back(t);
    }
};

struct Ev {
    hipEvent_t e = nullptr;
    bool recorded = false;
    int id = -1;
    Tracer *tr = nullptr;
    hipError_t record(hipStream_t s)
    {
        recorded = true;
        if (tr) { tr->event(kTrRecord, s, id); return hipSuccess; }
        return hipEventRecord(e, s);
    }
    hipError_t wait(hipStream_t s) const
    {
        if (!recorded) return hipSuccess;
        if (tr) { tr->event(kTrWait, s, id); return hipSuccess; }
        return hipStreamWaitEvent(s, e, 0);
    }
};

// Bytes an A/C part [r0, r1) occupies in its buffer (each array on a
// 256-byte boundary), and the same for a B part.
size_t ac_extent(const spgemm_csr *A, const spgemm_csr *C, int32_t r0, int32_t r1)
{
    const size_t na = (size_t)((int64_t)A->row_ptr[r1] - A->row_ptr[r0]);
    const size_t nc = (size_t)((int64_t)C->row_ptr[r1] - C->row_ptr[r0]);
    const size_t rows = (size_t)(r1 - r0 + 1);
    return 2 * al(4 * rows) + al(4 * na) + al(8 * na) + al(4 * nc) + 8 * nc;
}

size_t b_extent(const spgemm_csr *B, int32_t r0, int32_t r1)
{
    const size_t nb = (size_t)((int64_t)B->row_ptr[r1] - B->row_ptr[r0]);
    return al(4 * (size_t)(r1 - r0 + 1)) + al(4 * nb) + 8 * nb;
}

void place_ac(AcBuf &b, const spgemm_csr *A, const spgemm_csr *C, int32_t r0, int32_t r1)
{
    b.r0 = r0;
    b.r1 = r1;
    const int64_t na = (int64_t)A->row_ptr[r1] - A->row_ptr[r0];
    const int64_t nc = (int64_t)C->row_ptr[r1] - C->row_ptr[r0];
    char *p = b.base;
    b.arp = (int32_t *)p; p += al(4 * (size_t)(r1 - r0 + 1));
    b.aci = (int32_t *)p; p += al(4 * (size_t)na);
    b.aval = (double *)p; p += al(8 * (size_t)na);
    b.crp = (int32_t *)p; p += al(4 * (size_t)(r1 - r0 + 1));
    b.cci = (int32_t *)p; p += al(4 * (size_t)nc);
    b.cval = (double *)p;
    b.nnz_c = nc;
}

void place_b(BBuf &b, const spgemm_csr *B, int32_t r0, int32_t r1)
{
    b.r0 = r0;
    b.r1 = r1;
    const int64_t nb = (int64_t)B->row_ptr[r1] - B->row_ptr[r0];
    char *p = b.base;
    b.brp = (int32_t *)p; p += al(4 * (size_t)(r1 - r0 + 1));
    b.bci = (int32_t *)p; p += al(4 * (size_t)nb);
    b.bval = (double *)p;
}

// Device addresses of a matrix the kernels use in place (chunkknl's A and C):
// page-locked host memory through its device mapping, or device memory.
// *on_host tells whether its row pointers can be read on the host.
spgemm_status device_csr(spgemm_csr &M, int dev, bool *on_host)
{
    bool host = false;
    const void *q = nullptr;
    spgemm_status st = device_view(M.row_ptr, dev, &q, &host);
    if (st != SPGEMM_OK) return st;
    *on_host = host;
    M.row_ptr = (int32_t *)q;
    if (M.nnz > 0) {
        if ((st = device_view(M.col_idx, dev, &q, &host)) != SPGEMM_OK) return st;
        M.col_idx = (int32_t *)q;
        if ((st = device_view(M.values, dev, &q, &host)) != SPGEMM_OK) return st;
        M.values = (double *)q;
    }
    return SPGEMM_OK;
}

// A matrix the executor copies from or to: every array must be page-locked
// host memory.
spgemm_status pinned_csr(const spgemm_csr &M, int dev)
{
    const void *arrays[3] = {M.row_ptr, M.nnz > 0 ? M.col_idx : nullptr, M.nnz > 0 ? M.values : nullptr};
    for (const void *p : arrays) {
        if (!p) continue;
        bool host = false;
        const void *q = nullptr;
        spgemm_status st = device_view(p, dev, &q, &host);
        if (st != SPGEMM_OK) return st;
        if (!host) return SPGEMM_ERR_INVALID_ARG;
    }
    return SPGEMM_OK;
}

// Host row pointers of an operand: start at 0, never decrease, end at nnz.
bool row_ptr_ok(const int32_t *rp, int32_t n, int64_t nnz)
{
    if (rp[0] != 0) return false;
    for (int32_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return false;
    return (int64_t)rp[n] == nnz;
}

}  // namespace

namespace mls {

// One kernel step of a chunked run over the A/C rows in b. With keep, the
// rows' binning lives in part `part`'s slice of the per-row arrays and its
// own bin-count entry of the table; only the part's first step (`first`)
// computes it. The error word accumulates over the whole run.
spgemm_status numeric_launch(const Batch &b, double avg_b, char *ws, const Layout &L, int32_t *bin_tbl, bool keep,
                             int part, int32_t row0, bool first, hipStream_t s)
{
    Sched sc = make_sched(ws, L);
    if (keep) {
        sc.val += row0;
        sc.cls += row0;
        sc.perm += row0;
        sc.bin_count = bin_tbl + (size_t)part * kNumBins;
    }
    // clear the scheduling counters, keep the error word
    if (first || !keep)
        launch_fill_i32((int32_t *)(ws + L.hdr + kHdrBinCount), 0, (kHdrBytes - kHdrBinCount) / 4, s);
    else
        launch_fill_i32((int32_t *)(ws + L.hdr + kHdrTaskCursor), 0, kNumBins * kXcd, s);
    if (first || !keep) launch_bin(b, kModeNumeric, sc, bin_force(), nullptr, s);
    launch_numeric(b, sc, choose_group(avg_b), s);
    return check_launch();
}

}  // namespace mls

namespace {

spgemm_status run_chunked(const spgemm_csr *A, const spgemm_csr *B, const spgemm_csr *C, spgemm_plan *plan,
                          void *ws_v, size_t ws_bytes, hipStream_t s_c, hipStream_t s_h, hipStream_t s_d, Tracer *tr)
{
    if (!A || !B || !C || !plan || !ws_v) return SPGEMM_ERR_INVALID_ARG;
    PlanImpl *P = reinterpret_cast<PlanImpl *>(plan);
    if (A->nrows != P->nA || B->nrows != P->nB || B->ncols != P->ncols || C->nrows != A->nrows) return SPGEMM_ERR_DIM_MISMATCH;
    if (A->ncols != B->nrows || C->ncols != B->ncols) return SPGEMM_ERR_DIM_MISMATCH;
    if (!A->row_ptr || !B->row_ptr || !C->row_ptr) return SPGEMM_ERR_INVALID_ARG;
    if ((A->nnz > 0 && (!A->col_idx || !A->values)) || (B->nnz > 0 && (!B->col_idx || !B->values)) ||
        (C->nnz > 0 && (!C->col_idx || !C->values)))
        return SPGEMM_ERR_INVALID_ARG;
    if ((int64_t)ws_bytes < P->ws_bytes) return SPGEMM_ERR_WORKSPACE_TOO_SMALL;
    if (((uintptr_t)ws_v & 255) != 0) return SPGEMM_ERR_INVALID_ARG;
    if (P->nbuf_inner < 1 || P->nbuf_inner > kMaxBuf) return SPGEMM_ERR_INVALID_ARG;
    // the operands must be the ones the plan was cut for: same entry counts
    // and consistent row pointers (the part buffers are sized from them)
    if (A->nnz != P->nnzA || B->nnz != P->nnzB || C->nnz != P->nnzC) return SPGEMM_ERR_DIM_MISMATCH;
    const bool knl = P->algo == kAlgoKnl;
    // Algs. chunk1 / chunk2: the row pointers of A, B and C are host memory by
    // contract and must be consistent (the part buffers are sized from them);
    // checked here before any HIP call
    if (!knl && (!row_ptr_ok(A->row_ptr, A->nrows, A->nnz) || !row_ptr_ok(B->row_ptr, B->nrows, B->nnz) ||
                 !row_ptr_ok(C->row_ptr, C->nrows, C->nnz)))
        return SPGEMM_ERR_BAD_CSR;
    if (!knl) {
        // kernel steps carry B's row range, the others the rows of their matrix
        for (const spgemm_plan_step &stp : P->steps) {
            const int32_t rows = (stp.kind == kStepKernel || stp.matrix == kMatB) ? B->nrows : A->nrows;
            if (stp.row_begin < 0 || stp.row_end < stp.row_begin || stp.matrix < 0 || stp.matrix > 3 ||
                stp.row_end > rows)
                return SPGEMM_ERR_INVALID_ARG;
        }
        const size_t rac0 = al((size_t)P->max_ac) + kRegionSlack;
        const size_t rb0 = al((size_t)P->max_b) + kRegionSlack;
        for (const spgemm_plan_step &stp : P->steps) {
            if (stp.kind != kStepH2D) continue;
            if (stp.matrix == kMatA && ac_extent(A, C, stp.row_begin, stp.row_end) > rac0) return SPGEMM_ERR_DIM_MISMATCH;
            if (stp.matrix == kMatB && b_extent(B, stp.row_begin, stp.row_end) > rb0) return SPGEMM_ERR_DIM_MISMATCH;
        }
    }
    // B (and, except under chunkknl, A and C) are copied from and to
    // page-locked host memory; chunkknl's kernels use A and C in place. A
    // trace takes them as they are.
    spgemm_csr Ad = *A, Cd = *C;
    bool a_host = true, c_host = true;
    if (!tr) {
        int dev = 0;
        hipError_t ed = hipGetDevice(&dev);
        if (ed != hipSuccess) return hip_fail(ed);
        spgemm_status sv = pinned_csr(*B, dev);
        if (sv == SPGEMM_OK) sv = knl ? device_csr(Ad, dev, &a_host) : pinned_csr(*A, dev);
        if (sv == SPGEMM_OK) sv = knl ? device_csr(Cd, dev, &c_host) : pinned_csr(*C, dev);
        if (sv != SPGEMM_OK) return sv;
    }
    // chunkknl: B's row pointers, and those of A and C when they are in host
    // memory, must be consistent; A and C in device memory are used as they
    // are, like spgemm_numeric's operands
    if (knl && (!row_ptr_ok(B->row_ptr, B->nrows, B->nnz) || (a_host && !row_ptr_ok(A->row_ptr, A->nrows, A->nnz)) ||
                (c_host && !row_ptr_ok(C->row_ptr, C->nrows, C->nnz))))
        return SPGEMM_ERR_BAD_CSR;
    if (knl)
        for (const spgemm_plan_step &stp : P->steps)
            if (stp.row_begin < 0 || stp.row_end < stp.row_begin || stp.row_end > B->nrows ||
                (stp.kind == kStepH2D && b_extent(B, stp.row_begin, stp.row_end) > al((size_t)P->max_b) + kRegionSlack))
                return SPGEMM_ERR_DIM_MISMATCH;
    char *ws = (char *)ws_v;
    if (!tr) memo_forget(ws_v);

    const Layout L = make_layout(1, A->nrows, B->nrows, 0, B->ncols, false);
    int32_t *bin_tbl = (int32_t *)(ws + al(L.total));
    char *buf0 = ws + al(L.total) + binned_parts_bytes();
    const bool keep = (int64_t)P->p_ac.size() <= kMaxBinnedParts;
    std::vector<char> binned(P->p_ac.size(), 0);
    const int nbuf = P->nbuf_inner;
    const size_t rac = al((size_t)P->max_ac) + kRegionSlack;
    const size_t rb = al((size_t)P->max_b) + kRegionSlack;
    AcBuf acb[kMaxBuf];
    BBuf bb[kMaxBuf];
    size_t need;
    if (P->algo == kAlgoChunk1) {
        acb[0].base = buf0;
        for (int s = 0; s < nbuf; ++s) bb[s].base = buf0 + rac + s * rb;
        need = (size_t)(buf0 - ws) + rac + nbuf * rb;
    } else if (P->algo == kAlgoChunk2) {
        bb[0].base = buf0;
        for (int s = 0; s < nbuf; ++s) acb[s].base = buf0 + rb + s * rac;
        need = (size_t)(buf0 - ws) + rb + nbuf * rac;
    } else {
        for (int s = 0; s < nbuf; ++s) bb[s].base = buf0 + s * rb;
        need = (size_t)(buf0 - ws) + nbuf * rb;
    }
    if (need > ws_bytes) return SPGEMM_ERR_WORKSPACE_TOO_SMALL;
    // every part of the schedule must fit its buffer region, and every step
    // must name a part and a buffer of the plan, before anything is queued
    for (const spgemm_plan_step &stp : P->steps) {
        if (stp.slot < 0 || stp.slot >= nbuf) return SPGEMM_ERR_INVALID_ARG;
        if (stp.kind == kStepKernel && (stp.part < 0 || stp.part >= (int)P->p_ac.size())) return SPGEMM_ERR_INVALID_ARG;
        if (stp.kind != kStepH2D) continue;
        if (stp.row_begin < 0 || stp.row_end < stp.row_begin) return SPGEMM_ERR_INVALID_ARG;
        if (stp.matrix == kMatA && (knl || ac_extent(A, C, stp.row_begin, stp.row_end) > rac))
            return SPGEMM_ERR_DIM_MISMATCH;
        if (stp.matrix == kMatB && b_extent(B, stp.row_begin, stp.row_end) > rb) return SPGEMM_ERR_DIM_MISMATCH;
    }

    Ev ev_b_ready[kMaxBuf], ev_ac_ready[kMaxBuf], ev_kdone[kMaxBuf], ev_d2h[kMaxBuf];
    Ev ev_outer_free, ev_last_kernel, ev_last_d2h;
    std::vector<Ev *> all = {&ev_outer_free, &ev_last_kernel, &ev_last_d2h};
    for (int s = 0; s < kMaxBuf; ++s) {
        all.push_back(&ev_b_ready[s]);
        all.push_back(&ev_ac_ready[s]);
        all.push_back(&ev_kdone[s]);
        all.push_back(&ev_d2h[s]);
    }
    hipError_t e = hipSuccess;
    for (size_t k = 0; k < all.size(); ++k) {
        all[k]->id = (int)k + 1;
        all[k]->tr = tr;
        if (!tr && e == hipSuccess) e = hipEventCreateWithFlags(&all[k]->e, hipEventDisableTiming);
    }
    auto cleanup = [&]() {
        for (Ev *x : all)
            if (x->e) hipEventDestroy(x->e);
    };
    if (e != hipSuccess) { cleanup(); return hip_fail(e); }
    // the kernels' own region (header, per-row arrays, kept binnings), which
    // only work on the compute stream touches
    const size_t kern_bytes = (size_t)(buf0 - ws);
    if (tr) {   // work queued earlier on the compute stream may use all of the workspace
        tr->begin();
        tr->ws_range(kTrKernel, s_c, 1, ws, ws_bytes);
    }
    // the copy streams must not overwrite the workspace while work queued
    // earlier on the compute stream (an in-HBM product on the same
    // workspace, for instance) still reads it
    {
        Ev entry;
        entry.tr = tr;
        if (!tr) e = hipEventCreateWithFlags(&entry.e, hipEventDisableTiming);
        if (e == hipSuccess) e = entry.record(s_c);
        if (e == hipSuccess) e = entry.wait(s_h);
        if (e == hipSuccess) e = entry.wait(s_d);
        if (entry.e) hipEventDestroy(entry.e);
        if (e != hipSuccess) { cleanup(); return hip_fail(e); }
    }
    if (tr) {
        tr->begin();
        tr->ws_range(kTrFill, s_c, 1, ws, kern_bytes);
    } else {
        reset_header(ws, L, s_c);
    }

    const double avg_b = B->nrows > 0 ? (double)B->nnz / B->nrows : 1.0;
    int64_t issued_h = 0, issued_d = 0;
    spgemm_status st = SPGEMM_OK;
    auto h2d_on = [&](hipStream_t st_, void *dst, const void *src, size_t bytes) {
        if (bytes == 0 || e != hipSuccess) return;
        if (tr) {
            tr->begin();
            tr->ws_range(kTrH2D, st_, 1, dst, bytes);
            const char *hc = (const char *)tr->host_cval;
            if ((const char *)src >= hc && (const char *)src < hc + 8 * (size_t)C->nnz) {
                const int64_t lo = (const char *)src - hc;
                tr->access(kTrH2D, st_, kSpaceHostCVal, 0, lo, lo + (int64_t)bytes);
            }
        } else {
            e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st_);
        }
        issued_h += (int64_t)bytes;
    };
    auto h2d = [&](void *dst, const void *src, size_t bytes) { h2d_on(s_h, dst, src, bytes); };
    auto d2h = [&](double *dst, const void *src, size_t bytes) {
        if (bytes == 0 || e != hipSuccess) return;
        if (tr) {
            tr->begin();
            tr->ws_range(kTrD2H, s_d, 0, src, bytes);
            const int64_t lo = (const char *)dst - (const char *)tr->host_cval;
            tr->access(kTrD2H, s_d, kSpaceHostCVal, 1, lo, lo + (int64_t)bytes);
        } else {
            e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s_d);
        }
        issued_d += (int64_t)bytes;
    };
    const bool ac_outer = P->algo != kAlgoChunk2;   // chunk1 and chunkknl keep A/C in place over the B loop
    // Alg. chunk1: an A/C part's copies in follow the previous part's copy
    // back on the device-to-host stream (its buffer is free only then), so the
    // host-to-device stream keeps copying the next B parts meanwhile
    hipStream_t s_ac = ac_outer ? s_d : s_h;
    int kernels_done = 0;

    for (const spgemm_plan_step &stp : P->steps) {
        if (e != hipSuccess || st != SPGEMM_OK) break;
        const int slot = stp.slot;
        const int sac = ac_outer ? 0 : slot;   // buffer of the A/C part
        const int sb = ac_outer ? slot : 0;    // buffer of the B part
        const int32_t r0 = stp.row_begin, r1 = stp.row_end;
        switch (stp.kind) {
        case kStepH2D:
            if (stp.matrix == kMatA) {
                AcBuf &b = acb[sac];
                // chunk1: same stream as the previous part's copy back, which
                // waited for that part's last kernel
                if (!ac_outer) e = ev_d2h[sac].wait(s_ac);
                place_ac(b, A, C, r0, r1);
                const int64_t a0 = A->row_ptr[r0], a1 = A->row_ptr[r1];
                h2d_on(s_ac, b.arp, A->row_ptr + r0, 4 * (size_t)(r1 - r0 + 1));
                h2d_on(s_ac, b.aci, A->col_idx + a0, 4 * (size_t)(a1 - a0));
                h2d_on(s_ac, b.aval, A->values + a0, 8 * (size_t)(a1 - a0));
            } else if (stp.matrix == kMatCStruct) {
                AcBuf &b = acb[sac];
                const int64_t c0 = C->row_ptr[r0], c1 = C->row_ptr[r1];
                h2d_on(s_ac, b.crp, C->row_ptr + r0, 4 * (size_t)(r1 - r0 + 1));
                h2d_on(s_ac, b.cci, C->col_idx + c0, 4 * (size_t)(c1 - c0));
                if (e == hipSuccess) e = ev_ac_ready[sac].record(s_ac);
            } else if (stp.matrix == kMatCVal) {
                AcBuf &b = acb[sac];
                if (e == hipSuccess) e = ev_last_d2h.wait(s_h);
                const int64_t c0 = C->row_ptr[r0], c1 = C->row_ptr[r1];
                h2d(b.cval, C->values + c0, 8 * (size_t)(c1 - c0));
                if (e == hipSuccess) e = ev_ac_ready[sac].record(s_h);
            } else {   // B part
                BBuf &b = bb[sb];
                e = ac_outer ? ev_kdone[sb].wait(s_h) : ev_last_kernel.wait(s_h);
                place_b(b, B, r0, r1);
                const int64_t q0 = B->row_ptr[r0], q1 = B->row_ptr[r1];
                h2d(b.brp, B->row_ptr + r0, 4 * (size_t)(r1 - r0 + 1));
                h2d(b.bci, B->col_idx + q0, 4 * (size_t)(q1 - q0));
                h2d(b.bval, B->values + q0, 8 * (size_t)(q1 - q0));
                if (e == hipSuccess) e = ev_b_ready[sb].record(s_h);
            }
            break;
        case kStepZero: {
            AcBuf &b = acb[sac];
            e = ac_outer ? ev_outer_free.wait(s_c) : ev_d2h[sac].wait(s_c);
            const int64_t nc = (int64_t)C->row_ptr[r1] - C->row_ptr[r0];
            if (e == hipSuccess && tr) {
                tr->begin();
                tr->ws_range(kTrFill, s_c, 1, b.cval, 8 * (size_t)nc);
            } else if (e == hipSuccess) {
                launch_fill_f64(b.cval, 0.0, nc, s_c);
            }
            break;
        }
        case kStepKernel: {
            BBuf &bq = bb[sb];
            e = ev_b_ready[sb].wait(s_c);
            Batch bt;
            std::memset(&bt, 0, sizeof(bt));
            bt.nprob = 1;
            bt.max_ncols = g_opt.wide_table ? 0 : B->ncols;
            Prob &q = bt.p0;
            int32_t a_r0, a_r1;
            if (knl) {
                // A and C in place, all rows; the first B part writes C's
                // values, the later ones add onto them
                a_r0 = 0;
                a_r1 = A->nrows;
                q.arp = Ad.row_ptr; q.aci = Ad.col_idx; q.aval = Ad.values;
                q.crp = Cd.row_ptr; q.cci = Cd.col_idx; q.cval = Cd.values;
                q.a_off = 0;
                q.c_off = 0;
                q.accumulate = kernels_done > 0 ? 1 : 0;
            } else {
                AcBuf &a = acb[sac];
                if (e == hipSuccess) e = ev_ac_ready[sac].wait(s_c);
                a_r0 = a.r0;
                a_r1 = a.r1;
                q.arp = a.arp; q.aci = a.aci; q.aval = a.aval;
                q.crp = a.crp; q.cci = a.cci; q.cval = a.cval;
                q.a_off = A->row_ptr[a.r0];
                q.c_off = C->row_ptr[a.r0];
                q.accumulate = 1;
            }
            if (e != hipSuccess) break;
            bt.na = a_r1 - a_r0;
            q.brp = bq.brp; q.bci = bq.bci; q.bval = bq.bval;
            q.nrows = a_r1 - a_r0;
            q.ncols = B->ncols;
            q.krows = bq.r1 - bq.r0;
            q.b_off = B->row_ptr[bq.r0];
            q.k_lo = bq.r0;
            q.k_hi = bq.r1;
            q.ranged = (bq.r0 > 0 || bq.r1 < B->nrows) ? 1 : 0;
            const bool first = !binned[stp.part];
            if (tr) {
                tr->begin();
                tr->ws_range(kTrKernel, s_c, 1, ws, kern_bytes);
                tr->ws_range(kTrKernel, s_c, 0, bq.base, (size_t)((const char *)(bq.bval + (B->row_ptr[bq.r1] - B->row_ptr[bq.r0])) - bq.base));
                if (knl) {   // C's values rewritten in place in host memory
                    tr->access(kTrKernel, s_c, kSpaceHostCVal, 1, 0, 8 * C->nnz);
                } else {
                    AcBuf &a = acb[sac];
                    tr->ws_range(kTrKernel, s_c, 0, a.base, (size_t)((const char *)a.cval - a.base));
                    tr->ws_range(kTrKernel, s_c, 1, a.cval, 8 * (size_t)a.nnz_c);
                }
            } else {
                st = numeric_launch(bt, avg_b, ws, L, bin_tbl, keep, stp.part, a_r0, first, s_c);
            }
            binned[stp.part] = 1;
            ++kernels_done;
            if (st == SPGEMM_OK) e = ev_kdone[ac_outer ? sb : sac].record(s_c);
            if (e == hipSuccess) e = ev_last_kernel.record(s_c);
            break;
        }
        case kStepD2H: {
            AcBuf &b = acb[sac];
            e = ac_outer ? ev_last_kernel.wait(s_d) : ev_kdone[sac].wait(s_d);
            const int64_t c0 = C->row_ptr[r0], c1 = C->row_ptr[r1];
            d2h(C->values + c0, b.cval, 8 * (size_t)(c1 - c0));
            if (e == hipSuccess) e = ev_d2h[sac].record(s_d);
            if (e == hipSuccess) e = ev_last_d2h.record(s_d);
            if (e == hipSuccess && ac_outer) e = ev_outer_free.record(s_d);
            break;
        }
        }
    }
    if (tr) return e == hipSuccess ? st : hip_fail(e);
    hipError_t e2 = hipStreamSynchronize(s_c);
    hipError_t e3 = hipStreamSynchronize(s_h);
    hipError_t e4 = hipStreamSynchronize(s_d);
    cleanup();
    P->issued_h2d = issued_h;
    P->issued_d2h = issued_d;
    if (e != hipSuccess) return hip_fail(e);
    if (e2 != hipSuccess) return hip_fail(e2);
    if (e3 != hipSuccess) return hip_fail(e3);
    if (e4 != hipSuccess) return hip_fail(e4);
    if (st != SPGEMM_OK) return st;
    // structure errors flagged by the kernels
    return read_errors(ws, L, s_c);
}

}  // namespace

extern "C" spgemm_status spgemm_numeric_chunked(const spgemm_csr *A, const spgemm_csr *B, spgemm_csr *C,
                                                spgemm_plan *plan, void *ws_v, size_t ws_bytes, hipStream_t s_c,
                                                hipStream_t s_h, hipStream_t s_d)
{
    return run_chunked(A, B, C, plan, ws_v, ws_bytes, s_c, s_h, s_d, nullptr);
}

extern "C" spgemm_status spgemm_numeric_chunked_trace(const spgemm_csr *A, const spgemm_csr *B, const spgemm_csr *C,
                                                      spgemm_plan *plan, spgemm_trace_entry *out,
                                                      int64_t max_entries, int64_t *n_entries)
{
    if (!plan || !n_entries || !C || (max_entries > 0 && !out)) return SPGEMM_ERR_INVALID_ARG;
    PlanImpl *P = reinterpret_cast<PlanImpl *>(plan);
    Tracer tr;
    // a stand-in workspace base: ranges are reported relative to it and
    // nothing at it is ever read or written
    tr.ws = reinterpret_cast<const char *>((uintptr_t)1 << 20);
    tr.host_cval = C->values;
    tr.sc = reinterpret_cast<hipStream_t>((uintptr_t)0x10);
    tr.sh = reinterpret_cast<hipStream_t>((uintptr_t)0x20);
    tr.sd = reinterpret_cast<hipStream_t>((uintptr_t)0x30);
    const int64_t saved_h = P->issued_h2d, saved_d = P->issued_d2h;
    spgemm_status st = run_chunked(A, B, C, plan, (void *)tr.ws, (size_t)P->ws_bytes, tr.sc, tr.sh, tr.sd, &tr);
    P->issued_h2d = saved_h;
    P->issued_d2h = saved_d;
    if (st != SPGEMM_OK) return st;
    *n_entries = (int64_t)tr.v.size();
    for (int64_t k = 0; k < max_entries && k < (int64_t)tr.v.size(); ++k) out[k] = tr.v[(size_t)k];
    return SPGEMM_OK;
}
