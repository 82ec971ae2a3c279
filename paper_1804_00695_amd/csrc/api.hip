// api.hip -- C ABI: workspace layout and the launch sequences of the plain
// and batched two-phase product (Sec. 2.1).
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/mlspgemm.h"
#include "common.h"
#include "launch.h"
#include "internal.h"

using namespace mls;

namespace mls {

thread_local int g_last_hip_error = 0;
Options g_opt;

spgemm_status hip_fail(hipError_t e)
{
    g_last_hip_error = (int)e;
    return SPGEMM_ERR_HIP;
}

spgemm_status check_launch()
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPGEMM_OK : hip_fail(e);
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int pow2_group(double avg)
{
    int g = 8;
    while (g < 64 && g < avg) g <<= 1;
    return g;
}

// Workspace regions for a batch run over na A-rows, nb B-rows, zb B-entries.
Layout make_layout(int64_t nprob, int64_t na, int64_t nb, int64_t zb, int64_t max_ncols, bool need_bw)
{
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes); return o; };
    L.hdr = take(kHdrBytes);
    L.totals = take(sizeof(int64_t) * (size_t)std::max<int64_t>(nprob, 1));
    L.nnz_tab = take(sizeof(int64_t) * 2 * (size_t)std::max<int64_t>(nprob, 1));
    L.probs = take(sizeof(Prob) * (size_t)std::max<int64_t>(nprob, 1));
    L.abase = take(sizeof(int32_t) * (size_t)(nprob + 1));
    L.bbase = take(sizeof(int32_t) * (size_t)(nprob + 1));
    L.val = take(sizeof(int32_t) * (size_t)std::max<int64_t>(na, 1));
    L.cls = take((size_t)std::max<int64_t>(na, 1));
    L.perm = take(sizeof(int32_t) * (size_t)std::max<int64_t>(na, 1));
    L.nblk = (int32_t)((std::max<int64_t>(na, 1) + kBinRowsPerWG - 1) / kBinRowsPerWG);
    L.blk = take(sizeof(int32_t) * (size_t)kNumBins * (size_t)L.nblk);
    L.prefix = take(sizeof(int64_t) * (size_t)(na + 1));
    L.tiles = take(sizeof(int64_t) * (size_t)scan_tiles((int)std::min<int64_t>(na, 0x7fffffff)));
    if (need_bw) {
        L.bw = take(sizeof(uint2) * (size_t)std::max<int64_t>(zb, 1));
        L.bwc = take(sizeof(int32_t) * (size_t)std::max<int64_t>(nb, 1));
        int64_t words = (std::max<int64_t>(max_ncols, 1) + 31) / 32;
        int64_t slots = (int64_t)(256ll << 20) / (words * 4);
        slots = std::max<int64_t>(1, std::min<int64_t>(64, slots));
        L.spill_words = words;
        L.spill_slots = (int)slots;
        L.spill = take(sizeof(uint32_t) * (size_t)(words * slots));
    }
    L.total_min = off;
    if (need_bw) {
        L.scnt = take(sizeof(int32_t) * (size_t)std::max<int64_t>(na, 1));
        L.scr = take(sizeof(uint2) * (size_t)kScratchWords * (size_t)std::max<int64_t>(na, 1));
    }
    L.total = off;
    return L;
}

// The count pass may leave compressed B and the rows' set words in the
// workspace; a fill pass on the same workspace and the same operands uses them
// instead of recomputing. Any other call on that workspace forgets them.
namespace {
std::mutex g_memo_mu;
struct SymMemo {
    const void *ws = nullptr;
    std::vector<uint64_t> key;
    bool valid = false;
} g_memo;
}  // namespace

void memo_forget(const void *ws)
{
    std::lock_guard<std::mutex> lk(g_memo_mu);
    if (g_memo.ws == ws) g_memo.valid = false;
}

Sched make_sched(char *ws, const Layout &L)
{
    Sched sc;
    sc.err = (uint32_t *)(ws + L.hdr + kHdrErr);
    sc.bin_count = (int32_t *)(ws + L.hdr + kHdrBinCount);
    sc.blk_cnt = (int32_t *)(ws + L.blk);
    sc.nblk = L.nblk;
    sc.task_cursor = (int32_t *)(ws + L.hdr + kHdrTaskCursor);
    sc.val = (int32_t *)(ws + L.val);
    sc.cls = (uint8_t *)(ws + L.cls);
    sc.perm = (int32_t *)(ws + L.perm);
    sc.scr = L.has_scratch ? (uint2 *)(ws + L.scr) : nullptr;
    sc.scnt = L.has_scratch ? (int32_t *)(ws + L.scnt) : nullptr;
    sc.wstart = (int32_t *)(ws + L.prefix);   // the row-pointer scan's array, idle outside the symbolic phase
    return sc;
}

void reset_header(char *ws, const Layout &L, hipStream_t s)
{
    launch_fill_i32((int32_t *)(ws + L.hdr), 0, kHdrBytes / 4, s);
}

spgemm_status read_errors(char *ws, const Layout &L, hipStream_t s)
{
    uint32_t err = 0;
    hipError_t e = hipMemcpyAsync(&err, ws + L.hdr + kHdrErr, sizeof(err), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e);
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    return err_status(err);
}

spgemm_status err_status(uint32_t err)
{
    if (err & kErrBadCsr) return SPGEMM_ERR_BAD_CSR;
    if (err & kErrOverflow) return SPGEMM_ERR_INDEX_OVERFLOW;
    if (err & kErrStructure) return SPGEMM_ERR_STRUCTURE;
    if (err & kErrTable) return SPGEMM_ERR_STRUCTURE;
    return SPGEMM_OK;
}

static bool csr_ok(const spgemm_csr *M, bool need_values)
{
    if (!M || M->nrows < 0 || M->ncols < 0 || M->nnz < 0 || M->nnz >= 0x7fffffffLL) return false;
    if (!M->row_ptr) return false;
    if (M->nnz > 0 && !M->col_idx) return false;
    if (need_values && M->nnz > 0 && !M->values) return false;
    return true;
}

// Host-side description of a batch call; uploads the descriptors when
// there is more than one product.
spgemm_status prepare_batch(int32_t nbatch, const spgemm_csr *A, const spgemm_csr *B, const spgemm_csr *C,
                            bool need_values, bool need_bw, char *ws, size_t ws_bytes, hipStream_t s,
                            BatchHost &out, bool upload)
{
    if (nbatch < 1 || !A || !B) return SPGEMM_ERR_INVALID_ARG;
    int64_t na = 0, nb = 0, zb = 0, maxc = 0, za = 0;
    for (int t = 0; t < nbatch; ++t) {
        if (!csr_ok(&A[t], need_values) || !csr_ok(&B[t], need_values)) return SPGEMM_ERR_INVALID_ARG;
        if (A[t].ncols != B[t].nrows) return SPGEMM_ERR_DIM_MISMATCH;
        na += A[t].nrows;
        nb += B[t].nrows;
        zb += B[t].nnz;
        za += A[t].nnz;
        maxc = std::max<int64_t>(maxc, B[t].ncols);
    }
    if (na >= 0x7fffffff || nb >= 0x7fffffff) return SPGEMM_ERR_INDEX_OVERFLOW;
    out.layout = make_layout(nbatch, na, nb, zb, maxc, need_bw);
    if (!ws || ws_bytes < out.layout.total_min) return SPGEMM_ERR_WORKSPACE_TOO_SMALL;
    out.layout.has_scratch = need_bw && ws_bytes >= out.layout.total;
    if (((uintptr_t)ws & 255) != 0) return SPGEMM_ERR_INVALID_ARG;
    out.probs.assign(nbatch, Prob{});
    out.abase.assign(nbatch + 1, 0);
    out.bbase.assign(nbatch + 1, 0);
    out.nnz_tab.assign(2 * (size_t)nbatch, 0);
    int64_t eb = 0;
    for (int t = 0; t < nbatch; ++t) {
        Prob &P = out.probs[t];
        P.arp = A[t].row_ptr; P.aci = A[t].col_idx; P.aval = A[t].values;
        P.brp = B[t].row_ptr; P.bci = B[t].col_idx; P.bval = B[t].values;
        if (need_bw) {
            P.bw = (uint2 *)(ws + out.layout.bw) + eb;
            P.bwc = (int32_t *)(ws + out.layout.bwc) + out.bbase[t];
        }
        if (C) { P.crp = C[t].row_ptr; P.cci = C[t].col_idx; P.cval = C[t].values; }
        P.nrows = A[t].nrows;
        P.ncols = B[t].ncols;
        P.krows = B[t].nrows;
        P.k_lo = 0;
        P.k_hi = B[t].nrows;
        out.abase[t + 1] = out.abase[t] + A[t].nrows;
        out.bbase[t + 1] = out.bbase[t] + B[t].nrows;
        out.nnz_tab[2 * t] = A[t].nnz;
        out.nnz_tab[2 * t + 1] = B[t].nnz;
        eb += B[t].nnz;
    }
    Batch &bt = out.batch;
    std::memset(&bt, 0, sizeof(bt));
    bt.nprob = nbatch;
    bt.na = (int32_t)na;
    bt.nb = (int32_t)nb;
    // 0 keeps the numeric phase on the wide hash slots
    if (!g_opt.wide_table)
        for (int t = 0; t < nbatch; ++t) bt.max_ncols = std::max(bt.max_ncols, B[t].ncols);
    bt.p0 = out.probs[0];
    bt.probs = (const Prob *)(ws + out.layout.probs);
    bt.abase = (const int32_t *)(ws + out.layout.abase);
    bt.bbase = (const int32_t *)(ws + out.layout.bbase);
    out.avg_a = na > 0 ? (double)za / (double)na : 1.0;
    out.avg_b = nb > 0 ? (double)zb / (double)nb : 1.0;
    std::vector<uint64_t> &key = out.key;
    key.clear();
    key.push_back((uint64_t)nbatch);
    key.push_back((uint64_t)ws_bytes);
    for (int t = 0; t < nbatch; ++t) {
        key.push_back((uint64_t)(uintptr_t)A[t].row_ptr);
        key.push_back((uint64_t)(uintptr_t)A[t].col_idx);
        key.push_back((uint64_t)(uintptr_t)B[t].row_ptr);
        key.push_back((uint64_t)(uintptr_t)B[t].col_idx);
        key.push_back((uint64_t)(uint32_t)A[t].nrows);
        key.push_back((uint64_t)(uint32_t)A[t].ncols);
        key.push_back((uint64_t)(uint32_t)B[t].nrows);
        key.push_back((uint64_t)(uint32_t)B[t].ncols);
        key.push_back((uint64_t)A[t].nnz);
        key.push_back((uint64_t)B[t].nnz);
        key.push_back(C ? (uint64_t)(uintptr_t)C[t].row_ptr : 0ull);
    }
    if (!upload) return nbatch == 1 ? SPGEMM_OK : SPGEMM_ERR_INVALID_ARG;
    hipError_t e = hipSuccess;
    e = hipMemcpyAsync(ws + out.layout.nnz_tab, out.nnz_tab.data(), sizeof(int64_t) * out.nnz_tab.size(),
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess && nbatch > 1) {
        e = hipMemcpyAsync(ws + out.layout.probs, out.probs.data(), sizeof(Prob) * nbatch, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws + out.layout.abase, out.abase.data(), sizeof(int32_t) * (nbatch + 1),
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws + out.layout.bbase, out.bbase.data(), sizeof(int32_t) * (nbatch + 1),
                               hipMemcpyHostToDevice, s);
    }
    if (e != hipSuccess) return hip_fail(e);
    return SPGEMM_OK;
}

int choose_group(double avg)
{
    if (g_opt.group_size) return (int)g_opt.group_size;
    return pow2_group(avg);
}

// Symbolic count or fill over a prepared batch.
spgemm_status run_symbolic(BatchHost &bh, char *ws, int fill, int64_t *nnz_host, hipStream_t s)
{
    Layout &L = bh.layout;
    bool reuse = false;
    {
        std::lock_guard<std::mutex> lk(g_memo_mu);
        reuse = fill && g_memo.valid && g_memo.ws == ws && g_memo.key == bh.key;
        if (g_memo.ws == ws) g_memo.valid = false;
    }
    if (fill && !reuse) L.has_scratch = false;   // nothing to expand: recompute every row
    Sched sc = make_sched(ws, L);
    reset_header(ws, L, s);
    if (!fill && g_opt.validate) {
        launch_validate(bh.batch, 0, (const int64_t *)(ws + L.nnz_tab), sc.err, s);
        // B is checked by the same rules as A: skip it when every B_t is A_t itself
        bool same = true;
        for (int t = 0; t < bh.batch.nprob && same; ++t) {
            const Prob &q = bh.probs[t];
            same = q.arp == q.brp && q.aci == q.bci && q.nrows == q.krows && q.ncols == q.krows &&
                   q.a_off == q.b_off && bh.nnz_tab[2 * t] == bh.nnz_tab[2 * t + 1];
        }
        if (!same) launch_validate(bh.batch, 1, (const int64_t *)(ws + L.nnz_tab), sc.err, s);
        spgemm_status st = check_launch();
        if (st != SPGEMM_OK) return st;
        st = read_errors(ws, L, s);
        if (st != SPGEMM_OK) return st;
    }
    if (!reuse) launch_compress(bh.batch, s);
    launch_bin(bh.batch, fill ? kModeFill : kModeCount, sc, bin_force(), nullptr, s);
    if (fill) launch_sym_expand(bh.batch, sc, s);
    launch_symbolic(bh.batch, sc, fill, choose_group(bh.avg_a), s);
    spgemm_status st = check_launch();
    if (st != SPGEMM_OK) return st;
    if (fill) {
        if (reuse) {   // the words stay valid for another fill pass on the same operands
            std::lock_guard<std::mutex> lk(g_memo_mu);
            g_memo.ws = ws; g_memo.key = bh.key; g_memo.valid = true;
        }
        return SPGEMM_OK;
    }
    for (int t = 0; t < bh.batch.nprob; ++t)
        if (bh.probs[t].nrows == 0) launch_fill_i32(bh.probs[t].crp, 0, 1, s);
    int64_t *prefix = (int64_t *)(ws + L.prefix);
    launch_scan(sc.val, bh.batch.na, (int64_t *)(ws + L.tiles), prefix, s);
    launch_write_rowptr(bh.batch, prefix, (int64_t *)(ws + L.totals), sc.err, s);
    st = check_launch();
    if (st != SPGEMM_OK) return st;
    std::vector<int64_t> tot(bh.batch.nprob, 0);
    uint32_t err = 0;
    hipError_t e = hipMemcpyAsync(tot.data(), ws + L.totals, sizeof(int64_t) * tot.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&err, ws + L.hdr + kHdrErr, sizeof(err), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    // products with no rows never write their total
    for (int t = 0; t < bh.batch.nprob; ++t)
        if (bh.probs[t].nrows == 0) tot[t] = 0;
    if (nnz_host) std::memcpy(nnz_host, tot.data(), sizeof(int64_t) * tot.size());
    for (int t = 0; t < bh.batch.nprob; ++t)
        if (tot[t] >= 0x7fffffffLL) return SPGEMM_ERR_INDEX_OVERFLOW;
    st = err_status(err);
    if (st == SPGEMM_OK) {
        std::lock_guard<std::mutex> lk(g_memo_mu);
        g_memo.ws = ws; g_memo.key = bh.key; g_memo.valid = true;
    }
    return st;
}

spgemm_status run_numeric(BatchHost &bh, char *ws, hipStream_t s)
{
    memo_forget(ws);
    const Layout &L = bh.layout;
    Sched sc = make_sched(ws, L);
    reset_header(ws, L, s);
    launch_bin(bh.batch, kModeNumeric, sc, bin_force(), nullptr, s);
    launch_numeric(bh.batch, sc, choose_group(bh.avg_b), s);
    return check_launch();
}

}  // namespace mls

// ===========================================================================
// extern "C"

extern "C" {

const char *spgemm_status_string(spgemm_status s)
{
    switch (s) {
    case SPGEMM_OK: return "ok";
    case SPGEMM_ERR_INVALID_ARG: return "invalid argument";
    case SPGEMM_ERR_BAD_CSR: return "invalid CSR matrix";
    case SPGEMM_ERR_DIM_MISMATCH: return "dimension mismatch";
    case SPGEMM_ERR_INDEX_OVERFLOW: return "index overflow (2^31)";
    case SPGEMM_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case SPGEMM_ERR_BUDGET: return "HBM budget too small";
    case SPGEMM_ERR_HIP: return "HIP runtime error";
    case SPGEMM_ERR_UNSUPPORTED: return "unsupported";
    case SPGEMM_ERR_STRUCTURE: return "output structure misses a reached column";
    }
    return "unknown status";
}

int spgemm_last_hip_error(void) { return g_last_hip_error; }

int spgemm_version(void) { return 10000; }

spgemm_status spgemm_set_option(spgemm_option opt, int64_t value)
{
    switch (opt) {
    case SPGEMM_OPT_VALIDATE: g_opt.validate = value != 0; return SPGEMM_OK;
    case SPGEMM_OPT_FORCE_SPILL: g_opt.force_spill = value != 0; return SPGEMM_OK;
    case SPGEMM_OPT_GROUP_SIZE:
        if (value != 0 && value != 8 && value != 16 && value != 32 && value != 64) return SPGEMM_ERR_INVALID_ARG;
        g_opt.group_size = value;
        return SPGEMM_OK;
    case SPGEMM_OPT_FORCE_CLASS:
        if (value < -1 || value >= kNumClasses) return SPGEMM_ERR_INVALID_ARG;
        g_opt.force_class = (int)value;
        return SPGEMM_OK;
    case SPGEMM_OPT_PROFILE: g_opt.profile = value != 0; return SPGEMM_OK;
    case SPGEMM_OPT_WIDE_TABLE: g_opt.wide_table = value != 0; return SPGEMM_OK;
    }
    return SPGEMM_ERR_INVALID_ARG;
}

int64_t spgemm_get_option(spgemm_option opt)
{
    switch (opt) {
    case SPGEMM_OPT_VALIDATE: return g_opt.validate;
    case SPGEMM_OPT_FORCE_SPILL: return g_opt.force_spill;
    case SPGEMM_OPT_GROUP_SIZE: return g_opt.group_size;
    case SPGEMM_OPT_PROFILE: return g_opt.profile;
    case SPGEMM_OPT_WIDE_TABLE: return g_opt.wide_table;
    case SPGEMM_OPT_FORCE_CLASS: return g_opt.force_class;
    default: return 0;
    }
}

spgemm_status spgemm_validate_host(const spgemm_csr *M)
{
    if (!M || M->nrows < 0 || M->ncols < 0 || !M->row_ptr) return SPGEMM_ERR_INVALID_ARG;
    if (M->row_ptr[0] != 0) return SPGEMM_ERR_BAD_CSR;
    for (int32_t i = 0; i < M->nrows; ++i) {
        int32_t s = M->row_ptr[i], e = M->row_ptr[i + 1];
        if (e < s) return SPGEMM_ERR_BAD_CSR;
        for (int32_t p = s; p < e; ++p) {
            int32_t c = M->col_idx[p];
            if (c < 0 || c >= M->ncols) return SPGEMM_ERR_BAD_CSR;
            if (p > s && c <= M->col_idx[p - 1]) return SPGEMM_ERR_BAD_CSR;
        }
    }
    if ((int64_t)M->row_ptr[M->nrows] != M->nnz) return SPGEMM_ERR_BAD_CSR;
    return SPGEMM_OK;
}

spgemm_status spgemm_workspace_size(const spgemm_csr *A, const spgemm_csr *B, size_t *bytes)
{
    return spgemm_batch_workspace_size(1, A, B, bytes);
}

spgemm_status spgemm_batch_workspace_size(int32_t nbatch, const spgemm_csr *A, const spgemm_csr *B, size_t *bytes)
{
    if (nbatch < 1 || !A || !B || !bytes) return SPGEMM_ERR_INVALID_ARG;
    int64_t na = 0, nb = 0, zb = 0, maxc = 0;
    for (int t = 0; t < nbatch; ++t) {
        na += A[t].nrows;
        nb += B[t].nrows;
        zb += B[t].nnz;
        maxc = std::max<int64_t>(maxc, B[t].ncols);
    }
    *bytes = make_layout(nbatch, na, nb, zb, maxc, true).total;
    return SPGEMM_OK;
}

spgemm_status spgemm_row_work(const spgemm_csr *A, const spgemm_csr *B, int32_t *work, int64_t *total_host,
                              void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!work) return SPGEMM_ERR_INVALID_ARG;
    BatchHost bh;
    memo_forget(ws);
    spgemm_status st = prepare_batch(1, A, B, nullptr, false, false, (char *)ws, ws_bytes, stream, bh);
    if (st != SPGEMM_OK) return st;
    char *w = (char *)ws;
    Sched sc = make_sched(w, bh.layout);
    sc.val = work;
    reset_header(w, bh.layout, stream);
    unsigned long long *tot = (unsigned long long *)(w + bh.layout.hdr + kHdrTotal);
    launch_bin(bh.batch, kModeWork, sc, 0, tot, stream);
    st = check_launch();
    if (st != SPGEMM_OK) return st;
    unsigned long long t = 0;
    hipError_t e = hipMemcpyAsync(&t, tot, sizeof(t), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return hip_fail(e);
    st = read_errors(w, bh.layout, stream);
    if (total_host) *total_host = (int64_t)t;
    return st;
}

spgemm_status spgemm_compress(const spgemm_csr *B, uint32_t *words, int32_t *count, void *ws, size_t ws_bytes,
                              hipStream_t stream)
{
    (void)ws; (void)ws_bytes;
    if (!csr_ok(B, false) || !count || (B->nnz > 0 && !words)) return SPGEMM_ERR_INVALID_ARG;
    Batch b;
    std::memset(&b, 0, sizeof(b));
    b.nprob = 1;
    b.nb = B->nrows;
    b.p0.brp = B->row_ptr;
    b.p0.bci = B->col_idx;
    b.p0.bw = (uint2 *)words;
    b.p0.bwc = count;
    b.p0.ncols = B->ncols;
    b.p0.krows = B->nrows;
    launch_compress(b, stream);
    return check_launch();
}

spgemm_status spgemm_symbolic(const spgemm_csr *A, const spgemm_csr *B, int32_t *C_row_ptr, int32_t *C_col_idx,
                              int64_t *nnzC_host, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!C_row_ptr) return SPGEMM_ERR_INVALID_ARG;
    spgemm_csr C;
    std::memset(&C, 0, sizeof(C));
    C.nrows = A ? A->nrows : 0;
    C.ncols = B ? B->ncols : 0;
    C.row_ptr = C_row_ptr;
    C.col_idx = C_col_idx;
    return spgemm_batch_symbolic(1, A, B, &C, C_col_idx != nullptr, nnzC_host, ws, ws_bytes, stream);
}

spgemm_status spgemm_batch_symbolic(int32_t nbatch, const spgemm_csr *A, const spgemm_csr *B, spgemm_csr *C,
                                    int32_t fill, int64_t *nnzC_host, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!C) return SPGEMM_ERR_INVALID_ARG;
    for (int t = 0; t < nbatch; ++t) {
        if (!C[t].row_ptr) return SPGEMM_ERR_INVALID_ARG;
        if (fill && !C[t].col_idx) return SPGEMM_ERR_INVALID_ARG;
    }
    BatchHost bh;
    spgemm_status st = prepare_batch(nbatch, A, B, C, false, true, (char *)ws, ws_bytes, stream, bh);
    if (st != SPGEMM_OK) return st;
    return run_symbolic(bh, (char *)ws, fill ? 1 : 0, nnzC_host, stream);
}

spgemm_status spgemm_numeric(const spgemm_csr *A, const spgemm_csr *B, spgemm_csr *C, void *ws, size_t ws_bytes,
                             hipStream_t stream)
{
    return spgemm_batch_numeric(1, A, B, C, ws, ws_bytes, stream);
}

spgemm_status spgemm_batch_numeric(int32_t nbatch, const spgemm_csr *A, const spgemm_csr *B, spgemm_csr *C,
                                   void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!C) return SPGEMM_ERR_INVALID_ARG;
    for (int t = 0; t < nbatch; ++t) {
        if (C[t].nrows != A[t].nrows || C[t].ncols != B[t].ncols) return SPGEMM_ERR_DIM_MISMATCH;
        if (!C[t].row_ptr || (C[t].nnz > 0 && (!C[t].col_idx || !C[t].values))) return SPGEMM_ERR_INVALID_ARG;
    }
    BatchHost bh;
    spgemm_status st = prepare_batch(nbatch, A, B, C, true, false, (char *)ws, ws_bytes, stream, bh);
    if (st != SPGEMM_OK) return st;
    return run_numeric(bh, (char *)ws, stream);
}

spgemm_status spgemm_check_errors(void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!ws || ws_bytes < kHdrBytes) return SPGEMM_ERR_INVALID_ARG;
    Layout L;
    std::memset(&L, 0, sizeof(L));
    L.hdr = 0;
    spgemm_status st = read_errors((char *)ws, L, stream);
    if (st == SPGEMM_OK || st == SPGEMM_ERR_BAD_CSR || st == SPGEMM_ERR_INDEX_OVERFLOW ||
        st == SPGEMM_ERR_STRUCTURE) {
        launch_fill_i32((int32_t *)((char *)ws + kHdrErr), 0, 1, stream);
        spgemm_status st2 = check_launch();
        if (st == SPGEMM_OK) st = st2;
    }
    return st;
}

}  // extern "C"
