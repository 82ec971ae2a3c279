// symbolic_chunked.hip -- the symbolic phase (Sec. 2.1) under an HBM budget,
// for products whose structure does not fit the fast memory. The paper
// chunks only the numeric phase; here the same row-part idea carries the
// symbolic phase: the compressed pattern of B (Sec. 2.1) stays resident in
// HBM and row parts of A stream through, each counted (and, in the fill
// pass, expanded into sorted columns) by the LDS kernels of the in-HBM path,
// with its results copied back to host memory.
//
// Workspace (the budget): the kernels' header and per-row arrays for the
// largest part, B's row pointers, its compressed words and word counts, and
// a staging area that first takes B's column indices part by part (to
// compress them) and then the parts of A (row pointers and columns) and of C
// (row pointers; columns in the fill pass). One stream; every part is
// validated on the device before its kernels run.
#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/mlspgemm.h"
#include "common.h"
#include "internal.h"
#include "launch.h"

using namespace mls;

namespace {

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct Region {
    Layout L;            // kernels' header and per-row arrays (rows_cap rows)
    size_t brp = 0, bw = 0, bwc = 0, stage = 0, stage_bytes = 0;
    int32_t rows_cap = 0;
};

// Layout for parts of at most rows_cap rows; false when it does not fit.
bool make_region(const spgemm_csr *B, int32_t rows_cap, size_t ws_bytes, Region &R)
{
    R.rows_cap = rows_cap;
    R.L = make_layout(1, rows_cap, B->nrows, 0, B->ncols, false);
    size_t off = al(R.L.total_min);
    R.brp = off; off += al(4 * ((size_t)B->nrows + 1));
    R.bw = off; off += al(8 * (size_t)std::max<int64_t>(B->nnz, 1));
    R.bwc = off; off += al(4 * (size_t)std::max<int32_t>(B->nrows, 1));
    R.stage = off;
    if (off >= ws_bytes) return false;
    R.stage_bytes = ws_bytes - off;
    return true;
}

// Greedy maximal parts [r0, r1) of n rows with at most cap rows and
// bytes(r0, r1) <= limit; false when one row alone does not fit.
template <class F>
bool cut(int32_t n, int32_t cap, size_t limit, F bytes, std::vector<std::pair<int32_t, int32_t>> &out)
{
    out.clear();
    int32_t r0 = 0;
    while (r0 < n) {
        int32_t lo = r0, hi = std::min<int64_t>(n, (int64_t)r0 + cap);
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo + 1) / 2;
            if (bytes(r0, mid) <= limit) lo = mid; else hi = mid - 1;
        }
        if (lo == r0) return false;
        out.push_back({r0, lo});
        r0 = lo;
    }
    return true;
}

bool host_rp_ok(const int32_t *rp, int32_t n, int64_t nnz)
{
    if (rp[0] != 0) return false;
    for (int32_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return false;
    return (int64_t)rp[n] == nnz;
}

spgemm_status sync_errors(char *ws, const Layout &L, hipStream_t s)
{
    spgemm_status st = check_launch();
    if (st != SPGEMM_OK) return st;
    return read_errors(ws, L, s);
}

}  // namespace

extern "C" spgemm_status spgemm_symbolic_chunked(const spgemm_csr *A, const spgemm_csr *B, int32_t *C_row_ptr,
                                                 int32_t *C_col_idx, int64_t *nnzC_host, void *ws_v,
                                                 size_t ws_bytes, hipStream_t s)
{
    if (!A || !B || !C_row_ptr || !ws_v) return SPGEMM_ERR_INVALID_ARG;
    if (A->nrows < 0 || A->ncols < 0 || B->nrows < 0 || B->ncols < 0) return SPGEMM_ERR_INVALID_ARG;
    if (A->ncols != B->nrows) return SPGEMM_ERR_DIM_MISMATCH;
    if (!A->row_ptr || !B->row_ptr || (A->nnz > 0 && !A->col_idx) || (B->nnz > 0 && !B->col_idx))
        return SPGEMM_ERR_INVALID_ARG;
    if (A->nnz >= 0x7fffffffLL || B->nnz >= 0x7fffffffLL) return SPGEMM_ERR_INDEX_OVERFLOW;
    if (((uintptr_t)ws_v & 255) != 0) return SPGEMM_ERR_INVALID_ARG;
    // host row pointers (read here to cut the parts)
    if (!host_rp_ok(A->row_ptr, A->nrows, A->nnz) || !host_rp_ok(B->row_ptr, B->nrows, B->nnz))
        return SPGEMM_ERR_BAD_CSR;
    const bool fill = C_col_idx != nullptr;
    if (fill && !host_rp_ok(C_row_ptr, A->nrows, C_row_ptr[A->nrows])) return SPGEMM_ERR_BAD_CSR;
    char *ws = (char *)ws_v;
    memo_forget(ws_v);

    // rows per part: the per-row arrays take at most a quarter of the budget
    Region R;
    {
        const size_t per_row = make_layout(1, 1 << 20, B->nrows, 0, B->ncols, false).total_min / (1 << 20) + 1;
        int64_t cap = (int64_t)(ws_bytes / 4 / per_row);
        cap = std::max<int64_t>(1, std::min<int64_t>(cap, std::max<int32_t>(A->nrows, 1)));
        if (!make_region(B, (int32_t)cap, ws_bytes, R)) return SPGEMM_ERR_BUDGET;
    }
    // parts of B's column indices for the compression, and of A (and C)
    std::vector<std::pair<int32_t, int32_t>> pb, pa;
    const int32_t *brp_h = B->row_ptr, *arp_h = A->row_ptr;
    auto b_bytes = [&](int32_t r0, int32_t r1) { return al(4 * (size_t)((int64_t)brp_h[r1] - brp_h[r0])); };
    auto a_bytes = [&](int32_t r0, int32_t r1) {
        const size_t rows = (size_t)(r1 - r0 + 1);
        size_t b = 2 * al(4 * rows) + al(4 * (size_t)((int64_t)arp_h[r1] - arp_h[r0]));
        if (fill) b += al(4 * (size_t)((int64_t)C_row_ptr[r1] - C_row_ptr[r0]));
        return b;
    };
    if (B->nrows > 0 && !cut(B->nrows, B->nrows, R.stage_bytes, b_bytes, pb)) return SPGEMM_ERR_BUDGET;
    if (A->nrows > 0 && !cut(A->nrows, R.rows_cap, R.stage_bytes, a_bytes, pa)) return SPGEMM_ERR_BUDGET;

    const Layout &L = R.L;
    int32_t *d_brp = (int32_t *)(ws + R.brp);
    uint2 *d_bw = (uint2 *)(ws + R.bw);
    int32_t *d_bwc = (int32_t *)(ws + R.bwc);
    char *stage = ws + R.stage;
    hipError_t e = hipSuccess;
    int64_t nnz_tab[2] = {0, 0};
    auto h2d = [&](void *dst, const void *src, size_t bytes) {
        if (bytes && e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    };
    auto d2h = [&](void *dst, const void *src, size_t bytes) {
        if (bytes && e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
    };
    auto fail = [&]() { return hip_fail(e); };

    // 1. B's row pointers resident; its columns part by part, validated and compressed
    h2d(d_brp, brp_h, 4 * ((size_t)B->nrows + 1));
    for (auto [k0, k1] : pb) {
        const int64_t q0 = brp_h[k0], q1 = brp_h[k1];
        int32_t *d_bci = (int32_t *)stage;
        h2d(d_bci, B->col_idx + q0, 4 * (size_t)(q1 - q0));
        Batch bt;
        std::memset(&bt, 0, sizeof(bt));
        bt.nprob = 1;
        bt.nb = k1 - k0;
        Prob &q = bt.p0;
        q.brp = d_brp + k0;
        q.bci = d_bci;
        q.bw = d_bw + q0;
        q.bwc = d_bwc + k0;
        q.krows = k1 - k0;
        q.ncols = B->ncols;
        q.b_off = (int32_t)q0;
        if (g_opt.validate) {
            nnz_tab[0] = 0;
            nnz_tab[1] = q1 - q0;
            reset_header(ws, L, s);
            h2d(ws + L.nnz_tab, nnz_tab, sizeof(nnz_tab));
            if (e != hipSuccess) return fail();
            launch_validate(bt, 1, (const int64_t *)(ws + L.nnz_tab), (uint32_t *)(ws + L.hdr + kHdrErr), s);
            spgemm_status st = sync_errors(ws, L, s);   // also keeps nnz_tab alive until the copy is done
            if (st != SPGEMM_OK) return st;
        }
        launch_compress(bt, s);
        spgemm_status st = check_launch();
        if (st != SPGEMM_OK) return st;
        e = hipStreamSynchronize(s);   // the stage is reused by the next part
        if (e != hipSuccess) return fail();
    }

    // 2. parts of A: count (row pointers of C) or fill (columns of C)
    int64_t base = 0;
    std::vector<int32_t> crp_part;
    for (auto [r0, r1] : pa) {
        const int32_t rows = r1 - r0;
        const int64_t a0 = arp_h[r0], a1 = arp_h[r1];
        char *p = stage;
        int32_t *d_arp = (int32_t *)p; p += al(4 * ((size_t)rows + 1));
        int32_t *d_aci = (int32_t *)p; p += al(4 * (size_t)(a1 - a0));
        int32_t *d_crp = (int32_t *)p; p += al(4 * ((size_t)rows + 1));
        int32_t *d_cci = (int32_t *)p;
        h2d(d_arp, arp_h + r0, 4 * ((size_t)rows + 1));
        h2d(d_aci, A->col_idx + a0, 4 * (size_t)(a1 - a0));
        if (fill) h2d(d_crp, C_row_ptr + r0, 4 * ((size_t)rows + 1));
        Batch bt;
        std::memset(&bt, 0, sizeof(bt));
        bt.nprob = 1;
        bt.na = rows;
        bt.nb = B->nrows;
        bt.max_ncols = B->ncols;
        Prob &q = bt.p0;
        q.arp = d_arp;
        q.aci = d_aci;
        q.a_off = (int32_t)a0;
        q.brp = d_brp;
        q.bw = d_bw;
        q.bwc = d_bwc;
        q.crp = d_crp;
        q.cci = fill ? d_cci : nullptr;
        q.c_off = fill ? C_row_ptr[r0] : 0;
        q.nrows = rows;
        q.ncols = B->ncols;
        q.krows = B->nrows;
        q.k_lo = 0;
        q.k_hi = B->nrows;
        reset_header(ws, L, s);
        if (g_opt.validate) {
            nnz_tab[0] = a1 - a0;
            nnz_tab[1] = 0;
            h2d(ws + L.nnz_tab, nnz_tab, sizeof(nnz_tab));
            if (e != hipSuccess) return fail();
            launch_validate(bt, 0, (const int64_t *)(ws + L.nnz_tab), (uint32_t *)(ws + L.hdr + kHdrErr), s);
            spgemm_status st = sync_errors(ws, L, s);
            if (st != SPGEMM_OK) return st;
        }
        Sched sc = make_sched(ws, L);
        launch_bin(bt, fill ? kModeFill : kModeCount, sc, bin_force(), nullptr, s);
        launch_symbolic(bt, sc, fill ? 1 : 0, choose_group(rows > 0 ? (double)(a1 - a0) / rows : 1.0), s);
        if (!fill) {
            int64_t *prefix = (int64_t *)(ws + L.prefix);
            launch_scan(sc.val, rows, (int64_t *)(ws + L.tiles), prefix, s);
            launch_write_rowptr(bt, prefix, (int64_t *)(ws + L.totals), sc.err, s);
            spgemm_status st = check_launch();
            if (st != SPGEMM_OK) return st;
            crp_part.assign((size_t)rows + 1, 0);
            d2h(crp_part.data(), d_crp, 4 * ((size_t)rows + 1));
            if (e != hipSuccess) return fail();
            st = read_errors(ws, L, s);   // synchronises: crp_part is complete
            if (st != SPGEMM_OK) return st;
            if (r0 == 0) C_row_ptr[0] = 0;
            for (int32_t i = 1; i <= rows; ++i) {
                const int64_t v = base + crp_part[i];
                if (v >= 0x7fffffffLL) return SPGEMM_ERR_INDEX_OVERFLOW;
                C_row_ptr[r0 + i] = (int32_t)v;
            }
            base += crp_part[rows];
        } else {
            spgemm_status st = check_launch();
            if (st != SPGEMM_OK) return st;
            const int64_t c0 = C_row_ptr[r0], c1 = C_row_ptr[r1];
            d2h(C_col_idx + c0, d_cci, 4 * (size_t)(c1 - c0));
            if (e != hipSuccess) return fail();
            st = read_errors(ws, L, s);   // synchronises: the stage is free again
            if (st != SPGEMM_OK) return st;
        }
    }
    if (A->nrows == 0) C_row_ptr[0] = 0;
    if (!fill && nnzC_host) *nnzC_host = base;
    return SPGEMM_OK;
}
