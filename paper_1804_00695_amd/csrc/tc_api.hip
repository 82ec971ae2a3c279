// tc_api.hip -- triangle counting entry points (Sec. 4.1.2): host
// preprocessing (degree ordering, strict lower triangle) and the masked
// compressed product on the device.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

#include "../../include/mlspgemm.h"
#include "common.h"
#include "internal.h"
#include "launch.h"

using namespace mls;

extern "C" {

spgemm_status spgemm_tc_lower(const spgemm_csr *G, int32_t *perm, int32_t *lrp, int32_t *lci, int64_t *nnzL)
{
    if (!G || !G->row_ptr || !perm || !lrp || (G->nnz > 0 && (!G->col_idx || !lci))) return SPGEMM_ERR_INVALID_ARG;
    if (G->nrows != G->ncols || G->nrows < 0) return SPGEMM_ERR_DIM_MISMATCH;
    const int32_t n = G->nrows;
    const int32_t *rp = G->row_ptr, *ci = G->col_idx;
    // vertices by descending degree, ties by ascending id
    std::iota(perm, perm + n, 0);
    std::stable_sort(perm, perm + n, [&](int32_t a, int32_t b) { return rp[a + 1] - rp[a] > rp[b + 1] - rp[b]; });
    std::vector<int32_t> inv(n);
    for (int32_t i = 0; i < n; ++i) inv[perm[i]] = i;
    // row lengths of L: neighbours with a smaller new label
    lrp[0] = 0;
    int64_t tot = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t v = perm[i];
        int32_t c = 0;
        for (int32_t p = rp[v]; p < rp[v + 1]; ++p) {
            int32_t u = ci[p];
            if (u < 0 || u >= n || u == v) return SPGEMM_ERR_BAD_CSR;
            c += inv[u] < i;
        }
        tot += c;
        if (tot >= 0x7fffffffLL) return SPGEMM_ERR_INDEX_OVERFLOW;
        lrp[i + 1] = (int32_t)tot;
    }
    // fill rows in parallel, each sorted
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned w = 0; w < nt; ++w) {
        pool.emplace_back([&, w]() {
            for (int32_t i = (int32_t)w; i < n; i += (int32_t)nt) {
                const int32_t v = perm[i];
                int32_t *out = lci + lrp[i];
                int32_t c = 0;
                for (int32_t p = rp[v]; p < rp[v + 1]; ++p) {
                    int32_t j = inv[ci[p]];
                    if (j < i) out[c++] = j;
                }
                std::sort(out, out + c);
            }
        });
    }
    for (auto &t : pool) t.join();
    if (nnzL) *nnzL = tot;
    return SPGEMM_OK;
}

spgemm_status spgemm_tc_workspace_size(const spgemm_csr *L, size_t *bytes)
{
    if (!L || !bytes) return SPGEMM_ERR_INVALID_ARG;
    *bytes = make_layout(1, L->nrows, L->nrows, L->nnz, L->ncols, true).total_min;
    return SPGEMM_OK;
}

spgemm_status spgemm_tc(const spgemm_csr *L, int64_t *counts, int64_t *total_host, void *ws_v, size_t ws_bytes,
                        hipStream_t s)
{
    if (!L || !counts || !L->row_ptr || (L->nnz > 0 && !L->col_idx)) return SPGEMM_ERR_INVALID_ARG;
    if (L->nrows != L->ncols) return SPGEMM_ERR_DIM_MISMATCH;
    spgemm_csr Lp = *L;
    Lp.values = nullptr;
    memo_forget(ws_v);
    BatchHost bh;
    spgemm_status st = prepare_batch(1, &Lp, &Lp, nullptr, false, true, (char *)ws_v, ws_bytes, s, bh);
    if (st != SPGEMM_OK) return st;
    char *ws = (char *)ws_v;
    const Layout &Lay = bh.layout;
    Sched sc = make_sched(ws, Lay);
    reset_header(ws, Lay, s);
    launch_fill_i32((int32_t *)counts, 0, 2 * (int64_t)L->nrows, s);
    if (g_opt.validate) {
        launch_validate(bh.batch, 0, (const int64_t *)(ws + Lay.nnz_tab), sc.err, s);
        st = check_launch();
        if (st != SPGEMM_OK) return st;
        st = read_errors(ws, Lay, s);
        if (st != SPGEMM_OK) return st;
    }
    unsigned long long *tot = (unsigned long long *)(ws + Lay.hdr + kHdrTotal);
    launch_compress(bh.batch, s);
    launch_tc_bin(bh.batch, sc, bin_force(), s);
    launch_tc(bh.batch, sc, counts, tot, (uint32_t *)(ws + Lay.spill), Lay.spill_slots, Lay.spill_words, s);
    st = check_launch();
    if (st != SPGEMM_OK) return st;
    unsigned long long t = 0;
    hipError_t e = hipMemcpyAsync(&t, tot, sizeof(t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e);
    st = read_errors(ws, Lay, s);
    if (total_host) *total_host = (int64_t)t;
    return st;
}

}  // extern "C"
