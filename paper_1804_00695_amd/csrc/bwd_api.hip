// bwd_api.hip -- entry points of the adjoint and of its helpers (transpose,
// masked gather).
#include <algorithm>
#include <cstring>

#include "../../include/mlspgemm.h"
#include "common.h"
#include "internal.h"
#include "launch.h"

using namespace mls;

namespace {
inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

size_t transpose_ws(int64_t ncols)
{
    return al(4 * (size_t)std::max<int64_t>(ncols, 1)) * 2 + al(8 * (size_t)scan_tiles((int)ncols)) +
           al(8 * (size_t)(ncols + 1));
}

// Workspace of the deterministic adjoint: the header (error word), the
// transpose of A with its values, and the transpose's own scratch.
struct DetLayout {
    size_t trp = 0, tci = 0, tv = 0, cnt = 0, cursor = 0, tiles = 0, prefix = 0, total = 0;
};

DetLayout det_layout(const spgemm_csr *A)
{
    DetLayout d;
    const int64_t nc = std::max<int64_t>(A->ncols, 0), nz = std::max<int64_t>(A->nnz, 1);
    size_t off = al(kHdrBytes);
    d.trp = off; off += al(4 * (size_t)(nc + 1));
    d.tci = off; off += al(4 * (size_t)nz);
    d.tv = off; off += al(8 * (size_t)nz);
    d.cnt = off; off += al(4 * (size_t)std::max<int64_t>(nc, 1));
    d.cursor = off; off += al(4 * (size_t)std::max<int64_t>(nc, 1));
    d.tiles = off; off += al(8 * (size_t)scan_tiles((int)nc));
    d.prefix = off; off += al(8 * (size_t)(nc + 1));
    d.total = off;
    return d;
}
}  // namespace

extern "C" {

spgemm_status spgemm_backward_workspace_size(const spgemm_csr *A, const spgemm_csr *B, const spgemm_csr *W,
                                             int32_t deterministic, size_t *bytes)
{
    if (!A || !B || !W || !bytes) return SPGEMM_ERR_INVALID_ARG;
    if (deterministic) {
        DetLayout d = det_layout(A);
        *bytes = d.total;
    } else {
        *bytes = make_layout(1, A->nrows, B->nrows, 0, B->ncols, false).total;
    }
    return SPGEMM_OK;
}

spgemm_status spgemm_backward(const spgemm_csr *A, const spgemm_csr *B, const spgemm_csr *W, double *dA,
                              double *dB, int32_t deterministic, void *ws_v, size_t ws_bytes, hipStream_t s)
{
    if (!W || !W->row_ptr || (W->nnz > 0 && (!W->col_idx || !W->values))) return SPGEMM_ERR_INVALID_ARG;
    if (!A || !B || W->nrows != A->nrows || W->ncols != B->ncols) return SPGEMM_ERR_DIM_MISMATCH;
    memo_forget(ws_v);
    if (deterministic) {
        if (A->ncols != B->nrows) return SPGEMM_ERR_DIM_MISMATCH;
        if (!A->row_ptr || !B->row_ptr || A->nrows < 0 || B->nrows < 0) return SPGEMM_ERR_INVALID_ARG;
        if ((A->nnz > 0 && (!A->col_idx || !A->values)) || (B->nnz > 0 && (!B->col_idx || !B->values)))
            return SPGEMM_ERR_INVALID_ARG;
        const DetLayout d = det_layout(A);
        if (!ws_v || ws_bytes < d.total) return SPGEMM_ERR_WORKSPACE_TOO_SMALL;
        if (((uintptr_t)ws_v & 255) != 0) return SPGEMM_ERR_INVALID_ARG;
        char *w = (char *)ws_v;
        launch_fill_i32((int32_t *)w, 0, kHdrBytes / 4, s);   // error word
        int32_t *trp = (int32_t *)(w + d.trp);
        int32_t *tci = (int32_t *)(w + d.tci);
        double *tv = (double *)(w + d.tv);
        if (dB)
            launch_transpose(A->nrows, A->ncols, A->row_ptr, A->col_idx, A->values, trp, tci, tv,
                             (int32_t *)(w + d.cursor), (int64_t *)(w + d.tiles), (int64_t *)(w + d.prefix),
                             (int32_t *)(w + d.cnt), s);
        launch_backward_det(A->nrows, B->nrows, A->row_ptr, A->col_idx, B->row_ptr, B->col_idx, B->values,
                            W->row_ptr, W->col_idx, W->values, trp, tci, tv, dA, dB, (uint32_t *)w, s);
        return check_launch();
    }
    BatchHost bh;
    spgemm_status st = prepare_batch(1, A, B, W, true, false, (char *)ws_v, ws_bytes, s, bh);
    if (st != SPGEMM_OK) return st;
    char *ws = (char *)ws_v;
    Sched sc = make_sched(ws, bh.layout);
    if (dA) launch_fill_f64(dA, 0.0, A->nnz, s);
    if (dB) launch_fill_f64(dB, 0.0, B->nnz, s);
    reset_header(ws, bh.layout, s);
    launch_bin(bh.batch, kModeNumeric, sc, bin_force(), nullptr, s);
    launch_backward(bh.batch, sc, W->values, dA, dB, choose_group(bh.avg_b), s);
    return check_launch();
}

spgemm_status spgemm_transpose_workspace_size(const spgemm_csr *M, size_t *bytes)
{
    if (!M || !bytes) return SPGEMM_ERR_INVALID_ARG;
    *bytes = transpose_ws(M->ncols);
    return SPGEMM_OK;
}

spgemm_status spgemm_transpose(const spgemm_csr *M, spgemm_csr *T, void *ws_v, size_t ws_bytes, hipStream_t s)
{
    if (!M || !T || !M->row_ptr || !T->row_ptr || (M->nnz > 0 && (!M->col_idx || !T->col_idx)))
        return SPGEMM_ERR_INVALID_ARG;
    if (T->nrows != M->ncols || T->ncols != M->nrows || T->nnz != M->nnz) return SPGEMM_ERR_DIM_MISMATCH;
    if (M->values && !T->values && M->nnz > 0) return SPGEMM_ERR_INVALID_ARG;
    if (!ws_v || ws_bytes < transpose_ws(M->ncols) || ((uintptr_t)ws_v & 255)) return SPGEMM_ERR_WORKSPACE_TOO_SMALL;
    memo_forget(ws_v);
    char *w = (char *)ws_v;
    const size_t a = al(4 * (size_t)std::max<int64_t>(M->ncols, 1));
    int32_t *cnt = (int32_t *)w;
    int32_t *cursor = (int32_t *)(w + a);
    int64_t *tiles = (int64_t *)(w + 2 * a);
    int64_t *prefix = (int64_t *)(w + 2 * a + al(8 * (size_t)scan_tiles(M->ncols)));
    launch_transpose(M->nrows, M->ncols, M->row_ptr, M->col_idx, M->values, T->row_ptr, T->col_idx,
                     M->values ? T->values : nullptr, cursor, tiles, prefix, cnt, s);
    return check_launch();
}

spgemm_status spgemm_mask_gather(const spgemm_csr *X, const spgemm_csr *Pt, double *out, hipStream_t s)
{
    if (!X || !Pt || !out || !X->row_ptr || !Pt->row_ptr) return SPGEMM_ERR_INVALID_ARG;
    if (X->nrows != Pt->nrows || X->ncols != Pt->ncols) return SPGEMM_ERR_DIM_MISMATCH;
    if (X->nnz > 0 && (!X->col_idx || !X->values)) return SPGEMM_ERR_INVALID_ARG;
    launch_mask_gather(X->nrows, X->row_ptr, X->col_idx, X->values, Pt->row_ptr, Pt->col_idx, out, s);
    return check_launch();
}

}  // extern "C"
