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
}  // namespace

extern "C" {

spgemm_status spgemm_backward_workspace_size(const spgemm_csr *A, const spgemm_csr *B, const spgemm_csr *W,
                                             size_t *bytes)
{
    if (!A || !B || !W || !bytes) return SPGEMM_ERR_INVALID_ARG;
    *bytes = make_layout(1, A->nrows, B->nrows, 0, B->ncols, false).total;
    return SPGEMM_OK;
}

spgemm_status spgemm_backward(const spgemm_csr *A, const spgemm_csr *B, const spgemm_csr *W, double *dA,
                              double *dB, void *ws_v, size_t ws_bytes, hipStream_t s)
{
    if (!W || !W->row_ptr || (W->nnz > 0 && (!W->col_idx || !W->values))) return SPGEMM_ERR_INVALID_ARG;
    if (!A || !B || W->nrows != A->nrows || W->ncols != B->ncols) return SPGEMM_ERR_DIM_MISMATCH;
    memo_forget(ws_v);
    BatchHost bh;
    spgemm_status st = prepare_batch(1, A, B, W, true, false, (char *)ws_v, ws_bytes, s, bh);
    if (st != SPGEMM_OK) return st;
    char *ws = (char *)ws_v;
    Sched sc = make_sched(ws, bh.layout);
    if (dA) launch_fill_f64(dA, 0.0, A->nnz, s);
    if (dB) launch_fill_f64(dB, 0.0, B->nnz, s);
    reset_header(ws, bh.layout, s);
    launch_bin(bh.batch, kModeNumeric, sc, (int)g_opt.force_spill, nullptr, s);
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
