// launch.h -- host-side launchers of the gfx950 kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace mls {

enum { kModeCount = 0, kModeFill = 1, kModeNumeric = 2, kModeWork = 3 };

void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
void launch_validate(const Batch &b, int which, const int64_t *nnz_tab, uint32_t *err, hipStream_t s);
void launch_compress(const Batch &b, hipStream_t s);
void launch_bin(const Batch &b, int mode, const Sched &sc, int force, unsigned long long *total,
                hipStream_t s);
int scan_tiles(int n);
void launch_scan(const int32_t *val, int n, int64_t *tile_sum, int64_t *prefix, hipStream_t s);
void launch_write_rowptr(const Batch &b, const int64_t *prefix, int64_t *totals, uint32_t *err, hipStream_t s);

// Symbolic phase: count (fill == 0) or fill (fill == 1) over the binned rows.
// G = lanes per row for the LDS classes.
void launch_symbolic(const Batch &b, const Sched &sc, int fill, int G, hipStream_t s);

// Fill pass from the count pass's scratch words (rows with scnt >= 0).
void launch_sym_expand(const Batch &b, const Sched &sc, hipStream_t s);

// Windows of the spill bin's rows, ceil(size / m) per row: sc.wstart[r] = the
// first window of the r-th spill row, sc.wstart[n] = their total (one workgroup).
__global__ void k_win_scan(Batch b, Sched sc, int m);

// Numeric phase (row-range fused multiply-add) over the binned rows.
void launch_numeric(const Batch &b, const Sched &sc, int G, hipStream_t s);
// The same with the lanes per row of the first (G1) and second (G2) LDS classes given.
void launch_numeric_groups(const Batch &b, const Sched &sc, int G1, int G2, hipStream_t s);

// Triangle counting over the binned rows of L (A = B = L in the batch).
void launch_tc(const Batch &b, const Sched &sc, int64_t *counts, unsigned long long *total,
               uint32_t *spill_bitmaps, int spill_slots, int64_t spill_words, hipStream_t s);
void launch_tc_bin(const Batch &b, const Sched &sc, int force, hipStream_t s);
void launch_scatter(int na, const Sched &sc, hipStream_t s);

// Backward (adjoint) over the binned rows of W (= pattern of C).
void launch_backward(const Batch &b, const Sched &sc, const double *wval, double *dA, double *dB, int G,
                     hipStream_t s);

// Deterministic adjoint (one lane per output entry, sequential sums; W_ij by
// binary search in W_i). trp/tci/tv: the transpose of A with its values.
void launch_backward_det(int32_t m, int32_t kb, const int32_t *arp, const int32_t *aci, const int32_t *brp,
                         const int32_t *bci, const double *bval, const int32_t *wrp, const int32_t *wci,
                         const double *wval, const int32_t *trp, const int32_t *tci, const double *tv, double *dA,
                         double *dB, uint32_t *err, hipStream_t s);

// Transpose and masked gather helpers.
void launch_transpose(int32_t nrows, int32_t ncols, const int32_t *rp, const int32_t *ci, const double *v,
                      int32_t *trp, int32_t *tci, double *tv, int32_t *cursor, int64_t *tile_sum,
                      int64_t *prefix, int32_t *cnt, hipStream_t s);
void launch_mask_gather(int32_t nrows, const int32_t *xrp, const int32_t *xci, const double *xv,
                        const int32_t *prp, const int32_t *pci, double *out, hipStream_t s);

// Persistent grid sizes (workgroups) per kernel shape.
int device_cu_count();
int device_max_lds();   // LDS bytes one workgroup may allocate

// Workgroups of a persistent grid: resident workgroups per CU times the CUs,
// for a kernel of kWG threads with `smem` bytes of dynamic LDS.
template <typename K>
inline int spill_grid(K kernel, int smem)
{
    static int cus = device_cu_count();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWG, (size_t)smem) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

}  // namespace mls
