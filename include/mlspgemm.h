/*
 * mlspgemm.h -- C ABI of the MI355X (gfx950) two-phase SpGEMM library.
 *
 * Method: Deveci, Hammond, Wolf, Rajamanickam, "Sparse Matrix-Matrix
 * Multiplication on Multilevel Memory Architectures: Algorithms and
 * Experiments" (arXiv 1804.00695).
 *
 *   C = A * B on CSR, row-wise (Gustavson), in two phases (Sec. 2.1): a
 *   symbolic phase that finds the structure of C from compressed column
 *   masks of B, and a numeric phase that accumulates a_ik * B_k per row in
 *   an on-chip hash accumulator. Chunked execution (Sec. 3.3.1, Algs.
 *   "chunker", "chunk1", "chunk2") streams row parts of A, B and C between
 *   pinned host memory (the slow tier) and HBM (the fast tier) under a
 *   caller-chosen HBM budget.
 *
 * Conventions for every entry point:
 *   - Indices are int32, values fp64. Row pointers start at 0 and are
 *     non-decreasing; the columns of each row are strictly increasing and
 *     lie in [0, ncols). Structural entries of C are kept even when their
 *     value sums to 0.0; the columns of each row of C come out ascending.
 *   - Pointers inside spgemm_csr are device pointers unless the function
 *     says "host". The caller owns all memory. The library never allocates
 *     device memory: every entry point that needs scratch space takes a
 *     workspace (ws, ws_bytes) whose minimum size a *_workspace_size call
 *     returns; the workspace must be 256-byte aligned and must not be used
 *     by anything else until the work queued on the stream has finished.
 *   - Work is queued on the given stream(s). A function returns before the
 *     queued work ends unless it says it synchronises.
 *   - Every function returns an spgemm_status and never aborts. After
 *     SPGEMM_ERR_HIP, spgemm_last_hip_error() holds the HIP error code.
 *   - Floating point: products are rounded before they are added (no fused
 *     multiply-add) and the terms of each c_ij are added in ascending k,
 *     the order of the row-wise formulation; results are deterministic.
 */
#ifndef MLSPGEMM_H
#define MLSPGEMM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPGEMM_OK = 0,
    SPGEMM_ERR_INVALID_ARG = 1,        /* NULL pointer, negative size, bad option */
    SPGEMM_ERR_BAD_CSR = 2,            /* row_ptr not starting at 0 / decreasing, column out of range,
                                          columns of a row not strictly increasing */
    SPGEMM_ERR_DIM_MISMATCH = 3,       /* A.ncols != B.nrows, or C not shaped A.nrows x B.ncols */
    SPGEMM_ERR_INDEX_OVERFLOW = 4,     /* nnz(C), a row's work or a row pointer would reach 2^31 */
    SPGEMM_ERR_WORKSPACE_TOO_SMALL = 5,
    SPGEMM_ERR_BUDGET = 6,             /* a single row or part cannot fit the HBM budget */
    SPGEMM_ERR_HIP = 7,                /* a HIP runtime call failed; see spgemm_last_hip_error() */
    SPGEMM_ERR_UNSUPPORTED = 8,
    SPGEMM_ERR_STRUCTURE = 9           /* C's structure does not contain a column that A*B reaches */
} spgemm_status;

/* A CSR matrix. nnz must equal row_ptr[nrows] (host copy of it). */
typedef struct {
    int32_t nrows;
    int32_t ncols;
    int64_t nnz;
    int32_t *row_ptr;      /* nrows + 1 */
    int32_t *col_idx;      /* nnz */
    double *values;        /* nnz, or NULL for a pattern-only matrix */
} spgemm_csr;

const char *spgemm_status_string(spgemm_status s);
int spgemm_last_hip_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int spgemm_version(void);

/* Process-wide options (not thread safe; set before queueing work). */
typedef enum {
    SPGEMM_OPT_VALIDATE = 0,      /* 1 (default): the symbolic phase checks A and B on the device */
    SPGEMM_OPT_FORCE_SPILL = 1,   /* 1: every row takes the global-memory accumulator path (test knob) */
    SPGEMM_OPT_GROUP_SIZE = 2,    /* 0 (default): lanes per row chosen from row lengths; else 8/16/32/64 */
    SPGEMM_OPT_FORCE_CLASS = 3,   /* -1 (default): rows binned by size; c in 0..4: every row of the
                                     symbolic, numeric and adjoint phases whose size class is below c
                                     runs in LDS class c instead (test knob: every class kernel then
                                     sees rows of every size; results are unchanged) */
    SPGEMM_OPT_PROFILE = 4,       /* 1: time every kernel launch with a HIP event pair on its stream */
    SPGEMM_OPT_WIDE_TABLE = 5     /* 1: the numeric phase keeps 8-byte (column, position) hash slots
                                     even where column and position fit one 32-bit slot (test knob) */
} spgemm_option;
spgemm_status spgemm_set_option(spgemm_option opt, int64_t value);
int64_t spgemm_get_option(spgemm_option opt);

/* Kernel timing collected while SPGEMM_OPT_PROFILE is on: per kernel name,
 * the number of launches and the summed elapsed time between the events
 * recorded just before and just after each launch on the launch stream.
 * spgemm_profile_read waits for the pending events, folds them into the
 * totals and copies up to max_entries entries; it returns the number of
 * distinct kernels. spgemm_profile_reset clears the totals. */
typedef struct {
    char name[64];
    int64_t calls;
    double total_ms;
} spgemm_profile_entry;
int32_t spgemm_profile_read(spgemm_profile_entry *out, int32_t max_entries);
void spgemm_profile_reset(void);

/* Host-only CSR check of a matrix in host memory (same rules as the device
 * check). Returns SPGEMM_OK or SPGEMM_ERR_BAD_CSR. */
spgemm_status spgemm_validate_host(const spgemm_csr *M_host);

/* ------------------------------------------------------------------------
 * Plain product, everything in HBM (Sec. 2.1)
 * --------------------------------------------------------------------- */

/* Workspace for spgemm_row_work, spgemm_compress, spgemm_symbolic and
 * spgemm_numeric on these shapes (only nrows, ncols, nnz are read). The
 * size returned includes a per-row scratch (64 words of 8 bytes per row of
 * A) in which the symbolic count pass keeps each row's compressed column
 * set for the fill pass; a smaller workspace still works down to the size
 * without that scratch (the fill pass then recomputes every row), and
 * below that calls return SPGEMM_ERR_WORKSPACE_TOO_SMALL. */
spgemm_status spgemm_workspace_size(const spgemm_csr *A, const spgemm_csr *B, size_t *bytes);

/* Row work estimate (the input of row binning): work[i] = number of
 * multiply-adds of row i of C, sum over k in row i of A of nnz(row k of B).
 * work: device int32[A.nrows]. *total_host receives the int64 sum and the
 * call synchronises the stream. Errors: SPGEMM_ERR_INDEX_OVERFLOW if a
 * single row's work reaches 2^31. */
spgemm_status spgemm_row_work(const spgemm_csr *A, const spgemm_csr *B, int32_t *work,
                              int64_t *total_host, void *ws, size_t ws_bytes, hipStream_t stream);

/* Column compression of B's pattern (Sec. 2.1: several columns of a row of
 * B encoded with fewer integers so that unions are bitwise ORs). Column j
 * is bit (j & 31) of the word of set (j >> 5). Row k's words are written,
 * sets ascending, at words[2*(B.row_ptr[k] + w)] = set and
 * words[2*(B.row_ptr[k] + w) + 1] = mask for w < count[k] (a row never has
 * more words than entries, so the words of row k live inside row k's entry
 * range). words: device uint32[2 * B.nnz]; count: device int32[B.nrows].
 * Does not synchronise. */
spgemm_status spgemm_compress(const spgemm_csr *B, uint32_t *words, int32_t *count,
                              void *ws, size_t ws_bytes, hipStream_t stream);

/* Symbolic phase (Sec. 2.1). Two passes:
 *   count pass (C_col_idx == NULL): writes C_row_ptr[A.nrows + 1] (device)
 *     and *nnzC_host; synchronises the stream (the caller needs nnz(C) to
 *     allocate C). Validates A and B first when SPGEMM_OPT_VALIDATE is on.
 *   fill pass (C_col_idx != NULL): C_row_ptr must hold the count pass's
 *     result; writes the ascending, unique columns of every row of C into
 *     C_col_idx[nnz(C)]. nnzC_host may be NULL. Does not synchronise.
 *     When it directly follows a count pass on the same operands (same
 *     pointers, shapes and workspace, and no other call on that workspace
 *     in between), it reuses the compressed B and the per-row column sets
 *     that the count pass left in the workspace; A and B must not have
 *     been modified in between. Otherwise it recomputes them.
 * Errors: SPGEMM_ERR_BAD_CSR, SPGEMM_ERR_DIM_MISMATCH,
 * SPGEMM_ERR_INDEX_OVERFLOW (nnz(C) >= 2^31). */
spgemm_status spgemm_symbolic(const spgemm_csr *A, const spgemm_csr *B, int32_t *C_row_ptr,
                              int32_t *C_col_idx, int64_t *nnzC_host, void *ws, size_t ws_bytes,
                              hipStream_t stream);

/* Symbolic phase under an HBM budget, for products whose structure does not
 * fit the fast memory (the paper chunks only the numeric phase; this carries
 * its row-part idea over to Sec. 2.1's symbolic phase). A_host and B_host
 * hold host arrays (row_ptr, col_idx; values unused); C_row_ptr_host and
 * C_col_idx_host are host arrays too. The workspace (device memory) is the
 * budget: B's compressed pattern (8 bytes per entry of B plus 8 per row)
 * stays in it while row parts of A stream through, so every byte the call
 * uses lies in [ws, ws + ws_bytes). Same two passes as spgemm_symbolic:
 *   count (C_col_idx_host == NULL): writes C_row_ptr_host[A.nrows + 1] and
 *     *nnzC_host (may be NULL);
 *   fill (C_col_idx_host != NULL): C_row_ptr_host must hold the count
 *     pass's result; writes the ascending, unique columns of every row.
 * A and B are validated on the device part by part when SPGEMM_OPT_VALIDATE
 * is on. Synchronises the stream (one synchronisation per part). The result
 * equals spgemm_symbolic's. Errors: SPGEMM_ERR_BUDGET when B's compressed
 * pattern and one row of A (and of C) do not fit ws_bytes, SPGEMM_ERR_BAD_CSR,
 * SPGEMM_ERR_DIM_MISMATCH, SPGEMM_ERR_INDEX_OVERFLOW (nnz(C) >= 2^31). */
spgemm_status spgemm_symbolic_chunked(const spgemm_csr *A_host, const spgemm_csr *B_host,
                                      int32_t *C_row_ptr_host, int32_t *C_col_idx_host, int64_t *nnzC_host,
                                      void *ws, size_t ws_bytes, hipStream_t stream);

/* Numeric phase (Sec. 2.1, Fig. "spgemmexp"): C->values[e] = sum over k of
 * a_ik * b_kj for every stored (i, j) of C, terms added in ascending k.
 * C->row_ptr and C->col_idx must be the symbolic phase's result (any
 * superset structure with ascending columns also works: columns not
 * reached get 0.0). A and B must carry values. Does not synchronise. A
 * column reached by A*B but missing from C sets an error that the next
 * synchronising call reports as SPGEMM_ERR_STRUCTURE. */
spgemm_status spgemm_numeric(const spgemm_csr *A, const spgemm_csr *B, spgemm_csr *C,
                             void *ws, size_t ws_bytes, hipStream_t stream);

/* Data placement (Sec. 3.3, Table "gpudp"): spgemm_numeric with any of A, B
 * and C left in page-locked host memory, read (A, B, C's structure) and
 * written (C's values) in place by the kernels over the host link, with no
 * copy -- the paper's A_Pin, B_Pin, C_Pin and HostPin placements. Each array
 * pointer must be device memory of the current device or host memory
 * allocated page-locked with hipHostMalloc (torch's pin_memory), which is
 * used through its device mapping; pageable host memory, managed memory and
 * memory of another device give SPGEMM_ERR_INVALID_ARG before anything is
 * queued. The workspace must be device memory of the current device (same
 * size as for spgemm_numeric). *placement_out (may be NULL) receives bit 0,
 * 1, 2 set when an array of A, B, C is in host memory. Same kernels and the
 * same results, bit for bit, as spgemm_numeric. Does not synchronise. */
spgemm_status spgemm_numeric_placed(const spgemm_csr *A, const spgemm_csr *B, spgemm_csr *C,
                                    uint32_t *placement_out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Reports and clears the device-side error flag of a workspace (the word at
 * its start) after the work queued on the stream has finished (synchronises
 * the stream). */
spgemm_status spgemm_check_errors(void *ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): spgemm_numeric with
 * no workspace argument. Same kernels, same results bit for bit. Its scratch
 * is a fixed 64 MiB array in device memory that each GPU the library runs on
 * holds until the process ends (the per-row arrays take about 17 bytes per
 * row of A, so A may have up to about 3.9 million rows); a larger A returns
 * SPGEMM_ERR_WORKSPACE_TOO_SMALL before anything is queued. Allocates no
 * device memory and makes no host-to-device copy. The caller still owns A, B
 * and C (device memory, C's structure from the symbolic phase). Every call on
 * one GPU uses that GPU's same array: calls that overlap in time on one GPU
 * (two streams, two threads) race and give wrong results; serialise them.
 * Device-side errors (a column missing from C) are recorded in the array's
 * first word and are not reported by this call. Does not synchronise. */
spgemm_status spgemm_numeric_noalloc(const spgemm_csr *A, const spgemm_csr *B, spgemm_csr *C,
                                     hipStream_t stream);

/* ------------------------------------------------------------------------
 * Chunked execution between pinned host memory and HBM (Sec. 3.3.1)
 * --------------------------------------------------------------------- */

typedef struct spgemm_plan spgemm_plan;

typedef struct {
    int32_t algo;            /* 1 = Alg. chunk1 (A/C parts in place, B streams),
                                2 = Alg. chunk2 (B parts in place, A/C stream),
                                3 = Alg. chunkknl (B streams; A and C stay in host
                                    memory and the kernels access them in place) */
    int32_t branch;          /* which case of Alg. chunker decided (1..4; 0 for chunkknl) */
    int32_t n_ac_parts;      /* |P_AC| */
    int32_t n_b_parts;       /* |P_B| */
    int32_t nbuf_inner;      /* buffers of the inner-loop matrix (1 to 4) */
    int32_t n_steps;
    int64_t fast_bytes;      /* FastSize handed to the partition heuristic */
    int64_t h2d_bytes;       /* bytes the schedule copies host -> device */
    int64_t d2h_bytes;       /* bytes the schedule copies device -> host */
    int64_t cost_chunk1;     /* total copy bytes of chunk1 over these parts */
    int64_t cost_chunk2;     /* total copy bytes of chunk2 over these parts */
    int64_t chunk_bytes;     /* HBM of the part buffers */
    int64_t ws_bytes;        /* workspace spgemm_numeric_chunked needs (<= budget) */
    int64_t issued_h2d;      /* bytes the last execution actually queued host -> device */
    int64_t issued_d2h;      /* bytes the last execution actually queued device -> host */
    int64_t zero_copy_bytes; /* chunkknl: bytes the kernels read and write in place in host
                                memory (A and C's structure read and C's values written by
                                every pass, C's values read by every pass after the first) */
} spgemm_plan_info;

/* One step of the schedule, in issue order. */
typedef struct {
    int32_t kind;            /* 0 = copy host->device, 1 = copy device->host, 2 = kernel, 3 = zero C values */
    int32_t matrix;          /* 0 = A, 1 = B, 2 = C structure (row_ptr + col_idx), 3 = C values */
    int32_t part;            /* index into P_AC (A, C, kernel) or P_B (B) */
    int32_t row_begin;       /* row range [row_begin, row_end) of that matrix; for a kernel, of B */
    int32_t row_end;
    int32_t slot;            /* buffer of the inner-loop matrix */
    int64_t bytes;
} spgemm_plan_step;

/* Alg. "chunker" (Partition) on host data: A_host and B_host give the row
 * pointers (host) and shapes; C_row_ptr_host is the symbolic phase's row
 * pointer of C (host). The HBM budget bounds the workspace that
 * spgemm_numeric_chunked will need; FastSize is the budget less a reserve
 * for the kernels' own per-row arrays. nbuf = 1 reproduces the paper's
 * single-buffered loops; nbuf = 2..4 gives the inner-loop matrix that many
 * buffers so its copies overlap the kernels (double, triple, quadruple
 * buffering; the paper names these as future work, Sec. 4.2). min_parts >= 1
 * cuts the inner-loop matrix into at least that many parts (pipelining when
 * it fits whole). Host only, no GPU needed. Errors: SPGEMM_ERR_BUDGET when a
 * single row does not fit its portion. The plan is owned by the caller
 * (spgemm_plan_destroy). */
spgemm_status spgemm_chunked_plan(const spgemm_csr *A_host, const spgemm_csr *B_host,
                                  const int32_t *C_row_ptr_host, size_t hbm_budget_bytes,
                                  int32_t nbuf, int32_t min_parts, spgemm_plan **plan_out);
/* Alg. "chunkknl" (Sec. 3.2.2): only B is partitioned. The number of parts is
 * ceil(size(B) / portion) (at least min_parts), the balanced part size is
 * size(B) over that number, and BinarySearch cuts B's rows into parts of at
 * most that size; portion = FastSize / nbuf. A and C are not copied: the
 * row-range kernels read A and C's structure and accumulate C's values in
 * place, over the host link when they are in host memory (with everything
 * but B in host memory this is the paper's KNL scheme; with B whole in HBM,
 * its data-placement method). Same arguments and errors as
 * spgemm_chunked_plan; the plan reports algo = 3. */
spgemm_status spgemm_chunked_plan_knl(const spgemm_csr *A_host, const spgemm_csr *B_host,
                                      const int32_t *C_row_ptr_host, size_t hbm_budget_bytes,
                                      int32_t nbuf, int32_t min_parts, spgemm_plan **plan_out);
spgemm_status spgemm_plan_info_get(const spgemm_plan *plan, spgemm_plan_info *out);
/* Copies min(max_parts, n) (begin, end) pairs of P_AC (which = 0) or P_B
 * (which = 1) into ranges[2*i], ranges[2*i+1]. */
spgemm_status spgemm_plan_parts(const spgemm_plan *plan, int32_t which, int32_t *ranges, int32_t max_parts);
spgemm_status spgemm_plan_steps(const spgemm_plan *plan, spgemm_plan_step *steps, int32_t max_steps);
void spgemm_plan_destroy(spgemm_plan *plan);

/* Chunked numeric phase (Algs. chunk1 / chunk2 with the row-range fused
 * multiply-add kernel, C_r += A_r[:, P_B] * B_b, Sec. 3.2.2/3.3.1). A_host,
 * B_host and C_host hold host pointers to pinned memory (row_ptr, col_idx,
 * values); C_host's structure is the symbolic result and its values are
 * written. For a chunkknl plan (algo 3) A and C are used in place: each of
 * their arrays must be page-locked host memory from hipHostMalloc (torch's
 * pin_memory) or device memory of the current device (else
 * SPGEMM_ERR_INVALID_ARG before anything is queued). ws must hold
 * info.ws_bytes of device memory. Copies host->device are queued on s_h2d,
 * device->host on s_d2h, kernels on s_compute (they may be the same stream);
 * events order them. The row binning of an A/C part is done by its first
 * kernel step and reused by the others. Synchronises all three streams
 * before returning and records the issued byte counts in the plan. The
 * result equals spgemm_numeric's bit for bit. */
spgemm_status spgemm_numeric_chunked(const spgemm_csr *A_host, const spgemm_csr *B_host,
                                     spgemm_csr *C_host, spgemm_plan *plan, void *ws, size_t ws_bytes,
                                     hipStream_t s_compute, hipStream_t s_h2d, hipStream_t s_d2h);

/* Test support: what spgemm_numeric_chunked would queue for this plan and
 * these host operands, recorded instead of queued (no GPU call; nothing is
 * read but the host row pointers, nothing is written but out). Each entry is
 * one access of one operation, in issue order: op numbers the operation;
 * kind 0 copy host->device, 1 copy device->host, 2 kernel (the first
 * operation, kernel on the whole workspace, stands for work queued earlier
 * on the compute stream), 3 fill, 4 event record, 5 event wait; stream 0
 * compute, 1 host->device, 2 device->host; event (record / wait) an id, else
 * -1; space 0 the workspace, 1 C's values in host memory, -1 none; write 1
 * for a write, 0 for a read; [lo, hi) the byte range in that space. A
 * checker can derive the happens-before order from stream order and the
 * events and verify that conflicting accesses are ordered. *n_entries
 * receives the count; at most max_entries are copied. */
typedef struct {
    int32_t op, kind, stream, event, space, write;
    int64_t lo, hi;
} spgemm_trace_entry;
spgemm_status spgemm_numeric_chunked_trace(const spgemm_csr *A_host, const spgemm_csr *B_host,
                                           const spgemm_csr *C_host, spgemm_plan *plan, spgemm_trace_entry *out,
                                           int64_t max_entries, int64_t *n_entries);

/* ------------------------------------------------------------------------
 * Triangle counting (Sec. 4.1.2)
 * --------------------------------------------------------------------- */

/* Host preprocessing: relabel the vertices of the symmetric pattern G_host
 * (no self loops) by descending degree, ties by ascending id, and build L,
 * the strict lower triangle in the new labels (row i holds the new labels
 * j < i of its neighbours, ascending). perm_host[new] = old id. L_row_ptr_host
 * has nv+1 entries, L_col_idx_host nnz(G)/2. */
spgemm_status spgemm_tc_lower(const spgemm_csr *G_host, int32_t *perm_host, int32_t *L_row_ptr_host,
                              int32_t *L_col_idx_host, int64_t *nnzL_host);

spgemm_status spgemm_tc_workspace_size(const spgemm_csr *L, size_t *bytes);

/* Masked product (L * compressed(L)) o L, summed per row: counts[i] =
 * sum over k in row i of L of |row k of L intersected with row i of L|
 * (device int64[L.nrows]); *total_host = number of triangles. Pattern only
 * (values ignored). Synchronises the stream. */
spgemm_status spgemm_tc(const spgemm_csr *L, int64_t *counts, int64_t *total_host, void *ws,
                        size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched products (many independent C_t = A_t * B_t in each launch)
 * --------------------------------------------------------------------- */

/* The arrays A, B, C hold nbatch handles (host arrays of device CSR). */
spgemm_status spgemm_batch_workspace_size(int32_t nbatch, const spgemm_csr *A, const spgemm_csr *B,
                                          size_t *bytes);
/* Count pass over all products in one set of launches and one readback:
 * writes every C[t].row_ptr and nnzC_host[t]; synchronises. With
 * fill != 0, C[t].col_idx must be allocated and the columns are written
 * instead (no synchronisation). */
spgemm_status spgemm_batch_symbolic(int32_t nbatch, const spgemm_csr *A, const spgemm_csr *B,
                                    spgemm_csr *C, int32_t fill, int64_t *nnzC_host, void *ws,
                                    size_t ws_bytes, hipStream_t stream);
spgemm_status spgemm_batch_numeric(int32_t nbatch, const spgemm_csr *A, const spgemm_csr *B,
                                   spgemm_csr *C, void *ws, size_t ws_bytes, hipStream_t stream);

/* Reusable numeric plan for a batch with fixed structure (multigrid setup
 * reuse): the row binning is done once, the launches are captured into a
 * HIP graph, and spgemm_batch_plan_run replays them. The plan keeps
 * pointers to the caller's arrays and its part of the workspace; both must
 * stay valid until spgemm_batch_plan_destroy.
 * group_size 8/16/32/64: lanes per row of the first LDS class, rows binned by
 * size. group_size 0: autotuned -- every combination of the lanes per row of
 * the first LDS class (8, 16, 32, 64), of the second (32, 64), and of the
 * row-bin threshold between the two smallest classes (rows binned by size,
 * or every row of the smallest class moved up to the next) is timed on the
 * batch with HIP events and the fastest kept; all give identical results.
 * The choice is cached in the process by the batch's shape, and, when
 * tune_cache_path is not NULL, read from and appended to that text file
 * (lines "batch <nbatch> <rows of A> <rows of B> <nnz A> <nnz C> <device>
 * <g1> <g2> <floor>"; unreadable lines are ignored), so that other processes
 * on the same kind of GPU skip the search. Tuning synchronises the stream. */
typedef struct spgemm_batch_plan spgemm_batch_plan;
spgemm_status spgemm_batch_plan_create(int32_t nbatch, const spgemm_csr *A, const spgemm_csr *B,
                                       spgemm_csr *C, int32_t group_size, int32_t use_graph,
                                       const char *tune_cache_path, void *ws, size_t ws_bytes,
                                       hipStream_t stream, spgemm_batch_plan **out);
spgemm_status spgemm_batch_plan_run(spgemm_batch_plan *plan, hipStream_t stream);
/* Lanes per row the plan uses for its first LDS class (the autotuned value
 * when created with group_size 0). */
int32_t spgemm_batch_plan_group_size(const spgemm_batch_plan *plan);
/* The plan's whole schedule: lanes per row of the first and second LDS
 * classes and the row-bin floor (-1: rows binned by size; 1: the smallest
 * class's rows moved up to the next). */
spgemm_status spgemm_batch_plan_schedule(const spgemm_batch_plan *plan, int32_t *g1, int32_t *g2, int32_t *floor);
void spgemm_batch_plan_destroy(spgemm_batch_plan *plan);

/* ------------------------------------------------------------------------
 * Adjoint (backward) of loss = sum_ij W_ij (A*B)_ij
 * --------------------------------------------------------------------- */

/* Workspace for spgemm_backward in the given mode (deterministic != 0: the
 * transpose of A with its values plus the transpose's scratch; otherwise the
 * row binning of W). */
spgemm_status spgemm_backward_workspace_size(const spgemm_csr *A, const spgemm_csr *B,
                                             const spgemm_csr *W, int32_t deterministic, size_t *bytes);
/* W holds dLoss/dC on the pattern of C = A*B (its row_ptr/col_idx are C's).
 * dA_values[nnz(A)] receives dA_ik = sum_j W_ij b_kj (masked to pat(A));
 * dB_values[nnz(B)] receives dB_kj = sum_i a_ik W_ij (masked to pat(B)).
 * Either output may be NULL. Does not synchronise.
 *   deterministic == 0: fused kernel, dB accumulated with device atomics, so
 *     the order of dB's sums (and its last bits) may change between calls.
 *   deterministic != 0: each entry is one sequential sum in a fixed order
 *     (dA_ik over j ascending; dB_kj over i ascending, gathered through the
 *     transpose of A), products rounded before they are added; repeated calls
 *     give identical bits.
 * A column of A*B missing from W sets the structure error, which the next
 * synchronising call (spgemm_check_errors) reports as SPGEMM_ERR_STRUCTURE. */
spgemm_status spgemm_backward(const spgemm_csr *A, const spgemm_csr *B, const spgemm_csr *W,
                              double *dA_values, double *dB_values, int32_t deterministic, void *ws,
                              size_t ws_bytes, hipStream_t stream);

/* CSR transpose of M into T (T shaped M.ncols x M.nrows, T.row_ptr/col_idx/
 * values allocated by the caller with nnz(M) entries); columns of T come out
 * ascending. Used by the unfused adjoint path. */
spgemm_status spgemm_transpose_workspace_size(const spgemm_csr *M, size_t *bytes);
spgemm_status spgemm_transpose(const spgemm_csr *M, spgemm_csr *T, void *ws, size_t ws_bytes,
                               hipStream_t stream);
/* out[e] = value of X at (row, col) of the e-th entry of pattern P, 0.0 when X
 * has no such entry (X and P have the same shape; X's columns ascending). */
spgemm_status spgemm_mask_gather(const spgemm_csr *X, const spgemm_csr *P, double *out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* MLSPGEMM_H */
