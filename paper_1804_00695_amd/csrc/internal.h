// internal.h -- host-side structures shared by the ABI translation units.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/mlspgemm.h"
#include "common.h"

namespace mls {

struct Options {
    bool validate = true;
    bool force_spill = false;
    bool wide_table = false;
    int64_t group_size = 0;
    bool profile = false;
    int force_class = -1;   // test knob: rows move up to this LDS class (-1: off)
};
extern Options g_opt;

// Binning override handed to the binning kernels: kBinSpill when every row
// must spill, else the forced class floor (-1 = natural classes).
inline int bin_force() { return g_opt.force_spill ? kBinSpill : g_opt.force_class; }
extern thread_local int g_last_hip_error;

// Header region at the start of every workspace.
constexpr size_t kHdrBytes = 1024;
constexpr size_t kHdrErr = 0;
constexpr size_t kHdrBinCount = 64;
constexpr size_t kHdrTaskCursor = 192;   // kNumBins * kXcd int32 (up to 224 bytes)
constexpr size_t kHdrTotal = 512;        // uint64

struct Layout {
    size_t hdr = 0, totals = 0, nnz_tab = 0, probs = 0, abase = 0, bbase = 0;
    size_t val = 0, cls = 0, perm = 0, prefix = 0, tiles = 0, blk = 0;
    int32_t nblk = 0;
    size_t bw = 0, bwc = 0, spill = 0;
    int64_t spill_words = 0;
    int spill_slots = 0;
    size_t scr = 0, scnt = 0;   // symbolic scratch (after total_min)
    size_t total_min = 0;       // without the symbolic scratch
    size_t total = 0;           // with it
    bool has_scratch = false;   // the caller's workspace holds it
};

struct BatchHost {
    Layout layout;
    Batch batch;
    std::vector<Prob> probs;
    std::vector<int32_t> abase, bbase;
    std::vector<int64_t> nnz_tab;
    double avg_a = 1.0, avg_b = 1.0;
    std::vector<uint64_t> key;  // operands and shapes of the call, verbatim
};

spgemm_status hip_fail(hipError_t e);
spgemm_status check_launch();
spgemm_status err_status(uint32_t err);
Layout make_layout(int64_t nprob, int64_t na, int64_t nb, int64_t zb, int64_t max_ncols, bool need_bw);
Sched make_sched(char *ws, const Layout &L);
void reset_header(char *ws, const Layout &L, hipStream_t s);
spgemm_status read_errors(char *ws, const Layout &L, hipStream_t s);
// upload = false skips the host-to-device copies of the descriptor tables
// (only a single product's numeric phase can do without them: it passes its
// descriptor by value and never reads the entry-count table).
spgemm_status prepare_batch(int32_t nbatch, const spgemm_csr *A, const spgemm_csr *B, const spgemm_csr *C,
                            bool need_values, bool need_bw, char *ws, size_t ws_bytes, hipStream_t s,
                            BatchHost &out, bool upload = true);
spgemm_status run_symbolic(BatchHost &bh, char *ws, int fill, int64_t *nnz_host, hipStream_t s);
spgemm_status run_numeric(BatchHost &bh, char *ws, hipStream_t s);
int choose_group(double avg);
// Address the device uses for p: device memory of device `dev` unchanged,
// page-locked host memory through its device mapping (*on_host set);
// pageable, managed or another device's memory is SPGEMM_ERR_INVALID_ARG.
spgemm_status device_view(const void *p, int dev, const void **out, bool *on_host);
void memo_forget(const void *ws);
int pow2_group(double avg);

}  // namespace mls
