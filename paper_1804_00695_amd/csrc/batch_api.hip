// batch_api.hip -- reusable numeric plan for a batch of independent products
// with fixed structure (multigrid setup: the Galerkin products keep their
// sparsity while the values change). The rows of all products are binned
// once; each run re-zeroes only the per-XCD task cursors and launches the
// class kernels, all products in one launch per class. With use_graph the
// launches are captured once into a HIP graph and replayed.
//
// Autotuning (group_size 0): the schedule is chosen by timing, with HIP
// events on the actual batch, every combination of the lanes per row of the
// first LDS class (8, 16, 32, 64), of the second (32, 64) and of the row-bin
// threshold between the two smallest classes (rows binned by size, or every
// row of the smallest class moved up to the next); all of them give the same
// results bit for bit. The choice is cached in the process by the batch's
// shape and, given a cache file, persisted there (one line per shape and
// device) so that later processes skip the search.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/mlspgemm.h"
#include "common.h"
#include "internal.h"
#include "launch.h"

using namespace mls;

namespace {

struct Schedule {
    int g1 = 32;     // lanes per row, first LDS class
    int g2 = 32;     // lanes per row, second LDS class
    int floor = -1;  // row-bin floor: -1 rows binned by size, 1 the smallest class moved up
};

struct BatchPlanImpl {
    BatchHost bh;
    char *ws = nullptr;
    Schedule sch;
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using TuneKey = std::tuple<int32_t, int32_t, int32_t, int64_t, int64_t>;
std::mutex g_tune_mu;
std::map<TuneKey, Schedule> g_tune_cache;

void bin_rows(BatchPlanImpl &P, int floor, hipStream_t s)
{
    Sched sc = make_sched(P.ws, P.bh.layout);
    reset_header(P.ws, P.bh.layout, s);
    launch_bin(P.bh.batch, kModeNumeric, sc, g_opt.force_spill ? kBinSpill : std::max(floor, g_opt.force_class), nullptr,
               s);
}

void launch_run(BatchPlanImpl &P, hipStream_t s)
{
    Sched sc = make_sched(P.ws, P.bh.layout);
    // task cursors only: the bins (counts, perm) were computed once
    launch_fill_i32(sc.task_cursor, 0, kNumBins * kXcd, s);
    launch_numeric_groups(P.bh.batch, sc, P.sch.g1, P.sch.g2, s);
}

float time_schedule(BatchPlanImpl &P, const Schedule &c, hipStream_t s)
{
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return 1e30f;
    if (hipEventCreate(&b) != hipSuccess) { hipEventDestroy(a); return 1e30f; }
    const Schedule saved = P.sch;
    P.sch = c;
    launch_run(P, s);   // warm-up
    hipEventRecord(a, s);
    for (int r = 0; r < 3; ++r) launch_run(P, s);
    hipEventRecord(b, s);
    float ms = 1e30f;
    if (hipEventSynchronize(b) == hipSuccess) hipEventElapsedTime(&ms, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    P.sch = saved;
    return ms;
}

// Device name and CU count: a persisted choice is only reused on the same kind of GPU.
std::string device_tag()
{
    int dev = 0;
    hipDeviceProp_t pr;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
    std::string arch(pr.gcnArchName);
    for (char &ch : arch)
        if (ch == ' ' || ch == '\t') ch = '_';
    return arch + "/" + std::to_string(pr.multiProcessorCount);
}

// Cache file: lines "batch <nbatch> <na> <nb> <nnzA> <nnzC> <device> <g1> <g2> <floor>";
// other lines are ignored.
bool read_cached(const char *path, const TuneKey &k, const std::string &dev, Schedule &out)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        long long nb, na, nk, za, zc;
        char d[256];
        int g1, g2, fl;
        if (std::sscanf(line, "batch %lld %lld %lld %lld %lld %255s %d %d %d", &nb, &na, &nk, &za, &zc, d, &g1, &g2,
                        &fl) != 9)
            continue;
        if (nb != std::get<0>(k) || na != std::get<1>(k) || nk != std::get<2>(k) || za != std::get<3>(k) ||
            zc != std::get<4>(k) || dev != d)
            continue;
        const bool ok_g1 = g1 == 8 || g1 == 16 || g1 == 32 || g1 == 64, ok_g2 = g2 == 32 || g2 == 64;
        if (!ok_g1 || !ok_g2 || (fl != -1 && fl != 1)) continue;
        out.g1 = g1; out.g2 = g2; out.floor = fl;
        found = true;   // the last matching line wins
    }
    std::fclose(f);
    return found;
}

void write_cached(const char *path, const TuneKey &k, const std::string &dev, const Schedule &c)
{
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "batch %lld %lld %lld %lld %lld %s %d %d %d\n", (long long)std::get<0>(k),
                 (long long)std::get<1>(k), (long long)std::get<2>(k), (long long)std::get<3>(k),
                 (long long)std::get<4>(k), dev.c_str(), c.g1, c.g2, c.floor);
    std::fclose(f);
}

Schedule autotune(BatchPlanImpl &P, hipStream_t s)
{
    float best = 1e30f;
    Schedule bc;
    bc.g1 = pow2_group(P.bh.avg_b);
    bc.g2 = bc.g1 >= 64 ? 64 : 32;
    for (int floor : {-1, 1}) {
        bin_rows(P, floor, s);
        for (int g1 : {8, 16, 32, 64})
            for (int g2 : {32, 64}) {
                Schedule c;
                c.g1 = g1; c.g2 = g2; c.floor = floor;
                const float ms = time_schedule(P, c, s);
                if (ms < best) { best = ms; bc = c; }
            }
    }
    return bc;
}

}  // namespace

extern "C" {

spgemm_status spgemm_batch_plan_create(int32_t nbatch, const spgemm_csr *A, const spgemm_csr *B, spgemm_csr *C,
                                       int32_t group_size, int32_t use_graph, const char *tune_cache_path, void *ws,
                                       size_t ws_bytes, hipStream_t s, spgemm_batch_plan **out)
{
    if (!out || !C) return SPGEMM_ERR_INVALID_ARG;
    if (group_size != 0 && group_size != 8 && group_size != 16 && group_size != 32 && group_size != 64)
        return SPGEMM_ERR_INVALID_ARG;
    *out = nullptr;
    for (int t = 0; t < nbatch; ++t) {
        if (C[t].nrows != A[t].nrows || C[t].ncols != B[t].ncols) return SPGEMM_ERR_DIM_MISMATCH;
        if (!C[t].row_ptr || (C[t].nnz > 0 && (!C[t].col_idx || !C[t].values))) return SPGEMM_ERR_INVALID_ARG;
    }
    memo_forget(ws);
    BatchPlanImpl *P = new BatchPlanImpl();
    spgemm_status st = prepare_batch(nbatch, A, B, C, true, false, (char *)ws, ws_bytes, s, P->bh);
    if (st != SPGEMM_OK) { delete P; return st; }
    P->ws = (char *)ws;
    int64_t za = 0, zc = 0;
    for (int t = 0; t < nbatch; ++t) { za += A[t].nnz; zc += C[t].nnz; }
    if (group_size == 0 && g_opt.group_size) group_size = (int32_t)g_opt.group_size;
    if (group_size == 0) {
        TuneKey key(nbatch, P->bh.batch.na, P->bh.batch.nb, za, zc);
        const std::string dev = tune_cache_path ? device_tag() : std::string();
        bool have = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) { P->sch = it->second; have = true; }
        }
        // the file's line for this shape wins over the process's choice; a
        // choice made in this process is written when the file lacks it
        Schedule from_file;
        const bool in_file = tune_cache_path && read_cached(tune_cache_path, key, dev, from_file);
        if (in_file) {
            P->sch = from_file;
        } else {
            if (!have) P->sch = autotune(*P, s);
            if (tune_cache_path) write_cached(tune_cache_path, key, dev, P->sch);
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = P->sch;
    } else {
        P->sch.g1 = group_size;
        P->sch.g2 = group_size >= 64 ? 64 : 32;
        P->sch.floor = -1;
    }
    bin_rows(*P, P->sch.floor, s);
    st = check_launch();
    if (st != SPGEMM_OK) { delete P; return st; }
    P->use_graph = use_graph != 0;
    if (P->use_graph) {
        // one eager run first: the launch shapes are set up outside the capture
        launch_run(*P, s);
        hipError_t e = hipStreamSynchronize(s);
        // capture on a private stream (the caller's may be the legacy null
        // stream, which cannot be captured); the graph replays on any stream
        hipStream_t cs = nullptr;
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        const bool prof = g_opt.profile;   // no event records inside the captured graph
        g_opt.profile = false;
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            launch_run(*P, cs);
            e = hipStreamEndCapture(cs, &P->graph);
        }
        g_opt.profile = prof;
        if (cs) hipStreamDestroy(cs);
        if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            if (P->graph) hipGraphDestroy(P->graph);
            delete P;
            return hip_fail(e);
        }
    }
    st = check_launch();
    if (st != SPGEMM_OK) { spgemm_batch_plan_destroy((spgemm_batch_plan *)P); return st; }
    *out = reinterpret_cast<spgemm_batch_plan *>(P);
    return SPGEMM_OK;
}

spgemm_status spgemm_batch_plan_run(spgemm_batch_plan *plan, hipStream_t s)
{
    if (!plan) return SPGEMM_ERR_INVALID_ARG;
    BatchPlanImpl *P = reinterpret_cast<BatchPlanImpl *>(plan);
    if (P->use_graph) {
        hipError_t e = hipGraphLaunch(P->exec, s);
        return e == hipSuccess ? SPGEMM_OK : hip_fail(e);
    }
    launch_run(*P, s);
    return check_launch();
}

int32_t spgemm_batch_plan_group_size(const spgemm_batch_plan *plan)
{
    return plan ? reinterpret_cast<const BatchPlanImpl *>(plan)->sch.g1 : 0;
}

spgemm_status spgemm_batch_plan_schedule(const spgemm_batch_plan *plan, int32_t *g1, int32_t *g2, int32_t *floor)
{
    if (!plan || !g1 || !g2 || !floor) return SPGEMM_ERR_INVALID_ARG;
    const Schedule &c = reinterpret_cast<const BatchPlanImpl *>(plan)->sch;
    *g1 = c.g1;
    *g2 = c.g2;
    *floor = c.floor;
    return SPGEMM_OK;
}

void spgemm_batch_plan_destroy(spgemm_batch_plan *plan)
{
    BatchPlanImpl *P = reinterpret_cast<BatchPlanImpl *>(plan);
    if (!P) return;
    if (P->exec) hipGraphExecDestroy(P->exec);
    if (P->graph) hipGraphDestroy(P->graph);
    delete P;
}

}  // extern "C"
