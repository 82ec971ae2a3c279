// batch_api.hip -- reusable numeric plan for a batch of independent products
// with fixed structure (multigrid setup: the Galerkin products keep their
// sparsity while the values change). The rows of all products are binned
// once; each run re-zeroes only the per-XCD task cursors and launches the
// class kernels, all products in one launch per class. With use_graph the
// launches are captured once into a HIP graph and replayed. With group_size
// 0 the lanes-per-row of the first class is autotuned: every candidate is
// timed with HIP events on the actual batch and the fastest is kept (the
// choice is cached per process by the batch's shape).
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/mlspgemm.h"
#include "common.h"
#include "internal.h"
#include "launch.h"

using namespace mls;

namespace {

struct BatchPlanImpl {
    BatchHost bh;
    char *ws = nullptr;
    int group = 32;
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using TuneKey = std::tuple<int32_t, int32_t, int32_t, int64_t, int64_t>;
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune_cache;

void launch_run(BatchPlanImpl &P, hipStream_t s)
{
    Sched sc = make_sched(P.ws, P.bh.layout);
    // task cursors only: the bins (counts, perm) were computed once
    launch_fill_i32(sc.task_cursor, 0, kNumBins * kXcd, s);
    launch_numeric(P.bh.batch, sc, P.group, s);
}

float time_group(BatchPlanImpl &P, int G, hipStream_t s)
{
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return 1e30f;
    if (hipEventCreate(&b) != hipSuccess) { hipEventDestroy(a); return 1e30f; }
    const int saved = P.group;
    P.group = G;
    launch_run(P, s);   // warm-up
    hipEventRecord(a, s);
    for (int r = 0; r < 3; ++r) launch_run(P, s);
    hipEventRecord(b, s);
    float ms = 1e30f;
    if (hipEventSynchronize(b) == hipSuccess) hipEventElapsedTime(&ms, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    P.group = saved;
    return ms;
}

}  // namespace

extern "C" {

spgemm_status spgemm_batch_plan_create(int32_t nbatch, const spgemm_csr *A, const spgemm_csr *B, spgemm_csr *C,
                                       int32_t group_size, int32_t use_graph, void *ws, size_t ws_bytes,
                                       hipStream_t s, spgemm_batch_plan **out)
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
    Sched sc = make_sched(P->ws, P->bh.layout);
    reset_header(P->ws, P->bh.layout, s);
    launch_bin(P->bh.batch, kModeNumeric, sc, bin_force(), nullptr, s);
    st = check_launch();
    if (st != SPGEMM_OK) { delete P; return st; }
    int64_t za = 0, zc = 0;
    for (int t = 0; t < nbatch; ++t) { za += A[t].nnz; zc += C[t].nnz; }
    if (group_size == 0 && g_opt.group_size) group_size = (int32_t)g_opt.group_size;
    if (group_size == 0) {
        TuneKey key(nbatch, P->bh.batch.na, P->bh.batch.nb, za, zc);
        int cached = 0;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) cached = it->second;
        }
        if (cached) {
            P->group = cached;
        } else {
            float best = 1e30f;
            int bestG = pow2_group(P->bh.avg_b);
            for (int G : {8, 16, 32, 64}) {
                float ms = time_group(*P, G, s);
                if (ms < best) { best = ms; bestG = G; }
            }
            P->group = bestG;
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[key] = bestG;
        }
    } else {
        P->group = group_size;
    }
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
    return plan ? reinterpret_cast<const BatchPlanImpl *>(plan)->group : 0;
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
