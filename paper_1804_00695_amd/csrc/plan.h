// plan.h -- chunk plan object (internal).
#pragma once

#include <stdint.h>

#include <vector>

#include "../../include/mlspgemm.h"

namespace mls {

enum { kStepH2D = 0, kStepD2H = 1, kStepKernel = 2, kStepZero = 3 };
enum { kMatA = 0, kMatB = 1, kMatCStruct = 2, kMatCVal = 3 };

// alignment slack of the part buffers inside the workspace (each array of a
// part starts on a 256-byte boundary)
constexpr int64_t kChunkSlack = 64 * 1024;
// most buffers of the inner-loop matrix (double, triple, quadruple buffering)
constexpr int kMaxBuf = 4;
// the row binning of up to this many A/C parts is kept in the workspace and
// reused by every kernel step of the part (row sizes of C do not depend on
// the B part); beyond it each step bins its rows again
constexpr int kMaxBinnedParts = 4096;
// algorithm codes: Alg. chunk1, Alg. chunk2, Alg. chunkknl (B parts stream
// into HBM, A and C are accessed in place in host memory)
enum { kAlgoChunk1 = 1, kAlgoChunk2 = 2, kAlgoKnl = 3 };

struct Part {
    int32_t r0, r1;
};

struct PlanImpl {
    int algo = 0, branch = 0, nbuf_inner = 1;
    int32_t nA = 0, nB = 0, ncols = 0;
    int64_t nnzA = 0, nnzB = 0, nnzC = 0;   // of the operands the plan was made for
    int64_t fast = 0, reserve = 0;
    std::vector<Part> p_ac, p_b;
    int64_t h2d = 0, d2h = 0, cost1 = 0, cost2 = 0;
    int64_t zero_copy = 0;   // chunkknl: bytes the kernels move over the link in place (A, C)
    int64_t max_ac = 0, max_b = 0, chunk_bytes = 0, ws_bytes = 0;
    int32_t max_ac_rows = 0;
    std::vector<spgemm_plan_step> steps;
    int64_t issued_h2d = 0, issued_d2h = 0;
};

spgemm_status partition(PlanImpl &P, const int32_t *arp, int32_t nA, const int32_t *brp, int32_t nB,
                        const int32_t *crp, int64_t fast, int nbuf, int min_parts);
spgemm_status partition_knl(PlanImpl &P, const int32_t *arp, int32_t nA, const int32_t *brp, int32_t nB,
                            const int32_t *crp, int64_t fast, int nbuf, int min_parts);
// per-part binning tables that the workspace reserves after the kernels' layout
int64_t binned_parts_bytes();

}  // namespace mls
