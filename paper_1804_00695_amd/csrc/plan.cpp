// plan.cpp -- chunking decision of Sec. 3.3.1 (Alg. "chunker", the Partition
// heuristic) and the copy schedules of Algs. "chunk1" (A/C parts in place, B
// streams) and "chunk2" (B parts in place, A/C stream); and the partition of
// Sec. 3.2.2 (Alg. "chunkknl": only B is cut into parts that stream into fast
// memory, A and C stay in the slow tier and are accessed in place). Host only.
//
// Sizes: a row range [r0, r1) of a CSR matrix occupies 4*(r1 - r0 + 1) bytes
// of row pointers plus 12 bytes per entry (int32 index, fp64 value); C counts
// the same (its structure is known from the symbolic phase and its values
// accumulate in HBM). BinarySearch cuts greedy maximal row ranges whose size
// is at most the partition size (upper bound on the byte prefix). The
// "balanced partition size" of a total T over a portion S is
// ceil(T / max(ceil(T / S), min_parts)) (the portion itself when a single row
// is larger than that). After the outer-loop matrix is cut, what it leaves of
// the big portion goes to the inner-loop matrix. Copy costs count the bytes
// each schedule really moves, in both directions; ties go to the algorithm the
// branch favours. nbuf > 1 divides the inner matrix's portion among that many
// buffers (double, triple, quadruple buffering); min_parts > 1 cuts the inner
// matrix into at least that many parts so that transfers of consecutive parts
// overlap even when it fits whole.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/mlspgemm.h"
#include "common.h"
#include "internal.h"
#include "plan.h"

namespace mls {

static inline int64_t rows_bytes(const int32_t *rp, int32_t r0, int32_t r1)
{
    return 4ll * (r1 - r0 + 1) + 12ll * ((int64_t)rp[r1] - rp[r0]);
}

static inline int64_t struct_bytes(const int32_t *rp, int32_t r0, int32_t r1)
{
    return 4ll * (r1 - r0 + 1) + 4ll * ((int64_t)rp[r1] - rp[r0]);
}

// Greedy maximal parts of [0, n) with size(r0, r1) <= psize; false when a
// single row does not fit.
template <class SizeFn>
static bool cut_parts(SizeFn size, int32_t n, int64_t psize, std::vector<Part> &out)
{
    out.clear();
    if (n == 0) { out.push_back({0, 0}); return true; }
    int32_t r0 = 0;
    while (r0 < n) {
        int32_t lo = r0, hi = n;
        while (lo < hi) {   // largest r1 in (r0, n] with size <= psize
            int32_t mid = lo + (hi - lo + 1) / 2;
            if (size(r0, mid) <= psize) lo = mid; else hi = mid - 1;
        }
        if (lo == r0) return false;
        out.push_back({r0, lo});
        r0 = lo;
    }
    return true;
}

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

static bool balanced(int64_t total, int64_t portion, int64_t max_row, int64_t min_parts, int64_t &psize)
{
    if (portion <= 0) return false;
    int64_t np = std::max<int64_t>(std::max<int64_t>(ceil_div(total, portion), min_parts), 1);
    int64_t p = total > 0 ? ceil_div(total, np) : 0;
    if (p < max_row) p = portion;
    psize = p;
    return true;
}

void copy_bytes(int algo, const std::vector<Part> &pac, const std::vector<Part> &pb, const int32_t *arp,
                const int32_t *brp, const int32_t *crp, int32_t nA, int64_t &h2d, int64_t &d2h)
{
    int64_t ac = 0, b = 0;
    for (auto &p : pac) ac += rows_bytes(arp, p.r0, p.r1) + struct_bytes(crp, p.r0, p.r1);
    for (auto &p : pb) b += rows_bytes(brp, p.r0, p.r1);
    int64_t cval = 8ll * ((int64_t)crp[nA] - crp[0]);
    if (algo == 1) {
        h2d = ac + (int64_t)pac.size() * b;
        d2h = cval;
    } else {
        h2d = b + (int64_t)pb.size() * ac + ((int64_t)pb.size() - 1) * cval;
        d2h = (int64_t)pb.size() * cval;
    }
}

static void build_steps(PlanImpl &P, const int32_t *arp, const int32_t *brp, const int32_t *crp)
{
    P.steps.clear();
    auto add = [&](int kind, int mat, int part, int r0, int r1, int64_t bytes, int slot) {
        spgemm_plan_step s;
        s.kind = kind; s.matrix = mat; s.part = part; s.row_begin = r0; s.row_end = r1; s.slot = slot; s.bytes = bytes;
        P.steps.push_back(s);
    };
    int it = 0;
    if (P.algo == 1) {
        for (int r = 0; r < (int)P.p_ac.size(); ++r) {
            int r0 = P.p_ac[r].r0, r1 = P.p_ac[r].r1;
            add(kStepH2D, kMatA, r, r0, r1, rows_bytes(arp, r0, r1), 0);
            add(kStepH2D, kMatCStruct, r, r0, r1, struct_bytes(crp, r0, r1), 0);
            add(kStepZero, kMatCVal, r, r0, r1, 0, 0);
            for (int b = 0; b < (int)P.p_b.size(); ++b) {
                int slot = it % P.nbuf_inner;
                int b0 = P.p_b[b].r0, b1 = P.p_b[b].r1;
                add(kStepH2D, kMatB, b, b0, b1, rows_bytes(brp, b0, b1), slot);
                add(kStepKernel, kMatCVal, r, b0, b1, 0, slot);
                ++it;
            }
            add(kStepD2H, kMatCVal, r, r0, r1, 8ll * ((int64_t)crp[r1] - crp[r0]), 0);
        }
    } else {
        for (int b = 0; b < (int)P.p_b.size(); ++b) {
            int b0 = P.p_b[b].r0, b1 = P.p_b[b].r1;
            add(kStepH2D, kMatB, b, b0, b1, rows_bytes(brp, b0, b1), 0);
            for (int r = 0; r < (int)P.p_ac.size(); ++r) {
                int slot = it % P.nbuf_inner;
                int r0 = P.p_ac[r].r0, r1 = P.p_ac[r].r1;
                int64_t cv = 8ll * ((int64_t)crp[r1] - crp[r0]);
                add(kStepH2D, kMatA, r, r0, r1, rows_bytes(arp, r0, r1), slot);
                add(kStepH2D, kMatCStruct, r, r0, r1, struct_bytes(crp, r0, r1), slot);
                if (b == 0) add(kStepZero, kMatCVal, r, r0, r1, 0, slot);
                else add(kStepH2D, kMatCVal, r, r0, r1, cv, slot);
                add(kStepKernel, kMatCVal, r, b0, b1, 0, slot);
                add(kStepD2H, kMatCVal, r, r0, r1, cv, slot);
                ++it;
            }
        }
    }
}

spgemm_status partition(PlanImpl &P, const int32_t *arp, int32_t nA, const int32_t *brp, int32_t nB,
                        const int32_t *crp, int64_t fast, int nbuf, int min_parts)
{
    P.fast = fast;
    const int64_t sA = rows_bytes(arp, 0, nA), sB = rows_bytes(brp, 0, nB), sC = rows_bytes(crp, 0, nA);
    const int64_t big = (3 * fast) / 4, small = fast - big;
    auto size_ac = [&](int32_t r0, int32_t r1) { return rows_bytes(arp, r0, r1) + rows_bytes(crp, r0, r1); };
    auto size_b = [&](int32_t r0, int32_t r1) { return rows_bytes(brp, r0, r1); };
    int64_t max_row_ac = 0, max_row_b = 0;
    for (int32_t i = 0; i < nA; ++i)
        max_row_ac = std::max<int64_t>(max_row_ac, 16 + 12ll * ((int64_t)arp[i + 1] - arp[i] + crp[i + 1] - crp[i]));
    for (int32_t k = 0; k < nB; ++k) max_row_b = std::max<int64_t>(max_row_b, 8 + 12ll * ((int64_t)brp[k + 1] - brp[k]));
    auto maxpart = [&](const std::vector<Part> &parts, bool ac) {
        int64_t m = 0;
        for (auto &p : parts) m = std::max<int64_t>(m, ac ? size_ac(p.r0, p.r1) : size_b(p.r0, p.r1));
        return m;
    };
    int natural = 0;
    int64_t ps = 0;
    P.algo = 0;
    if (sB < big) {
        P.branch = 1; natural = 2;
        P.p_b.assign(1, Part{0, nB});
        if (!balanced(sA + sC, (fast - sB) / nbuf, max_row_ac, min_parts, ps) || !cut_parts(size_ac, nA, ps, P.p_ac))
            return SPGEMM_ERR_BUDGET;
        P.algo = 2;
    } else if (sA + sC < big) {
        P.branch = 2; natural = 1;
        P.p_ac.assign(1, Part{0, nA});
        if (!balanced(sB, (fast - sA - sC) / nbuf, max_row_b, min_parts, ps) || !cut_parts(size_b, nB, ps, P.p_b))
            return SPGEMM_ERR_BUDGET;
        P.algo = 1;
    } else if (sA + 2 * sC > sB) {
        P.branch = 3; natural = 1;
        if (!balanced(sA + sC, big, max_row_ac, 1, ps) || !cut_parts(size_ac, nA, ps, P.p_ac)) return SPGEMM_ERR_BUDGET;
        int64_t portion = (small + big - maxpart(P.p_ac, true)) / nbuf;
        if (!balanced(sB, portion, max_row_b, min_parts, ps) || !cut_parts(size_b, nB, ps, P.p_b)) return SPGEMM_ERR_BUDGET;
    } else {
        P.branch = 4; natural = 2;
        if (!balanced(sB, big, max_row_b, 1, ps) || !cut_parts(size_b, nB, ps, P.p_b)) return SPGEMM_ERR_BUDGET;
        int64_t portion = (small + big - maxpart(P.p_b, false)) / nbuf;
        if (!balanced(sA + sC, portion, max_row_ac, min_parts, ps) || !cut_parts(size_ac, nA, ps, P.p_ac))
            return SPGEMM_ERR_BUDGET;
    }
    int64_t h1, d1, h2, d2;
    copy_bytes(1, P.p_ac, P.p_b, arp, brp, crp, nA, h1, d1);
    copy_bytes(2, P.p_ac, P.p_b, arp, brp, crp, nA, h2, d2);
    P.cost1 = h1 + d1;
    P.cost2 = h2 + d2;
    if (P.algo == 0) P.algo = P.cost1 < P.cost2 ? 1 : (P.cost2 < P.cost1 ? 2 : natural);
    P.nbuf_inner = P.algo == natural ? nbuf : 1;
    P.h2d = P.algo == 1 ? h1 : h2;
    P.d2h = P.algo == 1 ? d1 : d2;
    P.max_ac = maxpart(P.p_ac, true);
    P.max_b = maxpart(P.p_b, false);
    P.chunk_bytes = P.algo == 1 ? P.max_ac + P.nbuf_inner * P.max_b : P.max_b + P.nbuf_inner * P.max_ac;
    for (auto &p : P.p_ac) {
        P.max_ac_rows = std::max(P.max_ac_rows, p.r1 - p.r0);
    }
    build_steps(P, arp, brp, crp);
    return SPGEMM_OK;
}

spgemm_status partition_knl(PlanImpl &P, const int32_t *arp, int32_t nA, const int32_t *brp, int32_t nB,
                            const int32_t *crp, int64_t fast, int nbuf, int min_parts)
{
    // np = ceil(size(B) / FastSize), pSize = size(B) / np, P_B = BinarySearch(B, pSize);
    // with nbuf buffers each part gets FastSize / nbuf
    P.fast = fast;
    P.branch = 0;
    P.algo = kAlgoKnl;
    P.nbuf_inner = nbuf;
    const int64_t sB = rows_bytes(brp, 0, nB);
    int64_t max_row_b = 0;
    for (int32_t k = 0; k < nB; ++k) max_row_b = std::max<int64_t>(max_row_b, 8 + 12ll * ((int64_t)brp[k + 1] - brp[k]));
    auto size_b = [&](int32_t r0, int32_t r1) { return rows_bytes(brp, r0, r1); };
    int64_t ps = 0;
    if (!balanced(sB, fast / nbuf, max_row_b, min_parts, ps) || !cut_parts(size_b, nB, ps, P.p_b)) return SPGEMM_ERR_BUDGET;
    P.p_ac.assign(1, Part{0, nA});
    int64_t b = 0;
    for (auto &p : P.p_b) b += rows_bytes(brp, p.r0, p.r1);
    P.h2d = b;
    P.d2h = 0;
    P.cost1 = P.cost2 = 0;
    const int64_t nparts = (int64_t)P.p_b.size();
    const int64_t cval = 8ll * ((int64_t)crp[nA] - crp[0]);
    // every pass reads A and C's structure in place and writes C's values;
    // passes after the first also read the values the previous one wrote
    P.zero_copy = nparts * (rows_bytes(arp, 0, nA) + struct_bytes(crp, 0, nA)) + nparts * cval + (nparts - 1) * cval;
    P.max_ac = 0;
    P.max_b = 0;
    for (auto &p : P.p_b) P.max_b = std::max<int64_t>(P.max_b, size_b(p.r0, p.r1));
    P.chunk_bytes = nbuf * P.max_b;
    P.max_ac_rows = nA;
    P.steps.clear();
    for (int q = 0; q < (int)P.p_b.size(); ++q) {
        spgemm_plan_step s;
        s.kind = kStepH2D; s.matrix = kMatB; s.part = q; s.row_begin = P.p_b[q].r0; s.row_end = P.p_b[q].r1;
        s.slot = q % nbuf; s.bytes = rows_bytes(brp, s.row_begin, s.row_end);
        P.steps.push_back(s);
        s.kind = kStepKernel; s.matrix = kMatCVal; s.part = 0; s.bytes = 0;
        P.steps.push_back(s);
    }
    return SPGEMM_OK;
}

int64_t binned_parts_bytes()
{
    return ((int64_t)kMaxBinnedParts * kNumBins * 4 + 255) & ~(int64_t)255;
}

}  // namespace mls

using namespace mls;

extern "C" {

static spgemm_status make_plan(const spgemm_csr *A, const spgemm_csr *B, const int32_t *C_row_ptr,
                               size_t hbm_budget_bytes, int32_t nbuf, int32_t min_parts, bool knl,
                               spgemm_plan **plan_out)
{
    if (!A || !B || !C_row_ptr || !plan_out || !A->row_ptr || !B->row_ptr) return SPGEMM_ERR_INVALID_ARG;
    if (nbuf < 1 || nbuf > kMaxBuf || min_parts < 1) return SPGEMM_ERR_INVALID_ARG;
    if (A->ncols != B->nrows) return SPGEMM_ERR_DIM_MISMATCH;
    *plan_out = nullptr;
    PlanImpl *P = new (std::nothrow) PlanImpl();
    if (!P) return SPGEMM_ERR_INVALID_ARG;
    P->nA = A->nrows;
    P->nB = B->nrows;
    P->ncols = B->ncols;
    P->nnzA = A->row_ptr[A->nrows];
    P->nnzB = B->row_ptr[B->nrows];
    P->nnzC = C_row_ptr[A->nrows];
    // reserve: the numeric kernels' per-row arrays for up to all rows of A,
    // the kept binnings of the A/C parts, and alignment slack of the part buffers
    P->reserve = (int64_t)make_layout(1, A->nrows, B->nrows, 0, B->ncols, false).total + binned_parts_bytes() +
                 kChunkSlack;
    int64_t fast = (int64_t)hbm_budget_bytes - P->reserve;
    if (fast <= 0) { delete P; return SPGEMM_ERR_BUDGET; }
    spgemm_status st = knl ? partition_knl(*P, A->row_ptr, A->nrows, B->row_ptr, B->nrows, C_row_ptr, fast, nbuf,
                                           min_parts)
                           : partition(*P, A->row_ptr, A->nrows, B->row_ptr, B->nrows, C_row_ptr, fast, nbuf,
                                       min_parts);
    if (st != SPGEMM_OK) { delete P; return st; }
    P->ws_bytes = P->reserve + P->chunk_bytes;
    *plan_out = reinterpret_cast<spgemm_plan *>(P);
    return SPGEMM_OK;
}

spgemm_status spgemm_chunked_plan(const spgemm_csr *A, const spgemm_csr *B, const int32_t *C_row_ptr,
                                  size_t hbm_budget_bytes, int32_t nbuf, int32_t min_parts, spgemm_plan **plan_out)
{
    return make_plan(A, B, C_row_ptr, hbm_budget_bytes, nbuf, min_parts, false, plan_out);
}

spgemm_status spgemm_chunked_plan_knl(const spgemm_csr *A, const spgemm_csr *B, const int32_t *C_row_ptr,
                                      size_t hbm_budget_bytes, int32_t nbuf, int32_t min_parts,
                                      spgemm_plan **plan_out)
{
    return make_plan(A, B, C_row_ptr, hbm_budget_bytes, nbuf, min_parts, true, plan_out);
}

spgemm_status spgemm_plan_info_get(const spgemm_plan *plan, spgemm_plan_info *out)
{
    if (!plan || !out) return SPGEMM_ERR_INVALID_ARG;
    const PlanImpl *P = reinterpret_cast<const PlanImpl *>(plan);
    std::memset(out, 0, sizeof(*out));
    out->algo = P->algo;
    out->branch = P->branch;
    out->n_ac_parts = (int32_t)P->p_ac.size();
    out->n_b_parts = (int32_t)P->p_b.size();
    out->nbuf_inner = P->nbuf_inner;
    out->n_steps = (int32_t)P->steps.size();
    out->fast_bytes = P->fast;
    out->h2d_bytes = P->h2d;
    out->d2h_bytes = P->d2h;
    out->cost_chunk1 = P->cost1;
    out->cost_chunk2 = P->cost2;
    out->chunk_bytes = P->chunk_bytes;
    out->ws_bytes = P->ws_bytes;
    out->issued_h2d = P->issued_h2d;
    out->issued_d2h = P->issued_d2h;
    out->zero_copy_bytes = P->zero_copy;
    return SPGEMM_OK;
}

spgemm_status spgemm_plan_parts(const spgemm_plan *plan, int32_t which, int32_t *ranges, int32_t max_parts)
{
    if (!plan || !ranges || (which != 0 && which != 1)) return SPGEMM_ERR_INVALID_ARG;
    const PlanImpl *P = reinterpret_cast<const PlanImpl *>(plan);
    const std::vector<Part> &v = which == 0 ? P->p_ac : P->p_b;
    for (int32_t i = 0; i < (int32_t)v.size() && i < max_parts; ++i) {
        ranges[2 * i] = v[i].r0;
        ranges[2 * i + 1] = v[i].r1;
    }
    return SPGEMM_OK;
}

spgemm_status spgemm_plan_steps(const spgemm_plan *plan, spgemm_plan_step *steps, int32_t max_steps)
{
    if (!plan || !steps) return SPGEMM_ERR_INVALID_ARG;
    const PlanImpl *P = reinterpret_cast<const PlanImpl *>(plan);
    for (int32_t i = 0; i < (int32_t)P->steps.size() && i < max_steps; ++i) steps[i] = P->steps[i];
    return SPGEMM_OK;
}

void spgemm_plan_destroy(spgemm_plan *plan)
{
    delete reinterpret_cast<PlanImpl *>(plan);
}

}  // extern "C"
