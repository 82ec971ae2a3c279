// common.h -- device-side descriptors and helpers shared by the gfx950 kernels.
//
// Every kernel works on a *batch* of independent products C_t = A_t * B_t
// (a single product is a batch of one). Rows of all A_t are numbered in one
// global row space: product t owns global rows [abase[t], abase[t+1]).
// The same holds for the rows of all B_t (bbase). A row-range restriction
// (k_lo, k_hi) and array offsets let the same kernels run on chunk parts
// (the row-range fused multiply-add kernel of the chunking algorithms).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mls {

constexpr int kWG = 256;          // threads per workgroup
constexpr int kWave = 64;         // gfx950 wavefront
constexpr int kXcd = 8;           // MI355X: 8 accelerator complex dies, 32 CUs each
constexpr int kNumClasses = 5;    // LDS classes
constexpr int kNumBins = 7;       // 5 LDS classes, spill, empty
constexpr int kBinSpill = 5;
constexpr int kBinEmpty = 6;

// Error bits (device flag).
constexpr uint32_t kErrBadCsr = 1u;
constexpr uint32_t kErrOverflow = 2u;
constexpr uint32_t kErrStructure = 4u;
constexpr uint32_t kErrTable = 8u;

// LDS capacities (hash slots) of the five classes, per phase. A row goes to
// the first class whose threshold holds; beyond class 3 it spills. The
// smallest class keeps many short rows in flight (small tables, 8 lanes).
//   count  : threshold on the word upper bound u, table = u slots at most
//   fill / numeric : threshold on the exact size n, table >= 2n slots
// (triangle counting keeps a table of its own, on the same rule)
constexpr int kCountCap[kNumClasses] = {64, 256, 512, 2048, 8192};
constexpr int kFillCap[kNumClasses] = {64, 256, 1024, 2048, 4096};

struct Prob {
    // A (or an A/C row part): row pointers hold global entry offsets; the
    // local entry index is row_ptr value - a_off.
    const int32_t *arp;
    const int32_t *aci;
    const double *aval;
    // B (or a B row part): local row = k - k_lo; local entry = brp - b_off.
    const int32_t *brp;
    const int32_t *bci;
    const double *bval;
    // Compressed B pattern, padded layout: row k's words at bw[brp[k]-b_off ...].
    uint2 *bw;
    int32_t *bwc;
    // C: row pointers with offset c_off.
    int32_t *crp;
    int32_t *cci;
    double *cval;
    int32_t nrows;   // rows of A / C
    int32_t ncols;   // columns of B / C
    int32_t krows;   // rows of B held (k_hi - k_lo)
    int32_t a_off, b_off, c_off;
    int32_t k_lo, k_hi;     // A columns outside [k_lo, k_hi) are skipped
    int32_t accumulate;     // numeric: 1 = add onto the values already in C
    int32_t ranged;         // numeric: [k_lo, k_hi) is part of B's rows; a row of at most one
                            // chunk with no entry in it is skipped (its values stay, or are
                            // set to 0 when not accumulating)
};

static_assert(sizeof(Prob) % 16 == 0, "Prob is copied in 16-byte words");

struct Batch {
    const Prob *probs;      // device array [nprob] (used when nprob > 1)
    Prob p0;                // the product when nprob == 1
    const int32_t *abase;   // device [nprob + 1]
    const int32_t *bbase;   // device [nprob + 1]
    int32_t nprob;
    int32_t na;             // total A rows
    int32_t nb;             // total B rows
    int32_t max_ncols;      // largest column count of C over the products (0 = unknown)
};

// Per-phase device state inside the workspace.
struct Sched {
    uint32_t *err;
    int32_t *bin_count;     // [kNumBins]
    int32_t *blk_cnt;       // [kNumBins * nblk]: rows of each bin per block of kBinRowsPerWG rows,
                            // then (after the bin scan) where those rows start in perm
    int32_t nblk;
    int32_t *task_cursor;   // [kNumBins * kXcd]
    int32_t *val;           // per global row: size used for binning / result
    uint8_t *cls;           // per global row: bin
    int32_t *perm;          // rows grouped by bin
    // symbolic scratch: the count pass leaves each row's compacted (set, mask)
    // words here (up to kScratchWords per row; scnt = -1 when a row has more)
    // and the fill pass expands them instead of recomputing the union
    uint2 *scr;             // nullptr when the workspace has no room for it
    int32_t *scnt;
    // numeric / adjoint spill path: first window of each spill row (position
    // in the spill bin), then the total; per-row scratch of na + 1 entries
    int32_t *wstart;
};

constexpr int kScratchWords = 64;

// Rows per binning block: every binning kernel assigns rows [b * kBinRowsPerWG,
// (b + 1) * kBinRowsPerWG) to workgroup b and leaves the block's row count per
// bin in blk_cnt, so that the bin scan and the scatter need no global atomics.
constexpr int kBinRowsPerWG = 1024;

// Pointers read out of descriptors are generic; loads through them compile
// to flat instructions, which make the compiler wait on LDS and vector memory
// together. Every kernel therefore casts them to the global address space.
#define MLS_G __attribute__((address_space(1)))
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <class T>
__device__ __forceinline__ const MLS_G T *gp(const T *p)
{
    return (const MLS_G T *)(p);
}

template <class T>
__device__ __forceinline__ MLS_G T *gpw(T *p)
{
    return (MLS_G T *)(p);
}

__device__ __forceinline__ int find_prob(const int32_t *base, int nprob, int g)
{
    // largest t with base[t] <= g
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (gp(base)[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// find_prob for a g that is the same in every lane of the wave, all lanes
// active: 64 candidates per step, so one or two dependent loads (up to 4096
// products) in place of log2(nprob).
__device__ __forceinline__ int find_prob_wave(const int32_t *base, int nprob, int g)
{
    if (nprob > 4096) return find_prob(base, nprob, g);
    const int lane = (int)(threadIdx.x & 63);
    const MLS_G int32_t *bs = gp(base);
    int t = 0;
    if (nprob > 64) {
        const int c = lane * 64;
        const int v = bs[c < nprob ? c : 0];
        const unsigned long long m = __ballot(c < nprob && v <= g);   // lane 0 always: base[0] = 0
        t = (63 - __clzll(m)) * 64;
    }
    const int c = t + lane;
    const int v = bs[c < nprob ? c : 0];
    const unsigned long long m = __ballot(c < nprob && v <= g);
    return t + (63 - __clzll(m));
}

// Product of row g when consecutive rows are spread over a wave (g = g_w +
// lane, g_w uniform): the product of the wave's first row serves every lane
// whose row lies before that product's end, the others search on their own.
// Call with every lane of the wave active.
__device__ __forceinline__ int find_prob_rows(const int32_t *base, int nprob, int g_w, int g)
{
    const int t = find_prob_wave(base, nprob, g_w);
    if (g < gp(base)[t + 1]) return t;
    return find_prob(base, nprob, g);
}

// Product lookup with a per-lane memory of the last product found: rows a
// lane takes in a row usually belong to the same product of a batch, and then
// two compares replace the binary search.
struct ProbCache {
    int t = 0, lo = 0, hi = 0;   // rows [lo, hi) belong to product t
};

__device__ __forceinline__ int find_prob_cached(const int32_t *base, int nprob, int g, ProbCache &c)
{
    if (g >= c.lo && g < c.hi) return c.t;
    c.t = find_prob(base, nprob, g);
    c.lo = gp(base)[c.t];
    c.hi = gp(base)[c.t + 1];
    return c.t;
}

// The descriptor of product t by value: from the kernel arguments for a
// single product, from global memory for a batch.
__device__ __forceinline__ Prob get_prob(const Batch &b, int t)
{
    if (b.nprob == 1) return b.p0;
    Prob P;
    const MLS_G u32x4 *src = (const MLS_G u32x4 *)(b.probs + t);
    u32x4 *dst = (u32x4 *)&P;
#pragma unroll
    for (int w = 0; w < (int)(sizeof(Prob) / 16); ++w) dst[w] = src[w];
    return P;
}

// get_prob for kernels specialised for batches: when every active lane of
// the wave asks for the same product (the rows of a wave are consecutive, so
// almost always), the descriptor is read once through the scalar cache
// (constant address space: the descriptors do not change while a kernel
// runs) and waits only on the scalar counter; otherwise each lane reads its
// own, and that wait stays inside its branch.
typedef const __attribute__((address_space(4))) u32x4 *MLS_K_u32x4p;

__device__ __forceinline__ Prob get_prob_batch(const Batch &b, int t)
{
    Prob P;
    u32x4 *dst = (u32x4 *)&P;
    const int t0 = __builtin_amdgcn_readfirstlane(t);
    if (__ballot(t != t0) == 0ull) {
        const MLS_K_u32x4p src = (MLS_K_u32x4p)(b.probs + t0);
#pragma unroll
        for (int w = 0; w < (int)(sizeof(Prob) / 16); ++w) dst[w] = src[w];
    } else {
        const MLS_G u32x4 *src = (const MLS_G u32x4 *)(b.probs + t);
#pragma unroll
        for (int w = 0; w < (int)(sizeof(Prob) / 16); ++w) dst[w] = src[w];
#pragma unroll
        for (int w = 0; w < (int)(sizeof(Prob) / 16); ++w) asm volatile("" ::"v"(dst[w]));
    }
    return P;
}

// get_prob_batch for kernels that serve both (the choice is made at run time).
__device__ __forceinline__ Prob get_prob_any(const Batch &b, int t)
{
    if (b.nprob == 1) return b.p0;
    return get_prob_batch(b, t);
}

// Multiplicative (Fibonacci) hashing of a 32-bit key into 2^logcap slots.
__device__ __forceinline__ uint32_t hslot(uint32_t key, int logcap)
{
    return (key * 0x9E3779B1u) >> (32 - logcap);
}

__device__ __forceinline__ int ilog2_ceil(int x)
{
    return x <= 1 ? 0 : 32 - __clz(x - 1);
}

// Cross-lane sums and scans over the G consecutive lanes of a group (G a
// power of two <= 64, groups aligned to G). Groups of at most 16 lanes lie in
// one 16-lane DPP row, where DPP moves read a neighbour's register directly
// (no LDS round trip): quad permutations and (half-)row mirrors for sums,
// row shifts for scans; every read stays inside the group (or is masked
// off). Wider groups use shuffles. All lanes of a group must be active.
template <int CTRL>
__device__ __forceinline__ int dpp_move(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v)
{
    if constexpr (G <= 16 && sizeof(T) == 4 && T(-1) < T(0)) {
        if constexpr (G >= 2) v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
        if constexpr (G >= 4) v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
        if constexpr (G >= 8) v += dpp_move<0x141>(v);   // row_half_mirror: the other quad of 8
        if constexpr (G >= 16) v += dpp_move<0x140>(v);  // row_mirror: the other half of 16
        return v;
    } else {
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
        return v;
    }
}

// the group's total, given a lane's value v and its inclusive prefix incl
template <int G>
__device__ __forceinline__ int group_total(int v, int incl)
{
    if constexpr (G <= 16) return group_sum<G>(v);
    else return __shfl(incl, G - 1, G);
}

// number of lower lanes of the group (G <= 16) whose key equals this lane's
template <int O, int G>
__device__ __forceinline__ void group_rank_step(int key, int lane, int &r)
{
    if constexpr (O < G) {
        const int y = dpp_move<0x110 + O>(key);   // row_shr:O
        r += (lane >= O && y == key) ? 1 : 0;
        group_rank_step<O + 1, G>(key, lane, r);
    }
}

template <int G>
__device__ __forceinline__ int group_rank(int key, int lane)
{
    static_assert(G <= 16, "one DPP row");
    int r = 0;
    group_rank_step<1, G>(key, lane, r);
    return r;
}

// inclusive prefix sum over the group; lane = position in the group
template <int G>
__device__ __forceinline__ int group_scan_incl(int v, int lane)
{
    if constexpr (G <= 16) {
        int y;
        if constexpr (G >= 2) { y = dpp_move<0x111>(v); if (lane >= 1) v += y; }   // row_shr:1
        if constexpr (G >= 4) { y = dpp_move<0x112>(v); if (lane >= 2) v += y; }   // row_shr:2
        if constexpr (G >= 8) { y = dpp_move<0x114>(v); if (lane >= 4) v += y; }   // row_shr:4
        if constexpr (G >= 16) { y = dpp_move<0x118>(v); if (lane >= 8) v += y; }  // row_shr:8
        return v;
    } else {
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
            const int y = __shfl_up(v, o, G);
            if (lane >= o) v += y;
        }
        return v;
    }
}

// Row at position pos of perm, or -1 (and an error bit) when the position or
// the row lies outside the batch -- which consistent bins never produce; the
// kernels then skip the row instead of dereferencing a bad index.
__device__ __forceinline__ int bin_row(const int32_t *perm, uint32_t *err, int na, int pos)
{
    if ((unsigned)pos >= (unsigned)na) { atomicOr(err, kErrTable); return -1; }
    const int g = gp(perm)[pos];
    if ((unsigned)g >= (unsigned)na) { atomicOr(err, kErrTable); return -1; }
    return g;
}

// Constant words read in place of an entry a lane does not need, so that a
// load needs no branch around it (a branch would make the wave wait for the
// load where the branches join): all ones (a column or row -1) and zeros.
static __device__ __attribute__((aligned(16))) int32_t k_ones4[4] = {-1, -1, -1, -1};
static __device__ __attribute__((aligned(16))) int32_t k_zeros4[4] = {0, 0, 0, 0};

// Pipelined form of bin_row: the perm load is only issued (a lane that wants
// no row reads -1), and bin_row_checked validates the value where it is first
// used, a row or more later. A position outside the batch never comes from
// consistent bins and is flagged at once.
__device__ __forceinline__ int bin_row_issue(const int32_t *perm, uint32_t *err, int na, int pos, bool want)
{
    const bool ok = want && (unsigned)pos < (unsigned)na;
    if (want && !ok) atomicOr(err, kErrTable);
    return *(ok ? gp(perm) + pos : (const MLS_G int32_t *)k_ones4);
}

__device__ __forceinline__ int bin_row_checked(uint32_t *err, int na, int g, bool want)
{
    if (!want) return -1;
    if ((unsigned)g >= (unsigned)na) { atomicOr(err, kErrTable); return -1; }
    return g;
}

// Bin start = exclusive prefix of the bin counts.
__device__ __forceinline__ int bin_start(const int32_t *bin_count, int bin)
{
    int s = 0;
    for (int c = 0; c < bin; ++c) s += bin_count[c];
    return s;
}

// Per-wave task schedule. Tasks of a bin are split into one contiguous slab
// per XCD (workgroup w runs on XCD w % 8, and the CUs of an XCD share one L2).
// Inside a slab, waves take blocks of kTaskBlock tasks from a per-XCD counter;
// block b holds the tasks base + c, base + c + S, ..., c = b mod S, base set
// by b div S, with S the number of waves the grid places on the XCD. While
// every wave is busy, the rows in flight on an XCD therefore form a narrow
// window of about S consecutive tasks (neighbouring rows share most of their
// rows of B, and a narrow window keeps that shared working set in the L2).
// A wave's first block is the one of its own index on the XCD (the grid is
// sized to be resident at once), so a launch does not start with every wave
// queued on the same counter; only the blocks after the first S are taken
// from the counter, and a slab that the first blocks cover takes none.
constexpr int kTaskBlock = 16;

//
// With log_chunk >= 0 the tasks are instead cut into chunks of 2^log_chunk
// consecutive tasks, dealt to the XCDs round-robin: each XCD then holds a
// uniform sample of the bin, for bins whose work per task drifts with the
// row index (the degree-ordered rows of a power-law graph), where contiguous
// slabs leave some XCDs idle while others still work.
struct TaskIter {
    int lo, hi, S, cur, left, x, lc, wid;
    bool first;
};

__device__ __forceinline__ TaskIter task_iter(int ntasks, int waves_per_wg, int log_chunk = -1)
{
    const int x = (int)(blockIdx.x % kXcd);
    TaskIter it;
    it.x = x;
    it.lc = log_chunk;
    if (log_chunk < 0) {
        it.lo = (int)(((int64_t)ntasks * x) / kXcd);
        it.hi = (int)(((int64_t)ntasks * (x + 1)) / kXcd);
    } else {
        // local tasks of XCD x: the full chunks x, x + 8, ... and the
        // partial last chunk when it falls on x
        const int nch = ntasks >> log_chunk;
        const int rem = ntasks & ((1 << log_chunk) - 1);
        const int full = nch > x ? (nch - x + kXcd - 1) / kXcd : 0;
        it.lo = 0;
        it.hi = (full << log_chunk) + (nch % kXcd == x ? rem : 0);
    }
    const int wgs_x = ((int)gridDim.x - x + kXcd - 1) / kXcd;   // workgroups on this XCD
    it.S = wgs_x * waves_per_wg;
    if (it.S < 1) it.S = 1;
    it.cur = 0;
    it.left = 0;
    // in [0, S); read from the first lane so that the compiler keeps it, and
    // every task index derived from it, in scalar registers
    it.wid = (int)(blockIdx.x / kXcd) * waves_per_wg + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    it.first = true;
    return it;
}

__device__ __forceinline__ int task_global(const TaskIter &it, int t)
{
    if (it.lc < 0) return t;
    return ((((t >> it.lc) * kXcd) + it.x) << it.lc) + (t & ((1 << it.lc) - 1));
}

// Next task of this wave, or -1. Uniform across the wave; call with all lanes
// active. cursor: the bin's kXcd counters, zero before the launch.
__device__ __forceinline__ int next_task_wave(int32_t *cursor, int ntasks, TaskIter &it)
{
    (void)ntasks;
    if (it.lo >= it.hi) return -1;   // empty slab: no counter traffic
    for (;;) {
        if (it.left > 0) {
            const int t = it.cur;
            it.cur += it.S;
            --it.left;
            if (t < it.hi) return task_global(it, t);
            it.left = 0;
        }
        int blk = 0;
        if (it.first) {
            blk = it.wid;
            it.first = false;
        } else {
            if ((int64_t)it.lo + (int64_t)it.S * kTaskBlock >= it.hi) return -1;   // no block past the first S
            if ((threadIdx.x & 63) == 0) blk = atomicAdd(cursor + blockIdx.x % kXcd, 1);
            blk = __builtin_amdgcn_readlane(blk, 0) + it.S;
        }
        const int64_t base = (int64_t)it.lo + (int64_t)(blk / it.S) * it.S * kTaskBlock + blk % it.S;
        if (base >= it.hi) return -1;
        it.cur = (int)base;
        it.left = kTaskBlock;
    }
}

}  // namespace mls
