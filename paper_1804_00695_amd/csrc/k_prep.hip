// k_prep.hip -- kernels around the two phases: CSR checks, column compression
// of B, per-row work estimate and binning, the row-pointer scan.
#include "common.h"
#include "launch.h"
#include "profile.h"

namespace mls {

// ---------------------------------------------------------------------------
// state reset (a fill kernel instead of hipMemsetAsync so that a captured
// graph replays it faithfully)

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_f64(double *p, double v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------------------
// Per-row helpers: one thread per short row, the whole wave per long row.

// CSR checks over the A rows (which = 0) or B rows (which = 1) of a batch:
// row_ptr[0] == 0, non-decreasing, row_ptr[n] == nnz, columns in range and
// strictly increasing. Column indices outside [0, nnz) are never read.
// One thread per row walks rows of up to kShortRow entries; rows of up to 16
// (32) entries are checked by 16 (32) lanes each, four (two) at a time; the
// wave checks longer rows together, one at a time, 64 entries per step.
constexpr int kShortRow = 4;
constexpr int kLongAhead = 4;   // long rows: steps of 64 entries whose loads are issued together

// 64 / GL rows per step, GL lanes per row (rows of at most GL entries); mm
// holds the lanes that own such rows. A row's verdict goes to its owner lane.
template <int GL>
__device__ __forceinline__ void validate_group_rows(unsigned long long mm, int lane, int len, int ncols,
                                                    const int32_t *ci_row, bool &bad)
{
    constexpr int NG = kWave / GL;
    constexpr uint32_t kAll = GL == 32 ? 0xffffffffu : ((1u << GL) - 1u);
    const int grp = lane / GL, gl = lane % GL;
    while (mm) {
        int pick = -1;
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            const int r = mm ? __ffsll((long long)mm) - 1 : -1;
            if (mm) mm &= mm - 1ull;
            if (j == grp) pick = r;
        }
        // every lane takes part in the shuffles (a group without a row reads lane 0)
        const int from = pick >= 0 ? pick : 0;
        int n = __shfl(len, from, kWave);
        if (pick < 0) n = 0;
        const int nc = __shfl(ncols, from, kWave);
        const uint64_t pa = ((uint64_t)(uint32_t)__shfl((int)((uint64_t)ci_row >> 32), from, kWave) << 32) |
                            (uint32_t)__shfl((int)(uint64_t)ci_row, from, kWave);
        const bool valid = gl < n;
        const int cq = valid ? ((const MLS_G int32_t *)pa)[gl] : 0;
        int prev = __shfl_up(cq, 1, GL);
        if (gl == 0) prev = -1;
        const bool bl = valid && (cq < 0 || cq >= nc || cq <= prev);
        const unsigned long long bb = __ballot(bl);
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            const int pj = __shfl(pick, j * GL, kWave);
            if (((uint32_t)(bb >> (j * GL)) & kAll) && lane == pj) bad = true;
        }
    }
}

__global__ __launch_bounds__(kWG) void k_validate(Batch b, int which, const int64_t *nnz_tab, uint32_t *err)
{
    const int lane = threadIdx.x & 63;
    const int total = which == 0 ? b.na : b.nb;
    const int g = blockIdx.x * kWG + threadIdx.x;
    bool bad = false, longrow = false, midrow = false;
    const int32_t *ci_row = nullptr;   // entries of this thread's row (long rows)
    int len = 0, ncols = 0;
    const int32_t *base = which == 0 ? b.abase : b.bbase;
    const int t_row = b.nprob == 1 ? 0 : find_prob_rows(base, b.nprob, g - lane, g);
    if (g < total) {
        const int t = t_row;
        const Prob P = get_prob_any(b, t);
        const int i = g - (b.nprob == 1 ? 0 : gp(base)[t]);
        const MLS_G int32_t *rp = gp(which == 0 ? P.arp : P.brp);
        const int32_t *ci = which == 0 ? P.aci : P.bci;
        const int off = which == 0 ? P.a_off : P.b_off;
        ncols = which == 0 ? P.k_hi : P.ncols;
        const int nrows = which == 0 ? P.nrows : P.krows;
        const int64_t nnz = gp(nnz_tab)[2 * t + which];
        const int s = rp[i], e = rp[i + 1];
        if (i == 0 && s != off) bad = true;
        if (i == nrows - 1 && (int64_t)e - off != nnz) bad = true;
        if (e < s || s < off || (int64_t)e - off > nnz) bad = true;
        if (!bad) {
            len = e - s;
            ci_row = ci + (s - off);
            if (len <= kShortRow) {
                const MLS_G int32_t *c = gp(ci_row);
                int prev = -1, q = 0;
                for (; q + 4 <= len; q += 4) {
                    const int c0 = c[q], c1 = c[q + 1], c2 = c[q + 2], c3 = c[q + 3];
                    bad |= c0 <= prev || c1 <= c0 || c2 <= c1 || c3 <= c2 || c0 < 0 || c3 >= ncols;
                    prev = c3;
                }
                for (; q < len; ++q) {
                    const int cq = c[q];
                    bad |= cq <= prev || cq < 0 || cq >= ncols;
                    prev = cq;
                }
            } else if (len <= kWave / 2) {
                midrow = true;
            } else {
                longrow = true;
            }
        }
    }
    // rows of kShortRow + 1 .. 16 entries four per step (16 lanes each), of
    // 17 .. 32 entries two per step (32 lanes each)
    validate_group_rows<16>(__ballot(midrow && len <= 16), lane, len, ncols, ci_row, bad);
    validate_group_rows<32>(__ballot(midrow && len > 16), lane, len, ncols, ci_row, bad);
    unsigned long long lm = __ballot(longrow);
    while (lm) {
        const int src = __ffsll((long long)lm) - 1;
        lm &= lm - 1ull;
        const int n = __builtin_amdgcn_readlane(len, src);
        const int nc = __builtin_amdgcn_readlane(ncols, src);
        const uint64_t pa = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)((uint64_t)ci_row >> 32), src) << 32) |
                            (uint32_t)__builtin_amdgcn_readlane((int)(uint64_t)ci_row, src);
        const MLS_G int32_t *c = (const MLS_G int32_t *)pa;
        int carry = -1;
        bool bl = false;
        for (int q4 = 0; q4 < n; q4 += kLongAhead * kWave) {
            // the loads of kLongAhead steps first
            int cqv[kLongAhead];
#pragma unroll
            for (int u = 0; u < kLongAhead; ++u) {
                const int q = q4 + u * kWave + lane;
                cqv[u] = q < n ? c[q] : 0;
            }
#pragma unroll
            for (int u = 0; u < kLongAhead; ++u) {
                const int q0 = q4 + u * kWave;
                if (q0 >= n) break;
                const bool valid = q0 + lane < n;
                const int cq = cqv[u];
                int prev = __shfl_up(cq, 1, kWave);
                if (lane == 0) prev = carry;
                if (valid && (cq < 0 || cq >= nc || cq <= prev)) bl = true;
                carry = __shfl(cq, kWave - 1, kWave);
            }
        }
        if (__ballot(bl)) bad = bad || lane == src;
    }
    if (bad) atomicOr(err, kErrBadCsr);
}

// Column compression of every B row (set = col >> 5, mask bit = col & 31),
// padded layout: the words of row k start at B's entry offset of row k.
// One thread per row walks rows of up to kCompressShort entries; rows of up to
// 16 (32) entries take 16 (32) lanes each, four (two) at a time; the wave takes
// longer rows together, 64 entries per step: a lane starts a word where its set differs
// from the previous entry's, masks are OR-ed in LDS, and the last word of a
// step stays open (it may continue in the next step).
constexpr int kCompressShort = 4;   // longest row a single thread compresses

// 64 / GL rows per step, GL lanes per row (rows of at most GL entries); mm
// holds the lanes that own such rows; wset / wmsk: the wave's 64 LDS slots.
template <int GL>
__device__ __forceinline__ void compress_group_rows(unsigned long long mm, int lane, int len, const int32_t *ci_row,
                                                    uint2 *out_row, int32_t *cnt_ptr, uint32_t *wset, uint32_t *wmsk)
{
    constexpr int NG = kWave / GL;
    constexpr uint32_t kAll = GL == 32 ? 0xffffffffu : ((1u << GL) - 1u);
    constexpr uint32_t kNone = 0xffffffffu;
    const int grp = lane / GL, gl = lane % GL;
    while (mm) {
        int pick = -1;
#pragma unroll
        for (int j = 0; j < NG; ++j) {
            const int r = mm ? __ffsll((long long)mm) - 1 : -1;
            if (mm) mm &= mm - 1ull;
            if (j == grp) pick = r;
        }
        // every lane takes part in the shuffles (a group without a row reads lane 0)
        const int from = pick >= 0 ? pick : 0;
        int n = __shfl(len, from, kWave);
        if (pick < 0) n = 0;
        const uint64_t pc_ = ((uint64_t)(uint32_t)__shfl((int)((uint64_t)ci_row >> 32), from, kWave) << 32) |
                             (uint32_t)__shfl((int)(uint64_t)ci_row, from, kWave);
        const uint64_t po_ = ((uint64_t)(uint32_t)__shfl((int)((uint64_t)out_row >> 32), from, kWave) << 32) |
                             (uint32_t)__shfl((int)(uint64_t)out_row, from, kWave);
        const uint64_t pn_ = ((uint64_t)(uint32_t)__shfl((int)((uint64_t)cnt_ptr >> 32), from, kWave) << 32) |
                             (uint32_t)__shfl((int)(uint64_t)cnt_ptr, from, kWave);
        const bool valid = gl < n;
        const uint32_t cv = valid ? (uint32_t)((const MLS_G int32_t *)pc_)[gl] : 0u;
        const uint32_t set = valid ? (cv >> 5) : kNone;
        uint32_t prev = __shfl_up(set, 1, GL);
        if (gl == 0) prev = kNone;
        const bool head = valid && set != prev;
        const uint32_t hm = (uint32_t)(__ballot(head) >> (GL * grp)) & kAll;
        const int lw = __popc(hm & ((2u << gl) - 1u)) - 1;   // word of this entry (entry 0 is a head)
        uint32_t *hs = wset + GL * grp;
        uint32_t *hk = wmsk + GL * grp;
        hk[gl] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (valid) {
            atomicOr(&hk[lw], 1u << (cv & 31u));
            if (head) hs[lw] = set;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        const int nh = __popc(hm);
        if (gl < nh) {
            u32x2 w; w.x = hs[gl]; w.y = hk[gl];
            ((MLS_G u32x2 *)po_)[gl] = w;
        }
        if (pick >= 0 && gl == 0) gpw((int32_t *)pn_)[0] = nh;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

__global__ __launch_bounds__(kWG) void k_compress(Batch b)
{
    __shared__ uint32_t s_set[kWG / kWave][kWave + 1];
    __shared__ uint32_t s_msk[kWG / kWave][kWave + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t *wset = s_set[wave];
    uint32_t *wmsk = s_msk[wave];
    const uint32_t kNone = 0xffffffffu;
    const int g = blockIdx.x * kWG + threadIdx.x;
    bool longrow = false, midrow = false;
    const int32_t *ci_row = nullptr;
    uint2 *out_row = nullptr;
    int32_t *cnt_ptr = nullptr;
    int len = 0;
    const int t_row = b.nprob == 1 ? 0 : find_prob_rows(b.bbase, b.nprob, g - (int)(threadIdx.x & 63), g);
    if (g < b.nb) {
        const int t = t_row;
        const Prob P = get_prob_any(b, t);
        const int k = g - (b.nprob == 1 ? 0 : gp(b.bbase)[t]);
        const int s0 = gp(P.brp)[k] - P.b_off;
        len = gp(P.brp)[k + 1] - P.b_off - s0;
        ci_row = P.bci + s0;
        out_row = P.bw + s0;
        cnt_ptr = P.bwc + k;
        if (len <= kCompressShort) {
            const MLS_G int32_t *c = gp(ci_row);
            MLS_G u32x2 *out = (MLS_G u32x2 *)out_row;
            uint32_t cur = kNone, msk = 0;
            int nout = 0;
            for (int q0 = 0; q0 < len; q0 += 4) {
                int cq[4];
#pragma unroll
                for (int d = 0; d < 4; ++d) cq[d] = q0 + d < len ? c[q0 + d] : -1;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    if (cq[d] < 0) continue;
                    const uint32_t set = (uint32_t)cq[d] >> 5;
                    if (set != cur) {
                        if (cur != kNone) { u32x2 w; w.x = cur; w.y = msk; out[nout++] = w; }
                        cur = set;
                        msk = 0;
                    }
                    msk |= 1u << (cq[d] & 31);
                }
            }
            if (cur != kNone) { u32x2 w; w.x = cur; w.y = msk; out[nout++] = w; }
            gpw(cnt_ptr)[0] = nout;
        } else if (len <= kWave / 2) {
            midrow = true;
        } else {
            longrow = true;
        }
    }
    // rows of kCompressShort + 1 .. 16 entries four per step (16 lanes each),
    // of 17 .. 32 entries two per step (32 lanes each)
    compress_group_rows<16>(__ballot(midrow && len <= 16), lane, len, ci_row, out_row, cnt_ptr, wset, wmsk);
    compress_group_rows<32>(__ballot(midrow && len > 16), lane, len, ci_row, out_row, cnt_ptr, wset, wmsk);
    unsigned long long lm = __ballot(longrow);
    while (lm) {
        const int src = __ffsll((long long)lm) - 1;
        lm &= lm - 1ull;
        const int n = __builtin_amdgcn_readlane(len, src);
        auto rl64 = [&](const void *p) {
            const uint64_t v = (uint64_t)p;
            return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), src) << 32) |
                   (uint32_t)__builtin_amdgcn_readlane((int)v, src);
        };
        const MLS_G int32_t *c = (const MLS_G int32_t *)rl64(ci_row);
        MLS_G u32x2 *out = (MLS_G u32x2 *)rl64(out_row);
        int32_t *cp = (int32_t *)rl64(cnt_ptr);
        uint32_t carry_set = kNone, carry_msk = 0;
        int nout = 0;
        uint32_t cvv[kLongAhead];
        for (int c0 = 0; c0 < n; c0 += kWave) {
            const int u = (c0 / kWave) % kLongAhead;
            if (u == 0) {   // the loads of the next kLongAhead steps
#pragma unroll
                for (int v = 0; v < kLongAhead; ++v) {
                    const int qv = c0 + v * kWave + lane;
                    cvv[v] = qv < n ? (uint32_t)c[qv] : 0u;
                }
            }
            const int q = c0 + lane;
            const bool valid = q < n;
            uint32_t cv = 0u;
#pragma unroll
            for (int v = 0; v < kLongAhead; ++v)
                if (v == u) cv = cvv[v];
            cv = valid ? cv : 0u;
            const uint32_t set = valid ? (cv >> 5) : kNone;
            uint32_t prev = __shfl_up(set, 1, kWave);
            if (lane == 0) prev = carry_set;
            const bool head = valid && set != prev;
            const unsigned long long hm = __ballot(head);
            const int lw = __popcll(hm & ((2ull << lane) - 1ull));   // 0 = continues the open word
            wmsk[lane] = 0u;
            if (lane == 0) wmsk[kWave] = 0u;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            if (valid) {
                atomicOr(&wmsk[lw], 1u << (cv & 31u));
                if (head) wset[lw] = set;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            const int nh = __popcll(hm);
            // word 0 continues the open word; words 1..nh-1 are complete; word nh stays open
            if (nh > 0 && carry_set != kNone && lane == 0) {
                u32x2 w; w.x = carry_set; w.y = carry_msk | wmsk[0];
                out[nout] = w;
            }
            const int base_out = nout + (carry_set != kNone ? 1 : 0);
            if (lane >= 1 && lane < nh) {
                u32x2 w; w.x = wset[lane]; w.y = wmsk[lane];
                out[base_out + lane - 1] = w;
            }
            if (nh > 0) {
                nout += (carry_set != kNone ? 1 : 0) + nh - 1;
                carry_set = wset[nh];
                carry_msk = wmsk[nh];
            } else {
                carry_msk |= wmsk[0];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        if (carry_set != kNone) {
            if (lane == 0) { u32x2 w; w.x = carry_set; w.y = carry_msk; out[nout] = w; }
            ++nout;
        }
        if (lane == 0) gpw(cp)[0] = nout;
    }
}

// ---------------------------------------------------------------------------
// Row sizes and bins.
//   kModeCount  : size = sum over in-range k of the word count of B_k (an
//                 upper bound of the distinct column sets of row i of C)
//   kModeFill   : size = min(that bound, nnz(C_i))
//   kModeNumeric: size = nnz(C_i)
//   kModeWork   : size = sum over in-range k of nnz(B_k) (multiply-adds)
// Threshold classes: kCountCap for count, kFillCap/2 for fill and numeric.

// force < 0: natural class; force = kBinSpill: every non-empty row spills;
// 0 <= force < kNumClasses: rows of a smaller natural class move up to class
// `force` (a larger table always holds a row; test knob).
__device__ __forceinline__ int class_of(int mode, int64_t size, int force)
{
    if (size == 0) return kBinEmpty;
    if (force == kBinSpill) return kBinSpill;
    int cls = kBinSpill;
    if (mode == kModeCount) {
        for (int c = 0; c < kNumClasses; ++c)
            if (size <= kCountCap[c]) { cls = c; break; }
    } else {
        for (int c = 0; c < kNumClasses; ++c)
            if (size <= kFillCap[c] / 2) { cls = c; break; }
    }
    if (force >= 0 && cls < force) cls = force;
    return cls;
}

constexpr int kBinRG = 4;                    // lanes per row where the size is gathered (measured: 2-16)
constexpr int kBinSlots = kWG / kBinRG;      // rows in flight per workgroup
constexpr int kBinLongRow = 512;             // rows of A longer than this are gathered by the workgroup
constexpr int kBinMaxLong = 64;              // such rows deferred per block (more are gathered in place)

// Per-block bin counts (LDS) written to blk_cnt[c * nblk + block].
__device__ __forceinline__ void bin_write_counts(const Sched &sc, const int *cnt)
{
    if (threadIdx.x < kNumBins) gpw(sc.blk_cnt)[threadIdx.x * sc.nblk + (int)blockIdx.x] = cnt[threadIdx.x];
}

// Bin of a row of known size (count, fill and work modes), by one thread.
__device__ __forceinline__ void bin_place(int mode, const Sched &sc, int force, const Prob &P, int g, int i,
                                          bool from_scratch, int64_t size, int *cnt, unsigned long long *tsum)
{
    int c;
    if (from_scratch) {
        c = kBinEmpty;
    } else {
        if (mode == kModeFill) {
            const int64_t nc = gp(P.crp)[i + 1] - gp(P.crp)[i];
            size = size < nc ? size : nc;
        }
        if (mode == kModeWork) {
            c = kBinEmpty;
            if (size >= 0x7fffffffLL) atomicOr(sc.err, kErrOverflow);
            atomicAdd(tsum, (unsigned long long)size);
        } else {
            c = class_of(mode, size, force);
            // a large row whose dense bitmap over C's columns is at most half
            // its class table takes the spill path's LDS bitmap instead
            if (c >= 3 && c < kNumClasses &&
                (int64_t)P.ncols <= 32 * (int64_t)(mode == kModeCount ? kCountCap[c] : kFillCap[c]))
                c = kBinSpill;
            // rows without work get no symbolic kernel: their scratch is empty
            if (mode == kModeCount && sc.scr && c == kBinEmpty) gpw(sc.scnt)[g] = 0;
        }
    }
    if (size >= 0x7fffffffLL) size = 0x7fffffff;
    gpw(sc.val)[g] = (int32_t)size;
    gpw(sc.cls)[g] = (uint8_t)c;
    atomicAdd(&cnt[c], 1);
}

__global__ __launch_bounds__(kWG) void k_bin(Batch b, int mode, Sched sc, int force,
                                             unsigned long long *total)
{
    __shared__ int cnt[kNumBins];
    __shared__ unsigned long long tsum;
    __shared__ int s_long[kBinMaxLong];
    __shared__ int s_nlong;
    __shared__ int64_t s_red[kWG / kWave];
    if (threadIdx.x < kNumBins) cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) { tsum = 0; s_nlong = 0; }
    __syncthreads();
    const int g0 = blockIdx.x * kBinRowsPerWG;
    ProbCache pc;
    if (b.nprob > 1) {
        // the product of the block's first row, searched once per wave: the
        // block's rows almost always belong to it
        pc.t = find_prob_wave(b.abase, b.nprob, g0);
        pc.lo = gp(b.abase)[pc.t];
        pc.hi = gp(b.abase)[pc.t + 1];
    }
    if (mode == kModeNumeric) {   // size = nnz(C_i): one thread per row
        for (int r = threadIdx.x; r < kBinRowsPerWG; r += kWG) {
            const int g = g0 + r;
            if (g >= b.na) break;
            const int t = b.nprob == 1 ? 0 : find_prob_cached(b.abase, b.nprob, g, pc);
            const Prob P = get_prob_any(b, t);
            const int i = g - (b.nprob == 1 ? 0 : pc.lo);
            const int nc = gp(P.crp)[i + 1] - gp(P.crp)[i];
            const int c = class_of(mode, nc, force);
            gpw(sc.val)[g] = nc;
            gpw(sc.cls)[g] = (uint8_t)c;
            atomicAdd(&cnt[c], 1);
        }
        __syncthreads();
        bin_write_counts(sc, cnt);
        return;
    }
    const int slot = threadIdx.x / kBinRG, lane = threadIdx.x % kBinRG;
    for (int r = slot; r < kBinRowsPerWG; r += kBinSlots) {
        const int g = g0 + r;
        if (g >= b.na) break;   // uniform per row group
        const int t = b.nprob == 1 ? 0 : find_prob_cached(b.abase, b.nprob, g, pc);
        const Prob P = get_prob_any(b, t);
        const int i = g - (b.nprob == 1 ? 0 : pc.lo);
        // fill pass: rows whose words the count pass kept are expanded, not binned
        const bool from_scratch = mode == kModeFill && sc.scr && gp(sc.scnt)[g] >= 0;
        int64_t size = 0;
        if (!from_scratch) {
            const int s = gp(P.arp)[i] - P.a_off, e = gp(P.arp)[i + 1] - P.a_off;
            if (e - s > kBinLongRow) {
                // long row: gathered below by the whole workgroup, unless the list is full
                int at = 0;
                if (lane == 0) {
                    at = atomicAdd(&s_nlong, 1);
                    if (at < kBinMaxLong) s_long[at] = r;
                }
                at = __shfl(at, 0, kBinRG);
                if (at < kBinMaxLong) continue;
            }
            const MLS_G int32_t *__restrict__ aci = gp(P.aci);
            const MLS_G int32_t *__restrict__ brp = gp(P.brp);
            const MLS_G int32_t *__restrict__ bwc = gp(P.bwc);
            const int k_lo = P.k_lo, k_hi = P.k_hi;
            // four entries per lane in flight: their columns, then the gathers
            for (int p0 = s + lane; p0 < e; p0 += 4 * kBinRG) {
                int kv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int p = p0 + u * kBinRG;
                    kv[u] = p < e ? aci[p] : -1;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (kv[u] < k_lo || kv[u] >= k_hi) continue;
                    const int kl = kv[u] - k_lo;
                    size += mode == kModeWork ? (int64_t)(brp[kl + 1] - brp[kl]) : (int64_t)bwc[kl];
                }
            }
            size = group_sum<kBinRG>(size);
        }
        if (lane == 0) bin_place(mode, sc, force, P, g, i, from_scratch, size, cnt, &tsum);
    }
    __syncthreads();
    // the deferred long rows, one at a time across the workgroup
    const int nlong = s_nlong < kBinMaxLong ? s_nlong : kBinMaxLong;
    for (int x = 0; x < nlong; ++x) {
        const int g = g0 + s_long[x];
        const int t = b.nprob == 1 ? 0 : find_prob_cached(b.abase, b.nprob, g, pc);
        const Prob P = get_prob_any(b, t);
        const int i = g - (b.nprob == 1 ? 0 : pc.lo);
        const MLS_G int32_t *__restrict__ aci = gp(P.aci);
        const MLS_G int32_t *__restrict__ brp = gp(P.brp);
        const MLS_G int32_t *__restrict__ bwc = gp(P.bwc);
        const int s = gp(P.arp)[i] - P.a_off, e = gp(P.arp)[i + 1] - P.a_off;
        int64_t size = 0;
        for (int p = s + (int)threadIdx.x; p < e; p += kWG) {
            const int k = aci[p];
            if (k < P.k_lo || k >= P.k_hi) continue;
            const int kl = k - P.k_lo;
            size += mode == kModeWork ? (int64_t)(brp[kl + 1] - brp[kl]) : (int64_t)bwc[kl];
        }
        size = group_sum<kWave>(size);
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = size;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t tot = 0;
            for (int w = 0; w < kWG / kWave; ++w) tot += s_red[w];
            bin_place(mode, sc, force, P, g, i, false, tot, cnt, &tsum);
        }
        __syncthreads();
    }
    bin_write_counts(sc, cnt);
    if (threadIdx.x == 0 && total && tsum) atomicAdd(total, tsum);
}

// One workgroup: bin totals into bin_count, and every block's count per bin
// replaced by the position in perm where that block's rows of the bin start
// (bins in order, blocks in order inside a bin). Only the nb blocks of this
// launch count: a launch over fewer rows than the workspace was laid out for
// (a chunk part) leaves the counts of later blocks from earlier launches.
// The bin scan runs as one workgroup of 1024 threads, 8192 blocks of counts
// per step (a batch of 22M rows has 21.5K blocks per bin)
constexpr int kScanWG = 1024;

__global__ __launch_bounds__(kScanWG) void k_bin_scan(Sched sc, int nb)
{
    __shared__ int64_t s_red[kScanWG / kWave];
    __shared__ int64_t s_start[kNumBins];
    __shared__ int64_t s_carry;
    MLS_G int32_t *blk = gpw(sc.blk_cnt);
    const int stride = sc.nblk;
    const int nblk = nb < stride ? nb : stride;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kPer = 8;   // consecutive blocks per thread and step
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    // bins in order, the running position spanning them: every block's count
    // becomes the position in perm where its rows of the bin start; a bin's
    // total is the difference of the positions where it and the next begin.
    // With at most kScanWG * kPer blocks, all bins' counts are loaded up front.
    const bool one_step = nblk <= kScanWG * kPer;
    int32_t pre[kNumBins][kPer];
    if (one_step) {
        const int xb = threadIdx.x * kPer;
#pragma unroll
        for (int c = 0; c < kNumBins; ++c)
#pragma unroll
            for (int d = 0; d < kPer; ++d) pre[c][d] = xb + d < nblk ? blk[c * stride + xb + d] : 0;
    }
#pragma unroll
    for (int c = 0; c < kNumBins; ++c) {
        if (threadIdx.x == 0) s_start[c] = s_carry;
        for (int x0 = 0; x0 < nblk; x0 += kScanWG * kPer) {
            const int xb = x0 + threadIdx.x * kPer;
            int32_t v[kPer];
            int64_t sum = 0;
#pragma unroll
            for (int d = 0; d < kPer; ++d) {
                v[d] = one_step ? pre[c][d] : (xb + d < nblk ? blk[c * stride + xb + d] : 0);
                sum += v[d];
            }
            int64_t incl = sum;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int64_t y = __shfl_up(incl, o, kWave);
                if (lane >= o) incl += y;
            }
            if (lane == 63) s_red[wave] = incl;
            __syncthreads();
            int64_t off = s_carry + incl - sum;
            for (int w = 0; w < wave; ++w) off += s_red[w];
#pragma unroll
            for (int d = 0; d < kPer; ++d) {
                if (xb + d < nblk) blk[c * stride + xb + d] = (int32_t)off;
                off += v[d];
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int64_t t = 0;
                for (int w = 0; w < kScanWG / kWave; ++w) t += s_red[w];
                s_carry += t;
            }
            __syncthreads();
        }
    }
    __syncthreads();
    if (threadIdx.x < kNumBins) {
        const int c = threadIdx.x;
        const int64_t end = c + 1 < kNumBins ? s_start[c + 1] : s_carry;
        gpw(sc.bin_count)[c] = (int32_t)(end - s_start[c]);
    }
}

// Group the rows by bin: perm[start of bin c ...] = global rows of bin c in
// ascending order (ranks by wave ballots, so the order is deterministic).
__global__ __launch_bounds__(kWG) void k_scatter(int na, Sched sc)
{
    __shared__ int s_wcnt[kWG / kWave][kNumBins];
    __shared__ int s_base[kNumBins];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x < kNumBins) s_base[threadIdx.x] = gp(sc.blk_cnt)[threadIdx.x * sc.nblk + (int)blockIdx.x];
    __syncthreads();
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int r0 = 0; r0 < kBinRowsPerWG; r0 += kWG) {
        const int g = blockIdx.x * kBinRowsPerWG + r0 + (int)threadIdx.x;
        const int c = g < na ? (int)gp(sc.cls)[g] : -1;
        int rank = 0;
#pragma unroll
        for (int cc = 0; cc < kNumBins; ++cc) {
            const unsigned long long m = __ballot(c == cc);
            if (c == cc) rank = __popcll(m & below);
            if (lane == 0) s_wcnt[wave][cc] = __popcll(m);
        }
        __syncthreads();
        if (c >= 0) {
            int off = s_base[c];
            for (int w = 0; w < wave; ++w) off += s_wcnt[w][c];
            gpw(sc.perm)[off + rank] = g;
        }
        __syncthreads();
        if (threadIdx.x < kNumBins) {
            int t = 0;
            for (int w = 0; w < kWG / kWave; ++w) t += s_wcnt[w][threadIdx.x];
            s_base[threadIdx.x] += t;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of the per-row counts into int64 prefixes, then the int32
// row pointers of each product.

constexpr int kScanTile = 2048;   // rows per workgroup (8 per thread)

__global__ void k_scan_tiles(const int32_t *val, int n, int64_t *tile_sum)
{
    __shared__ int64_t red[kWG / kWave];
    int64_t s = 0;
    int base = blockIdx.x * kScanTile;
    for (int r = threadIdx.x; r < kScanTile; r += kWG) {
        int g = base + r;
        if (g < n) s += val[g];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < kWG / kWave; ++w) t += red[w];
        tile_sum[blockIdx.x] = t;
    }
}

// One workgroup: exclusive scan of the tile sums in place.
__global__ void k_scan_sums(int64_t *tile_sum, int ntiles)
{
    __shared__ int64_t part[kWG];
    int per = (ntiles + kWG - 1) / kWG;
    int lo = threadIdx.x * per, hi = min(ntiles, lo + per);
    int64_t s = 0;
    for (int i = lo; i < hi; ++i) s += tile_sum[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int w = 0; w < kWG; ++w) { int64_t v = part[w]; part[w] = run; run += v; }
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int i = lo; i < hi; ++i) { int64_t v = tile_sum[i]; tile_sum[i] = run; run += v; }
}

__global__ void k_scan_apply(const int32_t *val, int n, const int64_t *tile_off, int64_t *prefix)
{
    // 256 threads x 8 consecutive rows
    __shared__ int64_t wsum[kWG / kWave];
    int base = blockIdx.x * kScanTile + threadIdx.x * 8;
    int64_t v[8];
    int64_t s = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        int g = base + r;
        v[r] = g < n ? val[g] : 0;
        s += v[r];
    }
    // inclusive scan of s across the wave
    int lane = threadIdx.x & 63;
    int64_t incl = s;
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[threadIdx.x >> 6] = incl;
    __syncthreads();
    int64_t off = tile_off[blockIdx.x];
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) off += wsum[w];
    int64_t run = off + incl - s;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        int g = base + r;
        if (g < n) prefix[g] = run;
        run += v[r];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kWG - 1) prefix[n] = run;
    if (base + 8 >= n && base < n) prefix[n] = run;
}

// Row pointers of every product from the global prefix; totals[t] = nnz(C_t).
__global__ void k_write_rowptr(Batch b, const int64_t *prefix, int64_t *totals, uint32_t *err)
{
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = b.nprob == 1 ? 0 : find_prob_rows(b.abase, b.nprob, g - (int)(threadIdx.x & 63), g);
    if (g >= b.na) return;
    const Prob P = get_prob_any(b, t);
    int r0 = b.nprob == 1 ? 0 : gp(b.abase)[t];
    int i = g - r0;
    int64_t v = prefix[g + 1] - prefix[r0];
    if (v >= 0x7fffffffLL) { atomicOr(err, kErrOverflow); v = 0x7fffffff; }
    gpw(P.crp)[i + 1] = (int32_t)v;
    if (i == 0) gpw(P.crp)[0] = 0;
    if (i == P.nrows - 1) totals[t] = prefix[g + 1] - prefix[r0];
}

// ---------------------------------------------------------------------------
// launchers

static inline int nblk(int64_t n, int per) { return (int)((n + per - 1) / per); }

void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    int grid = nblk(n, kWG);
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid), dim3(kWG), 0, s, p, v, n);
}

void launch_fill_f64(double *p, double v, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    int grid = nblk(n, kWG);
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid), dim3(kWG), 0, s, p, v, n);
}

void launch_validate(const Batch &b, int which, const int64_t *nnz_tab, uint32_t *err, hipStream_t s)
{
    int n = which == 0 ? b.na : b.nb;
    if (n <= 0) return;
    ProfScope ps("validate", s);
    hipLaunchKernelGGL(k_validate, dim3(nblk(n, kWG)), dim3(kWG), 0, s, b, which, nnz_tab, err);
}

void launch_compress(const Batch &b, hipStream_t s)
{
    if (b.nb <= 0) return;
    ProfScope ps("compress", s);
    hipLaunchKernelGGL(k_compress, dim3(nblk(b.nb, kWG)), dim3(kWG), 0, s, b);
}

void launch_bin(const Batch &b, int mode, const Sched &sc, int force, unsigned long long *total,
                hipStream_t s)
{
    if (b.na <= 0) return;
    {
        ProfScope ps("bin", s);
        hipLaunchKernelGGL(k_bin, dim3(nblk(b.na, kBinRowsPerWG)), dim3(kWG), 0, s, b, mode, sc, force, total);
    }
    launch_scatter(b.na, sc, s);
}

// Bin scan and scatter after a binning kernel (blocks of kBinRowsPerWG rows).
void launch_scatter(int na, const Sched &sc, hipStream_t s)
{
    if (na <= 0) return;
    ProfScope ps("scatter", s);
    const int nb = nblk(na, kBinRowsPerWG);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(kScanWG), 0, s, sc, nb);
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kWG), 0, s, na, sc);
}

int scan_tiles(int n) { return nblk(n > 0 ? n : 1, kScanTile); }

void launch_scan(const int32_t *val, int n, int64_t *tile_sum, int64_t *prefix, hipStream_t s)
{
    int nt = scan_tiles(n);
    ProfScope ps("scan", s);
    hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(kWG), 0, s, val, n, tile_sum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kWG), 0, s, tile_sum, nt);
    hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(kWG), 0, s, val, n, tile_sum, prefix);
}

void launch_write_rowptr(const Batch &b, const int64_t *prefix, int64_t *totals, uint32_t *err, hipStream_t s)
{
    if (b.na <= 0) return;
    ProfScope ps("write_rowptr", s);
    hipLaunchKernelGGL(k_write_rowptr, dim3(nblk(b.na, kWG)), dim3(kWG), 0, s, b, prefix, totals, err);
}

}  // namespace mls
