// k_tc.hip -- triangle counting as a masked product (Sec. 4.1.2): with L the
// strict lower triangle of the degree-ordered graph, t_i = sum over k in row i
// of L of |row k of L intersected with row i of L| = row i of (L*L) o L,
// summed. Only the pattern is used and no output matrix is formed; the right
// factor is the compressed L (32 columns per word), so each intersection
// step is a bitwise AND and a popcount.
//
// LDS path: G lanes own row i. The (set, mask) words of compressed row i go
// into an LDS hash keyed by set; each lane takes entries k of row i and, for
// every word (s, m) of compressed row k, adds popcount(m & mask_i[s]).
// Spill path: rows whose own word count exceeds the largest LDS class use a
// dense bitmap of row i in global memory, one workgroup per row.
#include <cstdio>

#include "common.h"
#include "launch.h"
#include "profile.h"

namespace mls {

constexpr uint32_t kTcEmpty = 0xffffffffu;
// own-word table sizes of the classes (a row's table has at least twice its
// own words); finer than the symbolic classes between 256 and 1024 slots,
// where most of the work of power-law graphs sits
constexpr int kTcCap[kNumClasses] = {64, 256, 512, 1024, 4096};

__device__ __forceinline__ void tc_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

constexpr int nw_tc(int row_bytes, int rows_per_wave)
{
    int per_wave = row_bytes * rows_per_wave;
    int nw = 65536 / per_wave;
    return nw > 4 ? 4 : (nw < 1 ? 1 : nw);
}

// A row of L as the pipeline holds it: index (-1 for none), own word count,
// entry range, the lane's first own word, and the lane's first staged entry
// k with the offset and word count of row k of comp(L).
struct TcRow {
    int i, size, ps, pe, k, st, nk;
    u32x2 w;
};

__device__ __forceinline__ TcRow tc_row(const MLS_G int32_t *lrp, const MLS_G int32_t *val, int g)
{
    TcRow r;
    r.i = g; r.size = 0; r.ps = 0; r.pe = 0; r.k = -1; r.st = 0; r.nk = 0;
    r.w.x = 0u; r.w.y = 0u;
    if (g >= 0) {
        r.size = val[g];
        r.ps = lrp[g];
        r.pe = lrp[g + 1];
    }
    return r;
}

__device__ __forceinline__ void tc_row_words(TcRow &r, const MLS_G int32_t *lrp, const MLS_G int32_t *lci,
                                             const MLS_G u32x2 *bw, int lane)
{
    (void)lrp;
    if (r.i < 0) return;
    if (lane < r.size) r.w = bw[r.ps + lane];
    if (r.ps + lane < r.pe) r.k = lci[r.ps + lane];
}

__device__ __forceinline__ void tc_row_entry(TcRow &r, const MLS_G int32_t *lrp, const MLS_G int32_t *bwc)
{
    if (r.i >= 0 && r.k >= 0) {
        r.st = lrp[r.k];
        r.nk = bwc[r.k];
    }
}

// LDS per row: the own-word table (key, mask) and the staged entries
constexpr int tc_row_bytes(int CAP, int G) { return CAP * 8 + G * 12 + 4; }

template <int G, int CAP, int PW, int PP, int WPE>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(WPE))) void k_tc_lds(Batch b, Sched sc, int bin, int64_t *counts)
{
    constexpr int W = kWave / G;
    constexpr int NW = nw_tc(tc_row_bytes(CAP, G), W);
    __shared__ uint32_t s_key[NW * W * CAP];
    __shared__ uint32_t s_msk[NW * W * CAP];
    __shared__ int s_poff[NW * W * (G + 1)];   // first piece of each staged entry, then the total
    __shared__ int s_st[NW * W * G];           // word offset of each staged entry's row
    __shared__ int s_nk[NW * W * G];           // its word count

    const int wave = threadIdx.x >> 6;
    if (wave >= NW) return;
    const int lw = threadIdx.x & 63;
    const int slot = lw / G, lane = lw % G;
    const int rs = wave * W + slot;
    uint32_t *key = s_key + rs * CAP;
    uint32_t *msk = s_msk + rs * CAP;
    int *poff = s_poff + rs * (G + 1);
    int *pst = s_st + rs * G;
    int *pnk = s_nk + rs * G;

    const Prob P = b.p0;
    const MLS_G int32_t *__restrict__ lrp = gp(P.arp);
    const MLS_G int32_t *__restrict__ lci = gp(P.aci);
    const MLS_G u32x2 *__restrict__ bw = (const MLS_G u32x2 *)P.bw;
    const MLS_G int32_t *__restrict__ bwc = gp(P.bwc);
    const MLS_G int32_t *val = gp(sc.val);
    const int n_bin = gp(sc.bin_count)[bin];
    const int start = bin_start(sc.bin_count, bin);
    const int ntasks = (n_bin + W - 1) / W;
    // the work of a row of L drifts with its degree rank: chunks of 32 tasks
    // dealt to the XCDs round-robin keep the XCDs evenly loaded
    TaskIter it = task_iter(ntasks, NW, 5);
    // the wave index as a per-lane value (the compiler then keeps the task
    // indices in vector registers): measured faster for these kernels
    // (R-MAT 22: 19.0 against 20.3 ms)
    it.wid = (int)(blockIdx.x / kXcd) * NW + (int)(threadIdx.x >> 6);
    // Rows are software-pipelined: while a row is counted, the next row's
    // index, sizes, first own word per lane and first staged entry per lane
    // (its row of comp(L): offset and word count) are loaded, so a row starts
    // with only its pieces' words to fetch.
    int task = next_task_wave(sc.task_cursor + bin * kXcd, ntasks, it);
    int gi = (task >= 0 && task * W + slot < n_bin) ? bin_row(sc.perm, sc.err, b.na, start + task * W + slot) : -1;
    TcRow cur = tc_row(lrp, val, gi);
    tc_row_words(cur, lrp, lci, bw, lane);
    tc_row_entry(cur, lrp, bwc);
    while (task >= 0) {
        const int task_n = next_task_wave(sc.task_cursor + bin * kXcd, ntasks, it);
        const int gn = (task_n >= 0 && task_n * W + slot < n_bin)
                           ? bin_row(sc.perm, sc.err, b.na, start + task_n * W + slot) : -1;
        const bool active = cur.i >= 0;
        const int i = active ? cur.i : 0;
        const int size = cur.size;
        int logcap = ilog2_ceil(2 * size);
        if (logcap < 5) logcap = 5;
        const int cap = 1 << logcap;
        const uint32_t cmask = (uint32_t)cap - 1u;
        for (int h = lane; h < cap; h += G) key[h] = kTcEmpty;
        tc_sync();
        const int ps = cur.ps, pe = cur.pe;
        if (active) {
            const MLS_G u32x2 *wi = bw + ps;
            for (int x = lane; x < size; x += G) {
                const u32x2 wd = x == lane ? cur.w : wi[x];
                uint32_t h = hslot(wd.x, logcap);
                for (uint32_t probe = 0; probe <= cmask; ++probe) {
                    if (atomicCAS(key + h, kTcEmpty, wd.x) == kTcEmpty) { msk[h] = wd.y; break; }
                    h = (h + 1u) & cmask;
                }
            }
        }
        TcRow nxt = tc_row(lrp, val, gn);
        tc_sync();
        uint32_t cnt = 0;
        // Entries k of row i are staged G at a time; the words of row k of
        // comp(L) are cut into pieces of PW words, and the pieces of the
        // chunk are dealt round-robin to the lanes, so that one long row of L
        // does not hold up the group. A piece's entry is found by binary
        // search over the staged first-piece offsets. Pieces hold PW words; PP
        // pieces per lane are in flight at once.
        bool first = true;
        for (int pc = ps; pc < pe; pc += G) {   // ps == pe for inactive rows
            int st = 0, nk = 0;
            if (first) {
                st = cur.st;
                nk = cur.nk;
                first = false;
                // the next row's own word and entry are in flight during this chunk
                tc_row_words(nxt, lrp, lci, bw, lane);
            } else if (pc + lane < pe) {
                const int k = lci[pc + lane];
                st = lrp[k];
                nk = bwc[k];
            }
            const int np = (nk + PW - 1) / PW;
            int incl = group_scan_incl<G>(np, lane);
            const int npieces = group_total<G>(np, incl);
            poff[lane] = incl - np;
            pst[lane] = st;
            pnk[lane] = nk;
            if (lane == 0) poff[G] = npieces;
            tc_sync();
            for (int q0 = lane; q0 < npieces; q0 += G * PP) {
                // PP pieces per round: their entries are found, their words loaded,
                // and only then looked up
                u32x2 wd[PP][PW];
                int len[PP];
#pragma unroll
                for (int r = 0; r < PP; ++r) {
                    const int q = q0 + r * G;
                    len[r] = 0;
                    if (q < npieces) {
                        int lo = 0, hi = G - 1;   // largest e with poff[e] <= q
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (poff[mid] <= q) lo = mid; else hi = mid - 1;
                        }
                        const int first = (q - poff[lo]) * PW;
                        len[r] = min(PW, pnk[lo] - first);
                        const MLS_G u32x2 *wk = bw + pst[lo] + first;
#pragma unroll
                        for (int d = 0; d < PW; ++d)
                            if (d < len[r]) wd[r][d] = wk[d];
                    }
                }
#pragma unroll
                for (int r = 0; r < PP; ++r) {
#pragma unroll
                    for (int d = 0; d < PW; ++d) {
                        if (d >= len[r]) continue;
                        uint32_t h = hslot(wd[r][d].x, logcap);
                        for (uint32_t probe = 0; probe <= cmask; ++probe) {
                            uint32_t kk = key[h];
                            if (kk == wd[r][d].x) { cnt += __popc(wd[r][d].y & msk[h]); break; }
                            if (kk == kTcEmpty) break;
                            h = (h + 1u) & cmask;
                        }
                    }
                }
            }
            tc_sync();
        }
        if (first) tc_row_words(nxt, lrp, lci, bw, lane);
        tc_row_entry(nxt, lrp, bwc);
        int64_t c = group_sum<G>((int64_t)cnt);
        if (active && lane == 0) gpw(counts)[i] = c;
        tc_sync();
        cur = nxt;
        task = task_n;
    }
}

__global__ __launch_bounds__(kWG) void k_tc_spill(Batch b, Sched sc, int64_t *counts, uint32_t *bitmaps,
                                                  int64_t words)
{
    __shared__ int64_t s_red[kWG / kWave];
    uint32_t *bm = bitmaps + (int64_t)blockIdx.x * words;
    const Prob P = b.p0;
    const MLS_G int32_t *__restrict__ lrp = gp(P.arp);
    const MLS_G int32_t *__restrict__ lci = gp(P.aci);
    const MLS_G u32x2 *__restrict__ bw = (const MLS_G u32x2 *)P.bw;
    const MLS_G int32_t *__restrict__ bwc = gp(P.bwc);
    const int n_bin = gp(sc.bin_count)[kBinSpill];
    const int start = bin_start(sc.bin_count, kBinSpill);
    const int nwords = (P.ncols + 31) >> 5;
    for (int r = blockIdx.x; r < n_bin; r += gridDim.x) {
        const int i = bin_row(sc.perm, sc.err, b.na, start + r);
        if (i < 0) continue;
        for (int w = threadIdx.x; w < nwords; w += kWG)
            __hip_atomic_store(bm + w, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        __syncthreads();
        const int ps = lrp[i], pe = lrp[i + 1];
        const int ni = bwc[i];
        for (int x = threadIdx.x; x < ni; x += kWG) {
            u32x2 wd = bw[ps + x];
            __hip_atomic_store(bm + wd.x, wd.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();
        __syncthreads();
        int64_t cnt = 0;
        for (int p = ps + threadIdx.x; p < pe; p += kWG) {
            const int k = lci[p];
            const MLS_G u32x2 *wk = bw + lrp[k];
            const int nk = bwc[k];
            for (int x = 0; x < nk; ++x) {
                u32x2 wd = wk[x];
                cnt += __popc(wd.y & __hip_atomic_load(bm + wd.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            }
        }
        cnt = group_sum<kWave>(cnt);
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t s = 0;
            for (int w = 0; w < kWG / kWave; ++w) s += s_red[w];
            gpw(counts)[i] = s;
        }
        __syncthreads();
    }
}

// Bins of L's rows by the word count of row i itself (the size of its hash
// table); rows without entries count zero triangles.
__global__ __launch_bounds__(kWG) void k_tc_bin(Batch b, Sched sc, int force)
{
    __shared__ int cnt[kNumBins];
    if (threadIdx.x < kNumBins) cnt[threadIdx.x] = 0;
    __syncthreads();
    const Prob P = b.p0;
    for (int r = threadIdx.x; r < kBinRowsPerWG; r += kWG) {
        const int i = blockIdx.x * kBinRowsPerWG + r;
        if (i >= b.na) break;
        int len = gp(P.arp)[i + 1] - gp(P.arp)[i];
        int size = gp(P.bwc)[i];
        int c;
        if (len == 0) c = kBinEmpty;
        else if (force == kBinSpill) c = kBinSpill;
        else {
            c = kBinSpill;
            for (int x = kNumClasses - 1; x >= 0; --x)
                if (size <= kTcCap[x] / 2) c = x;
            if (force >= 0 && c < force) c = force;   // test knob: a larger table holds any row
        }
        gpw(sc.val)[i] = size;
        gpw(sc.cls)[i] = (uint8_t)c;
        atomicAdd(&cnt[c], 1);
    }
    __syncthreads();
    if (threadIdx.x < kNumBins) gpw(sc.blk_cnt)[threadIdx.x * sc.nblk + (int)blockIdx.x] = cnt[threadIdx.x];
}

__global__ void k_sum_i64(const int64_t *x, int n, unsigned long long *total)
{
    __shared__ int64_t s_red[kWG / kWave];
    int64_t s = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) s += gp(x)[i];
    s = group_sum<kWave>(s);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < kWG / kWave; ++w) t += s_red[w];
        if (t) atomicAdd(total, (unsigned long long)t);
    }
}

template <typename K>
static int tc_grid(K kernel, int threads)
{
    static int cus = device_cu_count();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

template <int G, int CAP, int P, int PP, int WPE = 8>
static void launch_tc_class(const Batch &b, const Sched &sc, int bin, int64_t *counts, hipStream_t s)
{
    constexpr int W = kWave / G;
    constexpr int NW = nw_tc(tc_row_bytes(CAP, G), W);
    static int grid = tc_grid(k_tc_lds<G, CAP, P, PP, WPE>, NW * kWave);
    static char name[64];
    if (!name[0]) snprintf(name, sizeof(name), "tc_lds_G%d_C%d", G, CAP);
    ProfScope ps(name, s);
    hipLaunchKernelGGL((k_tc_lds<G, CAP, P, PP, WPE>), dim3(grid), dim3(NW * kWave), 0, s, b, sc, bin, counts);
}

void launch_tc_bin(const Batch &b, const Sched &sc, int force, hipStream_t s)
{
    if (b.na <= 0) return;
    int grid = (b.na + kBinRowsPerWG - 1) / kBinRowsPerWG;
    {
        ProfScope ps("tc_bin", s);
        hipLaunchKernelGGL(k_tc_bin, dim3(grid), dim3(kWG), 0, s, b, sc, force);
    }
    launch_scatter(b.na, sc, s);
}

void launch_tc(const Batch &b, const Sched &sc, int64_t *counts, unsigned long long *total, uint32_t *spill_bitmaps,
               int spill_slots, int64_t spill_words, hipStream_t s)
{
    if (b.na <= 0) return;
    // lanes per row, words per piece, pieces in flight per lane: measured on R-MAT
    launch_tc_class<32, kTcCap[0], 8, 1>(b, sc, 0, counts, s);
    launch_tc_class<64, kTcCap[1], 8, 1>(b, sc, 1, counts, s);
    launch_tc_class<64, kTcCap[2], 8, 1>(b, sc, 2, counts, s);
    launch_tc_class<64, kTcCap[3], 8, 1>(b, sc, 3, counts, s);
    launch_tc_class<64, kTcCap[4], 8, 1>(b, sc, 4, counts, s);
    {
        ProfScope ps("tc_spill", s);
        hipLaunchKernelGGL(k_tc_spill, dim3(spill_slots), dim3(kWG), 0, s, b, sc, counts, spill_bitmaps, spill_words);
    }
    ProfScope ps("tc_sum", s);
    hipLaunchKernelGGL(k_sum_i64, dim3(1024), dim3(kWG), 0, s, counts, b.na, total);
}

}  // namespace mls
