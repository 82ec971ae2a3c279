// k_symbolic.hip -- symbolic phase (Sec. 2.1): for every row i of C the union
// of the compressed column sets of the rows B_k, k in row i of A.
//
// LDS path: G lanes own one row; the lanes walk the entries of row i of A
// (one k per lane) and OR every (set, mask) word of compressed B_k into an
// open-addressing hash table in LDS keyed by set. Count pass: rownnz =
// sum of popcounts. Fill pass: the occupied (set, mask) pairs are compacted,
// sorted by set in LDS (bitonic network), and their bits expand into
// ascending columns at offsets from a scan of the popcounts.
//
// Spill path (rows whose word bound exceeds the largest LDS class, and large
// rows whose dense bitmap is smaller than their class table): one workgroup
// per row with a dense bitmap over C's columns in LDS (column windows when C
// is wider than the LDS holds); scanning the bitmap in order yields sorted
// columns directly.
#include <cstdio>

#include "common.h"
#include "launch.h"
#include "profile.h"

namespace mls {

constexpr uint32_t kEmptyKey = 0xffffffffu;
constexpr int kSymBatch = 6;   // words of one B_k row loaded before they are inserted (measured)
// fewer where 32 or more lanes own a row (their count kernels run at 6 waves per SIMD)
template <int G, bool FILL>
constexpr int sym_batch() { return (!FILL && (G >= 32 || G <= 8)) ? 4 : kSymBatch; }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

constexpr int nw_for(int row_bytes, int rows_per_wave)
{
    int per_wave = row_bytes * rows_per_wave;
    int nw = 65536 / per_wave;
    return nw > 4 ? 4 : (nw < 1 ? 1 : nw);
}

// OR mask m into the slot of set s, given the word k read from its home slot
// h (possibly before other lanes' inserts: an empty slot is claimed with a
// compare-and-swap, whose result is the slot's current key)
__device__ __forceinline__ void set_insert_at(uint32_t *key, uint32_t *msk, int logcap, uint32_t s, uint32_t m,
                                              uint32_t h, uint32_t k, uint32_t *err)
{
    const uint32_t cmask = (1u << logcap) - 1u;
    for (uint32_t probe = 0; probe <= cmask; ++probe) {
        if (k == kEmptyKey) k = atomicCAS(key + h, kEmptyKey, s);
        if (k == kEmptyKey || k == s) { atomicOr(msk + h, m); return; }
        h = (h + 1u) & cmask;
        k = __hip_atomic_load(key + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    atomicOr(err, kErrTable);
}

// Where a row of the bin lives: product t, local row i, its table size
// bound and its A entry range [ps, pe) (local); g < 0 for no row.
// The descriptor of product t: the kernel argument for a single product (the
// kernels are specialised for it), else read once per wave when the wave's
// rows share their product.
template <bool MULTI>
__device__ __forceinline__ Prob sym_prob(const Batch &b, int t)
{
    if (!MULTI) return b.p0;
    return get_prob_batch(b, t);
}

// Where a row of the bin lives: row g (-1: none), product t, local row i,
// output bound or size (size) and its A entry range [ps, pe). The loads are
// issued by sym_issue without a branch around them (a slot without a row
// reads zeros) and the offsets applied by sym_final, a row later.
struct SymRow {
    int g, t, i, size, ps, pe;
};

template <bool MULTI>
__device__ __forceinline__ SymRow sym_issue(const Batch &b, const Sched &sc, int g, ProbCache &pc)
{
    SymRow m{g, 0, 0, 0, 0, 0};
    const bool on = g >= 0;
    m.i = on ? g : 0;
    if (MULTI && on) {
        m.t = find_prob_cached(b.abase, b.nprob, g, pc);
        m.i = g - pc.lo;
    }
    const Prob P = sym_prob<MULTI>(b, m.t);
    const MLS_G int32_t *zero = (const MLS_G int32_t *)k_zeros4;
    const MLS_G int32_t *pv = on ? gp(sc.val) + g : zero;
    const MLS_G int32_t *pa = on ? gp(P.arp) + m.i : zero;
    m.size = *pv;
    m.ps = pa[0];
    m.pe = pa[1];
    return m;
}

template <bool MULTI>
__device__ __forceinline__ SymRow sym_final(const Batch &b, const SymRow &r)
{
    SymRow m = r;
    const int a_off = sym_prob<MULTI>(b, r.t).a_off;
    m.ps = r.ps - a_off;
    m.pe = r.pe - a_off;
    return m;
}

// The B row of entry ps + lane of a row of A (its first chunk), located in
// advance: the column (-1 past the row), then the word offset and count of
// its compressed row as loaded (zeros for a column outside [k_lo, k_hi): no
// words).
struct SymFirst {
    int k, q0, nw;
};

template <bool MULTI>
__device__ __forceinline__ void sym_first_a(const Batch &b, const SymRow &m, int lane, SymFirst &f)
{
    const bool on = m.ps + lane < m.pe;
    const MLS_G int32_t *pk = on ? gp(sym_prob<MULTI>(b, m.t).aci) + m.ps + lane : (const MLS_G int32_t *)k_ones4;
    f.k = *pk;
}

template <bool MULTI>
__device__ __forceinline__ void sym_first_b(const Batch &b, const SymRow &m, SymFirst &f)
{
    const Prob P = sym_prob<MULTI>(b, m.t);
    const bool in = f.k >= P.k_lo && f.k < P.k_hi;
    const int kl = in ? f.k - P.k_lo : 0;
    const MLS_G int32_t *zero = (const MLS_G int32_t *)k_zeros4;
    f.q0 = *(in ? gp(P.brp) + kl : zero);
    f.nw = *(in ? gp(P.bwc) + kl : zero);
}

// Waves per SIMD that the count kernel's LDS leaves resident (160 KB per CU,
// 4 SIMDs), at most 6 for 64 lanes per row and 5 otherwise, one fewer for
// batches (registers for the batched inserts and the row pipeline, without
// spills); the kernel is compiled to fit that many.
template <int G, int CAP, bool MULTI>
constexpr int sym_count_waves()
{
    constexpr int W = kWave / G;
    constexpr int NW = nw_for(CAP * 8, W);
    constexpr int wgs = 163840 / (NW * W * CAP * 8);
    constexpr int w = wgs * NW / 4;
    constexpr int cap = MULTI ? (G == 64 ? 5 : 4) : (G == 64 ? 6 : 5);
    return w > cap ? cap : (w < 1 ? 1 : w);
}

template <int G, int CAP, bool FILL, bool MULTI>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(FILL ? 1 : sym_count_waves<G, CAP, MULTI>())))
void k_sym_lds(Batch b, Sched sc, int bin)
{
    constexpr int W = kWave / G;
    constexpr int SB = sym_batch<G, FILL>();
    constexpr int ROWB = FILL ? CAP * 12 : CAP * 8;
    constexpr int NW = nw_for(ROWB, W);
    constexpr int LIST = FILL ? CAP / 2 : 1;
    // the fill pass's (set, mask) lists and counters follow the keys; the
    // count pass allocates nothing beyond the two tables, so that its
    // workgroups use exactly 16 or 32 KB and tile the 160 KB of LDS of a CU
    constexpr int EXTRA = FILL ? NW * W * (2 * LIST + 1) : 0;
    __shared__ __attribute__((aligned(16))) uint32_t s_key[NW * W * CAP + EXTRA];
    __shared__ __attribute__((aligned(16))) uint32_t s_msk[NW * W * CAP];
    uint2 *s_list = (uint2 *)(s_key + NW * W * CAP);
    int *s_cnt = (int *)(s_key + NW * W * CAP + NW * W * 2 * LIST);

    const int wave = threadIdx.x >> 6;
    if (wave >= NW) return;   // launched with NW waves; guard anyway
    const int lw = threadIdx.x & 63;
    const int slot = lw / G, lane = lw % G;
    const int rs = wave * W + slot;
    uint32_t *key = s_key + rs * CAP;
    uint32_t *msk = s_msk + rs * CAP;
    uint2 *list = s_list + rs * LIST;

    MLS_G int32_t *val = gpw(sc.val);
    const int n_bin = gp(sc.bin_count)[bin];
    const int start = bin_start(sc.bin_count, bin);
    const int ntasks = (n_bin + W - 1) / W;
    TaskIter it = task_iter(ntasks, NW);
    // Rows are software-pipelined, three of a slot in flight: the row after
    // next has its perm entry loading, the next row its size and row pointers,
    // then the B rows of its first chunk (the entries of A once this row's
    // words are inserted, the word offsets and counts after its count), so a
    // row starts with its dependent index loads done.
    int task = next_task_wave(sc.task_cursor + bin * kXcd, ntasks, it);
    const bool h_cur = task >= 0 && task * W + slot < n_bin;
    const int g_raw = bin_row_issue(sc.perm, sc.err, b.na, start + task * W + slot, h_cur);
    int task_n = task >= 0 ? next_task_wave(sc.task_cursor + bin * kXcd, ntasks, it) : -1;
    bool h_n = task_n >= 0 && task_n * W + slot < n_bin;
    int g_n = bin_row_issue(sc.perm, sc.err, b.na, start + task_n * W + slot, h_n);
    ProbCache pc;
    SymRow mr = sym_issue<MULTI>(b, sc, bin_row_checked(sc.err, b.na, g_raw, h_cur), pc);
    SymFirst f;
    {
        const SymRow m0 = sym_final<MULTI>(b, mr);
        sym_first_a<MULTI>(b, m0, lane, f);
        sym_first_b<MULTI>(b, m0, f);
    }
    // no prologue load is left pending into the loop (the wait counts at its
    // top are computed over both ways into it)
    asm volatile("" ::"v"(f.q0), "v"(f.nw), "v"(g_n), "v"(mr.size), "v"(mr.ps), "v"(mr.pe));
    while (task >= 0) {
        const int task_x = task_n >= 0 ? next_task_wave(sc.task_cursor + bin * kXcd, ntasks, it) : -1;
        const bool h_x = task_x >= 0 && task_x * W + slot < n_bin;
        const int g_x = bin_row_issue(sc.perm, sc.err, b.na, start + task_x * W + slot, h_x);
        const SymRow mr_n = sym_issue<MULTI>(b, sc, bin_row_checked(sc.err, b.na, g_n, h_n), pc);
        const SymRow m = sym_final<MULTI>(b, mr);
        const bool active = m.g >= 0;
        const int g = active ? m.g : 0;
        const int t = m.t;
        const Prob P = sym_prob<MULTI>(b, t);
        const int i = m.i;
        const int size = m.size;
        int logcap = ilog2_ceil(FILL ? 2 * size : size);
        if (logcap < 5) logcap = 5;
        const int cap = 1 << logcap;
        // table passes touch 4 slots per lane per access when the table is large enough
        const bool vec = cap >= 4 * G;
        if (vec) {
            for (int h = 4 * lane; h < cap; h += 4 * G) {
                *(uint4 *)(key + h) = make_uint4(kEmptyKey, kEmptyKey, kEmptyKey, kEmptyKey);
                *(uint4 *)(msk + h) = make_uint4(0u, 0u, 0u, 0u);
            }
        } else {
            for (int h = lane; h < cap; h += G) { key[h] = kEmptyKey; msk[h] = 0u; }
        }
        if (FILL && lane == 0) s_cnt[rs] = 0;
        wave_sync();
        if (active) {
            const MLS_G int32_t *__restrict__ aci = gp(P.aci);
            const MLS_G int32_t *__restrict__ brp = gp(P.brp);
            const MLS_G u32x2 *__restrict__ bw = (const MLS_G u32x2 *)P.bw;
            const MLS_G int32_t *__restrict__ bwc = gp(P.bwc);
            const int b_off = P.b_off, k_lo = P.k_lo, k_hi = P.k_hi;
            const int ps = m.ps, pe = m.pe;
            for (int p = ps + lane; p < pe; p += G) {
                int q0, nw;
                if (p == ps + lane) {   // first chunk: B row located during the previous row
                    q0 = f.q0 - b_off;
                    nw = f.nw;
                } else {
                    const int k = aci[p];
                    if (k < k_lo || k >= k_hi) continue;
                    const int kl = k - k_lo;
                    q0 = brp[kl] - b_off;
                    nw = bwc[kl];
                }
                const MLS_G u32x2 *w = bw + q0;
                // each lane starts at its own word of the row and wraps around:
                // neighbouring rows of B share most sets, and lanes ORing the same
                // set in one instruction would be serialized by the LDS
                const int rot = nw > 0 ? lane % nw : 0;
                for (int x = 0; x < nw; x += SB) {
                    u32x2 wd[SB];
#pragma unroll
                    for (int d = 0; d < SB; ++d)
                        if (x + d < nw) {
                            int e = x + d + rot;
                            if (e >= nw) e -= nw;
                            wd[d] = w[e];
                        }
                    // the home slots of all the words are read before any is
                    // updated, so their LDS latencies overlap
                    uint32_t hv[SB], kv[SB];
#pragma unroll
                    for (int d = 0; d < SB; ++d) hv[d] = x + d < nw ? hslot(wd[d].x, logcap) : 0u;
#pragma unroll
                    for (int d = 0; d < SB; ++d)
                        kv[d] = __hip_atomic_load(key + hv[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    // empty home slots claimed together, then the ORs; a word
                    // whose home slot holds another set probes on
#pragma unroll
                    for (int d = 0; d < SB; ++d)
                        if (x + d < nw && kv[d] == kEmptyKey) kv[d] = atomicCAS(key + hv[d], kEmptyKey, wd[d].x);
#pragma unroll
                    for (int d = 0; d < SB; ++d) {
                        if (x + d >= nw) continue;
                        if (kv[d] == kEmptyKey || kv[d] == wd[d].x)
                            atomicOr(msk + hv[d], wd[d].y);
                        else
                            set_insert_at(key, msk, logcap, wd[d].x, wd[d].y, hv[d], kv[d], sc.err);
                    }
                }
            }
        }
        wave_sync();
        // locate the next row's first chunk of B rows while this row is
        // finished: the entries of A now, the B rows' word offsets and counts
        // once they arrive
        const SymRow mn = sym_final<MULTI>(b, mr_n);
        sym_first_a<MULTI>(b, mn, lane, f);
        if (!FILL) {
            // one pass over the table: popcount of the union, and the occupied
            // (set, mask) words compacted in slot order into the row's scratch
            // slot for the fill pass (the first kScratchWords of them; a row
            // with more is marked and rebuilt there); each lane owns 4 (vec)
            // or 1 consecutive slots per step
            const int per = vec ? 4 : 1;
            MLS_G u32x2 *dst = sc.scr ? (MLS_G u32x2 *)sc.scr + (int64_t)g * kScratchWords : nullptr;
            int c = 0, base = 0;
            for (int h0 = 0; h0 < cap; h0 += per * G) {
                const int h = h0 + per * lane;
                uint32_t kk[4], mm[4];
                int nl = 0;
                if (h < cap) {
                    if (vec) {
                        const uint4 k4 = *(const uint4 *)(key + h);
                        const uint4 m4 = *(const uint4 *)(msk + h);
                        kk[0] = k4.x; kk[1] = k4.y; kk[2] = k4.z; kk[3] = k4.w;
                        mm[0] = m4.x; mm[1] = m4.y; mm[2] = m4.z; mm[3] = m4.w;
                    } else {
                        kk[0] = key[h]; mm[0] = msk[h];
                    }
                    for (int x = 0; x < per; ++x) {
                        nl += kk[x] != kEmptyKey;
                        c += __popc(mm[x]);
                    }
                }
                // exclusive prefix of nl over the group
                const int incl = group_scan_incl<G>(nl, lane);
                const int tot = group_total<G>(nl, incl);
                if (sc.scr && active && nl) {
                    int w = base + incl - nl;
                    for (int x = 0; x < per; ++x)
                        if (kk[x] != kEmptyKey) {
                            if (w < kScratchWords) {
                                u32x2 v; v.x = kk[x]; v.y = mm[x];
                                dst[w] = v;
                            }
                            ++w;
                        }
                }
                base += tot;
            }
            c = group_sum<G>(c);
            sym_first_b<MULTI>(b, mn, f);
            if (active && lane == 0) {
                val[g] = c;
                if (sc.scr) gpw(sc.scnt)[g] = base <= kScratchWords ? base : -1;
            }
        } else {
            sym_first_b<MULTI>(b, mn, f);
            for (int h = lane; h < cap; h += G) {
                uint32_t k = key[h];
                if (k != kEmptyKey) {
                    int e = atomicAdd(&s_cnt[rs], 1);
                    if (e < LIST) list[e] = make_uint2(k, msk[h]);
                    else atomicOr(sc.err, kErrTable);
                }
            }
            wave_sync();
            // sort the row's (set, mask) words by set (bitonic network over the
            // list padded to a power of two with sets that sort last), then
            // give each lane a contiguous run of words: an exclusive scan of
            // the runs' popcounts places every word's bits in the output row
            const int n = active ? min(s_cnt[rs], LIST) : 0;
            int npad = 1;
            while (npad < n) npad <<= 1;
            for (int e = n + lane; e < npad; e += G) list[e] = make_uint2(kEmptyKey, 0u);
            wave_sync();
            for (int kk = 2; kk <= npad; kk <<= 1) {
                for (int j = kk >> 1; j > 0; j >>= 1) {
                    for (int e = lane; e < npad; e += G) {
                        const int l = e ^ j;
                        if (l > e) {
                            const uint2 ae = list[e], al = list[l];
                            if ((ae.x > al.x) == ((e & kk) == 0)) { list[e] = al; list[l] = ae; }
                        }
                    }
                    wave_sync();
                }
            }
            const int per = (n + G - 1) / G;
            const int e0 = min(lane * per, n), e1 = min(e0 + per, n);
            int run = 0;
            for (int e = e0; e < e1; ++e) run += __popc(list[e].y);
            int incl = group_scan_incl<G>(run, lane);
            if (active) {
                const int cs = gp(P.crp)[i] - P.c_off;
                const int ce = gp(P.crp)[i + 1] - P.c_off;
                MLS_G int32_t *__restrict__ cci = gpw(P.cci);
                int pos = cs + incl - run;
                for (int e = e0; e < e1; ++e) {
                    const uint2 me = list[e];
                    uint32_t m = me.y;
                    while (m) {
                        const int bit = __ffs(m) - 1;
                        if (pos < ce) cci[pos] = (int32_t)(me.x * 32u + (uint32_t)bit);
                        else atomicOr(sc.err, kErrStructure);
                        ++pos;
                        m &= m - 1u;
                    }
                }
            }
        }
        wave_sync();
        task = task_n;
        task_n = task_x;
        g_n = g_x;
        h_n = h_x;
        mr = mr_n;
    }
}

// Spill path: rows whose word bound exceeds the largest LDS class. One
// workgroup per row, rows taken from a counter. The row's union is a dense
// bitmap in LDS over a window of columns: the whole column range whenever it
// fits (up to 2^20 columns with 128 KB), else one window after the other,
// each entry's words narrowed to the window by binary search (a row of
// comp(B) lists its sets in ascending order). The words of the staged
// entries are cut into pieces of kSpillPW, dealt to the threads round-robin,
// so that one long row of B does not hold up the workgroup; OR-ing is order-
// free. The fill pass reads the bitmap back in column order.
constexpr int kSpillPW = 4;

__device__ __forceinline__ int lower_set(const MLS_G u32x2 *w, int n, uint32_t set)
{
    // first word of w[0, n) whose set is >= set
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (w[mid].x < set) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kWG) void k_sym_spill(Batch b, Sched sc, int fill, int win_words)
{
    extern __shared__ uint32_t s_bm[];   // win_words words
    __shared__ int s_poff[kWG + 1];
    __shared__ int s_st[kWG];
    __shared__ int s_nk[kWG];
    __shared__ int s_red[kWG / kWave];
    __shared__ int s_row;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n_bin = gp(sc.bin_count)[kBinSpill];
    const int start = bin_start(sc.bin_count, kBinSpill);
    int32_t *cursor = sc.task_cursor + kBinSpill * kXcd;
    for (;;) {
        if (tid == 0) s_row = atomicAdd(cursor, 1);
        __syncthreads();
        const int r = s_row;
        __syncthreads();
        if (r >= n_bin) break;
        const int g = bin_row(sc.perm, sc.err, b.na, start + r);
        if (g < 0) continue;
        const int t = b.nprob == 1 ? 0 : find_prob(b.abase, b.nprob, g);
        const Prob P = get_prob_any(b, t);
        const int i = g - (b.nprob == 1 ? 0 : gp(b.abase)[t]);
        const MLS_G int32_t *__restrict__ aci = gp(P.aci);
        const MLS_G int32_t *__restrict__ brp = gp(P.brp);
        const MLS_G int32_t *__restrict__ bwc = gp(P.bwc);
        const MLS_G u32x2 *__restrict__ bw = (const MLS_G u32x2 *)P.bw;
        const int nwords = (P.ncols + 31) >> 5;
        const int ww = nwords < win_words ? nwords : win_words;
        const bool windowed = ww < nwords;
        const int ps = gp(P.arp)[i] - P.a_off, pe = gp(P.arp)[i + 1] - P.a_off;
        const int cs = fill ? gp(P.crp)[i] - P.c_off : 0;
        const int ce = fill ? gp(P.crp)[i + 1] - P.c_off : 0;
        int total = 0;   // columns found so far (uniform)
        bool bad = false;
        for (int w0 = 0; w0 < nwords; w0 += ww) {
            const int wn = nwords - w0 < ww ? nwords - w0 : ww;
            for (int x = tid; x < wn; x += kWG) s_bm[x] = 0u;
            __syncthreads();
            for (int pb = ps; pb < pe; pb += kWG) {
                int st = 0, nk = 0;
                const int p = pb + tid;
                if (p < pe) {
                    const int k = aci[p];
                    if (k >= P.k_lo && k < P.k_hi) {
                        const int kl = k - P.k_lo;
                        st = brp[kl] - P.b_off;
                        nk = bwc[kl];
                        if (windowed) {
                            const int lo = lower_set(bw + st, nk, (uint32_t)w0);
                            const int hi = lower_set(bw + st, nk, (uint32_t)(w0 + wn));
                            st += lo;
                            nk = hi - lo;
                        }
                    }
                }
                // exclusive scan of the piece counts over the workgroup
                const int np = (nk + kSpillPW - 1) / kSpillPW;
                int incl = np;
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) {
                    const int y = __shfl_up(incl, o, kWave);
                    if (lane >= o) incl += y;
                }
                if (lane == kWave - 1) s_red[wave] = incl;
                __syncthreads();
                int before = 0, all = 0;
#pragma unroll
                for (int x = 0; x < kWG / kWave; ++x) {
                    before += x < wave ? s_red[x] : 0;
                    all += s_red[x];
                }
                s_poff[tid] = before + incl - np;
                s_st[tid] = st;
                s_nk[tid] = nk;
                if (tid == 0) s_poff[kWG] = all;
                __syncthreads();
                for (int q = tid; q < all; q += kWG) {
                    int lo = 0, hi = kWG - 1;   // largest e with s_poff[e] <= q
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_poff[mid] <= q) lo = mid; else hi = mid - 1;
                    }
                    const int first = (q - s_poff[lo]) * kSpillPW;
                    const int len = min(kSpillPW, s_nk[lo] - first);
                    const MLS_G u32x2 *src = bw + s_st[lo] + first;
                    u32x2 wd[kSpillPW];
#pragma unroll
                    for (int d = 0; d < kSpillPW; ++d)
                        if (d < len) wd[d] = src[d];
#pragma unroll
                    for (int d = 0; d < kSpillPW; ++d) {
                        if (d >= len) continue;
                        const uint32_t x = wd[d].x - (uint32_t)w0;
                        if (x < (uint32_t)wn) atomicOr(s_bm + x, wd[d].y);
                        else bad = true;
                    }
                }
                __syncthreads();
            }
            // the window's columns: thread tid reads a run of consecutive words
            const int run = (wn + kWG - 1) / kWG;
            const int x0 = tid * run;
            const int x1 = x0 + run < wn ? x0 + run : wn;
            int c = 0;
            for (int x = x0; x < x1; ++x) c += __popc(s_bm[x]);
            int incl = c;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int y = __shfl_up(incl, o, kWave);
                if (lane >= o) incl += y;
            }
            if (lane == kWave - 1) s_red[wave] = incl;
            __syncthreads();
            int before = 0, all = 0;
#pragma unroll
            for (int x = 0; x < kWG / kWave; ++x) {
                before += x < wave ? s_red[x] : 0;
                all += s_red[x];
            }
            if (fill) {
                MLS_G int32_t *cci = gpw(P.cci);
                int pos = cs + total + before + incl - c;
                for (int x = x0; x < x1; ++x) {
                    uint32_t m = s_bm[x];
                    while (m) {
                        const int bit = __ffs(m) - 1;
                        if (pos < ce) cci[pos] = (w0 + x) * 32 + bit;
                        else bad = true;
                        ++pos;
                        m &= m - 1u;
                    }
                }
            }
            total += all;
            __syncthreads();
        }
        if (bad) atomicOr(sc.err, kErrStructure);
        if (!fill && tid == 0) {
            gpw(sc.val)[g] = total;
            if (sc.scr) gpw(sc.scnt)[g] = -1;   // recomputed by the fill pass
        }
        if (fill && tid == 0 && cs + total != ce) atomicOr(sc.err, kErrStructure);
    }
}

// Fill pass from the count pass's scratch: lane e holds word e of a row (a
// row keeps at most kScratchWords = 64 words). A word's output offset is the
// popcount sum of the words with smaller sets, accumulated from lane reads
// (no LDS); its bits then expand into ascending columns. Rows without scratch
// words (scnt < 0) are left to the recomputing fill kernels.
static_assert(kScratchWords == kWave, "one scratch word per lane");
constexpr int kExpandSmall = 16;   // rows with at most this many words take the 16-lane kernel
constexpr int kExpandMid = 32;     // rows with at most this many words take the 32-lane kernel
constexpr int kExpandStage = 256;  // columns of a row staged in LDS before the ordered write-out

struct ExpandRow {
    int cs, ce, t;
    u32x2 w;
};

// Scratch words (lane < n), product and C row bounds of global row g.
__device__ __forceinline__ ExpandRow expand_load(const Batch &b, const Sched &sc, int g, int n, int lane,
                                                 ProbCache &pc)
{
    ExpandRow r;
    r.cs = 0; r.ce = 0; r.t = 0;
    r.w.x = 0u; r.w.y = 0u;
    if (g < 0) return r;
    if (lane < n) r.w = ((const MLS_G u32x2 *)sc.scr)[(int64_t)g * kScratchWords + lane];
    int i = g;
    if (b.nprob > 1) {
        r.t = find_prob_cached(b.abase, b.nprob, g, pc);
        i = g - pc.lo;
    }
    const Prob P = get_prob_any(b, r.t);
    r.cs = gp(P.crp)[i] - P.c_off;
    r.ce = gp(P.crp)[i + 1] - P.c_off;
    return r;
}

// Rows of more than kExpandMid words: a wave reads the word counts of 64
// consecutive rows, then takes the large ones one at a time; the next large
// row's words are loaded while the current one is ranked and written.
__global__ __launch_bounds__(kWG) void k_sym_expand(Batch b, Sched sc)
{
    const int lane = threadIdx.x & 63;
    const int nw = (int)gridDim.x * (kWG / kWave);
    const int w0 = (int)((blockIdx.x * kWG + threadIdx.x) >> 6);
    const MLS_G int32_t *scnt = gp(sc.scnt);
    ProbCache pc;
    for (int base = w0 * kWave; base < b.na; base += nw * kWave) {
        const int gl = base + lane;
        const int nl = gl < b.na ? scnt[gl] : 0;
        unsigned long long big = __ballot(nl > kExpandMid);
        if (!big) continue;
        int r = __ffsll((long long)big) - 1;
        big &= big - 1ull;
        int n = __builtin_amdgcn_readlane(nl, r);
        ExpandRow cur = expand_load(b, sc, base + r, n, lane, pc);
        for (;;) {
            // prefetch the next large row of this chunk
            int rn = -1, nn = 0;
            if (big) {
                rn = __ffsll((long long)big) - 1;
                big &= big - 1ull;
                nn = __builtin_amdgcn_readlane(nl, rn);
            }
            const ExpandRow nxt = expand_load(b, sc, rn >= 0 ? base + rn : -1, nn, lane, pc);
            MLS_G int32_t *__restrict__ cci = gpw(get_prob_any(b, cur.t).cci);
            const uint32_t set = cur.w.x;
            // set < 2^26 (columns < 2^31) and a popcount <= 32 share one word:
            // set << 6 | popcount, so one lane read carries both, and
            // key_f < set << 6 exactly when set_f < set. Lanes at or past n
            // carry popcount 0, so the loop may run to a multiple of 4.
            const uint32_t kbase = set << 6;
            const uint32_t key = kbase | (uint32_t)(lane < n ? __popc(cur.w.y) : 0);
            int off = 0;
            for (int f = 0; f < n; f += 4) {
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const uint32_t kf = (uint32_t)__builtin_amdgcn_readlane((int)key, f + d);
                    off += kf < kbase ? (int)(kf & 63u) : 0;
                }
            }
            if (lane < n) {
                uint32_t m = cur.w.y;
                int pos = cur.cs + off;
                while (m) {
                    const int bit = __ffs(m) - 1;
                    if (pos < cur.ce) cci[pos] = (int32_t)(set * 32u + (uint32_t)bit);
                    else atomicOr(sc.err, kErrStructure);
                    ++pos;
                    m &= m - 1u;
                }
            }
            if (rn < 0) break;
            r = rn;
            n = nn;
            cur = nxt;
        }
    }
}

// Rows of (NLO, G] words, G at most kExpandMid: a wave reads the word counts
// of 64 consecutive rows and takes those rows 64 / G at a time, G lanes per
// row; the group's (set, popcount) keys go through LDS, where every lane
// reads all of them to rank its own word.
template <int G, int NLO>
__global__ __launch_bounds__(kWG) void k_sym_expand_small(Batch b, Sched sc)
{
    static_assert(G <= kExpandMid && NLO < G, "row sizes (NLO, G] of at most kExpandMid words");
    // the group's keys, exchanged through LDS (four per read) rather than by
    // one cross-lane shuffle per key
    __shared__ __attribute__((aligned(16))) uint32_t s_k[kWG];
    // a row's columns are placed in LDS first and written out in order, so
    // that the stores of a group are contiguous (rows of at most
    // kExpandStage columns; longer ones are written lane by lane)
    __shared__ int32_t s_col[(kWG / G) * kExpandStage];
    const int lane64 = threadIdx.x & 63;
    const int slot = lane64 / G, lane = lane64 % G;
    uint32_t *gk = s_k + (threadIdx.x & ~63) + slot * G;
    int32_t *gc = s_col + (threadIdx.x / G) * kExpandStage;
    const int nw = (int)gridDim.x * (kWG / kWave);
    const int w0 = (int)((blockIdx.x * kWG + threadIdx.x) >> 6);
    const MLS_G int32_t *scnt = gp(sc.scnt);
    const MLS_G u32x2 *scr = (const MLS_G u32x2 *)sc.scr;
    ProbCache pc;
    for (int base = w0 * kWave; base < b.na; base += nw * kWave) {
        const int gl = base + lane64;
        const int nl = gl < b.na ? scnt[gl] : 0;
        unsigned long long small = __ballot(nl > NLO && nl <= G);
        while (small) {
            // the next 64 / G rows of the chunk, one per group of G lanes
            int pick = -1;
#pragma unroll
            for (int j = 0; j < kWave / G; ++j) {
                const int r = small ? __ffsll((long long)small) - 1 : -1;
                if (small) small &= small - 1ull;
                if (j == slot) pick = r;
            }
            // every lane takes part in the shuffle: a source lane of a group without a row
            // must still provide its value
            int n = __shfl(nl, pick >= 0 ? pick : 0, kWave);
            if (pick < 0) n = 0;
            const int g = base + pick;
            u32x2 w;
            w.x = 0u; w.y = 0u;
            if (lane < n) w = scr[(int64_t)g * kScratchWords + lane];
            const uint32_t kb = w.x << 6;
            const uint32_t key = kb | (uint32_t)(lane < n ? __popc(w.y) : 0);
            gk[lane] = key;
            wave_sync();
            int off = 0, tot = 0;
#pragma unroll
            for (int f = 0; f < G; f += 4) {
                const uint4 q = *(const uint4 *)(gk + f);
                off += (q.x < kb ? (int)(q.x & 63u) : 0) + (q.y < kb ? (int)(q.y & 63u) : 0) +
                       (q.z < kb ? (int)(q.z & 63u) : 0) + (q.w < kb ? (int)(q.w & 63u) : 0);
                tot += (int)((q.x & 63u) + (q.y & 63u) + (q.z & 63u) + (q.w & 63u));
            }
            wave_sync();
            if (n > 0) {
                const int t = b.nprob == 1 ? 0 : find_prob_cached(b.abase, b.nprob, g, pc);
                // (per-lane read: this loop's LDS waits share the scalar
                // loads' counter, so a scalar descriptor read costs more here)
                const Prob P = get_prob(b, t);
                const int i = g - (b.nprob == 1 ? 0 : pc.lo);
                const int cs = gp(P.crp)[i] - P.c_off;
                const int ce = gp(P.crp)[i + 1] - P.c_off;
                MLS_G int32_t *__restrict__ cci = gpw(P.cci);
                if (tot <= kExpandStage && tot <= ce - cs) {
                    uint32_t m = lane < n ? w.y : 0u;
                    int pos = off;
                    while (m) {
                        gc[pos++] = (int32_t)(w.x * 32u + (uint32_t)(__ffs(m) - 1));
                        m &= m - 1u;
                    }
                    wave_sync();
                    for (int e = lane; e < tot; e += G) cci[cs + e] = gc[e];
                } else if (lane < n) {
                    uint32_t m = w.y;
                    int pos = cs + off;
                    while (m) {
                        const int bit = __ffs(m) - 1;
                        if (pos < ce) cci[pos] = (int32_t)(w.x * 32u + (uint32_t)bit);
                        else atomicOr(sc.err, kErrStructure);
                        ++pos;
                        m &= m - 1u;
                    }
                }
            }
            wave_sync();
        }
    }
}

void launch_sym_expand(const Batch &b, const Sched &sc, hipStream_t s)
{
    if (b.na <= 0 || !sc.scr) return;
    static int cus = device_cu_count();
    {
        // rows of 1-16 words take 16 lanes each (4 rows per step), rows of 17-32 words 32 lanes
        ProfScope ps("sym_expand_small", s);
        hipLaunchKernelGGL((k_sym_expand_small<kExpandSmall, 0>), dim3(cus * 8), dim3(kWG), 0, s, b, sc);
        hipLaunchKernelGGL((k_sym_expand_small<kExpandMid, kExpandSmall>), dim3(cus * 8), dim3(kWG), 0, s, b, sc);
    }
    ProfScope ps("sym_expand", s);
    hipLaunchKernelGGL(k_sym_expand, dim3(cus * 8), dim3(kWG), 0, s, b, sc);
}

// ---------------------------------------------------------------------------

template <typename K>
static int persistent_grid(K kernel, int threads)
{
    static int cus = device_cu_count();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

template <int G, int CAP, bool FILL>
static void launch_sym_class(const Batch &b, const Sched &sc, int bin, hipStream_t s)
{
    constexpr int W = kWave / G;
    constexpr int NW = nw_for(FILL ? CAP * 12 : CAP * 8, W);
    static char name[64];
    if (!name[0]) snprintf(name, sizeof(name), "sym_%s_lds_G%d_C%d", FILL ? "fill" : "count", G, CAP);
    ProfScope ps(name, s);
    if (b.nprob > 1) {
        static int grid = persistent_grid(k_sym_lds<G, CAP, FILL, true>, NW * kWave);
        hipLaunchKernelGGL((k_sym_lds<G, CAP, FILL, true>), dim3(grid), dim3(NW * kWave), 0, s, b, sc, bin);
    } else {
        static int grid = persistent_grid(k_sym_lds<G, CAP, FILL, false>, NW * kWave);
        hipLaunchKernelGGL((k_sym_lds<G, CAP, FILL, false>), dim3(grid), dim3(NW * kWave), 0, s, b, sc, bin);
    }
}

template <bool FILL>
static void launch_sym_all(const Batch &b, const Sched &sc, int G, hipStream_t s)
{
    constexpr int C0 = FILL ? kFillCap[0] : kCountCap[0];
    constexpr int C1 = FILL ? kFillCap[1] : kCountCap[1];
    constexpr int C2 = FILL ? kFillCap[2] : kCountCap[2];
    constexpr int C3 = FILL ? kFillCap[3] : kCountCap[3];
    constexpr int C4 = FILL ? kFillCap[4] : kCountCap[4];
    launch_sym_class<8, C0, FILL>(b, sc, 0, s);
    // the 256-slot count class runs with half the lanes per row (measured
    // faster on the 27-point stencil square, 1.88 -> 1.82 ms, and on the
    // Galerkin products)
    switch (!FILL && G >= 32 ? G / 2 : G) {
    case 8: launch_sym_class<8, C1, FILL>(b, sc, 1, s); break;
    case 16: launch_sym_class<16, C1, FILL>(b, sc, 1, s); break;
    case 64: launch_sym_class<64, C1, FILL>(b, sc, 1, s); break;
    default: launch_sym_class<32, C1, FILL>(b, sc, 1, s); break;
    }
    if (FILL) {   // fill tables are twice the row size: class 2 is already large
        if (G >= 64) launch_sym_class<64, C2, FILL>(b, sc, 2, s);
        else launch_sym_class<32, C2, FILL>(b, sc, 2, s);
    } else {
        switch (G) {
        case 8: launch_sym_class<8, C2, FILL>(b, sc, 2, s); break;
        case 16: launch_sym_class<16, C2, FILL>(b, sc, 2, s); break;
        case 64: launch_sym_class<64, C2, FILL>(b, sc, 2, s); break;
        default: launch_sym_class<32, C2, FILL>(b, sc, 2, s); break;
        }
    }
    if (G >= 64) launch_sym_class<64, C3, FILL>(b, sc, 3, s);
    else launch_sym_class<32, C3, FILL>(b, sc, 3, s);
    launch_sym_class<64, C4, FILL>(b, sc, 4, s);
}

void launch_symbolic(const Batch &b, const Sched &sc, int fill, int G, hipStream_t s)
{
    if (b.na <= 0) return;
    if (fill) launch_sym_all<true>(b, sc, G, s);
    else launch_sym_all<false>(b, sc, G, s);
    // bitmap window: every column of C when known and small, else the most the
    // workgroup's LDS holds next to the kernel's own arrays (at most 2^15 words)
    static int max_words = [] {
        int w = (device_max_lds() - 8192) / 4;
        return w < 4096 ? 4096 : (w > 32768 ? 32768 : w);
    }();
    int win = max_words;
    if (b.max_ncols > 0) {
        const int need = (b.max_ncols + 31) / 32;
        if (need < win) win = need < 64 ? 64 : need;
    }
    const int grid = spill_grid(k_sym_spill, win * 4);
    ProfScope ps(fill ? "sym_fill_spill" : "sym_count_spill", s);
    hipLaunchKernelGGL(k_sym_spill, dim3(grid), dim3(kWG), (size_t)win * 4, s, b, sc, fill, win);
}

int device_max_lds()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || n <= 0)
        return 65536;
    return n;
}

int device_cu_count()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

}  // namespace mls
