// k_numeric.hip -- numeric phase (Sec. 2.1, Fig. "spgemmexp") as the
// row-range fused multiply-add kernel of the chunking algorithms
// (Secs. 3.2.2 and 3.3.1): C_i += sum over k in row i of A, k in [k_lo, k_hi),
// of a_ik * B_k, optionally starting from the values already in C (the
// partial result of earlier row parts of B).
//
// LDS path: G lanes own a row of C. Its (sorted) columns are loaded once into
// an LDS hash mapping column -> position in the row, next to an LDS array of
// fp64 accumulators in row order. When C has few enough columns, a table slot
// packs column and position into one 32-bit word. The entries of row i of A are taken in
// stored order; for each, the G lanes take distinct entries of B_k, so no two
// lanes of a step touch the same accumulator and every c_ij receives its
// terms in ascending k -- the order of the row-wise formulation. Products are
// rounded before the add (compiled without contraction), so the result equals
// a sequential dense-accumulator evaluation bit for bit. The B loads of a
// batch of steps are all issued, without branches, before the first of them
// is used, to hide HBM/L2 latency.
//
// Spill path (rows with more outputs than the largest LDS class holds): the
// row's outputs are cut into windows of consecutive positions of C, each a
// task of its own with the LDS table and accumulators of one wave. A window
// streams the whole row of A, its rows of B narrowed to the window's column
// range (by binary search in B's sorted columns for long rows, by a range
// test for short ones), 64 (entry, B position) pairs per step; the adds of a
// step go in rounds so that every c_ij still gets its terms in ascending k.
#include <climits>
#include <cstdio>

#include "common.h"
#include "launch.h"
#include "postab.h"
#include "profile.h"

namespace mls {

constexpr int kNumDepth = 4;   // steps whose B loads are issued together (8 where LDS caps occupancy at 4)
constexpr int kNumWinCap = 1024;   // table slots of a spill window (CAP / 2 positions)
constexpr int kWinDepth = 2;       // spill window: batches of 64 pairs whose B loads are issued together
constexpr bool kNumFlat = true;    // flattened pairs for the classes of at most kNumFlatMaxG lanes per row
constexpr int kNumFlatMaxG = 8;

// all ones: read as a column it is -1 (no entry)
__device__ __attribute__((aligned(8))) int32_t k_num_void[2] = {-1, -1};

__device__ __forceinline__ void nwave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

constexpr int nw_num(int row_bytes, int rows_per_wave)
{
    int per_wave = row_bytes * rows_per_wave;
    int nw = 65536 / per_wave;
    return nw > 4 ? 4 : (nw < 1 ? 1 : nw);
}

// Hash a row's columns (column -> position) and set its accumulators (0, or
// the values already in C when accumulating). Each lane loads D of its
// columns (then values) before inserting them, so the loads overlap instead
// of each waiting on the previous insert (D = 2 for 32 or more lanes per
// row: few columns per lane, and few registers to spare at 8 waves per SIMD).
template <int G>
constexpr int ins_depth() { return G >= 32 ? 2 : 4; }

template <int G, typename TAB>
__device__ __forceinline__ void insert_row(TAB &tab, double *acc, int logcap,
                                           const MLS_G int32_t *__restrict__ cols,
                                           const MLS_G double *__restrict__ vals, int off, int n, int lane,
                                           bool accumulate)
{
    constexpr int kInsDepth = ins_depth<G>();
    if constexpr (kInsDepth == 1) {
        for (int e = lane; e < n; e += G) {
            tab.insert(logcap, cols[off + e], e);
            acc[e] = accumulate ? vals[off + e] : 0.0;
        }
        return;
    }
    for (int e0 = lane; e0 < n; e0 += G * kInsDepth) {
        int jv[kInsDepth];
#pragma unroll
        for (int u = 0; u < kInsDepth; ++u) {
            const int e = e0 + u * G;
            jv[u] = e < n ? cols[off + e] : -1;
        }
#pragma unroll
        for (int u = 0; u < kInsDepth; ++u)
            if (jv[u] >= 0) tab.insert(logcap, jv[u], e0 + u * G);
        if (accumulate) {
            double v[kInsDepth];
#pragma unroll
            for (int u = 0; u < kInsDepth; ++u) {
                const int e = e0 + u * G;
                v[u] = e < n ? vals[off + e] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kInsDepth; ++u) {
                const int e = e0 + u * G;
                if (e < n) acc[e] = v[u];
            }
        } else {
#pragma unroll
            for (int u = 0; u < kInsDepth; ++u) {
                const int e = e0 + u * G;
                if (e < n) acc[e] = 0.0;
            }
        }
    }
}

constexpr int num_row_bytes(int CAP, int G, bool PACK)
{
    return CAP * (PACK ? 4 : 8) + (CAP / 2) * 8 + G * 16;
}

// Where a row of the bin lives: product t, output size nc, the start of its
// C entries (cs) and its A entry range [ps, pe), all local (a slot without a
// row: nc = 0 and an empty range).
struct RowMeta {
    int t, nc, cs, ps, pe;
};

// The descriptor of product t: the kernel argument for a single product (its
// fields then live in scalar registers), else the batch's descriptor array.
template <bool MULTI>
__device__ __forceinline__ Prob prob_of(const Batch &b, int t)
{
    if (!MULTI) return b.p0;
    return get_prob_batch(b, t);
}

// Rows are software-pipelined across loop iterations, and every load of that
// pipeline is issued without a branch around it (a lane with nothing to load
// reads a constant word instead), so its first use can sit a row or more
// behind it: a use inside a branch would make the wave wait at the branch.

// A row's metadata as loaded: output size and row pointers before their
// offsets are subtracted (row_final), product t for a batch. A slot with no
// row reads zeros: no outputs and an empty range of A, so every step of the
// row loop is empty for it.
struct RowRaw {
    int t, nc, c0, a0, a1;
};

template <bool MULTI>
__device__ __forceinline__ RowRaw row_issue(const Batch &b, const Sched &sc, int g, ProbCache &pc)
{
    RowRaw r{0, 0, 0, 0, 0};
    const bool on = g >= 0;
    int i = g;
    if (MULTI && on) {
        r.t = find_prob_cached(b.abase, b.nprob, g, pc);
        i = g - pc.lo;
    }
    const Prob P = prob_of<MULTI>(b, r.t);
    const MLS_G int32_t *zero = (const MLS_G int32_t *)k_zeros4;
    const MLS_G int32_t *pv = on ? gp(sc.val) + g : zero;
    const MLS_G int32_t *pcr = on ? gp(P.crp) + i : zero;
    const MLS_G int32_t *par = on ? gp(P.arp) + i : zero;
    r.nc = *pv;
    r.c0 = *pcr;
    r.a0 = par[0];
    r.a1 = par[1];
    return r;
}

template <bool MULTI>
__device__ __forceinline__ RowMeta row_final(const Batch &b, const RowRaw &r)
{
    const Prob P = prob_of<MULTI>(b, r.t);
    RowMeta m;
    m.t = r.t;
    m.nc = r.nc;
    m.cs = r.c0 - P.c_off;
    m.ps = r.a0 - P.a_off;
    m.pe = r.a1 - P.a_off;
    return m;
}

// The first chunk of a row: entries ps + lane of row i of A (column -1 past
// the row) and the row pointers of B at their columns, as loaded (zeros for
// columns outside [k_lo, k_hi), which then give an empty range).
struct FirstChunk {
    int ka;
    double sa;
    int r0, r1;
};

__device__ __forceinline__ void first_a(const Prob &P, const RowMeta &m, int lane, FirstChunk &f)
{
    const bool on = m.ps + lane < m.pe;
    const MLS_G int32_t *pk = on ? gp(P.aci) + m.ps + lane : (const MLS_G int32_t *)k_num_void;
    const MLS_G double *pa = on ? gp(P.aval) + m.ps + lane : (const MLS_G double *)k_zeros4;
    f.ka = *pk;
    f.sa = *pa;
}

__device__ __forceinline__ void first_b(const Prob &P, FirstChunk &f)
{
    const bool in = f.ka >= P.k_lo && f.ka < P.k_hi;
    const MLS_G int32_t *pb = in ? gp(P.brp) + (f.ka - P.k_lo) : (const MLS_G int32_t *)k_zeros4;
    f.r0 = pb[0];
    f.r1 = pb[1];
}

// FLAT: the (entry, B position) pairs of a staged chunk are flattened, G at a
// time, one per lane (for rows of B shorter than G, which would leave lanes
// idle); the adds of a step go in rounds by the number of lower lanes with
// the same output position, so the terms still arrive in ascending k. The
// staged pair offsets follow the tables in LDS.
constexpr int num_flat_words(int G) { return G; }

// Waves per SIMD that the LDS of one workgroup (NW waves) leaves resident:
// 160 KB per CU, 4 SIMDs, at most 8 waves each.
constexpr int lds_waves_per_simd(int wg_bytes, int nw)
{
    int wgs = 163840 / wg_bytes;
    int w = wgs * nw / 4;
    return w > 8 ? 8 : (w < 1 ? 1 : w);
}

template <int G, int CAP, bool PACK, bool MULTI, bool FLAT>
struct NumShape {
    static constexpr int W = kWave / G;
    static constexpr int XW = FLAT ? num_flat_words(G) : 0;
    static constexpr int NW = nw_num(num_row_bytes(CAP, G, PACK) + 4 * XW, W);
    static constexpr int OCC = lds_waves_per_simd(NW * W * (num_row_bytes(CAP, G, PACK) + 4 * XW), NW);
    // where LDS already limits a SIMD to 4 waves, registers are free for
    // twice the steps in flight
    static constexpr int DEPTH = OCC <= 4 ? 2 * kNumDepth : kNumDepth;
    // waves per SIMD the kernel is compiled for: the LDS bound, capped so the
    // row pipeline's registers fit without spills (a reload from scratch
    // would wait for every load issued before it): 7 waves (72 VGPRs), 5
    // (96) for the flattened steps or for batches
    static constexpr int OCC_CAP = (FLAT || MULTI) ? 5 : 7;
    static constexpr int OCC_R = OCC < OCC_CAP ? OCC : OCC_CAP;
    // the next row's first chunk is prefetched where registers allow (at
    // most 5 waves per SIMD); otherwise a row loads its first chunk when it
    // starts
    static constexpr bool PF = !MULTI && OCC_R <= 5;
};

template <int G, int CAP, bool PACK, bool MULTI, bool FLAT>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(
    NumShape<G, CAP, PACK, MULTI, FLAT>::OCC_R))) void k_num_lds(Batch b, Sched sc, int bin)
{
    constexpr int kNumDepth = NumShape<G, CAP, PACK, MULTI, FLAT>::DEPTH;
    constexpr bool PF = NumShape<G, CAP, PACK, MULTI, FLAT>::PF;
    static_assert(FLAT || G % kNumDepth == 0, "the staged entries are read kNumDepth at a time");
    constexpr int W = kWave / G;
    constexpr int XW = FLAT ? num_flat_words(G) : 0;
    constexpr int NW = nw_num(num_row_bytes(CAP, G, PACK) + 4 * XW, W);
    constexpr int TW = PACK ? CAP : 2 * CAP;   // table words per row
    __shared__ __attribute__((aligned(16))) uint32_t s_tab[NW * W * (TW + XW)];
    __shared__ double s_acc[NW * W * (CAP / 2)];
    __shared__ int4 s_par[NW * W * G];   // staged entries of row i of A: (q0, q1, a)

    const int wave = threadIdx.x >> 6;
    if (wave >= NW) return;
    const int lw = threadIdx.x & 63;
    const int slot = lw / G, lane = lw % G;
    const int rs = wave * W + slot;
    // 2-slot buckets where 32 or more lanes own a row (measured on the
    // 27-point stencil square), 4-slot ones for narrower groups
    PosTab<CAP, PACK, (G >= 32 ? 2 : 4)> tab{s_tab + rs * TW};
    double *acc = s_acc + rs * (CAP / 2);
    int4 *par = s_par + rs * G;
    int *poff = (int *)(s_tab + NW * W * TW) + rs * XW;   // FLAT only: staged pair offsets

    const int n_bin = gp(sc.bin_count)[bin];
    const int start = bin_start(sc.bin_count, bin);
    const int ntasks = (n_bin + W - 1) / W;
    TaskIter it = task_iter(ntasks, NW);
    // Rows of a slot overlap: with PF three are in flight (the row after next
    // has its perm entry loading; the next row its metadata, then its first
    // chunk: A entries during this row's insert and steps, B row pointers
    // after them), so a row starts with all of its dependent index loads
    // done. Without PF (fewer registers), the next row's perm entry loads
    // from the start of a row and its metadata from the middle.
    int task = next_task_wave(sc.task_cursor + bin * kXcd, ntasks, it);
    const bool h_cur = task >= 0 && task * W + slot < n_bin;
    const int g_raw = bin_row_issue(sc.perm, sc.err, b.na, start + task * W + slot, h_cur);
    int task_n = -1, g_n = -1;
    bool h_n = false;
    if constexpr (PF) {
        task_n = task >= 0 ? next_task_wave(sc.task_cursor + bin * kXcd, ntasks, it) : -1;
        h_n = task_n >= 0 && task_n * W + slot < n_bin;
        g_n = bin_row_issue(sc.perm, sc.err, b.na, start + task_n * W + slot, h_n);
    }
    ProbCache pc;
    RowRaw mr = row_issue<MULTI>(b, sc, bin_row_checked(sc.err, b.na, g_raw, h_cur), pc);
    FirstChunk f;
    if constexpr (PF) {
        const RowMeta m0 = row_final<MULTI>(b, mr);
        const Prob P0 = prob_of<MULTI>(b, m0.t);
        first_a(P0, m0, lane, f);
        first_b(P0, f);
        asm volatile("" ::"v"(f.ka), "v"(f.sa), "v"(f.r0), "v"(f.r1), "v"(g_n));
    }
    // the loop starts with no load of the prologue pending: the wait counts
    // at the top of the loop are computed over both ways into it, and a load
    // pending from the prologue would make the first use there also wait
    // for the loads the previous row issued last
    asm volatile("" ::"v"(mr.nc), "v"(mr.c0), "v"(mr.a0), "v"(mr.a1));
    while (task >= 0) {
        // PF: the row after next; else the next row
        const int task_x = (!PF || task_n >= 0) ? next_task_wave(sc.task_cursor + bin * kXcd, ntasks, it) : -1;
        const bool h_x = task_x >= 0 && task_x * W + slot < n_bin;
        const int g_x = bin_row_issue(sc.perm, sc.err, b.na, start + task_x * W + slot, h_x);
        RowRaw mr_n;
        if constexpr (PF) mr_n = row_issue<MULTI>(b, sc, bin_row_checked(sc.err, b.na, g_n, h_n), pc);

        const RowMeta m = row_final<MULTI>(b, mr);
        const Prob P = prob_of<MULTI>(b, m.t);
        const int nc = m.nc;
        int logcap = ilog2_ceil(2 * nc);
        if (logcap < 5) logcap = 5;
        const int cap = 1 << logcap;
        tab.clear(cap, lane, G);
        // descriptor fields into registers once per row, as global pointers
        const MLS_G int32_t *__restrict__ aci = gp(P.aci);
        const MLS_G double *__restrict__ aval = gp(P.aval);
        const MLS_G int32_t *__restrict__ brp = gp(P.brp);
        const MLS_G int32_t *__restrict__ bci = gp(P.bci);
        const MLS_G double *__restrict__ bval = gp(P.bval);
        const MLS_G int32_t *__restrict__ cci = gp(P.cci);
        MLS_G double *__restrict__ cval = gpw(P.cval);
        const int b_off = P.b_off, k_lo = P.k_lo, k_hi = P.k_hi;
        const bool accumulate = P.accumulate != 0;
        const int cs = m.cs, ps = m.ps, pe = m.pe;
        // the first chunk of row i of A: loaded during the previous row (PF),
        // else its entries now and its B row pointers after the insert
        if constexpr (!PF) first_a(P, m, lane, f);
        // a step over a part of B's rows skips the rows (of one chunk) with no
        // entry in it: most rows of A reach only a few parts
        bool skip = false;
        if (P.ranged) {
            // (the empty asm keeps the test, and the wait for the entries,
            // inside this branch)
            int kk = f.ka;
            asm volatile("" : "+v"(kk));
            const unsigned long long bal = __ballot(kk >= k_lo && kk < k_hi);
            const unsigned long long gm = (G == 64 ? ~0ull : ((1ull << G) - 1ull)) << (slot * G);
            skip = pe - ps <= G && (bal & gm) == 0ull;
        }
        nwave_sync();
        if (!skip) insert_row<G>(tab, acc, logcap, cci, cval, cs, nc, lane, accumulate);
        nwave_sync();
        if constexpr (!PF) {
            mr_n = row_issue<MULTI>(b, sc, bin_row_checked(sc.err, b.na, g_x, h_x), pc);
            first_b(P, f);
        }
        int ka = f.ka;
        double sa = f.sa;
        bool bad = false;
        const int pe_w = skip ? ps : pe;
        // stage a chunk: (q0, q1, a) of its entry pc + lane, from the B row
        // pointers as loaded; FLAT: the group's pair offsets and pair count
        auto stage = [&](int q0r, int q1r, double a) -> int {
            const int sq0 = q0r - b_off, sq1 = q1r - b_off;
            par[lane] = make_int4(sq0, sq1, __double2loint(a), __double2hiint(a));
            int tot = 0;
            if constexpr (FLAT) {
                const int np = sq1 > sq0 ? sq1 - sq0 : 0;
                const int incl = group_scan_incl<G>(np, lane);
                tot = group_total<G>(np, incl);
                poff[lane] = incl - np;
            }
            return tot;
        };
        // the first chunk is staged here from what was loaded during the
        // previous row (unused when the row has no chunk), the later ones in
        // the chunk loop: no loaded value reaches a point where the two ways
        // join, where its wait would also cover the loads issued since
        int total = stage(f.r0, f.r1, f.sa);
        // PF: the next row's first A entries load during this row's steps
        RowMeta mn{};
        Prob Pn{};
        if constexpr (PF) {
            mn = row_final<MULTI>(b, mr_n);
            Pn = prob_of<MULTI>(b, mn.t);
            first_a(Pn, mn, lane, f);
        }
        for (int pc = ps; pc < pe_w; pc += G) {
            if (pc != ps) {
                // a later chunk: the B row pointers of the entries of A loaded
                // during the previous chunk
                const bool in = ka >= k_lo && ka < k_hi;
                const MLS_G int32_t *pb = in ? brp + (ka - k_lo) : (const MLS_G int32_t *)k_zeros4;
                total = stage(pb[0], pb[1], sa);
            }
            nwave_sync();
            // the next chunk's entries of A are in flight during this chunk's
            // steps (loaded without a branch: a default written into their
            // registers before a conditional load would wait for the loads of
            // the previous chunk, and with them for everything issued since)
            {
                const bool on = pc + G + lane < pe;
                ka = *(on ? aci + pc + G + lane : (const MLS_G int32_t *)k_ones4);
                sa = *(on ? aval + pc + G + lane : (const MLS_G double *)k_zeros4);
            }
            const int n = FLAT ? 0 : min(G, pe - pc);
            if constexpr (FLAT) {
                // the group's pair offsets in registers: a pair's entry is the
                // last one whose offset is at most the pair's index
                static_assert(G % 4 == 0 && G <= 16, "offsets read four at a time");
                int pofv[G];
#pragma unroll
                for (int x = 0; x < G; x += 4) {
                    const int4 v = *(const int4 *)(poff + x);
                    pofv[x] = v.x; pofv[x + 1] = v.y; pofv[x + 2] = v.z; pofv[x + 3] = v.w;
                }
                for (int base = 0; base < total; base += G * kNumDepth) {
                    int jv[kNumDepth];
                    double av[kNumDepth], bv[kNumDepth];
                    // loads without branches (pairs past the chunk read the
                    // all-ones dummy: column -1), all issued before any use
#pragma unroll
                    for (int d = 0; d < kNumDepth; ++d) {
                        const int pp = base + d * G + lane;
                        int lo = -1, po = 0;
#pragma unroll
                        for (int x = 0; x < G; ++x) {
                            const bool le = pofv[x] <= pp;
                            lo += le ? 1 : 0;
                            po = le ? pofv[x] : po;
                        }
                        const int4 pr = par[lo];
                        const int q = pr.x + (pp - po);
                        const bool ok = pp < total;
                        const MLS_G int32_t *pj = ok ? bci + q : (const MLS_G int32_t *)k_num_void;
                        const MLS_G double *pv = ok ? bval + q : (const MLS_G double *)k_num_void;
                        jv[d] = *pj;
                        bv[d] = *pv;
                        av[d] = __hiloint2double(pr.w, pr.z);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    int posv[kNumDepth];
                    tab.template lookup_n<kNumDepth>(logcap, jv, posv);
#pragma unroll
                    for (int d = 0; d < kNumDepth; ++d) asm volatile("" ::"v"(bv[d]));
#pragma unroll
                    for (int d = 0; d < kNumDepth; ++d)
                        if (posv[d] == -1) bad = true;
                    // lanes of a step holding the same output add in lane (= term)
                    // order: a lane's round is the number of lower lanes of its
                    // group with the same position, and one wave's LDS adds take
                    // effect in program order
#pragma unroll
                    for (int d = 0; d < kNumDepth; ++d) {
                        const int rank = group_rank<G>(posv[d], lane);
                        const int rk = posv[d] >= 0 ? rank : -1;
                        const double t = av[d] * bv[d];
                        for (int rr = 0;; ++rr) {
                            if (rk == rr) atomicAdd(acc + posv[d], t);
                            if (!__ballot(rk > rr)) break;
                        }
                    }
                }
            }
            for (int u0 = 0; u0 < n; u0 += kNumDepth) {
                // issue the B loads of kNumDepth steps, then accumulate them in order.
                // The staged entries are read together (all G are written every
                // chunk, those past the row as empty ranges, and G is a multiple of
                // kNumDepth).
                int2 qr[kNumDepth];
#pragma unroll
                for (int d = 0; d < kNumDepth; ++d) qr[d] = *(const int2 *)(par + u0 + d);
                bool longs = false;   // a step whose row of B is longer than G
#pragma unroll
                for (int d = 0; d < kNumDepth; ++d) longs |= qr[d].y - qr[d].x > G;
                if (__ballot(longs)) {
                    // one step at a time, each through all of its row of B: its
                    // entries have distinct columns, so the order is kept
#pragma unroll 1
                    for (int d = 0; d < kNumDepth; ++d) {
                        const int4 pr = par[u0 + d];
                        const double a = __hiloint2double(pr.w, pr.z);
                        for (int q = pr.x + lane; q < pr.y; q += G) {
                            const int pos = tab.lookup(logcap, bci[q]);
                            if (pos >= 0) atomicAdd(acc + pos, a * bval[q]);
                            else bad = true;
                        }
                    }
                    continue;
                }
                int jv[kNumDepth];
                double bv[kNumDepth], av[kNumDepth];
                // lanes past their row of B load the all-ones dummy instead
                // (column -1: no lookup, no add), so no branch surrounds the loads
#pragma unroll
                for (int d = 0; d < kNumDepth; ++d) {
                    const int q = qr[d].x + lane;
                    const bool ok = q < qr[d].y;
                    const MLS_G int32_t *pj = ok ? bci + q : (const MLS_G int32_t *)k_num_void;
                    const MLS_G double *pv = ok ? bval + q : (const MLS_G double *)k_num_void;
                    jv[d] = *pj;
                    bv[d] = *pv;
                }
                // keep the scheduler from hoisting uses of the loaded columns
                // above the later loads (each would wait for a load)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int d = 0; d < kNumDepth; ++d) av[d] = *((const double *)(par + u0 + d) + 1);
                // positions first (independent LDS reads), then the adds in step
                // order; within a step the lanes hold distinct columns of B_k, so
                // no two lanes add to the same slot and every slot gets its terms
                // in ascending k. The LDS fp64 add rounds like a plain add.
                int posv[kNumDepth];
                tab.template lookup_n<kNumDepth>(logcap, jv, posv);
                // every loaded value is consumed on every path (an empty asm
                // use), so no load is left pending into the next batch
#pragma unroll
                for (int d = 0; d < kNumDepth; ++d) asm volatile("" ::"v"(bv[d]));
#pragma unroll
                for (int d = 0; d < kNumDepth; ++d) {
                    if (posv[d] >= 0) atomicAdd(acc + posv[d], av[d] * bv[d]);
                    else if (posv[d] == -1) bad = true;
                }
            }
            nwave_sync();
        }
        // the next row's metadata is taken before this row's stores are
        // issued (a wait for it at the next row's start would also wait for
        // the stores: the counter covers both)
        asm volatile("" ::"v"(mr_n.nc), "v"(mr_n.c0), "v"(mr_n.a0), "v"(mr_n.a1));
        // PF: the next row's B row pointers (its A entries arrived during the steps)
        if constexpr (PF) first_b(Pn, f);
        if (bad) atomicOr(sc.err, kErrStructure);
        if (!skip)
            for (int e = lane; e < nc; e += G) cval[cs + e] = acc[e];
        else if (!accumulate)
            for (int e = lane; e < nc; e += G) cval[cs + e] = 0.0;
        nwave_sync();
        if constexpr (PF) {
            task = task_n;
            task_n = task_x;
            g_n = g_x;
            h_n = h_x;
        } else {
            task = task_x;
        }
        mr = mr_n;
    }
}

// first position in cols[lo, hi) whose column is >= j
__device__ __forceinline__ int lower_col(const MLS_G int32_t *cols, int lo, int hi, int j)
{
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cols[mid] < j) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Windows of the spill rows: wstart[r] = first window of the r-th row of the
// spill bin (ceil(nc / m) windows per row), wstart[n] = the total. One
// workgroup.
__global__ __launch_bounds__(kWG) void k_win_scan(Batch b, Sched sc, int m)
{
    __shared__ int s_red[kWG / kWave];
    __shared__ int s_carry;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = gp(sc.bin_count)[kBinSpill];
    const int start = bin_start(sc.bin_count, kBinSpill);
    MLS_G int32_t *ws = gpw(sc.wstart);
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int r0 = 0; r0 < n; r0 += kWG) {
        const int r = r0 + (int)threadIdx.x;
        int c = 0;
        if (r < n) {
            const int g = bin_row(sc.perm, sc.err, b.na, start + r);
            if (g >= 0) c = (gp(sc.val)[g] + m - 1) / m;
        }
        int incl = c;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += y;
        }
        if (lane == kWave - 1) s_red[wave] = incl;
        __syncthreads();
        int before = s_carry, all = 0;
#pragma unroll
        for (int x = 0; x < kWG / kWave; ++x) {
            before += x < wave ? s_red[x] : 0;
            all += s_red[x];
        }
        if (r < n) ws[r] = before + incl - c;
        __syncthreads();
        if (threadIdx.x == 0) s_carry += all;
        __syncthreads();
    }
    if (threadIdx.x == 0) ws[n] = s_carry;
}

constexpr int kWinBlock = 2;   // consecutive windows a wave takes per counter grab

// LDS of one spill window: table, accumulators, staged entries, their first
// pair and the per-position lane marks of the ordered adds
constexpr int win_bytes(int CAP, bool PACK)
{
    return CAP * (PACK ? 4 : 8) + (CAP / 2) * 8 + kWave * 16 + (kWave + 1) * 4 + (CAP / 2) * 4;
}

// A window's terms are flattened: the (entry, B position) pairs of a staged
// chunk of A's row, entry-major (so in ascending k), are taken 64 at a time,
// one per lane, with coalesced loads of B. Two lanes of a batch may hit the
// same output, so the adds are applied in rounds: in each round the lowest
// pending lane of every output position adds (an LDS min over lane ids
// finds it), which keeps every c_ij's terms in ascending k.
template <int CAP, bool PACK, bool MULTI>
__global__ __launch_bounds__(kWG) void k_num_win(Batch b, Sched sc)
{
    constexpr int G = kWave;
    constexpr int M = CAP / 2;   // positions of C per window
    constexpr int NW = nw_num(win_bytes(CAP, PACK), 1);
    constexpr int TW = PACK ? CAP : 2 * CAP;
    __shared__ __attribute__((aligned(16))) uint32_t s_tab[NW * TW];
    __shared__ double s_acc[NW * M];
    __shared__ int4 s_par[NW * G];        // staged entries: (first B position, -, a)
    __shared__ int s_poff[NW * (G + 1)];  // first pair of each staged entry, then the total
    __shared__ int s_own[NW * M];

    const int wave = threadIdx.x >> 6;
    if (wave >= NW) return;
    const int lane = threadIdx.x & 63;
    PosTab<CAP, PACK, 2> tab{s_tab + wave * TW};
    double *acc = s_acc + wave * M;
    int4 *par = s_par + wave * G;
    int *poff = s_poff + wave * (G + 1);
    int *own = s_own + wave * M;

    const int n_bin = gp(sc.bin_count)[kBinSpill];
    const int start = bin_start(sc.bin_count, kBinSpill);
    const MLS_G int32_t *wst = gp(sc.wstart);
    const int nwin = n_bin > 0 ? wst[n_bin] : 0;
    // one counter over all windows: their work varies too much (a hub row's
    // windows are consecutive and long) for per-XCD slabs
    if (nwin == 0) return;
    int32_t *cursor = sc.task_cursor + kBinSpill * kXcd;
    ProbCache pcache;
    for (;;) {
        int u0 = 0;
        if (lane == 0) u0 = atomicAdd(cursor, 1) * kWinBlock;
        u0 = __builtin_amdgcn_readlane(u0, 0);
        if (u0 >= nwin) break;
        int r = 0;   // largest r with wst[r] <= u0: the row holding window u0
        {
            int hi = n_bin - 1;
            while (r < hi) {
                const int mid = (r + hi + 1) >> 1;
                if (wst[mid] <= u0) r = mid; else hi = mid - 1;
            }
        }
        const int u1 = min(u0 + kWinBlock, nwin);
        for (int u = u0; u < u1; ++u) {
            while (wst[r + 1] <= u) ++r;
            const int g = bin_row(sc.perm, sc.err, b.na, start + r);
            if (g < 0) continue;
            int t = 0, i = g;
            if (MULTI) {
                t = find_prob_cached(b.abase, b.nprob, g, pcache);
                i = g - pcache.lo;
            }
            const Prob P = prob_of<MULTI>(b, t);
            const MLS_G int32_t *__restrict__ aci = gp(P.aci);
            const MLS_G double *__restrict__ aval = gp(P.aval);
            const MLS_G int32_t *__restrict__ brp = gp(P.brp);
            const MLS_G int32_t *__restrict__ bci = gp(P.bci);
            const MLS_G double *__restrict__ bval = gp(P.bval);
            const MLS_G int32_t *__restrict__ cci = gp(P.cci);
            MLS_G double *__restrict__ cval = gpw(P.cval);
            const int b_off = P.b_off, k_lo = P.k_lo, k_hi = P.k_hi;
            const bool accumulate = P.accumulate != 0;
            const int nc = gp(sc.val)[g];
            const int c0 = (u - wst[r]) * M;   // first position of the window in the row
            const int cs = gp(P.crp)[i] - P.c_off + c0;
            const int n = min(M, nc - c0);
            const int ps = gp(P.arp)[i] - P.a_off, pe = gp(P.arp)[i + 1] - P.a_off;
            const bool narrow = nc > M;
            // columns the window takes: from its first to its last column, open
            // below for the row's first window and above for its last, so that
            // a column outside the whole row still fails the lookup
            const int jlo = c0 == 0 ? INT_MIN : cci[cs];
            const int jhi = c0 + n == nc ? INT_MAX : cci[cs + n - 1];
            int logcap = ilog2_ceil(2 * n);
            if (logcap < 5) logcap = 5;
            tab.clear(1 << logcap, lane, G);
            nwave_sync();
            insert_row<G>(tab, acc, logcap, cci, cval, cs, n, lane, accumulate);
            nwave_sync();
            bool bad = false;
            for (int pc = ps; pc < pe; pc += G) {
                // stage the chunk: entry pc + lane's row of B, narrowed to the
                // window's columns when it is long, and its pair count
                int sq0 = 0, sq1 = 0;
                double sa = 0.0;
                if (pc + lane < pe) {
                    const int ka = aci[pc + lane];
                    sa = aval[pc + lane];
                    if (ka >= k_lo && ka < k_hi) {
                        sq0 = brp[ka - k_lo] - b_off;
                        sq1 = brp[ka - k_lo + 1] - b_off;
                        if (narrow && sq1 - sq0 > 32) {
                            if (jlo != INT_MIN) sq0 = lower_col(bci, sq0, sq1, jlo);
                            if (jhi != INT_MAX) sq1 = lower_col(bci, sq0, sq1, jhi + 1);
                        }
                    }
                }
                const int np = sq1 > sq0 ? sq1 - sq0 : 0;
                int incl = group_scan_incl<G>(np, lane);
                const int total = group_total<G>(np, incl);
                poff[lane] = incl - np;
                if (lane == 0) poff[G] = total;
                par[lane] = make_int4(sq0, 0, __double2loint(sa), __double2hiint(sa));
                nwave_sync();
                for (int base = 0; base < total; base += G * kWinDepth) {
                    // kWinDepth batches of 64 pairs: loads first, then lookups,
                    // then the ordered adds batch by batch
                    int jv[kWinDepth];
                    double tv[kWinDepth];
#pragma unroll
                    for (int d = 0; d < kWinDepth; ++d) {
                        jv[d] = -1;
                        tv[d] = 0.0;
                        const int pp = base + d * G + lane;
                        if (pp < total) {
                            int lo = 0, hi = G - 1;   // largest e with poff[e] <= pp
                            while (lo < hi) {
                                const int mid = (lo + hi + 1) >> 1;
                                if (poff[mid] <= pp) lo = mid; else hi = mid - 1;
                            }
                            const int4 pr = par[lo];
                            const int q = pr.x + (pp - poff[lo]);
                            jv[d] = bci[q];
                            tv[d] = __hiloint2double(pr.w, pr.z) * bval[q];
                        }
                    }
                    int jw[kWinDepth], posv[kWinDepth];
#pragma unroll
                    for (int d = 0; d < kWinDepth; ++d) jw[d] = (jv[d] >= jlo && jv[d] <= jhi) ? jv[d] : -1;
                    tab.template lookup_n<kWinDepth>(logcap, jw, posv);
#pragma unroll
                    for (int d = 0; d < kWinDepth; ++d)
                        if (posv[d] == -1) bad = true;
#pragma unroll
                    for (int d = 0; d < kWinDepth; ++d) {
                        bool pend = posv[d] >= 0;
                        while (__ballot(pend)) {
                            if (pend) own[posv[d]] = G;
                            nwave_sync();
                            if (pend) atomicMin(own + posv[d], lane);
                            nwave_sync();
                            if (pend && own[posv[d]] == lane) {
                                atomicAdd(acc + posv[d], tv[d]);
                                pend = false;
                            }
                            nwave_sync();
                        }
                    }
                }
                nwave_sync();
            }
            if (bad) atomicOr(sc.err, kErrStructure);
            for (int e = lane; e < n; e += G) cval[cs + e] = acc[e];
            nwave_sync();
        }
    }
}

// ---------------------------------------------------------------------------

template <typename K>
static int persistent_grid_n(K kernel, int threads)
{
    static int cus = device_cu_count();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

template <int G, int CAP, bool PACK, bool MULTI, bool FLAT>
static void launch_num_variant(const Batch &b, const Sched &sc, int bin, hipStream_t s)
{
    constexpr int W = kWave / G;
    constexpr int XW = FLAT ? num_flat_words(G) : 0;
    constexpr int NW = nw_num(num_row_bytes(CAP, G, PACK) + 4 * XW, W);
    static int grid = persistent_grid_n(k_num_lds<G, CAP, PACK, MULTI, FLAT>, NW * kWave);
    static char name[64];
    if (!name[0])
        snprintf(name, sizeof(name), "num_lds_G%d_C%d%s%s%s", G, CAP, PACK ? "_p" : "", MULTI ? "_b" : "", FLAT ? "_f" : "");
    ProfScope ps(name, s);
    hipLaunchKernelGGL((k_num_lds<G, CAP, PACK, MULTI, FLAT>), dim3(grid), dim3(NW * kWave), 0, s, b, sc, bin);
}

template <int G, int CAP, bool PACK>
static void launch_num_multi(const Batch &b, const Sched &sc, int bin, hipStream_t s)
{
    constexpr bool FLAT = kNumFlat && G <= kNumFlatMaxG;
    if (b.nprob > 1) launch_num_variant<G, CAP, PACK, true, FLAT>(b, sc, bin, s);
    else launch_num_variant<G, CAP, PACK, false, FLAT>(b, sc, bin, s);
}

// The packed table needs every column index below PackBits<CAP>::kMaxCols.
template <int G, int CAP>
static void launch_num_class(const Batch &b, const Sched &sc, int bin, hipStream_t s)
{
    if (b.max_ncols > 0 && (uint32_t)b.max_ncols <= PackBits<CAP>::kMaxCols)
        launch_num_multi<G, CAP, true>(b, sc, bin, s);
    else
        launch_num_multi<G, CAP, false>(b, sc, bin, s);
}

template <int CAP, bool PACK, bool MULTI>
static void launch_num_win(const Batch &b, const Sched &sc, hipStream_t s)
{
    constexpr int NW = nw_num(win_bytes(CAP, PACK), 1);
    static int grid = persistent_grid_n(k_num_win<CAP, PACK, MULTI>, NW * kWave);
    static char name[64];
    if (!name[0]) snprintf(name, sizeof(name), "num_spill_C%d%s%s", CAP, PACK ? "_p" : "", MULTI ? "_b" : "");
    ProfScope ps(name, s);
    hipLaunchKernelGGL(k_win_scan, dim3(1), dim3(kWG), 0, s, b, sc, CAP / 2);
    hipLaunchKernelGGL((k_num_win<CAP, PACK, MULTI>), dim3(grid), dim3(NW * kWave), 0, s, b, sc);
}

static void launch_num_spill(const Batch &b, const Sched &sc, hipStream_t s)
{
    constexpr int CAP = kNumWinCap;
    const bool pack = b.max_ncols > 0 && (uint32_t)b.max_ncols <= PackBits<CAP>::kMaxCols;
    if (b.nprob > 1) {
        if (pack) launch_num_win<CAP, true, true>(b, sc, s);
        else launch_num_win<CAP, false, true>(b, sc, s);
    } else {
        if (pack) launch_num_win<CAP, true, false>(b, sc, s);
        else launch_num_win<CAP, false, false>(b, sc, s);
    }
}

void launch_numeric_groups(const Batch &b, const Sched &sc, int G1, int G2, hipStream_t s)
{
    if (b.na <= 0) return;
    launch_num_class<8, kFillCap[0]>(b, sc, 0, s);
    switch (G1) {
    case 8: launch_num_class<8, kFillCap[1]>(b, sc, 1, s); break;
    case 16: launch_num_class<16, kFillCap[1]>(b, sc, 1, s); break;
    case 64: launch_num_class<64, kFillCap[1]>(b, sc, 1, s); break;
    default: launch_num_class<32, kFillCap[1]>(b, sc, 1, s); break;
    }
    if (G2 >= 64) launch_num_class<64, kFillCap[2]>(b, sc, 2, s);
    else launch_num_class<32, kFillCap[2]>(b, sc, 2, s);
    launch_num_class<64, kFillCap[3]>(b, sc, 3, s);
    launch_num_class<64, kFillCap[4]>(b, sc, 4, s);
    launch_num_spill(b, sc, s);
}

void launch_numeric(const Batch &b, const Sched &sc, int G, hipStream_t s)
{
    launch_numeric_groups(b, sc, G, G >= 64 ? 64 : 32, s);
}

}  // namespace mls
