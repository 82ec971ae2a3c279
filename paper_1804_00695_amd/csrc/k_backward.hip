// k_backward.hip -- adjoint of loss(A, B) = sum_ij W_ij (A*B)_ij with W given
// on the pattern of C = A*B (the product's reverse mode; not in the paper):
//   dA_ik = sum_{j in B_k} W_ij b_kj      (only on the pattern of A)
//   dB_kj = sum_{i : k in A_i} a_ik W_ij  (only on the pattern of B)
// Fused, with no dense or product-sized intermediate: G lanes own row i;
// W_i goes into an LDS hash (column -> W value); the pairs (entry (i, k),
// entry of B_k) of a chunk of A_i are flattened, one per lane: each looks up
// W_ij, adds W_ij b_kj to the entry's dA sum in LDS and a_ik W_ij into dB
// with a device fp64 atomic.
// Rows of W too long for LDS are cut into windows of consecutive positions of
// W_i, each a task of one wave with its own LDS hash; a window streams the
// row of A with its rows of B narrowed to the window's column range, and adds
// its part of dA_ik with a device atomic.
//
// Also here: CSR transpose (count, scan, scatter, per-row sort) and a masked
// gather out[e] = X(row(e), col(e)) over a pattern, used by the unfused
// per-call adjoint (W B^T masked to pat(A), A^T W masked to pat(B)).
#include <climits>
#include <cstdio>

#include "common.h"
#include "launch.h"
#include "postab.h"
#include "profile.h"

namespace mls {

constexpr int kBwdUnroll = 4;

// all ones: read as a column it is -1 (no entry)
__device__ __attribute__((aligned(8))) int32_t k_bwd_void[2] = {-1, -1};

__device__ __forceinline__ void bwd_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

constexpr int nw_bwd(int row_bytes, int rows_per_wave)
{
    int per_wave = row_bytes * rows_per_wave;
    int nw = 65536 / per_wave;
    return nw > 4 ? 4 : (nw < 1 ? 1 : nw);
}

// W_i's hash: column keys (-1 empty) in buckets of 4 slots (16 bytes), W
// values beside them. A column takes the first empty slot at or after the
// start of its home bucket, so a bucket's filled slots are a prefix of it and
// a bucket whose last slot is empty ends a search.
__device__ __forceinline__ uint32_t w_home(int logcap, int j) { return hslot((uint32_t)j, logcap - 2) << 2; }

__device__ __forceinline__ void w_insert(int *key, double *wv, int logcap, int j, double w)
{
    const uint32_t cmask = (1u << logcap) - 1u;
    uint32_t h = w_home(logcap, j);
    for (uint32_t probe = 0; probe <= cmask; probe += 4) {
        const int4 k = *(const int4 *)(key + h);
        int sl = k.x == -1 ? 0 : (k.y == -1 ? 1 : (k.z == -1 ? 2 : (k.w == -1 ? 3 : 4)));
        for (; sl < 4; ++sl)
            if (atomicCAS(key + h + sl, -1, j) == -1) { wv[h + sl] = w; return; }
        h = (h + 4u) & cmask;
    }
}

// slot of column j given the keys k of its home bucket h, or -1 when absent
__device__ __forceinline__ int w_slot(const int *key, int logcap, int j, uint32_t h, int4 k)
{
    const int sl = k.x == j ? 0 : (k.y == j ? 1 : (k.z == j ? 2 : (k.w == j ? 3 : -1)));
    if (sl >= 0) return (int)h + sl;
    if (k.w == -1) return -1;
    const uint32_t cmask = (1u << logcap) - 1u;
    for (uint32_t probe = 4; probe <= cmask; probe += 4) {   // the home bucket is full: rarely
        h = (h + 4u) & cmask;
        const int4 v = *(const int4 *)(key + h);
        const int s2 = v.x == j ? 0 : (v.y == j ? 1 : (v.z == j ? 2 : (v.w == j ? 3 : -1)));
        if (s2 >= 0) return (int)h + s2;
        if (v.w == -1) return -1;
    }
    return -1;
}

// slots of D columns (-2 where jv < 0), the home buckets of a pair read
// before either is searched, then the W values of all D read together
template <int D>
__device__ __forceinline__ void w_lookup_n(const int *key, const double *wv, int logcap, const int (&jv)[D],
                                           int (&sl)[D], double (&w)[D])
{
    static_assert(D % 2 == 0, "looked up in pairs");
#pragma unroll
    for (int d0 = 0; d0 < D; d0 += 2) {
        uint32_t hv[2];
        int4 kv[2];
#pragma unroll
        for (int d = 0; d < 2; ++d) hv[d] = jv[d0 + d] >= 0 ? w_home(logcap, jv[d0 + d]) : 0u;
#pragma unroll
        for (int d = 0; d < 2; ++d) kv[d] = *(const int4 *)(key + hv[d]);
#pragma unroll
        for (int d = 0; d < 2; ++d) sl[d0 + d] = jv[d0 + d] >= 0 ? w_slot(key, logcap, jv[d0 + d], hv[d], kv[d]) : -2;
    }
#pragma unroll
    for (int d = 0; d < D; ++d) w[d] = wv[sl[d] >= 0 ? sl[d] : 0];
}

// LDS of one row: W_i's hash (wide: key and value per slot; packed: a
// column -> position table and the values by position), the staged entries
// of A (first B position, a_ik, their dA sums) and the staged entries' first
// pairs
constexpr int bwd_row_bytes(int CAP, int G, bool PACK)
{
    return (PACK ? CAP * 4 + (CAP / 2) * 8 : CAP * 12) + G * 20 + (G + 4) * 4;
}

// Waves per workgroup that keep the most waves resident on a CU (160 KB of
// LDS, 32 waves), given the LDS of one wave.
constexpr int nw_bwd_best(int wave_bytes)
{
    int best = 1, best_w = 0;
    for (int nw = 1; nw <= 4; ++nw) {
        int wgs = 163840 / (nw * wave_bytes);
        int w = wgs * nw;
        if (w > 32) w = 32;
        if (65536 < nw * wave_bytes) w = 0;   // a workgroup's static LDS stays within 64 KB
        if (w >= best_w) { best = nw; best_w = w; }
    }
    return best;
}

// Rows of W in LDS: G lanes own row i. The pairs (entry of A_i, position in
// B_k) of a staged chunk of A_i are flattened and taken G at a time, one per
// lane: W_ij is looked up, a_ik W_ij goes to dB with a device atomic and
// W_ij b_kj to the entry's dA sum in LDS, written out once per entry.
// Latency: a row's metadata (size, row pointers of W and A) is loaded while
// the previous row runs, the first chunk of A_i while W_i is hashed, each
// lane's columns and values of W_i kInsDepth at a time before they are
// inserted, and the next chunk of A_i while the current one's pairs run.
constexpr int kBwdInsDepth = 4;

struct BwdMeta {
    int nw, ws0, ps, pe;
};

// The loads of a row's metadata (size of W_i, row pointers of W and A),
// issued without a branch around them (a slot without a row reads zeros: no
// entries) so that their first use can sit a row later.
__device__ __forceinline__ BwdMeta bwd_meta_issue(const Prob &P, const Sched &sc, int g)
{
    const bool on = g >= 0;
    const MLS_G int32_t *zero = (const MLS_G int32_t *)k_zeros4;
    const MLS_G int32_t *pv = on ? gp(sc.val) + g : zero;
    const MLS_G int32_t *pc = on ? gp(P.crp) + g : zero;
    const MLS_G int32_t *pa = on ? gp(P.arp) + g : zero;
    BwdMeta m;
    m.nw = *pv;
    m.ws0 = *pc;
    m.ps = pa[0];
    m.pe = pa[1];
    return m;
}

// A row's first chunk, located in advance: entries ps + lane of A_i (column
// -1 and value 0 past the row), then their rows' bounds in B (zeros past the
// row: no pairs).
struct BwdFirst {
    int ka;
    double sa;
    int q0, q1;
};

__device__ __forceinline__ void bwd_first_a(const Prob &P, const BwdMeta &m, int lane, BwdFirst &f)
{
    const bool on = m.ps + lane < m.pe;
    f.ka = *(on ? gp(P.aci) + m.ps + lane : (const MLS_G int32_t *)k_ones4);
    f.sa = *(on ? gp(P.aval) + m.ps + lane : (const MLS_G double *)k_zeros4);
}

__device__ __forceinline__ void bwd_first_b(const Prob &P, BwdFirst &f)
{
    const MLS_G int32_t *pb = f.ka >= 0 ? gp(P.brp) + f.ka : (const MLS_G int32_t *)k_zeros4;
    f.q0 = pb[0];
    f.q1 = pb[1];
}

template <int G, int CAP, bool PACK>
__global__ __launch_bounds__(kWG) void k_bwd_lds(Batch b, Sched sc, int bin, double *dA, double *dB)
{
    constexpr int W = kWave / G;
    constexpr int NW = nw_bwd_best(bwd_row_bytes(CAP, G, PACK) * W);
    constexpr int WV = PACK ? CAP / 2 : CAP;   // W values per row: by position, or by slot
    __shared__ __attribute__((aligned(16))) int s_key[NW * W * CAP];
    __shared__ double s_wv[NW * W * WV];
    __shared__ double s_pa[NW * W * G];
    __shared__ double s_da[NW * W * G];
    __shared__ int s_pq[NW * W * G];
    __shared__ __attribute__((aligned(16))) int s_poff[NW * W * (G + 4)];   // read four at a time

    const int wave = threadIdx.x >> 6;
    if (wave >= NW) return;
    const int lw = threadIdx.x & 63;
    const int slot = lw / G, lane = lw % G;
    const int rs = wave * W + slot;
    int *key = s_key + rs * CAP;
    double *wv = s_wv + rs * WV;
    PosTab<CAP, true, 4> ptab{(uint32_t *)key};   // PACK: column -> position of W_i
    double *pa = s_pa + rs * G;
    double *da = s_da + rs * G;
    int *pq = s_pq + rs * G;
    int *poff = s_poff + rs * (G + 4);

    const Prob P = b.p0;
    const MLS_G int32_t *__restrict__ aci = gp(P.aci);
    const MLS_G double *__restrict__ aval = gp(P.aval);
    const MLS_G int32_t *__restrict__ brp = gp(P.brp);
    const MLS_G int32_t *__restrict__ bci = gp(P.bci);
    const MLS_G double *__restrict__ bval = gp(P.bval);
    const MLS_G int32_t *__restrict__ wci = gp(P.cci);
    const MLS_G double *__restrict__ wval = gp(P.cval);
    MLS_G double *__restrict__ gdA = gpw(dA);
    const int n_bin = gp(sc.bin_count)[bin];
    const int start = bin_start(sc.bin_count, bin);
    const int ntasks = (n_bin + W - 1) / W;
    TaskIter it = task_iter(ntasks, NW);
    // Three rows of a slot are in flight: the row after next has its perm
    // entry loading, the next row its metadata, then its first chunk (entries
    // of A_i while this row's W_i is hashed, their B row bounds after this
    // row's pairs), so a row starts with its dependent index loads done.
    int task = next_task_wave(sc.task_cursor + bin * kXcd, ntasks, it);
    const bool h_cur = task >= 0 && task * W + slot < n_bin;
    const int g_raw = bin_row_issue(sc.perm, sc.err, b.na, start + task * W + slot, h_cur);
    int task_n = task >= 0 ? next_task_wave(sc.task_cursor + bin * kXcd, ntasks, it) : -1;
    bool h_n = task_n >= 0 && task_n * W + slot < n_bin;
    int g_n = bin_row_issue(sc.perm, sc.err, b.na, start + task_n * W + slot, h_n);
    BwdMeta m = bwd_meta_issue(P, sc, bin_row_checked(sc.err, b.na, g_raw, h_cur));
    BwdFirst f;
    bwd_first_a(P, m, lane, f);
    bwd_first_b(P, f);
    // no prologue load is left pending into the loop (the wait counts at its
    // top are computed over both ways into it)
    asm volatile("" ::"v"(f.q0), "v"(f.q1), "v"(f.sa), "v"(g_n), "v"(m.nw), "v"(m.ws0), "v"(m.ps), "v"(m.pe));
    while (task >= 0) {
        const int task_x = task_n >= 0 ? next_task_wave(sc.task_cursor + bin * kXcd, ntasks, it) : -1;
        const bool h_x = task_x >= 0 && task_x * W + slot < n_bin;
        const int g_x = bin_row_issue(sc.perm, sc.err, b.na, start + task_x * W + slot, h_x);
        const BwdMeta mn = bwd_meta_issue(P, sc, bin_row_checked(sc.err, b.na, g_n, h_n));
        const int nw = m.nw, ws0 = m.ws0, ps = m.ps, pe = m.pe;
        int logcap = ilog2_ceil(2 * nw);
        if (logcap < 5) logcap = 5;
        const int cap = 1 << logcap;
        if constexpr (PACK) {
            ptab.clear(cap, lane, G);
        } else {
            for (int h = lane; h < cap; h += G) key[h] = -1;
        }
        // this row's first chunk was located during the previous row
        int ka = f.ka;
        double sa = f.sa;
        int fq0 = f.q0, fq1 = f.q1;
        bwd_sync();
        for (int e0 = lane; e0 < nw; e0 += G * kBwdInsDepth) {
            int jv[kBwdInsDepth];
            double wj[kBwdInsDepth];
#pragma unroll
            for (int u = 0; u < kBwdInsDepth; ++u) {
                const int e = e0 + u * G;
                jv[u] = -1;
                wj[u] = 0.0;
                if (e < nw) { jv[u] = wci[ws0 + e]; wj[u] = wval[ws0 + e]; }
            }
#pragma unroll
            for (int u = 0; u < kBwdInsDepth; ++u) {
                if (jv[u] < 0) continue;
                if constexpr (PACK) {
                    ptab.insert(logcap, jv[u], e0 + u * G);
                    wv[e0 + u * G] = wj[u];
                } else {
                    w_insert(key, wv, logcap, jv[u], wj[u]);
                }
            }
        }
        bwd_sync();
        bool bad = false;
        // the chunk loop runs to the wave's longest row, so that the group
        // scans (cross-lane shuffles) run with every lane present
        int nch = (pe - ps + G - 1) / G;
        for (int o = 32; o >= 1; o >>= 1) nch = max(nch, __shfl_xor(nch, o, kWave));
        // stage a chunk: its entries' first B positions, pair offsets, a_ik
        // and zeroed dA sums; returns the chunk's pair count
        auto stage = [&](int q0, int q1, double a) -> int {
            const int np = q1 > q0 ? q1 - q0 : 0;
            const int incl = group_scan_incl<G>(np, lane);
            const int tot = group_total<G>(np, incl);
            poff[lane] = incl - np;
            if (lane == 0) poff[G] = tot;
            pq[lane] = q0;
            pa[lane] = a;
            da[lane] = 0.0;
            return tot;
        };
        // the first chunk from what was located during the previous row, the
        // later ones in the loop: no loaded value reaches a point where two
        // ways join (its wait there would cover every load issued since)
        int total = stage(fq0, fq1, sa);
        // the next row's first entries of A load during this row's pairs
        bwd_first_a(P, mn, lane, f);
        for (int c = 0; c < nch; ++c) {
            const int pc = ps + c * G;
            if (c > 0) {
                const MLS_G int32_t *pb = pc + lane < pe ? brp + ka : (const MLS_G int32_t *)k_zeros4;
                total = stage(pb[0], pb[1], sa);
            }
            // the next chunk's entries of A are in flight during this chunk's
            // pairs (no branch: see the numeric kernel's chunk loop)
            {
                const bool on = pc + G + lane < pe;
                ka = *(on ? aci + pc + G + lane : (const MLS_G int32_t *)k_ones4);
                sa = *(on ? aval + pc + G + lane : (const MLS_G double *)k_zeros4);
            }
            bwd_sync();
            // groups of at most 16 lanes keep the pair offsets in registers: a
            // pair's entry is the last one whose offset is at most its index
            constexpr int RG = G <= 16 ? G : 4;
            int pofv[RG];
            if constexpr (G <= 16) {
#pragma unroll
                for (int x = 0; x < G; x += 4) {
                    const int4 v = *(const int4 *)(poff + x);
                    pofv[x] = v.x; pofv[x + 1] = v.y; pofv[x + 2] = v.z; pofv[x + 3] = v.w;
                }
            }
            // the dB adds of a batch are issued after the next batch's loads:
            // the wait for those loads then does not include them (the
            // counter covers loads and atomics in issue order)
            int dq[kBwdUnroll];
            double dv[kBwdUnroll];
#pragma unroll
            for (int d = 0; d < kBwdUnroll; ++d) { dq[d] = -1; dv[d] = 0.0; }
            for (int base = 0; base < total; base += G * kBwdUnroll) {
                int qv[kBwdUnroll], ev[kBwdUnroll], jv[kBwdUnroll];
                double bv[kBwdUnroll];
                // loads without branches (pairs past the chunk read the all-ones
                // dummy: column -1), all issued before any use
#pragma unroll
                for (int d = 0; d < kBwdUnroll; ++d) {
                    const int pp = base + d * G + lane;
                    int lo, po;
                    if constexpr (G <= 16) {
                        lo = -1;
                        po = 0;
#pragma unroll
                        for (int x = 0; x < G; ++x) {
                            const bool le = pofv[x] <= pp;
                            lo += le ? 1 : 0;
                            po = le ? pofv[x] : po;
                        }
                    } else {
                        lo = 0;
                        int hi = G - 1;   // largest e with poff[e] <= pp
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (poff[mid] <= pp) lo = mid; else hi = mid - 1;
                        }
                        po = poff[lo];
                    }
                    const bool ok = pp < total;
                    ev[d] = lo;
                    qv[d] = pq[lo] + (pp - po);
                    const MLS_G int32_t *pj = ok ? bci + qv[d] : (const MLS_G int32_t *)k_bwd_void;
                    const MLS_G double *pv = ok ? bval + qv[d] : (const MLS_G double *)k_bwd_void;
                    jv[d] = *pj;
                    bv[d] = *pv;
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int d = 0; d < kBwdUnroll; ++d)
                    if (dq[d] >= 0) atomicAdd(dB + dq[d], dv[d]);
                int sl[kBwdUnroll];
                double w[kBwdUnroll];
                if constexpr (PACK) {
                    // positions in W_i's row, then the values by position
                    ptab.template lookup_n<kBwdUnroll>(logcap, jv, sl);
#pragma unroll
                    for (int d = 0; d < kBwdUnroll; ++d) w[d] = wv[sl[d] >= 0 ? sl[d] : 0];
                } else {
                    w_lookup_n<kBwdUnroll>(key, wv, logcap, jv, sl, w);
                }
#pragma unroll
                for (int d = 0; d < kBwdUnroll; ++d) asm volatile("" ::"v"(bv[d]));
#pragma unroll
                for (int d = 0; d < kBwdUnroll; ++d) {
                    if (sl[d] == -1) bad = true;
                    dq[d] = -1;
                    if (sl[d] < 0) continue;
                    if (dA) atomicAdd(da + ev[d], w[d] * bv[d]);
                    if (dB) { dq[d] = qv[d]; dv[d] = pa[ev[d]] * w[d]; }
                }
            }
#pragma unroll
            for (int d = 0; d < kBwdUnroll; ++d)
                if (dq[d] >= 0) atomicAdd(dB + dq[d], dv[d]);
            bwd_sync();
            if (dA && pc + lane < pe) gdA[pc + lane] = da[lane];
            bwd_sync();
        }
        // the next row's B row bounds (its entries of A arrived during the pairs)
        bwd_first_b(P, f);
        if (bad) atomicOr(sc.err, kErrStructure);
        bwd_sync();
        task = task_n;
        task_n = task_x;
        g_n = g_x;
        h_n = h_x;
        m = mn;
    }
}

__device__ __forceinline__ int bsearch_w(const MLS_G int32_t *cols, int n, int j)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (cols[mid] < j) lo = mid + 1; else hi = mid;
    }
    return (lo < n && cols[lo] == j) ? lo : -1;
}

// first position in cols[lo, hi) whose column is >= j
__device__ __forceinline__ int lower_col_w(const MLS_G int32_t *cols, int lo, int hi, int j)
{
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cols[mid] < j) lo = mid + 1; else hi = mid;
    }
    return lo;
}

constexpr int kBwdWinCap = 1024;   // table slots of a spill window (CAP / 2 positions of W_i)
constexpr int kBwdWinDepth = 2;    // batches of 64 pairs whose B loads are issued together
constexpr int kBwdWinBlock = 4;    // consecutive windows a wave takes per counter grab

// LDS of one spill window: hash keys and W values, staged entries, their
// first pair, and the entries' dA parts
constexpr int bwd_win_bytes(int CAP) { return CAP * 12 + kWave * 16 + (kWave + 1) * 4 + kWave * 8; }

// Windows of the spill rows come from k_win_scan (same rule: ceil(nnz(W_i) / M)).
// A window's (entry, B position) pairs are flattened, 64 per step: each pair
// adds a_ik W_ij into dB with a device atomic and W_ij b_kj into its entry's
// dA part in LDS; the parts go to dA with one device atomic per entry.
template <int CAP>
__global__ __launch_bounds__(kWG) void k_bwd_win(Batch b, Sched sc, double *dA, double *dB)
{
    constexpr int G = kWave;
    constexpr int M = CAP / 2;
    constexpr int NW = nw_bwd(bwd_win_bytes(CAP), 1);
    __shared__ __attribute__((aligned(16))) int s_key[NW * CAP];
    __shared__ double s_wv[NW * CAP];
    __shared__ int4 s_par[NW * G];        // staged entries: (first B position, -, a)
    __shared__ int s_poff[NW * (G + 1)];  // first pair of each staged entry, then the total
    __shared__ double s_da[NW * G];

    const int wave = threadIdx.x >> 6;
    if (wave >= NW) return;
    const int lane = threadIdx.x & 63;
    int *key = s_key + wave * CAP;
    double *wv = s_wv + wave * CAP;
    int4 *par = s_par + wave * G;
    int *poff = s_poff + wave * (G + 1);
    double *da = s_da + wave * G;

    const Prob P = b.p0;
    const MLS_G int32_t *__restrict__ arp = gp(P.arp);
    const MLS_G int32_t *__restrict__ aci = gp(P.aci);
    const MLS_G double *__restrict__ aval = gp(P.aval);
    const MLS_G int32_t *__restrict__ brp = gp(P.brp);
    const MLS_G int32_t *__restrict__ bci = gp(P.bci);
    const MLS_G double *__restrict__ bval = gp(P.bval);
    const MLS_G int32_t *__restrict__ wrp = gp(P.crp);
    const MLS_G int32_t *__restrict__ wci = gp(P.cci);
    const MLS_G double *__restrict__ wval = gp(P.cval);
    const int n_bin = gp(sc.bin_count)[kBinSpill];
    const int start = bin_start(sc.bin_count, kBinSpill);
    const MLS_G int32_t *wst = gp(sc.wstart);
    const int nwin = n_bin > 0 ? wst[n_bin] : 0;
    // one counter over all windows: their work varies too much (a hub row's
    // windows are consecutive and long) for per-XCD slabs
    if (nwin == 0) return;
    int32_t *cursor = sc.task_cursor + kBinSpill * kXcd;
    for (;;) {
        int u0 = 0;
        if (lane == 0) u0 = atomicAdd(cursor, 1) * kBwdWinBlock;
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
        const int u1 = min(u0 + kBwdWinBlock, nwin);
        for (int u = u0; u < u1; ++u) {
            while (wst[r + 1] <= u) ++r;
            const int i = bin_row(sc.perm, sc.err, b.na, start + r);
            if (i < 0) continue;
            const int nw = gp(sc.val)[i];
            const int c0 = (u - wst[r]) * M;
            const int ws0 = wrp[i] + c0;
            const int n = min(M, nw - c0);
            const bool narrow = nw > M;
            // open below for the row's first window and above for its last, so
            // that a column outside the whole row still fails the lookup
            const int jlo = c0 == 0 ? INT_MIN : wci[ws0];
            const int jhi = c0 + n == nw ? INT_MAX : wci[ws0 + n - 1];
            int logcap = ilog2_ceil(2 * n);
            if (logcap < 5) logcap = 5;
            const int cap = 1 << logcap;
            for (int h = lane; h < cap; h += G) key[h] = -1;
            bwd_sync();
            for (int e0 = lane; e0 < n; e0 += G * kBwdInsDepth) {
                int jv[kBwdInsDepth];
                double wj[kBwdInsDepth];
#pragma unroll
                for (int u = 0; u < kBwdInsDepth; ++u) {
                    const int e = e0 + u * G;
                    jv[u] = -1;
                    wj[u] = 0.0;
                    if (e < n) { jv[u] = wci[ws0 + e]; wj[u] = wval[ws0 + e]; }
                }
#pragma unroll
                for (int u = 0; u < kBwdInsDepth; ++u)
                    if (jv[u] >= 0) w_insert(key, wv, logcap, jv[u], wj[u]);
            }
            bwd_sync();
            bool bad = false;
            const int ps = arp[i], pe = arp[i + 1];
            for (int pc = ps; pc < pe; pc += G) {
                int sq0 = 0, sq1 = 0;
                double sa = 0.0;
                if (pc + lane < pe) {
                    const int k = aci[pc + lane];
                    sa = aval[pc + lane];
                    sq0 = brp[k];
                    sq1 = brp[k + 1];
                    if (narrow && sq1 - sq0 > 32) {
                        if (jlo != INT_MIN) sq0 = lower_col_w(bci, sq0, sq1, jlo);
                        if (jhi != INT_MAX) sq1 = lower_col_w(bci, sq0, sq1, jhi + 1);
                    }
                }
                const int np = sq1 > sq0 ? sq1 - sq0 : 0;
                int incl = group_scan_incl<G>(np, lane);
                const int total = group_total<G>(np, incl);
                poff[lane] = incl - np;
                if (lane == 0) poff[G] = total;
                par[lane] = make_int4(sq0, 0, __double2loint(sa), __double2hiint(sa));
                da[lane] = 0.0;
                bwd_sync();
                for (int base = 0; base < total; base += G * kBwdWinDepth) {
                    int ev[kBwdWinDepth], qv[kBwdWinDepth], jv[kBwdWinDepth];
                    double bv[kBwdWinDepth], av[kBwdWinDepth];
#pragma unroll
                    for (int d = 0; d < kBwdWinDepth; ++d) {
                        jv[d] = -1; ev[d] = 0; qv[d] = 0; bv[d] = 0.0; av[d] = 0.0;
                        const int pp = base + d * G + lane;
                        if (pp < total) {
                            int lo = 0, hi = G - 1;   // largest e with poff[e] <= pp
                            while (lo < hi) {
                                const int mid = (lo + hi + 1) >> 1;
                                if (poff[mid] <= pp) lo = mid; else hi = mid - 1;
                            }
                            const int4 pr = par[lo];
                            ev[d] = lo;
                            qv[d] = pr.x + (pp - poff[lo]);
                            av[d] = __hiloint2double(pr.w, pr.z);
                            jv[d] = bci[qv[d]];
                            bv[d] = bval[qv[d]];
                        }
                    }
                    int jw[kBwdWinDepth], sl[kBwdWinDepth];
                    double w[kBwdWinDepth];
#pragma unroll
                    for (int d = 0; d < kBwdWinDepth; ++d) jw[d] = (jv[d] >= jlo && jv[d] <= jhi) ? jv[d] : -1;
                    w_lookup_n<kBwdWinDepth>(key, wv, logcap, jw, sl, w);
#pragma unroll
                    for (int d = 0; d < kBwdWinDepth; ++d) {
                        if (sl[d] == -1) bad = true;
                        if (sl[d] < 0) continue;
                        if (dA) atomicAdd(da + ev[d], w[d] * bv[d]);
                        if (dB) atomicAdd(dB + qv[d], av[d] * w[d]);
                    }
                }
                bwd_sync();
                if (dA && pc + lane < pe && da[lane] != 0.0) atomicAdd(dA + pc + lane, da[lane]);
                bwd_sync();
            }
            if (bad) atomicOr(sc.err, kErrStructure);
        }
    }
}

template <typename K>
static int bwd_grid(K kernel, int threads)
{
    static int cus = device_cu_count();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

template <int G, int CAP, bool PACK>
static void launch_bwd_variant(const Batch &b, const Sched &sc, int bin, double *dA, double *dB, hipStream_t s)
{
    constexpr int W = kWave / G;
    constexpr int NW = nw_bwd_best(bwd_row_bytes(CAP, G, PACK) * W);
    static int grid = bwd_grid(k_bwd_lds<G, CAP, PACK>, NW * kWave);
    static char name[64];
    if (!name[0]) snprintf(name, sizeof(name), "bwd_lds_G%d_C%d%s", G, CAP, PACK ? "_p" : "");
    ProfScope ps(name, s);
    hipLaunchKernelGGL((k_bwd_lds<G, CAP, PACK>), dim3(grid), dim3(NW * kWave), 0, s, b, sc, bin, dA, dB);
}

// The packed table needs every column index of W below PackBits<CAP>::kMaxCols.
template <int G, int CAP>
static void launch_bwd_class(const Batch &b, const Sched &sc, int bin, double *dA, double *dB, hipStream_t s)
{
    if (b.max_ncols > 0 && (uint32_t)b.max_ncols <= PackBits<CAP>::kMaxCols)
        launch_bwd_variant<G, CAP, true>(b, sc, bin, dA, dB, s);
    else
        launch_bwd_variant<G, CAP, false>(b, sc, bin, dA, dB, s);
}

void launch_backward(const Batch &b, const Sched &sc, const double *wval, double *dA, double *dB, int G,
                     hipStream_t s)
{
    (void)wval;
    if (b.na <= 0) return;
    launch_bwd_class<8, kFillCap[0]>(b, sc, 0, dA, dB, s);
    switch (G) {
    case 8: launch_bwd_class<8, kFillCap[1]>(b, sc, 1, dA, dB, s); break;
    case 16: launch_bwd_class<16, kFillCap[1]>(b, sc, 1, dA, dB, s); break;
    case 64: launch_bwd_class<64, kFillCap[1]>(b, sc, 1, dA, dB, s); break;
    default: launch_bwd_class<32, kFillCap[1]>(b, sc, 1, dA, dB, s); break;
    }
    if (G >= 64) launch_bwd_class<64, kFillCap[2]>(b, sc, 2, dA, dB, s);
    else launch_bwd_class<32, kFillCap[2]>(b, sc, 2, dA, dB, s);
    launch_bwd_class<64, kFillCap[3]>(b, sc, 3, dA, dB, s);
    launch_bwd_class<64, kFillCap[4]>(b, sc, 4, dA, dB, s);
    constexpr int NWW = nw_bwd(bwd_win_bytes(kBwdWinCap), 1);
    static int win_grid = bwd_grid(k_bwd_win<kBwdWinCap>, NWW * kWave);
    ProfScope ps("bwd_spill", s);
    hipLaunchKernelGGL(k_win_scan, dim3(1), dim3(kWG), 0, s, b, sc, kBwdWinCap / 2);
    hipLaunchKernelGGL(k_bwd_win<kBwdWinCap>, dim3(win_grid), dim3(NWW * kWave), 0, s, b, sc, dA, dB);
}

// ---------------------------------------------------------------------------
// Deterministic adjoint: every entry of dA and of dB is the sequential sum of
// one lane, in the order of the row-wise formulation -- dA_ik over the columns
// j of B_k in ascending order, dB_kj over the rows i of column k of A in
// ascending order (read from the transpose of A) -- with each product rounded
// before it is added. The result does not depend on scheduling, so repeated
// calls agree bit for bit. W_ij is found by binary search in W_i's ascending
// columns (no LDS table, no atomics on the outputs); a triple whose column j
// is missing from W_i sets the structure error.

constexpr int kDetLanes = 8;   // lanes per row; a lane takes every 8th entry

__global__ __launch_bounds__(kWG) void k_bwd_det_da(int32_t m, const int32_t *arp, const int32_t *aci,
                                                    const int32_t *brp, const int32_t *bci, const double *bval,
                                                    const int32_t *wrp, const int32_t *wci, const double *wval,
                                                    double *dA, uint32_t *err)
{
    const int64_t g = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const int64_t i = g / kDetLanes;
    if (i >= m) return;
    const int l = (int)(g % kDetLanes);
    const int ws = gp(wrp)[i], wn = gp(wrp)[i + 1] - ws;
    const MLS_G int32_t *wc = gp(wci) + ws;
    const MLS_G double *wv = gp(wval) + ws;
    bool bad = false;
    const int pe = gp(arp)[i + 1];
    for (int p = gp(arp)[i] + l; p < pe; p += kDetLanes) {
        const int k = gp(aci)[p];
        const int qs = gp(brp)[k], qe = gp(brp)[k + 1];
        double sum = 0.0;
        int lo = 0;   // the columns of B_k ascend, so each search starts past the last hit
        for (int q = qs; q < qe; ++q) {
            const int j = gp(bci)[q];
            lo = lower_col_w(wc, lo, wn, j);
            if (lo >= wn || wc[lo] != j) { bad = true; break; }
            sum += wv[lo] * gp(bval)[q];
        }
        gpw(dA)[p] = sum;
    }
    if (bad) atomicOr(err, kErrStructure);
}

__global__ __launch_bounds__(kWG) void k_bwd_det_db(int32_t kb, const int32_t *trp, const int32_t *tci,
                                                    const double *tv, const int32_t *brp, const int32_t *bci,
                                                    const int32_t *wrp, const int32_t *wci, const double *wval,
                                                    double *dB, uint32_t *err)
{
    const int64_t g = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const int64_t k = g / kDetLanes;
    if (k >= kb) return;
    const int l = (int)(g % kDetLanes);
    const int rs = gp(trp)[k], re = gp(trp)[k + 1];
    bool bad = false;
    const int qe = gp(brp)[k + 1];
    for (int q = gp(brp)[k] + l; q < qe; q += kDetLanes) {
        const int j = gp(bci)[q];
        double sum = 0.0;
        for (int r = rs; r < re; ++r) {   // rows i of column k of A, ascending
            const int i = gp(tci)[r];
            const int ws = gp(wrp)[i], wn = gp(wrp)[i + 1] - ws;
            const int pos = lower_col_w(gp(wci) + ws, 0, wn, j);
            if (pos >= wn || gp(wci)[ws + pos] != j) { bad = true; break; }
            sum += gp(tv)[r] * gp(wval)[ws + pos];
        }
        gpw(dB)[q] = sum;
    }
    if (bad) atomicOr(err, kErrStructure);
}

void launch_backward_det(int32_t m, int32_t kb, const int32_t *arp, const int32_t *aci, const int32_t *brp,
                         const int32_t *bci, const double *bval, const int32_t *wrp, const int32_t *wci,
                         const double *wval, const int32_t *trp, const int32_t *tci, const double *tv, double *dA,
                         double *dB, uint32_t *err, hipStream_t s)
{
    if (dA && m > 0) {
        ProfScope ps("bwd_det_dA", s);
        const int64_t blocks = ((int64_t)m * kDetLanes + kWG - 1) / kWG;
        hipLaunchKernelGGL(k_bwd_det_da, dim3((unsigned)blocks), dim3(kWG), 0, s, m, arp, aci, brp, bci, bval, wrp,
                           wci, wval, dA, err);
    }
    if (dB && kb > 0) {
        ProfScope ps("bwd_det_dB", s);
        const int64_t blocks = ((int64_t)kb * kDetLanes + kWG - 1) / kWG;
        hipLaunchKernelGGL(k_bwd_det_db, dim3((unsigned)blocks), dim3(kWG), 0, s, kb, trp, tci, tv, brp, bci, wrp,
                           wci, wval, dB, err);
    }
}

// ---------------------------------------------------------------------------
// transpose

__global__ void k_tr_count(int32_t nrows, const int32_t *rp, const int32_t *ci, int32_t *cnt)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    for (int p = gp(rp)[i]; p < gp(rp)[i + 1]; ++p) atomicAdd(cnt + gp(ci)[p], 1);
}

__global__ void k_tr_rowptr(int32_t n, const int64_t *prefix, int32_t *trp)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) gpw(trp)[i] = (int32_t)gp(prefix)[i];
}

__global__ void k_tr_scatter(int32_t nrows, const int32_t *rp, const int32_t *ci, const double *v, const int32_t *trp,
                             int32_t *cursor, int32_t *tci, double *tv)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    for (int p = gp(rp)[i]; p < gp(rp)[i + 1]; ++p) {
        int c = gp(ci)[p];
        int pos = gp(trp)[c] + atomicAdd(cursor + c, 1);
        gpw(tci)[pos] = i;
        if (v) gpw(tv)[pos] = gp(v)[p];
    }
}

// per-row insertion sort of (column, value) pairs (rows of a transpose are
// short for the workloads here; long rows still sort correctly, just slowly)
__global__ void k_tr_sort(int32_t n, const int32_t *trp, int32_t *tci, double *tv)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int s = gp(trp)[r], e = gp(trp)[r + 1];
    MLS_G int32_t *c = gpw(tci);
    MLS_G double *v = gpw(tv);
    for (int a = s + 1; a < e; ++a) {
        int key = c[a];
        double kv = tv ? v[a] : 0.0;
        int b2 = a - 1;
        while (b2 >= s && c[b2] > key) {
            c[b2 + 1] = c[b2];
            if (tv) v[b2 + 1] = v[b2];
            --b2;
        }
        c[b2 + 1] = key;
        if (tv) v[b2 + 1] = kv;
    }
}

void launch_transpose(int32_t nrows, int32_t ncols, const int32_t *rp, const int32_t *ci, const double *v,
                      int32_t *trp, int32_t *tci, double *tv, int32_t *cursor, int64_t *tile_sum, int64_t *prefix,
                      int32_t *cnt, hipStream_t s)
{
    ProfScope ps("transpose", s);
    launch_fill_i32(cnt, 0, ncols, s);
    launch_fill_i32(cursor, 0, ncols, s);
    if (nrows > 0)
        hipLaunchKernelGGL(k_tr_count, dim3((nrows + kWG - 1) / kWG), dim3(kWG), 0, s, nrows, rp, ci, cnt);
    launch_scan(cnt, ncols, tile_sum, prefix, s);
    hipLaunchKernelGGL(k_tr_rowptr, dim3((ncols + kWG) / kWG), dim3(kWG), 0, s, ncols, prefix, trp);
    if (nrows > 0)
        hipLaunchKernelGGL(k_tr_scatter, dim3((nrows + kWG - 1) / kWG), dim3(kWG), 0, s, nrows, rp, ci, v, trp, cursor,
                           tci, tv);
    if (ncols > 0) hipLaunchKernelGGL(k_tr_sort, dim3((ncols + kWG - 1) / kWG), dim3(kWG), 0, s, ncols, trp, tci, tv);
}

// out[e] = X(r, c) for the e-th entry (r, c) of pattern P, else 0.0
__global__ void k_mask_gather(int32_t nrows, const int32_t *xrp, const int32_t *xci, const double *xv,
                              const int32_t *prp, const int32_t *pci, double *out)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const int xs = gp(xrp)[r], xn = gp(xrp)[r + 1] - xs;
    for (int p = gp(prp)[r]; p < gp(prp)[r + 1]; ++p) {
        int pos = bsearch_w(gp(xci) + xs, xn, gp(pci)[p]);
        gpw(out)[p] = pos >= 0 ? gp(xv)[xs + pos] : 0.0;
    }
}

void launch_mask_gather(int32_t nrows, const int32_t *xrp, const int32_t *xci, const double *xv, const int32_t *prp,
                        const int32_t *pci, double *out, hipStream_t s)
{
    if (nrows <= 0) return;
    ProfScope ps("mask_gather", s);
    hipLaunchKernelGGL(k_mask_gather, dim3((nrows + kWG - 1) / kWG), dim3(kWG), 0, s, nrows, xrp, xci, xv, prp, pci,
                       out);
}

}  // namespace mls
