// k_numeric.hip -- numeric phase (Sec. 2.1, Fig. "spgemmexp") as the
// row-range fused multiply-add kernel of the chunking algorithms
// (Secs. 3.2.2 and 3.3.1): C_i += sum over k in row i of A, k in [k_lo, k_hi),
// of a_ik * B_k, optionally starting from the values already in C (the
// partial result of earlier row parts of B).
//
// LDS path: G lanes own a row of C. Its (sorted) columns are loaded once into
// an LDS hash mapping column -> position in the row, next to an LDS array of
// fp64 accumulators in row order. The entries of row i of A are taken in
// stored order; for each, the G lanes take distinct entries of B_k, so no two
// lanes of a step touch the same accumulator and every c_ij receives its
// terms in ascending k -- the order of the row-wise formulation. Products are
// rounded before the add (compiled without contraction), so the result equals
// a sequential dense-accumulator evaluation bit for bit. Loads for U entries
// of A are issued before their accumulation steps to hide HBM/L2 latency.
//
// Spill path (rows with more than the largest LDS class of outputs): one
// workgroup per row accumulates directly in C's value array (global memory),
// locating positions by binary search in C's sorted columns, one k per step
// with a workgroup barrier between steps.
#include <cstdio>

#include "common.h"
#include "launch.h"
#include "profile.h"

namespace mls {

constexpr int kNumDepth = 8;   // steps whose B loads are issued together

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

__device__ __forceinline__ int pos_lookup(const int2 *tab, int logcap, int j)
{
    const uint32_t cmask = (1u << logcap) - 1u;
    uint32_t h = hslot((uint32_t)j, logcap);
    for (uint32_t probe = 0; probe <= cmask; ++probe) {
        int2 v = tab[h];
        if (v.x == j) return v.y;
        if (v.x == -1) return -1;
        h = (h + 1u) & cmask;
    }
    return -1;
}

__device__ __forceinline__ void pos_insert(int2 *tab, int logcap, int j, int pos)
{
    const uint32_t cmask = (1u << logcap) - 1u;
    uint32_t h = hslot((uint32_t)j, logcap);
    for (uint32_t probe = 0; probe <= cmask; ++probe) {
        int old = atomicCAS(&tab[h].x, -1, j);
        if (old == -1) { tab[h].y = pos; return; }
        h = (h + 1u) & cmask;
    }
}

template <int G, int CAP>
__global__ __launch_bounds__(kWG) void k_num_lds(Batch b, Sched sc, int bin)
{
    constexpr int W = kWave / G;
    constexpr int NW = nw_num(CAP * 12 + G * 16, W);
    __shared__ int2 s_tab[NW * W * CAP];
    __shared__ double s_acc[NW * W * (CAP / 2)];
    __shared__ int4 s_par[NW * W * G];   // staged entries of row i of A: (q0, q1, a)

    const int wave = threadIdx.x >> 6;
    if (wave >= NW) return;
    const int lw = threadIdx.x & 63;
    const int slot = lw / G, lane = lw % G;
    const int rs = wave * W + slot;
    int2 *tab = s_tab + rs * CAP;
    double *acc = s_acc + rs * (CAP / 2);
    int4 *par = s_par + rs * G;

    const MLS_G int32_t *perm = gp(sc.perm);
    const MLS_G int32_t *val = gp(sc.val);
    const int n_bin = gp(sc.bin_count)[bin];
    const int start = bin_start(sc.bin_count, bin);
    const int ntasks = (n_bin + W - 1) / W;
    TaskIter it = task_iter(ntasks, NW);
    for (;;) {
        int task = next_task_wave(sc.task_cursor + bin * kXcd, ntasks, it);
        if (task < 0) break;
        const int r = task * W + slot;
        const bool active = r < n_bin;
        int g = active ? perm[start + r] : 0;
        int t = (!active || b.nprob == 1) ? 0 : find_prob(b.abase, b.nprob, g);
        const Prob P = get_prob(b, t);
        int i = g - (b.nprob == 1 ? 0 : gp(b.abase)[t]);
        const int nc = active ? val[g] : 0;
        int logcap = ilog2_ceil(2 * nc);
        if (logcap < 5) logcap = 5;
        const int cap = 1 << logcap;
        for (int h = lane; h < cap; h += G) tab[h] = make_int2(-1, 0);
        nwave_sync();
        // descriptor fields into registers once per row, as global pointers
        const MLS_G int32_t *__restrict__ aci = gp(P.aci);
        const MLS_G double *__restrict__ aval = gp(P.aval);
        const MLS_G int32_t *__restrict__ brp = gp(P.brp);
        const MLS_G int32_t *__restrict__ bci = gp(P.bci);
        const MLS_G double *__restrict__ bval = gp(P.bval);
        const MLS_G int32_t *__restrict__ cci = gp(P.cci);
        MLS_G double *__restrict__ cval = gpw(P.cval);
        const int a_off = P.a_off, b_off = P.b_off, k_lo = P.k_lo, k_hi = P.k_hi;
        const bool accumulate = P.accumulate != 0;
        int cs = 0, ps = 0, pe = 0;
        if (active) {
            cs = gp(P.crp)[i] - P.c_off;
            ps = gp(P.arp)[i] - a_off;
            pe = gp(P.arp)[i + 1] - a_off;
            for (int e = lane; e < nc; e += G) {
                pos_insert(tab, logcap, cci[cs + e], e);
                acc[e] = accumulate ? cval[cs + e] : 0.0;
            }
        }
        nwave_sync();
        bool bad = false;
        for (int pc = ps; pc < pe; pc += G) {
            // stage a chunk of row i of A: one round of loads for G entries
            {
                const int p = pc + lane;
                int q0 = 0, q1 = 0;
                double a = 0.0;
                if (p < pe) {
                    const int k = aci[p];
                    a = aval[p];
                    if (k >= k_lo && k < k_hi) {
                        q0 = brp[k - k_lo] - b_off;
                        q1 = brp[k - k_lo + 1] - b_off;
                    }
                }
                par[lane] = make_int4(q0, q1, __double2loint(a), __double2hiint(a));
            }
            nwave_sync();
            const int n = min(G, pe - pc);
            for (int u0 = 0; u0 < n; u0 += kNumDepth) {
                // issue the B loads of kNumDepth steps, then accumulate them in order
                int jv[kNumDepth], q1v[kNumDepth];
                double bv[kNumDepth], av[kNumDepth];
#pragma unroll
                for (int d = 0; d < kNumDepth; ++d) {
                    jv[d] = -1; bv[d] = 0.0; av[d] = 0.0; q1v[d] = 0;
                    if (u0 + d < n) {
                        const int4 pr = par[u0 + d];
                        av[d] = __hiloint2double(pr.w, pr.z);
                        q1v[d] = pr.y;
                        const int q = pr.x + lane;
                        if (q < pr.y) { jv[d] = bci[q]; bv[d] = bval[q]; }
                    }
                }
                // positions first (independent LDS reads), then the adds in step
                // order; within a step the lanes hold distinct columns of B_k, so
                // no two lanes add to the same slot and every slot gets its terms
                // in ascending k. The LDS fp64 add rounds like a plain add.
                int posv[kNumDepth];
#pragma unroll
                for (int d = 0; d < kNumDepth; ++d) posv[d] = jv[d] >= 0 ? pos_lookup(tab, logcap, jv[d]) : -2;
#pragma unroll
                for (int d = 0; d < kNumDepth; ++d) {
                    if (posv[d] >= 0) atomicAdd(acc + posv[d], av[d] * bv[d]);
                    else if (posv[d] == -1) bad = true;
                    if (u0 + d < n && q1v[d] - par[u0 + d].x > G) {   // rows of B longer than G
                        const int q0 = par[u0 + d].x;
                        for (int q = q0 + G + lane; q < q1v[d]; q += G) {
                            const int pos = pos_lookup(tab, logcap, bci[q]);
                            if (pos >= 0) atomicAdd(acc + pos, av[d] * bval[q]);
                            else bad = true;
                        }
                    }
                }
            }
            nwave_sync();
        }
        if (bad) atomicOr(sc.err, kErrStructure);
        if (active)
            for (int e = lane; e < nc; e += G) cval[cs + e] = acc[e];
        nwave_sync();
    }
}

__device__ __forceinline__ int bsearch_col(const MLS_G int32_t *cols, int n, int j)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (cols[mid] < j) lo = mid + 1; else hi = mid;
    }
    return (lo < n && cols[lo] == j) ? lo : -1;
}

__global__ __launch_bounds__(kWG) void k_num_spill(Batch b, Sched sc)
{
    const int n_bin = gp(sc.bin_count)[kBinSpill];
    const int start = bin_start(sc.bin_count, kBinSpill);
    for (int r = blockIdx.x; r < n_bin; r += gridDim.x) {
        int g = gp(sc.perm)[start + r];
        int t = b.nprob == 1 ? 0 : find_prob(b.abase, b.nprob, g);
        const Prob P = get_prob(b, t);
        int i = g - (b.nprob == 1 ? 0 : gp(b.abase)[t]);
        const int cs = gp(P.crp)[i] - P.c_off;
        const int nc = gp(P.crp)[i + 1] - gp(P.crp)[i];
        double *cv = P.cval + cs;
        const MLS_G int32_t *cc = gp(P.cci) + cs;
        const MLS_G int32_t *__restrict__ aci = gp(P.aci);
        const MLS_G double *__restrict__ aval = gp(P.aval);
        const MLS_G int32_t *__restrict__ brp = gp(P.brp);
        const MLS_G int32_t *__restrict__ bci = gp(P.bci);
        const MLS_G double *__restrict__ bval = gp(P.bval);
        if (!P.accumulate)
            for (int e = threadIdx.x; e < nc; e += kWG)
                __hip_atomic_store(cv + e, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        __syncthreads();
        bool bad = false;
        const int ps = gp(P.arp)[i] - P.a_off, pe = gp(P.arp)[i + 1] - P.a_off;
        for (int p = ps; p < pe; ++p) {
            int k = aci[p];
            if (k >= P.k_lo && k < P.k_hi) {
                double a = aval[p];
                int kl = k - P.k_lo;
                int q0 = brp[kl] - P.b_off, q1 = brp[kl + 1] - P.b_off;
                for (int q = q0 + threadIdx.x; q < q1; q += kWG) {
                    int pos = bsearch_col(cc, nc, bci[q]);
                    if (pos < 0) { bad = true; continue; }
                    double old = __hip_atomic_load(cv + pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(cv + pos, old + a * bval[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            __threadfence();
            __syncthreads();
        }
        if (bad) atomicOr(sc.err, kErrStructure);
        __syncthreads();
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

template <int G, int CAP>
static void launch_num_class(const Batch &b, const Sched &sc, int bin, hipStream_t s)
{
    constexpr int W = kWave / G;
    constexpr int NW = nw_num(CAP * 12 + G * 16, W);
    static int grid = persistent_grid_n(k_num_lds<G, CAP>, NW * kWave);
    static char name[64];
    if (!name[0]) snprintf(name, sizeof(name), "num_lds_G%d_C%d", G, CAP);
    ProfScope ps(name, s);
    hipLaunchKernelGGL((k_num_lds<G, CAP>), dim3(grid), dim3(NW * kWave), 0, s, b, sc, bin);
}

void launch_numeric(const Batch &b, const Sched &sc, int G, hipStream_t s)
{
    if (b.na <= 0) return;
    switch (G) {
    case 8: launch_num_class<8, kFillCap[0]>(b, sc, 0, s); break;
    case 16: launch_num_class<16, kFillCap[0]>(b, sc, 0, s); break;
    case 64: launch_num_class<64, kFillCap[0]>(b, sc, 0, s); break;
    default: launch_num_class<32, kFillCap[0]>(b, sc, 0, s); break;
    }
    if (G >= 64) launch_num_class<64, kFillCap[1]>(b, sc, 1, s);
    else launch_num_class<32, kFillCap[1]>(b, sc, 1, s);
    launch_num_class<64, kFillCap[2]>(b, sc, 2, s);
    static int spill_grid = device_cu_count();
    ProfScope ps("num_spill", s);
    hipLaunchKernelGGL(k_num_spill, dim3(spill_grid), dim3(kWG), 0, s, b, sc);
}

}  // namespace mls
