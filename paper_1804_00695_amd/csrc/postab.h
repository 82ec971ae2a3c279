// postab.h -- the column -> position hash table of one row held in LDS,
// shared by the numeric and adjoint kernels.
#pragma once

#include "common.h"

namespace mls {

// Column -> position table of one row of C, in one of two layouts:
//   wide  : int2 slots (column, position), any column count;
//   packed: one uint32 per slot, column << PB | position, with PB bits for the
//           position (positions < CAP/2). Usable when every column index of C
//           fits in the remaining bits; halves the bytes of every lookup.
// Empty slots hold -1 (all ones); a packed key never equals it because the
// column range excludes the all-ones column field.
template <int CAP>
struct PackBits {
    static constexpr int PB = CAP == 64 ? 5 : (CAP == 256 ? 7 : (CAP == 1024 ? 9 : (CAP == 2048 ? 10 : 11)));
    static_assert(CAP == 64 || CAP == 256 || CAP == 1024 || CAP == 2048 || CAP == 4096, "table class");
    static constexpr uint32_t kMaxCols = (1u << (32 - PB)) - 1u;   // columns < this fit
};

// Bucket words of a packed table: BK = 2 or 4 slots read in one LDS access.
template <int BK> struct BucketT;
template <> struct BucketT<2> {
    using T = uint2;
    __device__ __forceinline__ static uint32_t minx(T w, uint32_t k) { return min(w.x ^ k, w.y ^ k); }
    __device__ __forceinline__ static uint32_t last(T w) { return w.y; }
    __device__ __forceinline__ static int first_empty(T w, uint32_t e) { return w.x == e ? 0 : (w.y == e ? 1 : 2); }
};
template <> struct BucketT<4> {
    using T = uint4;
    __device__ __forceinline__ static uint32_t minx(T w, uint32_t k)
    {
        return min(min(w.x ^ k, w.y ^ k), min(w.z ^ k, w.w ^ k));
    }
    __device__ __forceinline__ static uint32_t last(T w) { return w.w; }
    __device__ __forceinline__ static int first_empty(T w, uint32_t e)
    {
        return w.x == e ? 0 : (w.y == e ? 1 : (w.z == e ? 2 : (w.w == e ? 3 : 4)));
    }
};

template <int CAP, bool PACK, int BK = 4>
struct PosTab {
    static_assert(BK == 2 || BK == 4, "bucket of 2 or 4 slots");
    using BT = BucketT<BK>;
    using BW = typename BT::T;
    static constexpr int LB = BK == 2 ? 1 : 2;   // log2 of the bucket width
    uint32_t *t;   // CAP words (packed) or 2*CAP words (wide)

    __device__ __forceinline__ void clear(int cap, int lane, int G)
    {
        if (PACK) {
            if (cap >= 4 * G) {
                for (int h = 4 * lane; h < cap; h += 4 * G)
                    *(uint4 *)(t + h) = make_uint4(0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu);
            } else {
                for (int h = lane; h < cap; h += G) t[h] = 0xffffffffu;
            }
        } else {
            for (int h = lane; h < cap; h += G) ((int2 *)t)[h] = make_int2(-1, 0);
        }
    }

    static constexpr uint32_t kEmpty = 0xffffffffu;

    // Packed tables are probed a bucket (BK slots, one LDS read) at a time: a key
    // takes the first empty slot at or after the start of its home bucket, so
    // the filled slots of every bucket are a prefix of it (a lane only claims
    // a slot after seeing every earlier one taken, and slots are never
    // emptied), and a bucket whose last slot is empty ends a search.
    __device__ __forceinline__ static uint32_t home(int logcap, int j)
    {
        return hslot((uint32_t)j, logcap - LB) << LB;
    }
    __device__ __forceinline__ BW bucket(uint32_t h) const { return *(const BW *)(t + h); }

    __device__ __forceinline__ void insert(int logcap, int j, int pos)
    {
        const uint32_t cmask = (1u << logcap) - 1u;
        if (PACK) {
            const uint32_t v = ((uint32_t)j << PackBits<CAP>::PB) | (uint32_t)pos;
            uint32_t h = home(logcap, j);
            for (uint32_t probe = 0; probe <= cmask; probe += BK) {
                int sl = BT::first_empty(bucket(h), kEmpty);
                for (; sl < BK; ++sl)
                    if (atomicCAS(t + h + sl, kEmpty, v) == kEmpty) return;
                h = (h + BK) & cmask;
            }
        } else {
            uint32_t h = hslot((uint32_t)j, logcap);
            int2 *tab = (int2 *)t;
            for (uint32_t probe = 0; probe <= cmask; ++probe) {
                int old = atomicCAS(&tab[h].x, -1, j);
                if (old == -1) { tab[h].y = pos; return; }
                h = (h + 1u) & cmask;
            }
        }
    }

    // Packed: position of column j given the words w of its home bucket h, or
    // -1 when j is not in the row. A slot holds j iff its word XOR (j << PB)
    // is below 2^PB, and that value is then the position; at most one slot
    // of a bucket holds j, so the minimum over the bucket decides.
    __device__ __forceinline__ int find(int logcap, int j, uint32_t h, BW w, bool live = true) const
    {
        constexpr int PB = PackBits<CAP>::PB;
        const uint32_t key = (uint32_t)j << PB, pm = (1u << PB) - 1u;
        const uint32_t m = BT::minx(w, key);
        int p = m <= pm ? (int)m : -1;
        if (live && m > pm && BT::last(w) != kEmpty) p = find_more(logcap, key, h);
        return p;
    }

    // the search past a full home bucket h (rarely needed)
    __device__ __forceinline__ int find_more(int logcap, uint32_t key, uint32_t h) const
    {
        constexpr int PB = PackBits<CAP>::PB;
        const uint32_t pm = (1u << PB) - 1u, cmask = (1u << logcap) - 1u;
        for (uint32_t probe = BK; probe <= cmask; probe += BK) {
            h = (h + BK) & cmask;
            const BW v = bucket(h);
            const uint32_t mv = BT::minx(v, key);
            if (mv <= pm) return (int)mv;
            if (BT::last(v) == kEmpty) return -1;
        }
        return -1;
    }

    // position of column j in the row, or -1 when j is not in the row
    __device__ __forceinline__ int lookup(int logcap, int j) const
    {
        if (PACK) {
            const uint32_t h = home(logcap, j);
            return find(logcap, j, h, bucket(h));
        } else {
            const uint32_t cmask = (1u << logcap) - 1u;
            uint32_t h = hslot((uint32_t)j, logcap);
            const int2 *tab = (const int2 *)t;
            for (uint32_t probe = 0; probe <= cmask; ++probe) {
                const int2 v = tab[h];
                if (v.x == j) return v.y;
                if (v.x == -1) return -1;
                h = (h + 1u) & cmask;
            }
        }
        return -1;
    }

    // positions of D columns (-2 where jv < 0): the home buckets of all D are
    // read before any is searched
    template <int D>
    __device__ __forceinline__ void lookup_n(int logcap, const int (&jv)[D], int (&pos)[D]) const
    {
        static_assert(D % 2 == 0, "looked up in pairs");
        if (PACK) {
            // two at a time: four buckets in registers would cost 16 VGPRs
#pragma unroll
            for (int d0 = 0; d0 < D; d0 += 2) {
                uint32_t hv[2];
                BW wv[2];
#pragma unroll
                for (int d = 0; d < 2; ++d) hv[d] = jv[d0 + d] >= 0 ? home(logcap, jv[d0 + d]) : 0u;
#pragma unroll
                for (int d = 0; d < 2; ++d) wv[d] = bucket(hv[d]);
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    const bool live = jv[d0 + d] >= 0;
                    const int p = find(logcap, jv[d0 + d], hv[d], wv[d], live);
                    pos[d0 + d] = live ? p : -2;
                }
            }
        } else {
#pragma unroll
            for (int d = 0; d < D; ++d) pos[d] = jv[d] >= 0 ? lookup(logcap, jv[d]) : -2;
        }
    }
};

}  // namespace mls
