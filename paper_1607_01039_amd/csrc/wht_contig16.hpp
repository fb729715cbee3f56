// wht_contig16.hpp -- passes over tiles of 256 KiB (2^16 4-byte or 2^15
// 8-byte entries), twice what LDS holds in one piece.
//
// The tile lives in registers (1024 threads x 64 or 32 entries) and the top
// tile bit is a register bit in every layout ("pinned"): each transpose
// through LDS moves one half of the tile at a time (128 KiB + padding), the
// half given by the pinned bit.  The descriptions below are for 4-byte
// entries; 8-byte tiles have one bit less everywhere (strided "S15c6",
// "S15c7": 512-byte and 1 KiB row segments of 2^9 and 2^8 rows), and their
// layouts, five register bits each, need one transpose more for the same
// row bits (a CPU model of the 64 banks finds the one-word-per-32 padding
// free of conflicts for both strided 8-byte tiles).
//   * contiguous (CB = 0, "C16"): 2^16 consecutive entries, all 16 bits
//     transformed; layouts L0 {0, 1, 12 .. 15} (16-byte loads), L1 {2 .. 6, 15},
//     L2 {7 .. 11, 15}.
//   * strided (CB > 0, "S16c<CB>"): 2^CB contiguous columns (2^CB * 4 bytes
//     per row segment) of 2^(16 - CB) rows at a stride of 2^b entries; the
//     16 - CB row bits are transformed.  L0 as above, then one layout with the
//     remaining row bits (e.g. CB = 8: L1 {8 .. 11, 14, 15}).
// In both, the lanes of the last layout hold tile bits 0 .. 5, so every wave
// store covers 256 contiguous bytes.  Every candidate bit is transformed (the
// planner uses these variants at their full height only), so the layout
// sequence is fixed at compile time.  Like every pass, the butterflies on
// distinct bits commute (the regrouping of Fig. 2 and Fig. 3).
#pragma once
#include "wht_tile.hpp"

namespace fwht {

template <class S, int CB, bool TH, int NTM, int TBX = 0, int NTX = 1024>
struct Pinned16Kernel {
    static_assert(sizeof(S) == 4 || sizeof(S) == 8, "4- or 8-byte entries");
    // 256 KiB tiles: 2^16 entries of 4 bytes (64 per thread) or 2^15 of 8
    // bytes (32 per thread), half the register file either way; TBX / NTX
    // give other tile sizes and thread counts (C15p: 2^15 4-byte entries in
    // 512 threads, two workgroups per CU)
    static constexpr int TB = TBX ? TBX : sizeof(S) == 4 ? 16 : 15, NT = NTX, E = (1 << TB) / NT, K = clog2(E);
    static constexpr int VEC = 16 / (int)sizeof(S), VB = clog2(VEC);
    static constexpr bool COLS = CB == 0;
    static constexpr int R = TB - CB;  // transformed bits
    static constexpr LayoutList LS = make_pinned_layouts(TB, K, VB, CB);
    static constexpr int LAST = LS.n - 1;
    static constexpr uint32_t FULL = lowmask(TB);
    static constexpr uint32_t HALF = lowmask(TB - 1);
    // LDS padding, entries per 32: one, except two for the contiguous 8-byte
    // tile, whose second layout would otherwise read with 2-way bank
    // conflicts (CPU model of the 64 banks)
    static constexpr uint32_t PAD = sizeof(S) == 8 && COLS ? 2 : 1;
    static constexpr int LDS_ELEMS = (1 << (TB - 1)) + PAD * ((1 << (TB - 1)) / 32);
    static_assert(LS.n >= 2 && LS.n <= 4, "layout count");
    static_assert(lanes_contiguous(LS.m[LAST], 6), "last layout stores whole runs of 64 entries");
    static_assert(CB == 0 || CB >= VB + 5, "a wave's vector loads cover whole 512-byte row segments");

    template <int P>
    struct Split {
        static constexpr uint32_t TM = FULL & ~LS.m[P];
        static constexpr uint32_t LANE = low_set_bits(TM, 6);
        static constexpr uint32_t WAVE = TM & ~LANE;
    };

    // Global offset (entries) of tile index idx: rows of stride 2^b above the
    // CB column bits (the identity for a contiguous tile).  Linear over
    // disjoint bit sets, so register, wave and lane parts add up.
    __device__ static __forceinline__ uint64_t goff(uint32_t idx, uint32_t b)
    {
        if constexpr (COLS) return idx;
        else return ((uint64_t)(idx >> CB) << b) + (idx & lowmask(CB));
    }

    // Half H of the registers of layout P (those whose pinned bit is H) to
    // LDS, or back; the LDS index drops the pinned bit.
    // padded LDS index; additive over disjoint bit sets, so the thread part
    // and the register part are padded separately
    __device__ static __forceinline__ constexpr uint32_t pad(uint32_t i) { return i + PAD * (i >> 5); }

    template <int P, int H>
    __device__ static __forceinline__ void to_lds(S *lds, const S (&v)[E], uint32_t t)
    {
        constexpr uint32_t M = LS.m[P];
        const uint32_t tb = pad(pdep_rt<FULL & ~M>(t));
        static_for<H * (E / 2), (H + 1) * (E / 2)>([&](auto J) {
            constexpr uint32_t jp = cpdep((uint32_t)decltype(J)::value, M) & HALF;
            lds[tb + pad(jp)] = v[decltype(J)::value];
        });
    }
    template <int P, int H>
    __device__ static __forceinline__ void from_lds(const S *lds, S (&v)[E], uint32_t t)
    {
        constexpr uint32_t M = LS.m[P];
        const uint32_t tb = pad(pdep_rt<FULL & ~M>(t));
        static_for<H * (E / 2), (H + 1) * (E / 2)>([&](auto J) {
            constexpr uint32_t jp = cpdep((uint32_t)decltype(J)::value, M) & HALF;
            v[decltype(J)::value] = lds[tb + pad(jp)];
        });
    }
    template <int FROM, int TO>
    __device__ static __forceinline__ void transpose(S *lds, S (&v)[E], uint32_t t)
    {
        to_lds<FROM, 0>(lds, v, t);
        __syncthreads();
        from_lds<TO, 0>(lds, v, t);
        __syncthreads();
        to_lds<FROM, 1>(lds, v, t);
        __syncthreads();
        from_lds<TO, 1>(lds, v, t);
    }

    // Threshold epilogue around the final stores (as in the 2^15-entry tile
    // pass): whether any element of this thread is a hit before the stores;
    // after them, only in a wave with a hit, a uniform loop re-reads every
    // entry this thread has just written, tests it again and appends the hits.
    __device__ static __forceinline__ bool any_hit(const S (&v)[E], const PassArgs &a)
    {
        const HitTest<S> ht(a);
        bool any = false;
        static_for<0, E>([&](auto J) { any |= ht.above(v[decltype(J)::value]); });
        return any;
    }
    __device__ static __forceinline__ void emit(const S *buf, bool any, uint64_t lo, const PassArgs &a)
    {
        if (__ballot(any) == 0) return;
        const HitTest<S> ht(a);
#pragma unroll 1
        for (int j = 0; j < E; ++j) {
            const uint64_t off = lo + goff(pdep_rt<LS.m[LAST]>((uint32_t)j), a.b);
            const S val = any ? buf[off] : S(0);
            emit_hits<S>(any && ht.above(val), off, val, a);
        }
    }

    __device__ static __forceinline__ void tile(const S *src, S *dst, S *lds, uint32_t t, uint64_t base,
                                                const PassArgs &a)
    {
        const uint32_t lane = t & 63u;
        const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);
        S v[E];
        {
            constexpr uint32_t M0 = LS.m[0];
            const uint64_t lb = goff(pdep_rt<Split<0>::LANE>(lane), a.b);
            const uint64_t wb = base + goff(pdep_rt<Split<0>::WAVE>(wave), a.b);
            static_for<0, E / VEC>([&](auto JT) {
                constexpr int jt = decltype(JT)::value;
                constexpr uint32_t jp = cpdep((uint32_t)(jt << VB), M0);
                const v4u q = gload16<(NTM & NT_LOAD) != 0>(src + (wb + goff(jp, a.b)) + lb);
                const S *qs = reinterpret_cast<const S *>(&q);
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[jt * VEC + e] = qs[e];
            });
        }
        // Every load of the tile is issued before the first butterfly: the
        // previous tile's stores are still in flight, and the counter that
        // tracks loads also counts them, so consuming the first load early
        // would wait for all of them before the other loads were issued.
        __builtin_amdgcn_sched_barrier(0);
        reg_stages<S, LS.m[0], LS.fresh[0], E>(v, FULL);
        static_for<1, LS.n>([&](auto PP) {
            constexpr int P = decltype(PP)::value;
            if constexpr (P > 1) __syncthreads();  // the previous transpose's reads are done
            transpose<P - 1, P>(lds, v, t);
            reg_stages<S, LS.m[P], LS.fresh[P], E>(v, FULL);
        });
        if constexpr (std::is_same<S, float>::value) {
            if (a.do_scale) {
#pragma unroll
                for (int j = 0; j < E; ++j) v[j] *= a.scale;
            }
        }
        // opaque thread coordinates: store offsets are computed here, not
        // kept live from the loads
        uint32_t slane = lane, swave = wave;
        asm volatile("" : "+v"(slane));
        asm volatile("" : "+s"(swave));
        // The lanes of the last layout are tile bits 0 .. 5 (column bits), so a
        // store is a wave-uniform base plus the lane id as a 32-bit index.
        static_assert(Split<LAST>::LANE == lowmask(6), "lanes on tile bits 0 .. 5");
        const uint64_t wo = base + goff(pdep_rt<Split<LAST>::WAVE>(swave), a.b);
        S *ub = dst + wo;
        bool any = false;
        if constexpr (TH) any = any_hit(v, a);
        static_for<0, E>([&](auto J) {
            constexpr uint32_t jp = cpdep((uint32_t)decltype(J)::value, LS.m[LAST]);
            gstore1<(NTM & NT_STORE) != 0>(ub + goff(jp, a.b) + slane, v[decltype(J)::value]);
        });
        if constexpr (TH) emit(dst, any, wo + slane, a);
        __syncthreads();  // the next tile reuses the LDS buffer
    }

    __device__ static __forceinline__ void run(S *__restrict__ buf, const PassArgs &a)
    {
        __shared__ S lds[LDS_ELEMS];
        S *out = a.dst ? static_cast<S *>(a.dst) : buf;
        if (a.zero_first && blockIdx.x == 0 && threadIdx.x == 0) *a.zero_first = 0ull;
        const uint32_t cbl = (uint32_t)__builtin_ctzll(a.colblocks);  // colblocks = 2^cbl
        // Contiguous tiles in XCD-major order: workgroup w runs on XCD w mod 8,
        // and the workgroups of one XCD take one contiguous eighth of the
        // tiles (a contiguous in-place pass measured 3% faster this way).
        const bool xcd = COLS && (a.ntiles & 7) == 0 && (gridDim.x & 7) == 0;
        // scalar trip count (see the tile kernel's loop)
        const uint64_t first = blockIdx.x;
        const uint32_t iters = a.ntiles > first ? (uint32_t)((a.ntiles - first - 1) / gridDim.x + 1) : 0u;
        for (uint32_t k = 0; k < iters; ++k) {
            const uint64_t w = first + (uint64_t)k * gridDim.x;
            const uint64_t tl = xcd ? ((w & 7) * (a.ntiles >> 3) + (w >> 3)) : w;
            // opaque copies per tile: the offsets derived from them are
            // recomputed for each tile instead of being hoisted and kept live
            uint32_t t = threadIdx.x;
            asm volatile("" : "+v"(t));
            PassArgs at = a;
            asm volatile("" : "+s"(at.b));
            const uint64_t g = tl >> cbl, cb = tl & (a.colblocks - 1);
            const uint64_t base = COLS ? (tl << TB) : (((g << R) << at.b) + (cb << CB));
            tile(buf, out, lds, t, base, at);
        }
    }
};

template <class S, int CB, bool TH, int NTM, int TBX = 0, int NTX = 1024>
__global__ void __launch_bounds__(NTX, 1024 / NTX) wht_pinned16_kernel(S *__restrict__ buf, PassArgs a)
{
    Pinned16Kernel<S, CB, TH, NTM, TBX, NTX>::run(buf, a);
}

// Host launchers.  Every tile is full: the planner schedules these variants
// only over their full height, and the contiguous one only as the first pass
// of a transform of at least 2^17 entries, with no epilogue.
template <class S, int CB, int NTM, int TBX = 0, int NTX = 1024>
hipError_t launch_pinned16(void *buf, const PassArgs &a, hipStream_t s)
{
    constexpr int TB = Pinned16Kernel<S, CB, false, NTM, TBX, NTX>::TB;
    constexpr int R = TB - CB;
    if (a.act != (lowmask(R) << CB)) return hipErrorInvalidValue;
    if (CB == 0 && ((a.total & lowmask(TB)) || a.thresh)) return hipErrorInvalidValue;
    if (CB > 0 && (((a.total >> a.b) & lowmask(R)) || a.b < (uint32_t)CB)) return hipErrorInvalidValue;
    const uint64_t maxgrid = (1ull << 31) / NTX;  // work-items counted in 32 bits; grid-stride loop
    const uint64_t grid = a.ntiles < maxgrid ? a.ntiles : maxgrid;
    if (a.thresh)
        hipLaunchKernelGGL((wht_pinned16_kernel<S, CB, true, NTM, TBX, NTX>), dim3((uint32_t)grid), dim3(NTX), 0, s,
                           (S *)buf, a);
    else
        hipLaunchKernelGGL((wht_pinned16_kernel<S, CB, false, NTM, TBX, NTX>), dim3((uint32_t)grid), dim3(NTX), 0, s,
                           (S *)buf, a);
    return hipGetLastError();
}

template <class S, int NTM = 0>
hipError_t launch_contig16(void *buf, const PassArgs &a, hipStream_t s)
{
    return launch_pinned16<S, 0, NTM>(buf, a, s);
}

// 128 KiB tiles held the same way by 512 threads (64 registers of 4-byte or
// 32 of 8-byte entries) with half-tile transposes through 66-68 KiB of LDS,
// so that two workgroups share a CU and one's loads and stores overlap the
// other's LDS phases: "C15p" (2^15 4-byte entries) and "C14p" (2^14 8-byte
// entries), first passes only, over exactly their bits, no epilogue; and the
// strided 8-byte "S14c6p" (2^8 rows x 512 B).
template <class S, int NTM = 0>
hipError_t launch_contig15p(void *buf, const PassArgs &a, hipStream_t s)
{
    return launch_pinned16<S, 0, NTM, sizeof(S) == 4 ? 15 : 14, 512>(buf, a, s);
}
template <class S, int CB, int NTM = 0>
hipError_t launch_strided14p(void *buf, const PassArgs &a, hipStream_t s)
{
    static_assert(sizeof(S) == 8, "8-byte entries");
    return launch_pinned16<S, CB, NTM, 14, 512>(buf, a, s);
}
// The strided 4-byte counterparts "S15c7p" and "S15c8p": 2^8 rows x 512 B and
// 2^7 rows x 1 KiB, half-tile transposes through 66 KiB of LDS, two
// workgroups per CU.
template <class S, int CB, int NTM = 0>
hipError_t launch_strided15p(void *buf, const PassArgs &a, hipStream_t s)
{
    static_assert(sizeof(S) == 4, "4-byte entries");
    return launch_pinned16<S, CB, NTM, 15, 512>(buf, a, s);
}

}  // namespace fwht
