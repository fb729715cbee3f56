// wht_contig16.hpp -- contiguous pass over tiles of 2^16 consecutive 4-byte
// entries (256 KiB), transformed over all 16 tile bits in one HBM round trip.
//
// The tile is twice what LDS holds, so it lives in registers (1024 threads x
// 64 entries) and the top tile bit is a register bit in every layout
// ("pinned"): each transpose through LDS moves one half of the tile at a time
// (2^15 entries + padding), the half given by the pinned bit.  Layouts for 64
// entries per thread:
//   L0 {0, 1, 12, 13, 14, 15}: 16-byte vector loads (bits 0, 1 in a vector);
//   L1 {2 .. 6, 15};  L2 {7 .. 11, 15}: lanes hold bits 0 .. 5, so a wave's
//   stores cover 256 contiguous bytes.
// All 16 bits are transformed, so the layout sequence is fixed at compile
// time.  Like every pass, the butterflies on distinct bits commute (the
// regrouping of Fig. 2 and Fig. 3).
#pragma once
#include "wht_tile.hpp"

namespace fwht {

template <class S, int NTM = 0>
struct Contig16Kernel {
    static_assert(sizeof(S) == 4, "2^16 entries of 4 bytes fill half the register file");
    static constexpr int TB = 16, NT = 1024, E = (1 << TB) / NT, K = 6, VEC = 4, VB = 2;
    static constexpr LayoutList LS = make_pinned_layouts(TB, K, VB);
    static constexpr uint32_t FULL = lowmask(TB);
    static constexpr uint32_t HALF = lowmask(TB - 1);
    static constexpr int LDS_ELEMS = (1 << (TB - 1)) + (1 << (TB - 1)) / 32;
    static_assert(LS.n == 3, "three layouts");
    static_assert(lanes_contiguous(LS.m[2], 6), "last layout stores whole 256-byte runs");

    template <int P>
    struct Split {
        static constexpr uint32_t TM = FULL & ~LS.m[P];
        static constexpr uint32_t LANE = low_set_bits(TM, 6);
        static constexpr uint32_t WAVE = TM & ~LANE;
    };

    // Half H of the registers of layout P (those whose pinned bit is H) to
    // LDS, or back; the LDS index drops the pinned bit.
    template <int P, int H>
    __device__ static __forceinline__ void to_lds(S *lds, const S (&v)[E], uint32_t t)
    {
        constexpr uint32_t M = LS.m[P];
        const uint32_t tb = lds_pad(pdep_rt<FULL & ~M>(t));
        static_for<H * (E / 2), (H + 1) * (E / 2)>([&](auto J) {
            constexpr uint32_t jp = cpdep((uint32_t)decltype(J)::value, M) & HALF;
            lds[tb + jp + (jp >> 5)] = v[decltype(J)::value];
        });
    }
    template <int P, int H>
    __device__ static __forceinline__ void from_lds(const S *lds, S (&v)[E], uint32_t t)
    {
        constexpr uint32_t M = LS.m[P];
        const uint32_t tb = lds_pad(pdep_rt<FULL & ~M>(t));
        static_for<H * (E / 2), (H + 1) * (E / 2)>([&](auto J) {
            constexpr uint32_t jp = cpdep((uint32_t)decltype(J)::value, M) & HALF;
            v[decltype(J)::value] = lds[tb + jp + (jp >> 5)];
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

    __device__ static __forceinline__ void tile(const S *src, S *dst, S *lds, uint32_t t, const PassArgs &a)
    {
        const uint32_t lane = t & 63u;
        const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);
        S v[E];
        {
            constexpr uint32_t M0 = LS.m[0];
            const uint32_t lp = pdep_rt<Split<0>::LANE>(lane);
            const uint32_t wp = pdep_rt<Split<0>::WAVE>(wave);
            static_for<0, E / VEC>([&](auto JT) {
                constexpr int jt = decltype(JT)::value;
                constexpr uint32_t jp = cpdep((uint32_t)(jt << VB), M0);
                const v4u q = gload16<(NTM & NT_LOAD) != 0>(src + (jp | wp) + lp);
                const S *qs = reinterpret_cast<const S *>(&q);
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[jt * VEC + e] = qs[e];
            });
        }
        reg_stages<S, LS.m[0], LS.fresh[0], E>(v, FULL);
        transpose<0, 1>(lds, v, t);
        reg_stages<S, LS.m[1], LS.fresh[1], E>(v, FULL);
        __syncthreads();
        transpose<1, 2>(lds, v, t);
        reg_stages<S, LS.m[2], LS.fresh[2], E>(v, FULL);
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
        const uint32_t lp = pdep_rt<Split<2>::LANE>(slane);
        const uint32_t wp = pdep_rt<Split<2>::WAVE>(swave);
        static_for<0, E>([&](auto J) {
            constexpr uint32_t jp = cpdep((uint32_t)decltype(J)::value, LS.m[2]);
            gstore1<(NTM & NT_STORE) != 0>(dst + ((jp | wp) + lp), v[decltype(J)::value]);
        });
        __syncthreads();  // the next tile reuses the LDS buffer
    }

    __device__ static __forceinline__ void run(S *__restrict__ buf, const PassArgs &a)
    {
        __shared__ S lds[LDS_ELEMS];
        S *out = a.dst ? static_cast<S *>(a.dst) : buf;
        if (a.zero_first && blockIdx.x == 0 && threadIdx.x == 0) *a.zero_first = 0ull;
        for (uint64_t tl = blockIdx.x; tl < a.ntiles; tl += gridDim.x) {
            uint32_t t = threadIdx.x;
            asm volatile("" : "+v"(t));
            const uint64_t base = tl << TB;
            tile(buf + base, out + base, lds, t, a);
        }
    }
};

template <class S, int NTM>
__global__ void __launch_bounds__(1024, 1) wht_contig16_kernel(S *__restrict__ buf, PassArgs a)
{
    Contig16Kernel<S, NTM>::run(buf, a);
}

// Host launcher: every tile is full (the planner only schedules this variant
// as the first pass of a transform of at least 2^17 entries, over all 16
// bits, and never with an epilogue).
template <class S, int NTM = 0>
hipError_t launch_contig16(void *buf, const PassArgs &a, hipStream_t s)
{
    if (a.act != lowmask(16) || (a.total & lowmask(16)) || a.thresh) return hipErrorInvalidValue;
    const uint64_t maxgrid = (1ull << 31) / 1024;  // work-items counted in 32 bits; grid-stride loop
    const uint64_t grid = a.ntiles < maxgrid ? a.ntiles : maxgrid;
    hipLaunchKernelGGL((wht_contig16_kernel<S, NTM>), dim3((uint32_t)grid), dim3(1024), 0, s, (S *)buf, a);
    return hipGetLastError();
}

}  // namespace fwht
