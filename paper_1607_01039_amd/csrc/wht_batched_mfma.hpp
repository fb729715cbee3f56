// wht_batched_mfma.hpp -- the batched persistent transform with radix-16
// stages on the matrix cores (v_mfma_f32_16x16x16 with f16 or bf16 operands,
// FP32 accumulation).
//
// A radix-16 stage is the product H_16 X, where the 16 rows of X are the 16
// entries that differ in four index bits.  For the 16x16x16 MFMA, lane l
// holds B[k][n] for n = l mod 16 and k = 4 (l div 16) + i, i = 0..3 in four
// operand halves, and receives D[m][n] for m = 4 (l div 16) + i in four FP32
// registers: the output sits where its input row sat, so the stage is in
// place.  The four K bits are therefore two register bits (i) and lane bits
// 4 and 5; lane bits 0..3 index 16 independent columns.  The data is rounded
// to f16/bf16 at the input of each such stage; H_16 (entries +-1, scaled by
// an exact power of two) is exact in both formats.  Stage bits that a work
// item does not transform get an identity factor instead of H_2.
//
// Tile of 2^16 entries (as the FP32 kernel), 1024 threads, 64 entries per
// thread, two layouts (register bits listed in register-index order):
//   MA (load): registers {0,1,12,13,14,15}, lanes {2..7}, waves {8..11};
//        MFMA on {0,1,6,7} (registers 0,1 + lanes 4,5), VALU on {12..15}.
//   MB: registers {2,3,8,9,10,11}, lanes {0,1,6,7,4,5}, waves {12..15};
//        MFMA on {2,3,4,5}, VALU on {8..11}.
//   MC (store): registers {0,1,12,13,14,11}, lanes {2..7}, waves {8,9,10,15}:
//        16-byte stores of four consecutive entries.
// MA -> MB goes through LDS as f16/bf16: the values are the operands of MB's
// MFMA stage, which rounds them to that format anyway, so storing them
// rounded changes nothing and halves the LDS footprint (the whole 2^16 tile
// in 128 KiB).  MB -> MC goes through the same LDS as FP32 values in two
// halves: bit 11 is the last register bit of both, so each half of every
// thread's registers maps to one half of the tile.
#pragma once
#include "wht_batched.hpp"

#ifndef MFMA_GROUP_BLOCKS
#define MFMA_GROUP_BLOCKS 4
#endif

namespace fwht {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

struct XLayout {
    int reg[6];
    int lane[6];
    int wave[4];
};

constexpr XLayout XL_A{{0, 1, 12, 13, 14, 15}, {2, 3, 4, 5, 6, 7}, {8, 9, 10, 11}};
constexpr XLayout XL_B{{2, 3, 8, 9, 10, 11}, {0, 1, 6, 7, 4, 5}, {12, 13, 14, 15}};
constexpr XLayout XL_C{{0, 1, 12, 13, 14, 11}, {2, 3, 4, 5, 6, 7}, {8, 9, 10, 15}};

constexpr uint32_t xl_reg_part(const XLayout &L, uint32_t j)
{
    uint32_t r = 0;
    for (int q = 0; q < 6; ++q)
        if ((j >> q) & 1u) r |= 1u << L.reg[q];
    return r;
}
constexpr uint32_t xl_lane_mask(const XLayout &L)
{
    uint32_t r = 0;
    for (int q = 0; q < 6; ++q) r |= 1u << L.lane[q];
    return r;
}

template <int PREC>
__device__ __forceinline__ uint16_t to_half_bits(float x);
template <>
__device__ __forceinline__ uint16_t to_half_bits<FWHT_PREC_FP16_MFMA>(float x)
{
    _Float16 h = (_Float16)x;  // round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
template <>
__device__ __forceinline__ uint16_t to_half_bits<FWHT_PREC_BF16_MFMA>(float x)
{
    const __bf16 h = (__bf16)x;  // round to nearest even (gfx950 converts in hardware)
    return __builtin_bit_cast(uint16_t, h);
}

template <int PREC>
struct MfmaOp;
template <>
struct MfmaOp<FWHT_PREC_FP16_MFMA> {
    __device__ static __forceinline__ float4_t run(const uint16_t (&a)[4], const uint16_t (&b)[4])
    {
        half4_t av, bv;
        for (int i = 0; i < 4; ++i) {
            av[i] = __builtin_bit_cast(_Float16, a[i]);
            bv[i] = __builtin_bit_cast(_Float16, b[i]);
        }
        const float4_t z = {0.f, 0.f, 0.f, 0.f};
        return __builtin_amdgcn_mfma_f32_16x16x16f16(av, bv, z, 0, 0, 0);
    }
};
template <>
struct MfmaOp<FWHT_PREC_BF16_MFMA> {
    __device__ static __forceinline__ float4_t run(const uint16_t (&a)[4], const uint16_t (&b)[4])
    {
        short4_t av, bv;
        for (int i = 0; i < 4; ++i) {
            av[i] = (short)a[i];
            bv[i] = (short)b[i];
        }
        const float4_t z = {0.f, 0.f, 0.f, 0.f};
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, z, 0, 0, 0);
    }
};

template <int PREC>
struct BatchedMfmaKernel {
    static constexpr int MFMA_GROUP = MFMA_GROUP_BLOCKS;
    static constexpr int TB = 16, NT = 1024, E = 64, VEC = 4;
    // f16/bf16 tile with 4 halves of padding per 64 (see transpose_ab)
    static constexpr int LDS_HALFS = (1 << TB) + 4 * ((1 << TB) / 64);
    using Base = BatchedKernel<16, 1024>;  // address, fetch and item helpers

    template <int WHICH>
    __device__ static __forceinline__ uint32_t lane_part(uint32_t lane)
    {
        constexpr XLayout L = WHICH == 0 ? XL_A : WHICH == 1 ? XL_B : XL_C;
        uint32_t r = 0;
#pragma unroll
        for (int q = 0; q < 6; ++q) r |= ((lane >> q) & 1u) << L.lane[q];
        return r;
    }
    template <int WHICH>
    __device__ static __forceinline__ uint32_t wave_part(uint32_t wave)
    {
        constexpr XLayout L = WHICH == 0 ? XL_A : WHICH == 1 ? XL_B : XL_C;
        uint32_t r = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) r |= ((wave >> q) & 1u) << L.wave[q];
        return r;
    }

    // Padding of the 16-bit tile: 4 halves (8 bytes) after every 64.  The
    // four MA values of tile bits 0, 1 stay one aligned 8-byte store, and the
    // 32 words one MB read touches (lanes on tile bits 0, 1, 4, 5, 6, 7) fall
    // in 32 distinct banks: bits 6, 7 shift them by 2 and 4 words.  (Padding
    // by one half per 32 misaligned those stores and gave 3-way conflicts.)
    // The map is linear over disjoint bit sets, so thread and register parts
    // are padded separately and added.
    __device__ static __forceinline__ constexpr uint32_t hpad(uint32_t i) { return i + 4u * (i >> 6); }

    // MA -> MB through LDS in the operand format (see the file comment).
    __device__ static __forceinline__ void transpose_ab(uint16_t *lds, float (&v)[E], uint32_t lane, uint32_t wave)
    {
        const uint32_t ta = hpad(lane_part<0>(lane) | wave_part<0>(wave));
        const uint32_t tb = hpad(lane_part<1>(lane) | wave_part<1>(wave));
        __syncthreads();
        static_for<0, E>([&](auto J) {
            constexpr uint32_t jp = xl_reg_part(XL_A, decltype(J)::value);
            lds[ta + hpad(jp)] = to_half_bits<PREC>(v[decltype(J)::value]);
        });
        __syncthreads();
        static_for<0, E>([&](auto J) {
            constexpr uint32_t jp = xl_reg_part(XL_B, decltype(J)::value);
            v[decltype(J)::value] = from_half_bits(lds[tb + hpad(jp)]);
        });
    }

    // MB -> MC through LDS as FP32, one half (tile bit 11 = register index 5)
    // at a time; the half-tile index drops bit 11.
    __device__ static __forceinline__ uint32_t drop11(uint32_t i) { return (i & 0x7ffu) | ((i >> 1) & ~0x7ffu); }

    // Bank swizzle of the FP32 half tile (no padding): bits 5, 6, 7 of the
    // index are XORed into bits 1; 0 and 2; 3.  An MB store from 32 lanes
    // (tile bits 0, 1, 4, 6, 7) and an MC load from 32 lanes (tile bits 2 .. 6)
    // then each touch 32 distinct banks.  The map is linear over GF(2), so the
    // thread and register parts are swizzled separately and XORed.
    __device__ static __forceinline__ constexpr uint32_t swz(uint32_t q)
    {
        return q ^ (((q >> 5) & 1u) << 1) ^ (((q >> 6) & 1u) * 5u) ^ (((q >> 7) & 1u) << 3);
    }

    __device__ static __forceinline__ void transpose_bc(float *lds, float (&v)[E], uint32_t lane, uint32_t wave)
    {
        const uint32_t tb = swz(drop11(lane_part<1>(lane) | wave_part<1>(wave)));
        const uint32_t tc = swz(drop11(lane_part<2>(lane) | wave_part<2>(wave)));
        static_for<0, 2>([&](auto H0) {
            constexpr int H = decltype(H0)::value;
            __syncthreads();
            static_for<H * (E / 2), (H + 1) * (E / 2)>([&](auto J) {
                constexpr uint32_t jp = xl_reg_part(XL_B, decltype(J)::value);
                lds[tb ^ swz(drop11(jp))] = v[decltype(J)::value];
            });
            __syncthreads();
            static_for<H * (E / 2), (H + 1) * (E / 2)>([&](auto J) {
                constexpr uint32_t jp = xl_reg_part(XL_C, decltype(J)::value);
                v[decltype(J)::value] = lds[tc ^ swz(drop11(jp))];
            });
        });
    }

    __device__ static __forceinline__ float from_half_bits(uint16_t h)
    {
        if constexpr (PREC == FWHT_PREC_FP16_MFMA) return (float)__builtin_bit_cast(_Float16, h);
        else return __builtin_bit_cast(float, (uint32_t)h << 16);
    }

    // FP32 butterflies on register indices Q0..Q1-1 of the layout whose tile
    // bits are below MM.
    template <int WHICH, int Q0, int Q1, int MM>
    __device__ static __forceinline__ void valu_stages(float (&v)[E])
    {
        constexpr XLayout L = WHICH == 0 ? XL_A : WHICH == 1 ? XL_B : XL_C;
        static_for<Q0, Q1>([&](auto Q) {
            constexpr int q = decltype(Q)::value;
            if constexpr (L.reg[q] < MM) {
#pragma unroll
                for (int j = 0; j < E; ++j)
                    if (!((j >> q) & 1)) bfly(v[j], v[j | (1 << q)]);
            }
        });
    }

    // One MFMA stage over K = {register 0, register 1, lane 4, lane 5}:
    // A[m][k] = prod over the four bits b of (b < MM ? H_2[m_b][k_b] : [m_b == k_b]),
    // scaled by 2^-ceil(a/2) for a active bits (exact).  Returns ceil(a/2).
    template <int WHICH, int MM>
    __device__ static __forceinline__ int mfma_stage(float (&v)[E], uint32_t lane)
    {
        constexpr XLayout L = WHICH == 0 ? XL_A : WHICH == 1 ? XL_B : XL_C;
        constexpr uint32_t kb = (L.reg[0] < MM ? 1u : 0u) | (L.reg[1] < MM ? 2u : 0u) |
                                (L.lane[4] < MM ? 4u : 0u) | (L.lane[5] < MM ? 8u : 0u);
        constexpr int na = cpopc(kb);
        if constexpr (na == 0) {
            return 0;
        } else {
            constexpr int sh = (na + 1) / 2;
            // A operand: lane holds A[m = lane mod 16][k = 4 (lane div 16) + i].
            const uint32_t mrow = lane & 15u;
            const float sc = 1.0f / (float)(1u << sh);
            uint16_t a[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t k = 4u * (lane >> 4) + (uint32_t)i;
                float val = sc;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint32_t mb = (mrow >> b) & 1u, kk = (k >> b) & 1u;
                    if ((kb >> b) & 1u) {
                        if (mb & kk) val = -val;
                    } else if (mb != kk) {
                        val = 0.f;
                    }
                }
                a[i] = to_half_bits<PREC>(val);
            }
            // E/4 independent 16x16 blocks: register indices 2 and up.  A
            // scheduling fence after every MFMA_GROUP blocks bounds the
            // operands in flight while letting that many products overlap.
#pragma unroll
            for (int blk = 0; blk < E / 4; ++blk) {
                uint16_t b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) b[i] = to_half_bits<PREC>(v[(blk << 2) | i]);
                const float4_t d = MfmaOp<PREC>::run(a, b);
#pragma unroll
                for (int i = 0; i < 4; ++i) v[(blk << 2) | i] = d[i];
                if ((blk % MFMA_GROUP) == MFMA_GROUP - 1) __builtin_amdgcn_sched_barrier(0);
            }
            return sh;
        }
    }

    template <int MM>
    __device__ static __forceinline__ void load(const BArgs &a, const BItem &I, float (&v)[E], uint32_t lane,
                                                uint32_t wave)
    {
        constexpr uint32_t LM = xl_lane_mask(XL_A);
        const uint32_t lp = lane_part<0>(lane), wp = wave_part<0>(wave);
        // all loads first, the empty slots zeroed after every load has been
        // issued (as in the FP32 kernel)
        uint32_t okm = 0;
        static_for<0, E / VEC>([&](auto JT) {
            constexpr int jt = decltype(JT)::value;
            constexpr uint32_t jp = xl_reg_part(XL_A, (uint32_t)(jt << 2));
            bool ok;
            const float *p = Base::template addr<MM, LM>(a, I, jp, wp, lp, ok);
            const v4u q = *reinterpret_cast<const v4u *>(p);
            okm |= (uint32_t)ok << jt;
            const float *qs = reinterpret_cast<const float *>(&q);
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[jt * VEC + e] = qs[e];
        });
        __builtin_amdgcn_sched_barrier(0);
        static_for<0, E / VEC>([&](auto JT) {
            constexpr int jt = decltype(JT)::value;
            if (!((okm >> jt) & 1u)) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[jt * VEC + e] = 0.f;
            }
        });
    }

    // 16-byte stores from a layout whose register indices 0, 1 are tile bits
    // 0, 1 (MA or MC).
    template <int WHICH, int MM>
    __device__ static __forceinline__ void store_vec(const BArgs &a, const BItem &I, const float (&v)[E],
                                                     uint32_t lane, uint32_t wave)
    {
        constexpr XLayout L = WHICH == 0 ? XL_A : WHICH == 1 ? XL_B : XL_C;
        static_assert(L.reg[0] == 0 && L.reg[1] == 1, "vector layout");
        constexpr uint32_t LM = xl_lane_mask(L);
        const uint32_t lp = lane_part<WHICH>(lane), wp = wave_part<WHICH>(wave);
        static_for<0, E / VEC>([&](auto JT) {
            constexpr int jt = decltype(JT)::value;
            constexpr uint32_t jp = xl_reg_part(L, (uint32_t)(jt << 2));
            bool ok;
            float *p = Base::template addr<MM, LM>(a, I, jp, wp, lp, ok);
            v4u q;
            float *qs = reinterpret_cast<float *>(&q);
#pragma unroll
            for (int e = 0; e < VEC; ++e) qs[e] = v[jt * VEC + e];
            if (ok) *reinterpret_cast<v4u *>(p) = q;
        });
    }

    template <int WHICH, int MM>
    __device__ static __forceinline__ void store(const BArgs &a, const BItem &I, const float (&v)[E], uint32_t lane,
                                                 uint32_t wave)
    {
        constexpr XLayout L = WHICH == 0 ? XL_A : WHICH == 1 ? XL_B : XL_C;
        constexpr uint32_t LM = xl_lane_mask(L);
        const uint32_t lp = lane_part<WHICH>(lane), wp = wave_part<WHICH>(wave);
        static_for<0, E>([&](auto J) {
            constexpr int j = decltype(J)::value;
            constexpr uint32_t jp = xl_reg_part(L, (uint32_t)j);
            bool ok;
            float *p = Base::template addr<MM, LM>(a, I, jp, wp, lp, ok);
            if (ok) *p = v[j];
        });
    }

    template <int MM>
    __device__ static __forceinline__ void item(const BArgs &a, const BItem &I, uint16_t *lds, uint32_t t)
    {
        const uint32_t lane = t & 63u;
        const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);
        float v[E];
        load<MM>(a, I, v, lane, wave);
        int shift = mfma_stage<0, MM>(v, lane);
        valu_stages<0, 2, 6, MM>(v);
        constexpr bool needB = MM > 2;  // MB owns bits 2..5 and 8..11
        if constexpr (needB) {
            transpose_ab(lds, v, lane, wave);
            shift += mfma_stage<1, MM>(v, lane);
            valu_stages<1, 2, 6, MM>(v);
        }
        // Undo the stage scales; 2^(-m/2) when normalising.
        float sc = (float)(1u << shift);
        // an opaque copy of the flag, so that the scale of every size is not
        // precomputed for the whole persistent loop (15 live registers)
        int32_t nz = a.normalize;
        asm volatile("" : "+s"(nz));
        if (nz) sc *= (float)(1.0 / sqrt((double)(1ull << MM)));
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] *= sc;
        // Opaque copies of the thread coordinates: the store addresses are
        // then recomputed here instead of being kept live (and spilled) from
        // the loads.
        uint32_t slane = lane, swave = wave;
        asm volatile("" : "+v"(slane));
        asm volatile("" : "+s"(swave));
        if constexpr (needB) {
            transpose_bc(reinterpret_cast<float *>(lds), v, slane, swave);
            store_vec<2, MM>(a, I, v, slane, swave);
        } else {
            store_vec<0, MM>(a, I, v, slane, swave);
        }
    }

    __device__ static __forceinline__ void run(const BArgs &a)
    {
        __shared__ uint16_t lds[LDS_HALFS];
        const uint32_t t = threadIdx.x;
        // static cyclic assignment; each transpose starts with a barrier
        for (int32_t it = blockIdx.x; it < a.nitems; it += gridDim.x) {
            const BItem I = Base::read_item(a, it);
            // An opaque copy of the thread id per item: the per-layout lane,
            // wave and LDS offsets derived from it are recomputed for each
            // item rather than hoisted out of the loop and kept live.
            uint32_t tt = t;
            asm volatile("" : "+v"(tt));
            static_for<2, TB + 1>([&](auto M0) {
                constexpr int MM = decltype(M0)::value;
                if (I.m == MM) item<MM>(a, I, lds, tt);
            });
        }
    }
};

template <int PREC>
__global__ void __launch_bounds__(1024, 1) batched_mfma_kernel(BArgs a)
{
    BatchedMfmaKernel<PREC>::run(a);
}

}  // namespace fwht
