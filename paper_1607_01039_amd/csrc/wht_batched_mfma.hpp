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
// Tile of 2^14 entries, 512 threads, 32 entries per thread, two layouts:
//   MA (load/store): registers {0,1,11,12,13}, lanes {2..7}, waves {8,9,10};
//        MFMA on {0,1,6,7} (registers 0,1 + lanes 4,5), VALU on {11,12,13}.
//   MB: registers {2,3,8,9,10}, lanes {0,1,6,7,4,5}, waves {11,12,13};
//        MFMA on {2,3,4,5} (registers 2,3 + lanes 4,5), VALU on {8,9,10}.
// The remaining bits are FP32 VALU butterflies, as in the FP32 kernel.
#pragma once
#include "wht_batched.hpp"

namespace fwht {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

struct XLayout {
    int reg[5];
    int lane[6];
    int wave[3];
};

constexpr XLayout XL_A{{0, 1, 11, 12, 13}, {2, 3, 4, 5, 6, 7}, {8, 9, 10}};
constexpr XLayout XL_B{{2, 3, 8, 9, 10}, {0, 1, 6, 7, 4, 5}, {11, 12, 13}};

constexpr uint32_t xl_reg_part(const XLayout &L, uint32_t j)
{
    uint32_t r = 0;
    for (int q = 0; q < 5; ++q)
        if ((j >> q) & 1u) r |= 1u << L.reg[q];
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
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
    return (uint16_t)(u >> 16);
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
    static constexpr int TB = 14, NT = 512, E = 32, VEC = 4;
    static constexpr uint32_t FULL = lowmask(TB);
    static constexpr int LDS_ELEMS = (1 << TB) + (1 << TB) / 32;
    using Base = BatchedKernel<14, 512, FWHT_PREC_FP32>;  // address helpers

    // Thread part of the tile index in layout WHICH.
    template <int WHICH>
    __device__ static __forceinline__ uint32_t tpart(uint32_t t)
    {
        constexpr XLayout L = WHICH == 0 ? XL_A : XL_B;
        uint32_t r = 0;
#pragma unroll
        for (int q = 0; q < 6; ++q) r |= ((t >> q) & 1u) << L.lane[q];
#pragma unroll
        for (int q = 0; q < 3; ++q) r |= ((t >> (6 + q)) & 1u) << L.wave[q];
        return r;
    }

    template <int WHICH>
    __device__ static __forceinline__ void to_lds(float *lds, const float (&v)[E], uint32_t t)
    {
        constexpr XLayout L = WHICH == 0 ? XL_A : XL_B;
        const uint32_t tb = lds_pad(tpart<WHICH>(t));
        static_for<0, E>([&](auto J) {
            constexpr uint32_t jp = xl_reg_part(L, decltype(J)::value);
            lds[tb + jp + (jp >> 5)] = v[decltype(J)::value];
        });
    }

    template <int WHICH>
    __device__ static __forceinline__ void from_lds(const float *lds, float (&v)[E], uint32_t t)
    {
        constexpr XLayout L = WHICH == 0 ? XL_A : XL_B;
        const uint32_t tb = lds_pad(tpart<WHICH>(t));
        static_for<0, E>([&](auto J) {
            constexpr uint32_t jp = xl_reg_part(L, decltype(J)::value);
            v[decltype(J)::value] = lds[tb + jp + (jp >> 5)];
        });
    }

    // FP32 butterflies on register bits q = 2, 3, 4 of the layout that `act`
    // selects (tile bits L.reg[2..4]).
    template <int WHICH>
    __device__ static __forceinline__ void valu_stages(float (&v)[E], uint32_t act)
    {
        constexpr XLayout L = WHICH == 0 ? XL_A : XL_B;
        static_for<2, 5>([&](auto Q) {
            constexpr int q = decltype(Q)::value;
            if ((act >> L.reg[q]) & 1u) {
#pragma unroll
                for (int j = 0; j < E; ++j)
                    if (!((j >> q) & 1)) bfly(v[j], v[j | (1 << q)]);
            }
        });
    }

    // One MFMA stage over K = {reg 0, reg 1, lane 4, lane 5} of the layout:
    // A[m][k] = prod over the four bits b of (act_b ? H_2[m_b][k_b] : [m_b == k_b]),
    // times 2^-ceil(a/2) for a active bits (exact).  Returns the number of
    // active bits (0: nothing done).
    template <int WHICH>
    __device__ static __forceinline__ int mfma_stage(float (&v)[E], uint32_t act, uint32_t lane)
    {
        constexpr XLayout L = WHICH == 0 ? XL_A : XL_B;
        const uint32_t kb = ((act >> L.reg[0]) & 1u) | (((act >> L.reg[1]) & 1u) << 1) |
                            (((act >> L.lane[4]) & 1u) << 2) | (((act >> L.lane[5]) & 1u) << 3);
        const int na = __builtin_popcount(kb);
        if (na == 0) return 0;
        // A operand: lane holds A[m = lane mod 16][k = 4 (lane div 16) + i].
        const uint32_t mrow = lane & 15u;
        const float sc = 1.0f / (float)(1u << ((na + 1) / 2));
        uint16_t a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t k = 4u * (lane >> 4) + (uint32_t)i;
            float val = sc;
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
        // Eight independent 16x16 blocks: register bits 2, 3, 4.
#pragma unroll
        for (int blk = 0; blk < 8; ++blk) {
            uint16_t b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) b[i] = to_half_bits<PREC>(v[(blk << 2) | i]);
            const float4_t d = MfmaOp<PREC>::run(a, b);
#pragma unroll
            for (int i = 0; i < 4; ++i) v[(blk << 2) | i] = d[i];
        }
        return na;
    }

    template <int KIND>
    __device__ static __forceinline__ void load(const BArgs &a, const BItem &I, float (&v)[E], uint32_t t)
    {
        const uint32_t tp = tpart<0>(t);
        static_for<0, E / VEC>([&](auto JT) {
            constexpr int jt = decltype(JT)::value;
            constexpr uint32_t jp = xl_reg_part(XL_A, (uint32_t)(jt << 2));
            const int64_t off = Base::template addr<KIND>(I, a.segs, jp | tp);
            v4u q = {0u, 0u, 0u, 0u};
            if (off >= 0) q = *reinterpret_cast<const v4u *>(a.data + off);
            const float *qs = reinterpret_cast<const float *>(&q);
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[jt * VEC + e] = qs[e];
        });
    }

    template <int KIND>
    __device__ static __forceinline__ void store(const BArgs &a, const BItem &I, const float (&v)[E], uint32_t t)
    {
        const uint32_t tp = tpart<0>(t);
        static_for<0, E / VEC>([&](auto JT) {
            constexpr int jt = decltype(JT)::value;
            constexpr uint32_t jp = xl_reg_part(XL_A, (uint32_t)(jt << 2));
            const int64_t off = Base::template addr<KIND>(I, a.segs, jp | tp);
            v4u q;
            float *qs = reinterpret_cast<float *>(&q);
#pragma unroll
            for (int e = 0; e < VEC; ++e) qs[e] = v[jt * VEC + e];
            if (off >= 0) *reinterpret_cast<v4u *>(a.data + off) = q;
        });
    }

    template <int KIND>
    __device__ static __forceinline__ void item(const BArgs &a, const BItem &I, float *lds, uint32_t t)
    {
        uint32_t act;
        if constexpr (KIND == BK_TILE) act = lowmask(I.m);
        else if constexpr (KIND == BK_STEP1) act = FULL;
        else act = lowmask(I.m - TB) << (2 * TB - I.m);
        const uint32_t lane = t & 63u;
        float v[E];
        load<KIND>(a, I, v, t);
        // scale bookkeeping: the MFMA stages multiply by 2^-ceil(a/2) each
        int shift = mfma_stage<0>(v, act, lane);
        shift = (shift + 1) / 2;
        valu_stages<0>(v, act);
        constexpr uint32_t BBITS = (1u << 2) | (1u << 3) | (1u << 4) | (1u << 5) | (1u << 8) | (1u << 9) | (1u << 10);
        if (act & BBITS) {
            __syncthreads();
            to_lds<0>(lds, v, t);
            __syncthreads();
            from_lds<1>(lds, v, t);
            const int nb = mfma_stage<1>(v, act, lane);
            shift += (nb + 1) / 2;
            valu_stages<1>(v, act);
            __syncthreads();
            to_lds<1>(lds, v, t);
            __syncthreads();
            from_lds<0>(lds, v, t);
        }
        // Undo the stage scales; apply 2^(-m/2) on the last step.
        float sc = (float)(1u << shift);
        if (a.normalize && KIND != BK_STEP1) sc *= (float)(1.0 / sqrt((double)(1ull << I.m)));
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] *= sc;
        store<KIND>(a, I, v, t);
    }

    __device__ static __forceinline__ void run(const BArgs &a)
    {
        __shared__ float lds[LDS_ELEMS];
        __shared__ int32_t s_item;
        const uint32_t t = threadIdx.x;
        for (int32_t it = Base::fetch(a, &s_item, t); it < a.nitems; it = Base::fetch(a, &s_item, t)) {
            BItem I = a.items[it];
            I.kind = __builtin_amdgcn_readfirstlane(I.kind);
            I.m = __builtin_amdgcn_readfirstlane(I.m);
            I.sub = __builtin_amdgcn_readfirstlane(I.sub);
            I.tid = __builtin_amdgcn_readfirstlane(I.tid);
            I.seg0 = __builtin_amdgcn_readfirstlane(I.seg0);
            I.nseg = __builtin_amdgcn_readfirstlane(I.nseg);
            if (I.kind == BK_STEP2) {
                if (__builtin_amdgcn_readfirstlane(t >> 6) == 0) {
                    const int32_t need = 1 << (I.m - TB);
                    for (uint32_t spins = 0;; ++spins) {
                        const int32_t c = __builtin_amdgcn_readfirstlane(
                            __hip_atomic_load(&a.done[I.tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                        if (c >= need) break;
                        if (spins > (1u << 26)) {
                            if (t == 0) atomicExch(a.err, 1);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
                __syncthreads();
                __threadfence();
            }
            if (I.kind == BK_TILE) item<BK_TILE>(a, I, lds, t);
            else if (I.kind == BK_STEP1) item<BK_STEP1>(a, I, lds, t);
            else item<BK_STEP2>(a, I, lds, t);
            __syncthreads();  // LDS reuse by the next item
            if (I.kind == BK_STEP1) {
                __threadfence();
                __syncthreads();
                if (t == 0) atomicAdd(&a.done[I.tid], 1);
            }
        }
    }
};

template <int PREC>
__global__ void __launch_bounds__(512, 2) batched_mfma_kernel(BArgs a)
{
    BatchedMfmaKernel<PREC>::run(a);
}

}  // namespace fwht
