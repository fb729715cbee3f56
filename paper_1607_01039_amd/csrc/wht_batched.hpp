// wht_batched.hpp -- persistent kernel for many independent transforms of
// uneven sizes (2^2 .. 2^16 entries each) in one launch.
//
// Work comes from a host-built list of items, handed out through one atomic
// counter in list order (largest work first, as the equal-load principle of
// section 3 asks for sub-tasks of equal size):
//   TILE   2^(TB-m) transforms of one size 2^m <= 2^TB gathered into one tile
//          of 2^TB entries; all m bits of each are transformed in the tile.
//   STEP1  a contiguous 2^TB-entry chunk of a transform with m > TB: its low
//          TB bits.
//   STEP2  the remaining m - TB <= 2 high bits of such a transform, over a
//          tile of 2^(m-TB) rows x 2^(2TB-m) columns, after all STEP1 chunks
//          of that transform have been published.
// Every STEP1 item precedes every STEP2 item in the list, so a block that
// takes a STEP2 item only ever waits on items already taken by running
// blocks, which never wait themselves: the wait always ends.
#pragma once
#include "wht_tile.hpp"

namespace fwht {

enum : int32_t { BK_TILE = 0, BK_STEP1 = 1, BK_STEP2 = 2 };

struct BItem {
    int64_t off;   // STEP1/STEP2: first entry of the transform
    int32_t kind;
    int32_t m;     // transform size 2^m
    int32_t sub;   // STEP1: chunk index; STEP2: column block
    int32_t tid;   // STEP1/STEP2: completion-counter index
    int32_t seg0;  // TILE: first entry in the segment table
    int32_t nseg;  // TILE: number of transforms in the tile
};

struct BArgs {
    float *data;
    const BItem *items;
    const int64_t *segs;
    int32_t nitems;
    int32_t normalize;
    int32_t *queue;  // [1] next item
    int32_t *done;   // [ntid] published STEP1 chunks per transform
    int32_t *err;    // [1] set when a wait exceeds its bound
};

template <int TB, int NT, int PREC>
struct BatchedKernel {
    using S = float;
    static constexpr int E = (1 << TB) / NT;
    static constexpr int K = clog2(E);
    static constexpr int VEC = 4;
    static constexpr int VB = 2;
    static constexpr LayoutList LS = make_layouts(TB, 6, K, VB, true);
    static constexpr uint32_t FULL = lowmask(TB);
    static constexpr int LDS_ELEMS = (1 << TB) + (1 << TB) / 32;
    static_assert(LS.n <= 8, "too many layouts");

    // Global entry offset of tile index idx for item I; -1 when masked.
    template <int KIND>
    __device__ static __forceinline__ int64_t addr(const BItem &I, const int64_t *__restrict__ segs, uint32_t idx)
    {
        if constexpr (KIND == BK_TILE) {
            const uint32_t q = idx >> I.m;
            if ((int32_t)q >= I.nseg) return -1;
            return segs[I.seg0 + q] + (idx & lowmask(I.m));
        }
        if constexpr (KIND == BK_STEP1) return I.off + ((int64_t)I.sub << TB) + idx;
        const int r2 = I.m - TB;
        const uint32_t row = idx >> (TB - r2), col = idx & lowmask(TB - r2);
        return I.off + ((int64_t)row << TB) + ((int64_t)I.sub << (TB - r2)) + col;
    }

    template <int P>
    __device__ static __forceinline__ void to_lds(S *lds, const S (&v)[E], uint32_t t)
    {
        constexpr uint32_t M = LS.m[P];
        const uint32_t tb = lds_pad(pdep_rt<FULL & ~M>(t));
        static_for<0, E>([&](auto J) {
            constexpr uint32_t jp = cpdep((uint32_t)decltype(J)::value, M);
            lds[tb + jp + (jp >> 5)] = v[decltype(J)::value];
        });
    }

    template <int P>
    __device__ static __forceinline__ void from_lds(const S *lds, S (&v)[E], uint32_t t)
    {
        constexpr uint32_t M = LS.m[P];
        const uint32_t tb = lds_pad(pdep_rt<FULL & ~M>(t));
        static_for<0, E>([&](auto J) {
            constexpr uint32_t jp = cpdep((uint32_t)decltype(J)::value, M);
            v[decltype(J)::value] = lds[tb + jp + (jp >> 5)];
        });
    }

    __device__ static __forceinline__ void dispatch_to_lds(S *lds, const S (&v)[E], uint32_t t, int p)
    {
        static_for<0, LS.n>([&](auto PP) {
            constexpr int P = decltype(PP)::value;
            if (P == p) to_lds<P>(lds, v, t);
        });
    }

    // Load / store in layout L0 (16-byte accesses of 4 consecutive entries,
    // which always lie in one segment or row).
    template <int KIND>
    __device__ static __forceinline__ void load0(const BArgs &a, const BItem &I, S (&v)[E], uint32_t t)
    {
        constexpr uint32_t M0 = LS.m[0];
        const uint32_t tp = pdep_rt<FULL & ~M0>(t);
        static_for<0, E / VEC>([&](auto JT) {
            constexpr int jt = decltype(JT)::value;
            constexpr uint32_t jp = cpdep((uint32_t)(jt << VB), M0);
            const int64_t off = addr<KIND>(I, a.segs, jp | tp);
            v4u q = {0u, 0u, 0u, 0u};
            if (off >= 0) q = *reinterpret_cast<const v4u *>(a.data + off);
            const S *qs = reinterpret_cast<const S *>(&q);
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[jt * VEC + e] = qs[e];
        });
    }

    template <int P, int KIND>
    __device__ static __forceinline__ void store_layout(const BArgs &a, const BItem &I, const S (&v)[E], uint32_t t)
    {
        constexpr uint32_t M = LS.m[P];
        const uint32_t tp = pdep_rt<FULL & ~M>(t);
        if constexpr (P == 0) {
            static_for<0, E / VEC>([&](auto JT) {
                constexpr int jt = decltype(JT)::value;
                constexpr uint32_t jp = cpdep((uint32_t)(jt << VB), M);
                const int64_t off = addr<KIND>(I, a.segs, jp | tp);
                v4u q;
                S *qs = reinterpret_cast<S *>(&q);
#pragma unroll
                for (int e = 0; e < VEC; ++e) qs[e] = v[jt * VEC + e];
                if (off >= 0) *reinterpret_cast<v4u *>(a.data + off) = q;
            });
        } else {
            static_for<0, E>([&](auto J) {
                constexpr int j = decltype(J)::value;
                constexpr uint32_t jp = cpdep((uint32_t)j, M);
                const int64_t off = addr<KIND>(I, a.segs, jp | tp);
                if (off >= 0) a.data[off] = v[j];
            });
        }
    }

    template <int KIND>
    __device__ static __forceinline__ void dispatch_store(const BArgs &a, const BItem &I, const S (&v)[E],
                                                          uint32_t t, int p)
    {
        static_for<0, LS.n>([&](auto PP) {
            constexpr int P = decltype(PP)::value;
            if constexpr (P == 0 || lanes_contiguous(LS.m[P], 6)) {
                if (P == p) store_layout<P, KIND>(a, I, v, t);
            }
        });
    }

    __device__ static __forceinline__ bool store_ok(int p)
    {
        bool ok = false;
        static_for<0, LS.n>([&](auto PP) {
            constexpr int P = decltype(PP)::value;
            if (P == p) ok = P == 0 || lanes_contiguous(LS.m[P], 6);
        });
        return ok;
    }

    // One item: transform the `act` bits of the tile, scale when it is the
    // last step of its transforms, store.
    template <int KIND>
    __device__ static __forceinline__ void item(const BArgs &a, const BItem &I, S *lds, uint32_t t)
    {
        uint32_t act;
        if constexpr (KIND == BK_TILE) act = lowmask(I.m);
        else if constexpr (KIND == BK_STEP1) act = FULL;
        else act = lowmask(I.m - TB) << (2 * TB - I.m);
        S v[E];
        load0<KIND>(a, I, v, t);
        reg_stages<S, LS.m[0], LS.fresh[0], E>(v, act);
        int cur = 0;
        bool wrote = false;
        static_for<1, LS.n>([&](auto PP) {
            constexpr int P = decltype(PP)::value;
            if (act & LS.fresh[P]) {
                if (wrote) __syncthreads();
                dispatch_to_lds(lds, v, t, cur);
                __syncthreads();
                from_lds<P>(lds, v, t);
                wrote = true;
                cur = P;
                reg_stages<S, LS.m[P], LS.fresh[P], E>(v, act);
            }
        });
        if (!store_ok(cur)) {
            __syncthreads();
            dispatch_to_lds(lds, v, t, cur);
            __syncthreads();
            from_lds<0>(lds, v, t);
            cur = 0;
            wrote = true;
        }
        if (a.normalize && KIND != BK_STEP1) {
            const float sc = (float)(1.0 / sqrt((double)(1ull << I.m)));
#pragma unroll
            for (int j = 0; j < E; ++j) v[j] *= sc;
        }
        dispatch_store<KIND>(a, I, v, t, cur);
        if (wrote) __syncthreads();
    }

    // Next item index for the whole block (uniform: it steers branches that
    // contain barriers, so it travels through a scalar register).
    __device__ static __forceinline__ int32_t fetch(const BArgs &a, int32_t *s_item, uint32_t t)
    {
        if (t == 0) *s_item = atomicAdd(a.queue, 1);
        __syncthreads();
        const int32_t it = __builtin_amdgcn_readfirstlane(*s_item);
        __syncthreads();
        return it;
    }

    __device__ static __forceinline__ void run(const BArgs &a)
    {
        __shared__ S lds[LDS_ELEMS];
        __shared__ int32_t s_item;
        const uint32_t t = threadIdx.x;
        for (int32_t it = fetch(a, &s_item, t); it < a.nitems; it = fetch(a, &s_item, t)) {
            BItem I = a.items[it];
            I.kind = __builtin_amdgcn_readfirstlane(I.kind);
            I.m = __builtin_amdgcn_readfirstlane(I.m);
            I.sub = __builtin_amdgcn_readfirstlane(I.sub);
            I.tid = __builtin_amdgcn_readfirstlane(I.tid);
            I.seg0 = __builtin_amdgcn_readfirstlane(I.seg0);
            I.nseg = __builtin_amdgcn_readfirstlane(I.nseg);
            if (I.kind == BK_STEP2) {
                if (__builtin_amdgcn_readfirstlane(t >> 6) == 0) {
                    // Wave 0 waits (every lane, uniform control flow).
                    // Bounded: the producers were handed out earlier and
                    // never wait, so this ends; the bound only guards
                    // against a broken work list.
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
                __threadfence();  // acquire: see the STEP1 results of other CUs
            }
            if (I.kind == BK_TILE) item<BK_TILE>(a, I, lds, t);
            else if (I.kind == BK_STEP1) item<BK_STEP1>(a, I, lds, t);
            else item<BK_STEP2>(a, I, lds, t);
            if (I.kind == BK_STEP1) {
                __threadfence();  // release this thread's stores
                __syncthreads();
                if (t == 0) atomicAdd(&a.done[I.tid], 1);
            }
        }
    }
};

template <int TB, int NT, int PREC>
__global__ void __launch_bounds__(NT, 2) batched_kernel(BArgs a)
{
    BatchedKernel<TB, NT, PREC>::run(a);
}

}  // namespace fwht
