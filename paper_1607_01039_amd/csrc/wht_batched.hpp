// wht_batched.hpp -- persistent kernel for many independent transforms of
// uneven sizes (2^2 .. 2^16 entries each) in one launch.
//
// Work comes from a host-built list of tiles, largest transforms first.  A
// tile is 2^16 entries: the entries of 2^(16-m) transforms of one size 2^m,
// gathered from their own offsets, so every tile costs about the same and a
// static cyclic assignment (workgroup g takes tiles g, g + G, g + 2G, ...)
// balances the load (the equal-load principle of section 3) without a shared
// counter.  One workgroup transforms a whole tile, so no tile ever waits for
// another one: there is no communication between workgroups at all.
//
// The tile lives in registers (1024 threads x 64 entries).  Between layouts
// it is transposed through LDS in two halves: the top tile bit stays a
// register bit in every layout ("pinned"), so each half of every thread's
// registers goes to, and comes back from, one half of the tile.
#pragma once
#include "wht_tile.hpp"

namespace fwht {

struct BItem {
    int32_t m;     // transform size 2^m
    int32_t seg0;  // first entry in the segment table
    int32_t nseg;  // number of transforms gathered in this tile
    int32_t pad;
};

struct BArgs {
    float *data;
    const BItem *items;
    const int64_t *segs;
    int32_t nitems;
    int32_t normalize;
};

// The work list and the segment table are read-only during a launch; reading
// them through the constant address space lets the compiler use scalar loads
// for wave-uniform indices (vector loads, each waited for before the data
// access that needs its result, serialised the per-item address arithmetic).
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *as_const(const T *p)
{
    return (const __attribute__((address_space(4))) T *)p;
}

template <int TB, int NT>
struct BatchedKernel {
    using S = float;
    static constexpr int E = (1 << TB) / NT;
    static constexpr int K = clog2(E);
    static constexpr int VEC = 4;
    static constexpr int VB = 2;
    static constexpr LayoutList LS = make_pinned_layouts(TB, K, VB);
    static constexpr uint32_t FULL = lowmask(TB);
    static constexpr uint32_t HALF = lowmask(TB - 1);
    static constexpr int LDS_ELEMS = (1 << (TB - 1)) + (1 << (TB - 1)) / 32;
    static_assert(LS.n <= 8, "too many layouts");

    // Entry of tile index idx = (register part jp) | (wave part wp) | (lane
    // part lp) for transforms of size 2^MM.  `ok` is false for an empty slot
    // (past the tile's last transform); the pointer is then an entry of the
    // tile's first transform, so that it is always safe to load (the caller
    // discards the value) and the address needs no branch: the segment-table
    // reads of neighbouring entries stay shared.  When every lane bit lies
    // below MM the segment (and so the base address) is uniform.
    template <int MM, uint32_t LANEMASK>
    __device__ static __forceinline__ S *addr(const BArgs &a, const BItem &I, uint32_t jp, uint32_t wp, uint32_t lp,
                                              bool &ok)
    {
        if constexpr ((LANEMASK >> MM) == 0) {
            const uint32_t q = (jp | wp) >> MM;  // uniform: wp comes from the wave id
            ok = (int32_t)q < I.nseg;
            const uint32_t qc = ok ? q : 0u;
            return a.data + as_const(a.segs)[I.seg0 + qc] + ((jp | wp) & lowmask(MM)) + lp;
        } else {
            const uint32_t idx = jp | wp | lp;
            const uint32_t q = idx >> MM;
            ok = (int32_t)q < I.nseg;
            const uint32_t qc = ok ? q : 0u;
            return a.data + a.segs[I.seg0 + qc] + (idx & lowmask(MM));
        }
    }

    template <int P>
    struct Split {
        static constexpr uint32_t TM = FULL & ~LS.m[P];
        static constexpr uint32_t LANE = low_set_bits(TM, 6);
        static constexpr uint32_t WAVE = TM & ~LANE;
    };

    // Half H of the registers of layout P to LDS, or back.
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

    // Layout FROM -> layout TO through LDS, one half of the tile at a time.
    template <int FROM, int TO>
    __device__ static __forceinline__ void transpose(S *lds, S (&v)[E], uint32_t t)
    {
        static_assert((LS.m[FROM] >> (TB - 1)) & 1u, "pinned bit");
        static_assert((LS.m[TO] >> (TB - 1)) & 1u, "pinned bit");
        __syncthreads();
        to_lds<FROM, 0>(lds, v, t);
        __syncthreads();
        from_lds<TO, 0>(lds, v, t);
        __syncthreads();
        to_lds<FROM, 1>(lds, v, t);
        __syncthreads();
        from_lds<TO, 1>(lds, v, t);
    }

    __device__ static __forceinline__ void dispatch_transpose(S *lds, S (&v)[E], uint32_t t, int from, int to)
    {
        static_for<0, LS.n>([&](auto F0) {
            constexpr int FR = decltype(F0)::value;
            static_for<0, LS.n>([&](auto T0) {
                constexpr int TO = decltype(T0)::value;
                if constexpr (FR != TO) {
                    if (FR == from && TO == to) transpose<FR, TO>(lds, v, t);
                }
            });
        });
    }

    template <int MM>
    __device__ static __forceinline__ void load0(const BArgs &a, const BItem &I, S (&v)[E], uint32_t lane,
                                                 uint32_t wave)
    {
        constexpr uint32_t M0 = LS.m[0];
        const uint32_t lp = pdep_rt<Split<0>::LANE>(lane);
        const uint32_t wp = pdep_rt<Split<0>::WAVE>(wave);
        // all loads first, the empty slots zeroed only after every load has
        // been issued (see the scheduling barrier in item())
        uint32_t okm = 0;
        static_for<0, E / VEC>([&](auto JT) {
            constexpr int jt = decltype(JT)::value;
            constexpr uint32_t jp = cpdep((uint32_t)(jt << VB), M0);
            bool ok;
            const S *p = addr<MM, Split<0>::LANE>(a, I, jp, wp, lp, ok);
            const v4u q = *reinterpret_cast<const v4u *>(p);
            okm |= (uint32_t)ok << jt;
            const S *qs = reinterpret_cast<const S *>(&q);
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[jt * VEC + e] = qs[e];
        });
        __builtin_amdgcn_sched_barrier(0);
        static_for<0, E / VEC>([&](auto JT) {
            constexpr int jt = decltype(JT)::value;
            if (!((okm >> jt) & 1u)) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[jt * VEC + e] = S(0);
            }
        });
    }

    template <int P, int MM>
    __device__ static __forceinline__ void store_layout(const BArgs &a, const BItem &I, const S (&v)[E],
                                                        uint32_t lane, uint32_t wave)
    {
        constexpr uint32_t M = LS.m[P];
        const uint32_t lp = pdep_rt<Split<P>::LANE>(lane);
        const uint32_t wp = pdep_rt<Split<P>::WAVE>(wave);
        if constexpr (P == 0) {
            static_for<0, E / VEC>([&](auto JT) {
                constexpr int jt = decltype(JT)::value;
                constexpr uint32_t jp = cpdep((uint32_t)(jt << VB), M);
                bool ok;
                S *p = addr<MM, Split<0>::LANE>(a, I, jp, wp, lp, ok);
                v4u q;
                S *qs = reinterpret_cast<S *>(&q);
#pragma unroll
                for (int e = 0; e < VEC; ++e) qs[e] = v[jt * VEC + e];
                if (ok) *reinterpret_cast<v4u *>(p) = q;
            });
        } else {
            static_for<0, E>([&](auto J) {
                constexpr int j = decltype(J)::value;
                constexpr uint32_t jp = cpdep((uint32_t)j, M);
                bool ok;
                S *p = addr<MM, Split<P>::LANE>(a, I, jp, wp, lp, ok);
                if (ok) *p = v[j];
            });
        }
    }

    template <int MM>
    __device__ static __forceinline__ void dispatch_store(const BArgs &a, const BItem &I, const S (&v)[E],
                                                          uint32_t lane, uint32_t wave, int p)
    {
        static_for<0, LS.n>([&](auto PP) {
            constexpr int P = decltype(PP)::value;
            if constexpr (P == 0 || lanes_contiguous(LS.m[P], 6)) {
                if (P == p) store_layout<P, MM>(a, I, v, lane, wave);
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

    template <int MM>
    __device__ static __forceinline__ void item(const BArgs &a, const BItem &I, S *lds, uint32_t t)
    {
        constexpr uint32_t act = lowmask(MM);
        const uint32_t lane = t & 63u;
        const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);
        S v[E];
        // every load is issued before the first use: the counter that tracks
        // the loads also counts the previous item's stores, so consuming the
        // first load early would drain those stores before the others issue
        load0<MM>(a, I, v, lane, wave);
        reg_stages<S, LS.m[0], LS.fresh[0], E>(v, act);
        int cur = 0;
        static_for<1, LS.n>([&](auto PP) {
            constexpr int P = decltype(PP)::value;
            if constexpr ((act & LS.fresh[P]) != 0) {
                dispatch_transpose(lds, v, t, cur, P);
                cur = P;
                reg_stages<S, LS.m[P], LS.fresh[P], E>(v, act);
            }
        });
        if (!store_ok(cur)) {
            dispatch_transpose(lds, v, t, cur, 0);
            cur = 0;
        }
        int32_t nz = a.normalize;  // opaque copy: keeps the per-size scales out of the loop prologue
        asm volatile("" : "+s"(nz));
        if (nz) {
            const float sc = (float)(1.0 / sqrt((double)(1ull << MM)));
#pragma unroll
            for (int j = 0; j < E; ++j) v[j] *= sc;
        }
        // Opaque copies of the thread coordinates: the store addresses are
        // then recomputed here instead of being kept live (and spilled) from
        // the loads.
        uint32_t slane = lane, swave = wave;
        asm volatile("" : "+v"(slane));
        asm volatile("" : "+s"(swave));
        dispatch_store<MM>(a, I, v, slane, swave, cur);
    }

    // Transform sizes are a run-time property of each tile; the item code is
    // specialised per size so that its address arithmetic is as uniform as
    // the size allows.
    __device__ static __forceinline__ void item_any(const BArgs &a, const BItem &I, S *lds, uint32_t t)
    {
        static_for<2, TB + 1>([&](auto M0) {
            constexpr int MM = decltype(M0)::value;
            if (I.m == MM) item<MM>(a, I, lds, t);
        });
    }

    __device__ static __forceinline__ BItem read_item(const BArgs &a, int32_t it)
    {
        const __attribute__((address_space(4))) BItem *ip = as_const(a.items) + it;
        BItem I;
        I.m = __builtin_amdgcn_readfirstlane(ip->m);
        I.seg0 = __builtin_amdgcn_readfirstlane(ip->seg0);
        I.nseg = __builtin_amdgcn_readfirstlane(ip->nseg);
        I.pad = 0;
        return I;
    }

    __device__ static __forceinline__ void run(const BArgs &a)
    {
        __shared__ S lds[LDS_ELEMS];
        const uint32_t t = threadIdx.x;
        // static cyclic assignment; every transpose starts with a barrier, so
        // one item's last LDS reads finish before the next item's writes
        for (int32_t it = blockIdx.x; it < a.nitems; it += gridDim.x) {
            // An opaque copy of the thread id per item: the per-layout lane,
            // wave and LDS offsets derived from it are recomputed for each
            // item rather than hoisted out of the loop and kept live.
            uint32_t tt = t;
            asm volatile("" : "+v"(tt));
            item_any(a, read_item(a, it), lds, tt);
        }
    }
};

constexpr int BATCH_TB = 16;
constexpr int BATCH_NT = 1024;

}  // namespace fwht
