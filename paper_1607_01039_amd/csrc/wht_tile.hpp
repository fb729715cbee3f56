// wht_tile.hpp -- one HBM pass of the in-place Walsh-Hadamard transform on gfx950.
//
// A pass applies the radix-2 butterflies (a, b) -> (a + b, a - b) of the stages
// whose index bits fall in one bit range (section 3, Fig. 1: stage k pairs the
// entries pt and pt + 2^k).  Stages on distinct bits commute, so a transform of
// 2^n entries is any sequence of passes that together cover bits 0..n-1
// (the regrouping that Fig. 2 and Fig. 3 use across cores and disk passes).
//
// The array is viewed as rows of 2^b entries.  One workgroup owns a tile of
// 2^TB entries: 2^CB contiguous columns (tile bits 0..CB-1) of 2^(TB-CB)
// consecutive rows (tile bits CB..TB-1, global bits b..b+TB-CB-1).
//   * contiguous pass (b = CB, COLS): the tile is 2^TB consecutive entries and
//     all TB tile bits may be transformed;
//   * strided pass (b > CB): only the row bits are transformed; the CB column
//     bits give 2^CB * sizeof(S) contiguous bytes per row segment.
// Which tile bits are transformed is a run-time mask (`act`), so the same
// kernel also serves short transforms (several per tile) and partial passes.
//
// Inside the tile, every thread keeps E = 2^TB / NT entries in registers.  A
// "layout" says which tile bits are register bits (mask M); the other bits
// index the thread (lanes take the lowest ones, so a wave touches contiguous
// memory).  The kernel walks a compile-time list of layouts: L0 (vector-load
// layout: the low VB bits + the top bits are register bits), then groups of
// K = log2 E untransformed bits in ascending order.  Within a layout the
// butterflies on register bits are plain VALU add/sub; between layouts the
// tile is transposed through LDS, padded by one word per 32 so that every
// access pattern used here is free of bank conflicts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace fwht {

// ---------------------------------------------------------------- compile time
constexpr int cpopc(uint32_t m) { int c = 0; while (m) { c += m & 1u; m >>= 1; } return c; }
constexpr int clog2(uint32_t v) { int r = 0; while (v > 1) { v >>= 1; ++r; } return r; }
constexpr int nth_bit(uint32_t m, int q)
{
    for (int b = 0; b < 32; ++b)
        if ((m >> b) & 1u) { if (q == 0) return b; --q; }
    return 31;
}
constexpr uint32_t cpdep(uint32_t x, uint32_t m)
{
    uint32_t r = 0;
    int q = 0;
    for (int b = 0; b < 32; ++b)
        if ((m >> b) & 1u) { if ((x >> q) & 1u) r |= 1u << b; ++q; }
    return r;
}
constexpr uint32_t lowmask(int k) { return k >= 32 ? 0xffffffffu : ((1u << k) - 1u); }

struct LayoutList {
    uint32_t m[8];      // register bits of each layout
    uint32_t fresh[8];  // bits a layout transforms (its own group, not its filler)
    int n;
};

// L0 = low VB bits + top (K - VB) bits; then the remaining candidate bits in
// ascending groups of K, the last group topped up with the highest other bits.
constexpr LayoutList make_layouts(int TB, int CB, int K, int VB, bool cols)
{
    LayoutList L{};
    const uint32_t full = lowmask(TB);
    const int top = K - VB;
    L.m[0] = lowmask(VB) | (lowmask(top) << (TB - top));
    L.n = 1;
    const uint32_t cand = cols ? full : (full & ~lowmask(CB));
    L.fresh[0] = L.m[0] & cand;
    uint32_t rem = cand & ~L.m[0];
    while (rem) {
        uint32_t g = 0;
        int c = 0;
        for (int b = 0; b < TB && c < K; ++b)
            if ((rem >> b) & 1u) { g |= 1u << b; ++c; }
        rem &= ~g;
        L.fresh[L.n] = g;
        for (int b = TB - 1; b >= 0 && c < K; --b)
            if (!((g >> b) & 1u)) { g |= 1u << b; ++c; }
        L.m[L.n++] = g;
    }
    return L;
}

// The lowest `k` set bits of m.
constexpr uint32_t low_set_bits(uint32_t m, int k)
{
    uint32_t r = 0;
    for (int b = 0; b < 32 && k > 0; ++b)
        if ((m >> b) & 1u) { r |= 1u << b; --k; }
    return r;
}

// A layout is store-friendly when its lowest non-register bits are the low
// bits of the tile, i.e. the lanes of a wave write consecutive entries.
constexpr bool lanes_contiguous(uint32_t m, int nlanebits)
{
    return (m & lowmask(nlanebits)) == 0;
}

// Layouts of a 2^TB tile with K register bits per thread, the top tile bit
// pinned as a register bit in all of them: L0 = low VB bits + top K - VB bits;
// then ascending groups of K - 1 untransformed bits, each + the pinned bit,
// the last topped up with the highest other bits.  Only tile bits from LO up
// are transformed (LO = CB for a strided tile whose low bits are columns).
constexpr LayoutList make_pinned_layouts(int TB, int K, int VB, int LO = 0)
{
    LayoutList L{};
    const uint32_t cand = lowmask(TB) & ~lowmask(LO);
    const uint32_t pin = 1u << (TB - 1);
    const int top = K - VB;
    L.m[0] = lowmask(VB) | (lowmask(top) << (TB - top));
    L.fresh[0] = L.m[0] & cand;
    L.n = 1;
    uint32_t rem = cand & ~L.m[0];
    while (rem) {
        uint32_t g = 0;
        int c = 0;
        for (int b = 0; b < TB && c < K - 1; ++b)
            if ((rem >> b) & 1u) { g |= 1u << b; ++c; }
        rem &= ~g;
        L.fresh[L.n] = g;
        g |= pin;
        ++c;
        for (int b = TB - 2; b >= 0 && c < K; --b)
            if (!((g >> b) & 1u)) { g |= 1u << b; ++c; }
        L.m[L.n++] = g;
    }
    return L;
}

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

template <uint32_t MASK>
__device__ __forceinline__ uint32_t pdep_rt(uint32_t x)
{
    uint32_t r = 0;
    int q = 0;
#pragma unroll
    for (int b = 0; b < 32; ++b)
        if ((MASK >> b) & 1u) { r |= ((x >> q) & 1u) << b; ++q; }
    return r;
}

// ------------------------------------------------------------------ pass args
struct PassArgs {
    uint64_t total;      // entries in the array (batch * 2^n)
    uint64_t colblocks;  // 2^(b - CB): column blocks per row (a power of two)
    uint64_t ntiles;     // tiles in this pass
    uint32_t b;          // log2 of the row stride
    uint32_t act;        // transformed tile bits
    // epilogue (last pass only)
    int32_t do_scale;    // float: multiply by `scale`
    float scale;
    int32_t thresh;      // emit (k, y_k) with |y_k| > T
    int64_t T;           // integer threshold (T < 0: every entry)
    float Tf;            // float threshold, rounded toward -inf from double
    unsigned long long *hit_idx;
    void *hit_val;
    uint64_t cap;
    unsigned long long *count;
    // index of a hit: k = ((off >> kshift) << kL | off mod 2^kshift) + kbase,
    // the identity (k = off) when all three are 0; the streamed column phase
    // uses it to report positions in the whole array
    uint32_t kshift, kL;
    uint64_t kbase;
    // destination of the pass (nullptr: in place); same layout as the source
    void *dst;
    // when set, the first workgroup clears this counter before anything else
    // (the hit count of a threshold fused into a LATER pass of the same
    // transform, so that it needs no launch of its own)
    unsigned long long *zero_first;
};

// The threshold test |W_k| > T of one entry, set up once per launch.  For
// integers it is one add and one unsigned compare: with 0 <= T < 2^(w-1),
// |v| > T exactly when v lies outside [-T, T], i.e. when (v + T) mod 2^w
// >= 2T + 1 (v = -2^(w-1), whose magnitude is 2^(w-1), included); T < 0
// makes the bound 0 (every entry), and for int32 a T >= 2^31 matches nothing
// (no int32 magnitude exceeds 2^31).
template <class S> struct HitTest;
template <> struct HitTest<uint32_t> {
    uint32_t add, lim;
    bool none;
    __device__ explicit HitTest(const PassArgs &a)
        : add(a.T < 0 ? 0u : (uint32_t)a.T), lim(a.T < 0 ? 0u : 2u * (uint32_t)a.T + 1u), none(a.T >= (1ll << 31))
    {
    }
    __device__ bool above(uint32_t v) const { return !none && v + add >= lim; }
};
template <> struct HitTest<uint64_t> {
    uint64_t add, lim;
    __device__ explicit HitTest(const PassArgs &a)
        : add(a.T < 0 ? 0ull : (uint64_t)a.T), lim(a.T < 0 ? 0ull : 2ull * (uint64_t)a.T + 1ull)
    {
    }
    __device__ bool above(uint64_t v) const { return v + add >= lim; }
};
template <> struct HitTest<float> {
    float t;
    __device__ explicit HitTest(const PassArgs &a) : t(a.Tf) {}
    __device__ bool above(float v) const { return fabsf(v) > t; }
};

// Wave-aggregated append of one (index, value) hit per lane with `hit` set.
template <class S>
__device__ __forceinline__ void emit_hits(bool hit, uint64_t k, S v, const PassArgs &a)
{
    uint64_t m = __ballot(hit);
    if (m == 0) return;
    const uint32_t lane = __lane_id();
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    const int leader = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if ((int)lane == leader) base = atomicAdd(a.count, (unsigned long long)__popcll(m));
    base = __shfl(base, leader);
    if (hit) {
        unsigned long long slot = base + below;
        if (slot < a.cap) {
            k = (((k >> a.kshift) << a.kL) | (k & ((1ull << a.kshift) - 1ull))) + a.kbase;
            a.hit_idx[slot] = k;
            ((S *)a.hit_val)[slot] = v;
        }
    }
}

template <class S>
__device__ __forceinline__ void bfly(S &x, S &y)
{
    S a = x, b = y;
    x = a + b;
    y = a - b;
}

// Butterflies on the register bits of layout M that it owns (FRESH) and the
// pass transforms (act).
template <class S, uint32_t M, uint32_t FRESH, int E>
__device__ __forceinline__ void reg_stages(S (&v)[E], uint32_t act)
{
    constexpr int K = clog2(E);
    static_for<0, K>([&](auto Q) {
        constexpr int q = decltype(Q)::value;
        constexpr int bit = nth_bit(M, q);
        if (((FRESH >> bit) & 1u) && ((act >> bit) & 1u)) {
#pragma unroll
            for (int j = 0; j < E; ++j)
                if (!((j >> q) & 1)) bfly(v[j], v[j | (1 << q)]);
        }
    });
}

__device__ __forceinline__ uint32_t lds_pad(uint32_t i) { return i + (i >> 5); }

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// 16-byte global load / store; NT marks the access non-temporal (the data is
// streamed once per pass and will not be re-read before eviction).
template <bool NT>
__device__ __forceinline__ v4u gload16(const void *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const v4u *>(p));
    else return *reinterpret_cast<const v4u *>(p);
}
template <bool NT>
__device__ __forceinline__ void gstore16(void *p, v4u q)
{
    if constexpr (NT) __builtin_nontemporal_store(q, reinterpret_cast<v4u *>(p));
    else *reinterpret_cast<v4u *>(p) = q;
}
template <bool NT, class S>
__device__ __forceinline__ void gstore1(S *p, S x)
{
    if constexpr (NT) __builtin_nontemporal_store(x, p);
    else *p = x;
}

// Cache policy of a pass's global accesses (bit mask): non-temporal loads
// and/or stores.  Measured on the strided passes, streaming accesses keep
// the caches from holding lines that will not be reused before eviction.
constexpr int NT_LOAD = 1, NT_STORE = 2;

template <int TB, int CB, int NT, bool COLS, class S, bool TH, int NTM>
struct TileKernel {
    static constexpr int E = (1 << TB) / NT;
    static constexpr int K = clog2(E);
    static constexpr int VEC = 16 / (int)sizeof(S);
    static constexpr int VB = clog2(VEC);
    static constexpr int R = TB - CB;
    static constexpr LayoutList LS = make_layouts(TB, CB, K, VB, COLS);
    static constexpr uint32_t FULL = lowmask(TB);
    static constexpr int LDS_ELEMS = (1 << TB) + (1 << TB) / 32;
    // Lanes of a store-friendly layout write >= 256 contiguous bytes, or a
    // whole row segment when segments are shorter.
    static constexpr int SLB = (8 - clog2(sizeof(S))) < CB ? (8 - clog2(sizeof(S))) : CB;
    static_assert(E * NT == (1 << TB), "tile must split evenly");
    static_assert(E >= VEC, "a thread must hold at least one vector");
    static_assert(K - VB <= R, "top register bits must be row bits");
    static_assert(CB >= VB + 2, "a row segment must be at least 4 vectors");
    static_assert(NT % 64 == 0, "whole waves");
    static_assert(LS.n <= 8, "too many layouts");
    static_assert(lanes_contiguous(LS.m[LS.n - 1], SLB) || LS.n == 1, "store layout");

    // Global offset (entries) of tile bits `idx`; the row stride is 2^b
    // (2^CB for a contiguous pass, known at compile time).  The map is linear
    // over disjoint bit sets, so lane, wave and register parts add up.
    __device__ static __forceinline__ uint64_t goff(uint32_t idx, uint32_t b)
    {
        const uint32_t bb = COLS ? (uint32_t)CB : b;
        return ((uint64_t)(idx >> CB) << bb) + (idx & lowmask(CB));
    }

    // Per-layout split of the thread bits: lanes take the lowest six.
    template <uint32_t M>
    struct Split {
        static constexpr uint32_t TM = FULL & ~M;
        static constexpr uint32_t LANE = low_set_bits(TM, 6);
        static constexpr uint32_t WAVE = TM & ~LANE;
    };

    // Byte offset of this lane's part (small: it spans at most 64 entries of
    // a row and a few rows) and the wave-uniform part (entries) of a layout.
    template <uint32_t M>
    __device__ static __forceinline__ uint32_t lane_bytes(uint32_t lane, uint32_t b)
    {
        return (uint32_t)(goff(pdep_rt<Split<M>::LANE>(lane), b) * sizeof(S));
    }
    template <uint32_t M>
    __device__ static __forceinline__ uint64_t wave_off(uint32_t wave, uint32_t b)
    {
        return goff(pdep_rt<Split<M>::WAVE>(wave), b);
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

    __device__ static __forceinline__ bool store_ok(int p)
    {
        bool ok = false;
        static_for<0, LS.n>([&](auto PP) {
            constexpr int P = decltype(PP)::value;
            if (P == p) ok = lanes_contiguous(LS.m[P], SLB);
        });
        return ok;
    }

    // Threshold epilogue, in two parts around the final stores from layout M
    // (element j goes to global entry wb + lb/sizeof(S) + goff(pdep(j, M))).
    // Before the stores: whether any element of this thread is a hit (one add
    // and one compare per element, OR-ed into a lane flag).  After them, and
    // only in a wave where some lane has a hit (rare for thresholds in the
    // noise tail): a uniform loop over the elements re-reads each entry this
    // thread has just written, tests it again and appends the hits, so no
    // register array stays live for it.
    template <uint32_t M, bool FULLT>
    __device__ static __forceinline__ bool tile_any_hit(const S (&v)[E], uint64_t wb, uint32_t lb,
                                                        const PassArgs &a)
    {
        const HitTest<S> ht(a);
        const uint64_t lo = wb + lb / sizeof(S);
        bool any = false;
        static_for<0, E>([&](auto J) {
            constexpr int j = decltype(J)::value;
            const bool in = FULLT || lo + goff(cpdep((uint32_t)j, M), a.b) < a.total;
            any |= in && ht.above(v[j]);
        });
        return any;
    }
    template <uint32_t M, bool FULLT>
    __device__ static __forceinline__ void emit_tile_hits(const S *buf, bool any, uint64_t wb, uint32_t lb,
                                                          const PassArgs &a)
    {
        if (__ballot(any) == 0) return;
        const HitTest<S> ht(a);
        const uint64_t lo = wb + lb / sizeof(S);
#pragma unroll 1
        for (int j = 0; j < E; ++j) {
            const uint64_t off = lo + goff(pdep_rt<M>((uint32_t)j), a.b);
            const bool in = any && (FULLT || off < a.total);
            const S val = in ? buf[off] : S(0);
            emit_hits<S>(in && ht.above(val), off, val, a);
        }
    }

    template <bool FULLT>
    __device__ static __forceinline__ void load_vec(const S *__restrict__ buf, S (&v)[E], uint32_t lane,
                                                    uint32_t wave, uint64_t base, const PassArgs &a)
    {
        constexpr uint32_t M0 = LS.m[0];
        const uint32_t lb = lane_bytes<M0>(lane, a.b);
        const uint64_t wb = base + wave_off<M0>(wave, a.b);
        static_for<0, E / VEC>([&](auto JT) {
            constexpr int jt = decltype(JT)::value;
            constexpr uint32_t jp = cpdep((uint32_t)(jt << VB), M0);
            const S *p = buf + (wb + goff(jp, a.b));
            if (FULLT) {
                const v4u q = gload16<(NTM & NT_LOAD) != 0>(reinterpret_cast<const char *>(p) + lb);
                const S *qs = reinterpret_cast<const S *>(&q);
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[jt * VEC + e] = qs[e];
            } else {
                const uint64_t off = (uint64_t)(p - buf) + lb / sizeof(S);
                if (off + VEC <= a.total) {
                    const v4u q = gload16<(NTM & NT_LOAD) != 0>(buf + off);
                    const S *qs = reinterpret_cast<const S *>(&q);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) v[jt * VEC + e] = qs[e];
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) v[jt * VEC + e] = (off + e < a.total) ? buf[off + e] : S(0);
                }
            }
        });
    }

    template <bool FULLT>
    __device__ static __forceinline__ void store_vec(S *__restrict__ buf, const S (&v)[E], uint32_t lane,
                                                     uint32_t wave, uint64_t base, const PassArgs &a)
    {
        constexpr uint32_t M0 = LS.m[0];
        const uint32_t lb = lane_bytes<M0>(lane, a.b);
        const uint64_t wb = base + wave_off<M0>(wave, a.b);
        bool any = false;
        if constexpr (TH) any = tile_any_hit<M0, FULLT>(v, wb, lb, a);
        static_for<0, E / VEC>([&](auto JT) {
            constexpr int jt = decltype(JT)::value;
            constexpr uint32_t jp = cpdep((uint32_t)(jt << VB), M0);
            S *p = buf + (wb + goff(jp, a.b));
            const uint64_t off = (uint64_t)(p - buf) + lb / sizeof(S);
            v4u q;
            S *qs = reinterpret_cast<S *>(&q);
#pragma unroll
            for (int e = 0; e < VEC; ++e) qs[e] = v[jt * VEC + e];
            if (FULLT) {
                gstore16<(NTM & NT_STORE) != 0>(reinterpret_cast<char *>(p) + lb, q);
            } else if (off + VEC <= a.total) {
                gstore16<(NTM & NT_STORE) != 0>(buf + off, q);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    if (off + e < a.total) buf[off + e] = v[jt * VEC + e];
            }
        });
        if constexpr (TH) emit_tile_hits<M0, FULLT>(buf, any, wb, lb, a);
    }

    template <int P, bool FULLT>
    __device__ static __forceinline__ void store_layout(S *__restrict__ buf, const S (&v)[E], uint32_t lane,
                                                        uint32_t wave, uint64_t base, const PassArgs &a)
    {
        constexpr uint32_t M = LS.m[P];
        const uint32_t lb = lane_bytes<M>(lane, a.b);
        const uint64_t wb = base + wave_off<M>(wave, a.b);
        bool any = false;
        if constexpr (TH) any = tile_any_hit<M, FULLT>(v, wb, lb, a);
        static_for<0, E>([&](auto J) {
            constexpr int j = decltype(J)::value;
            constexpr uint32_t jp = cpdep((uint32_t)j, M);
            S *p = buf + (wb + goff(jp, a.b));
            if (FULLT) {
                gstore1<(NTM & NT_STORE) != 0>(reinterpret_cast<S *>(reinterpret_cast<char *>(p) + lb), v[j]);
            } else {
                const uint64_t off = (uint64_t)(p - buf) + lb / sizeof(S);
                if (off < a.total) buf[off] = v[j];
            }
        });
        if constexpr (TH) emit_tile_hits<M, FULLT>(buf, any, wb, lb, a);
    }

    template <bool FULLT>
    __device__ static __forceinline__ void dispatch_store(S *__restrict__ buf, const S (&v)[E], uint32_t lane,
                                                          uint32_t wave, uint64_t base, const PassArgs &a, int p)
    {
        static_for<1, LS.n>([&](auto PP) {
            constexpr int P = decltype(PP)::value;
            if constexpr (lanes_contiguous(LS.m[P], SLB)) {
                if (P == p) store_layout<P, FULLT>(buf, v, lane, wave, base, a);
            }
        });
    }

    template <bool FULLT>
    __device__ static __forceinline__ void tile_body(const S *buf, S *out, S *lds, uint32_t t, uint64_t base,
                                                     const PassArgs &a)
    {
        const uint32_t lane = t & 63u;
        const uint32_t wave = __builtin_amdgcn_readfirstlane(t >> 6);
        S v[E];
        load_vec<FULLT>(buf, v, lane, wave, base, a);
        // every load issued before the first butterfly (the previous tile's
        // stores share the counter that the first use would wait on)
        __builtin_amdgcn_sched_barrier(0);
        reg_stages<S, LS.m[0], LS.fresh[0], E>(v, a.act);
        // remaining layouts, skipping those that own no transformed bit
        int cur = 0;
        bool wrote = false;
        static_for<1, LS.n>([&](auto PP) {
            constexpr int P = decltype(PP)::value;
            if (a.act & LS.fresh[P]) {
                if (wrote) __syncthreads();
                dispatch_to_lds(lds, v, t, cur);
                __syncthreads();
                from_lds<P>(lds, v, t);
                wrote = true;
                cur = P;
                reg_stages<S, LS.m[P], LS.fresh[P], E>(v, a.act);
            }
        });
        if (cur != 0 && !store_ok(cur)) {
            __syncthreads();
            dispatch_to_lds(lds, v, t, cur);
            __syncthreads();
            from_lds<0>(lds, v, t);
            cur = 0;
        }
        if constexpr (std::is_same<S, float>::value) {
            if (a.do_scale) {
#pragma unroll
                for (int j = 0; j < E; ++j) v[j] *= a.scale;
            }
        }
        // The store addresses repeat the load addresses; an opaque copy of
        // the lane id makes the compiler recompute them here instead of
        // keeping 64-bit load addresses live (and spilled) across the tile.
        uint32_t slane = lane;
        asm volatile("" : "+v"(slane));
        if (cur == 0) store_vec<FULLT>(out, v, slane, wave, base, a);
        else dispatch_store<FULLT>(out, v, slane, wave, base, a, cur);
        if (wrote) __syncthreads();  // the next tile reuses the LDS buffer
    }

    __device__ static __forceinline__ void run(S *__restrict__ buf, const PassArgs &a)
    {
        __shared__ S lds[LDS_ELEMS];
        S *out = a.dst ? static_cast<S *>(a.dst) : buf;
        const uint32_t t = threadIdx.x;
        if (a.zero_first && blockIdx.x == 0 && t == 0) *a.zero_first = 0ull;
        const uint32_t b = COLS ? (uint32_t)CB : a.b;
        const uint32_t cbl = (uint32_t)__builtin_ctzll(a.colblocks);  // colblocks = 2^cbl
        // Scalar trip count: a 64-bit tile < ntiles test would be a vector
        // compare against a vector copy of ntiles, which the compiler may
        // rebuild at the loop latch in registers that the stores just read,
        // and then waits for every store to finish before the next tile.
        const uint64_t first = blockIdx.x;
        const uint32_t iters = a.ntiles > first ? (uint32_t)((a.ntiles - first - 1) / gridDim.x + 1) : 0u;
        for (uint32_t k = 0; k < iters; ++k) {
            const uint64_t tile = first + (uint64_t)k * gridDim.x;
            const uint64_t g = tile >> cbl;
            const uint64_t cb = tile & (a.colblocks - 1);
            const uint64_t base = ((g << R) << b) + (cb << CB);
            // An opaque copy of the row-stride exponent: every element's
            // offset depends on it, and without this the compiler hoists all
            // of them out of the tile loop and spills them.
            PassArgs at = a;
            asm volatile("" : "+s"(at.b));
            uint32_t tt = t;  // likewise for the offsets derived from the thread id
            asm volatile("" : "+v"(tt));
            if ((((g + 1) << R) << b) <= a.total) tile_body<true>(buf, out, lds, tt, base, at);
            else tile_body<false>(buf, out, lds, tt, base, at);
        }
    }
};

// Each variant is compiled to keep at least MINW waves per SIMD resident
// (register budget 512 / MINW), so that several tiles share a CU and one
// tile's LDS phases overlap another tile's HBM traffic.
template <int TB, int CB, int NT, bool COLS, class S, bool TH, int NTM, int MINW>
__global__ void __launch_bounds__(NT, MINW) wht_tile_kernel(S *__restrict__ buf, PassArgs a)
{
    TileKernel<TB, CB, NT, COLS, S, TH, NTM>::run(buf, a);
}

// Host-side launcher of one variant (threshold epilogue chosen per launch).
template <int TB, int CB, int NT, bool COLS, class S, int NTM>
hipError_t launch_tile(void *buf, const PassArgs &a, hipStream_t s)
{
    constexpr int MINW = 2;
    // The dispatch packet counts work-items in 32 bits; the tile loop is
    // grid-stride, so a capped grid still covers every tile.
    const uint64_t maxgrid = (1ull << 31) / NT;
    const uint64_t grid = a.ntiles < maxgrid ? a.ntiles : maxgrid;
    if (a.thresh)
        hipLaunchKernelGGL((wht_tile_kernel<TB, CB, NT, COLS, S, true, NTM, MINW>), dim3((uint32_t)grid), dim3(NT),
                           0, s, (S *)buf, a);
    else
        hipLaunchKernelGGL((wht_tile_kernel<TB, CB, NT, COLS, S, false, NTM, MINW>), dim3((uint32_t)grid), dim3(NT),
                           0, s, (S *)buf, a);
    return hipGetLastError();
}

}  // namespace fwht
