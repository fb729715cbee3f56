// fwht_fold.hip -- linear space reduction of the signal (section 5.1, WHT
// with an on-the-fly signal source).
//
// A rank-m linear map A : GF(2)^n -> GF(2)^m reduces a signal of 2^n entries
// to u_j = sum of x_i over the 2^(n-m) indices i with A i = j.  Since
// <A i, k'> = <i, A^T k'>, the 2^m-point transform of u at k' is the
// 2^n-point transform of x at A^T k': one reduction and one small transform
// give the coefficients on an m-dimensional subspace of the index space, and
// independent reductions cover the rest with high probability.
//
// Which coefficients are obtained depends only on the row space of A, so the
// host replaces the caller's rows by the unique reduced echelon basis of their
// span with pivots at the lowest bits p_0 < ... < p_{m-1} (returned to the
// caller; entry k' of the reduced transform then holds the coefficient at the
// XOR of basis[t] over the set bits t of k').  With Q = {q_r} the other n - m
// bit positions, the preimage of j is
//     i = D(j) xor g(h),   h in GF(2)^(n-m),
// where D deposits bit t of j at p_t and g(h) is the XOR of
// gamma_r = e_{q_r} xor (bits p_t of the basis rows that contain q_r) over the
// set bits r of h.  A thread owns a run of 2^VB consecutive j: when the
// lowest pivots are bits 0 .. VB-1, D moves such a run to 2^VB consecutive
// entries, so each step reads one 16-byte vector.  g(h) is the same for every
// thread of a wave, so its low VB bits only permute the vector (a
// wave-uniform selection) and its other bits move the whole wave to another
// run: every load is coalesced.  h is walked in Gray-code order (one gamma
// per step), with its low four bits unrolled for a stored signal (sixteen
// loads in flight per thread) and its low three bits for a generated one.
//
// Two sources: a signal stored in device memory (bound by HBM: 2^n reads and
// 2^m writes), and the planted signal of the synthetic inputs generated on
// the fly (bound by integer ALU: the signal never exists in memory, as in the
// paper's setting, where each machine has online access to the source).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "fwht_internal.hpp"

namespace fwht {

constexpr int kFoldMaxM = 36;       // reduced transforms of up to 2^36 entries
constexpr int kFoldMaxNStored = 40;  // stored signals of up to 2^40 entries
constexpr int kFoldMaxNGen = 48;     // generated signals of up to 2^48 entries

struct FoldArgs {
    const void *x;      // stored signal (unused by the generated source)
    void *u;            // reduced signal, 2^m entries
    uint64_t s;         // generated source: planted mask
    uint64_t state;     //   state of the noise stream
    uint32_t thr32;     //   noise bit = [top 32 bits < thr32] xor flip
    uint32_t flip;      //   (a threshold of 2^32 is thr32 = 0, flip = 1)
    uint64_t nvec;      // 2^jbits runs of 2^VB consecutive j
    uint32_t jbits;     // m - VB
    uint32_t cbits;     // each run's preimage is split over 2^cbits chunks
    uint32_t lbits;     // h bits walked by one thread (n - m - cbits)
    uint32_t atomic;    // chunks > 1: partial sums are added to a zeroed u
    uint64_t dep[kFoldMaxM];         // dep[t] = bit p_(t + VB)
    uint64_t gamma[kFoldMaxNGen];    // gamma_r, r < n - m
};

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output i of the stream with
// state S is mix(S + (i + 1) * 0x9E3779B97F4A7C15).  The planted signal's noise
// bit is [(output >> 32) < thr] and x_i = (-1)^(<s, i> xor noise_i).  Returns
// the top 32 bits of output i given state1 = S + 0x9E3779B97F4A7C15.
__device__ __forceinline__ uint32_t splitmix_hi32(uint64_t i, uint64_t state1)
{
    uint64_t z = state1 + i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    const uint32_t hi = (uint32_t)(z >> 32);
    return hi ^ (hi >> 31);
}

__device__ __forceinline__ uint32_t parity64(uint64_t v) { return (uint32_t)__popcll(v) & 1u; }

template <class U, int VB>
struct Vec;
template <>
struct Vec<uint32_t, 2> {
    using T = uint4;
};
template <>
struct Vec<uint64_t, 1> {
    using T = ulonglong2;
};

// 16-byte piece v of a run of E entries held in registers.
template <class U, int E>
__device__ __forceinline__ uint4 pack16(const U (&acc)[E], int v)
{
    if constexpr (sizeof(U) == 4)
        return make_uint4(acc[4 * v], acc[4 * v + 1], acc[4 * v + 2], acc[4 * v + 3]);
    else
        return make_uint4((uint32_t)acc[2 * v], (uint32_t)(acc[2 * v] >> 32), (uint32_t)acc[2 * v + 1],
                          (uint32_t)(acc[2 * v + 1] >> 32));
}

// v[e] <- v[e xor sig] for the E = 2^VB entries of a run.
template <class U, int VB>
__device__ __forceinline__ void xor_permute(U (&v)[1 << VB], uint32_t sig)
{
    if constexpr (VB >= 1) {
        const bool b0 = sig & 1u;
#pragma unroll
        for (int e = 0; e < (1 << VB); e += 2) {
            const U a = v[e], b = v[e + 1];
            v[e] = b0 ? b : a;
            v[e + 1] = b0 ? a : b;
        }
    }
    if constexpr (VB >= 2) {
        const bool b1 = sig & 2u;
#pragma unroll
        for (int e = 0; e < (1 << VB); e += 4) {
            const U a0 = v[e], a1 = v[e + 1], c0 = v[e + 2], c1 = v[e + 3];
            v[e] = b1 ? c0 : a0;
            v[e + 1] = b1 ? c1 : a1;
            v[e + 2] = b1 ? a0 : c0;
            v[e + 3] = b1 ? a1 : c1;
        }
    }
}

template <class U, int VB, int UB, bool GEN>
__global__ void __launch_bounds__(256) fold_kernel(FoldArgs a)
{
    constexpr int E = 1 << VB;
    constexpr int KN = 1 << UB;
    const uint64_t tau = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    const uint64_t jv = tau & (a.nvec - 1);
    const uint64_t chunk = tau >> a.jbits;
    if (chunk >> a.cbits) return;  // only when the whole job is smaller than one workgroup

    uint64_t base = 0;  // D(jv << VB); its low VB bits are zero
    for (uint32_t t = 0; t < a.jbits; ++t)
        if ((jv >> t) & 1u) base ^= a.dep[t];
    uint64_t g = 0;  // g(h) at the first h of this chunk
    for (uint32_t r = 0; r < a.cbits; ++r)
        if ((chunk >> r) & 1u) g ^= a.gamma[a.lbits + r];
    uint64_t G[KN];  // XOR combinations of gamma_0 .. gamma_(UB-1)
    G[0] = 0;
#pragma unroll
    for (int k = 1; k < KN; ++k) G[k] = G[k & (k - 1)] ^ a.gamma[__builtin_ctz(k)];

    const uint64_t nouter = 1ull << (a.lbits - UB);
    U acc[E];
    // generated source: cnt[e] counts the steps with noise xor <s, g> = 1;
    // entry e is -1 where that differs from pb[e] = <s, base xor e> xor flip
    uint32_t cnt[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        acc[e] = 0;
        cnt[e] = 0;
    }
    const uint64_t state1 = a.state + 0x9E3779B97F4A7C15ull;
    const U *x = static_cast<const U *>(a.x);
    for (uint64_t o = 0; o < nouter; ++o) {
        if (o) g ^= a.gamma[UB + __builtin_ctzll(o)];  // Gray code: one bit of h changes
        if constexpr (!GEN) {
            U v[KN][E];
#pragma unroll
            for (int k = 0; k < KN; ++k) {
                const uint64_t idx = base ^ g ^ G[k];
                // the signal is read exactly once: non-temporal loads (5-10%
                // faster than cached ones at 2^30 entries)
                if constexpr (VB == 0) {
                    v[k][0] = __builtin_nontemporal_load(x + idx);
                } else {
                    using VT = typename Vec<U, VB>::T;
                    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
                    const u32x4 w = __builtin_nontemporal_load(
                        reinterpret_cast<const u32x4 *>(x + (idx & ~(uint64_t)(E - 1))));
                    const VT q = *reinterpret_cast<const VT *>(&w);
                    const U *qs = reinterpret_cast<const U *>(&q);
#pragma unroll
                    for (int e = 0; e < E; ++e) v[k][e] = qs[e];
                }
            }
#pragma unroll
            for (int k = 0; k < KN; ++k) {
                if constexpr (VB > 0) xor_permute<U, VB>(v[k], (uint32_t)((g ^ G[k]) & (E - 1)));
#pragma unroll
                for (int e = 0; e < E; ++e) acc[e] += v[k][e];
            }
        } else {
#pragma unroll
            for (int k = 0; k < KN; ++k) {
                const uint64_t gk = g ^ G[k];
                const bool pg = parity64(a.s & gk);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const uint64_t i = base ^ gk ^ (uint64_t)e;
                    cnt[e] += (uint32_t)((splitmix_hi32(i, state1) < a.thr32) != pg);
                }
            }
        }
    }
    if constexpr (GEN) {
        const int64_t terms = (int64_t)1 << a.lbits;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const bool pb = parity64(a.s & (base ^ (uint64_t)e)) ^ a.flip;
            const int64_t neg = pb ? terms - (int64_t)cnt[e] : (int64_t)cnt[e];
            acc[e] = (U)(terms - 2 * neg);
        }
    }
    U *u = static_cast<U *>(a.u) + (jv << VB);
    if (a.atomic) {
#pragma unroll
        for (int e = 0; e < E; ++e) atomicAdd(u + e, acc[e]);
    } else if constexpr (E * sizeof(U) < 16) {
#pragma unroll
        for (int e = 0; e < E; ++e) u[e] = acc[e];
    } else {
#pragma unroll
        for (int v = 0; v < (int)(E * sizeof(U) / 16); ++v) reinterpret_cast<uint4 *>(u)[v] = pack16<U, E>(acc, v);
    }
}

__global__ void __launch_bounds__(256) fold_zero_kernel(uint4 *p, uint64_t nvec)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < nvec; i += (uint64_t)gridDim.x * 256u)
        p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void __launch_bounds__(256) fold_zero_small_kernel(unsigned char *p, uint64_t bytes)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < bytes; i += (uint64_t)gridDim.x * 256u) p[i] = 0;
}

struct RemapArgs {
    uint64_t *idx;
    const uint64_t *count;
    uint64_t cap;
    uint32_t m;
    uint64_t basis[kFoldMaxM];
};

// Reduced hit indices k' -> A^T k' (the XOR of basis[t] over the set bits t).
__global__ void __launch_bounds__(256) remap_hits_kernel(RemapArgs a)
{
    const uint64_t cnt = *a.count;
    const uint64_t nh = cnt < a.cap ? cnt : a.cap;
    for (uint64_t h = (uint64_t)blockIdx.x * 256u + threadIdx.x; h < nh; h += (uint64_t)gridDim.x * 256u) {
        const uint64_t kp = a.idx[h];
        uint64_t k = 0;
        for (uint32_t t = 0; t < a.m; ++t)
            if ((kp >> t) & 1u) k ^= a.basis[t];
        a.idx[h] = k;
    }
}

// Reduced echelon basis of the span of rows[0 .. m) with pivots at the lowest
// bits (row t's lowest set bit is p_t, p_0 < p_1 < ..., and bit p_t is clear
// in every other row).  False when the rows are linearly dependent.
static bool canonical_basis(const uint64_t *rows, int n, int m, uint64_t *out)
{
    uint64_t r[kFoldMaxM];
    for (int t = 0; t < m; ++t) r[t] = rows[t];
    int rank = 0;
    for (int bit = 0; bit < n && rank < m; ++bit) {
        int p = -1;
        for (int q = rank; q < m; ++q)
            if ((r[q] >> bit) & 1u) {
                p = q;
                break;
            }
        if (p < 0) continue;
        std::swap(r[rank], r[p]);
        for (int q = 0; q < m; ++q)
            if (q != rank && ((r[q] >> bit) & 1u)) r[q] ^= r[rank];
        ++rank;
    }
    if (rank < m) return false;
    for (int t = 0; t < m; ++t) out[t] = r[t];
    return true;
}

template <class U, int VB, int UB, bool GEN>
static hipError_t launch_fold_t(const FoldArgs &a, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL((fold_kernel<U, VB, UB, GEN>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <class U, bool GEN>
static hipError_t launch_fold_u(const FoldArgs &a, int vb, int ub, uint32_t grid, hipStream_t s)
{
    // stored source: one 16-byte vector per step; generated source: runs of 4
    constexpr int VBMAX = (GEN || sizeof(U) == 4) ? 2 : 1;
    if (vb == VBMAX) {
        if constexpr (!GEN)
            if (ub == 4) return launch_fold_t<U, VBMAX, 4, GEN>(a, grid, s);
        return ub ? launch_fold_t<U, VBMAX, 3, GEN>(a, grid, s) : launch_fold_t<U, VBMAX, 0, GEN>(a, grid, s);
    }
    return ub ? launch_fold_t<U, 0, 3, GEN>(a, grid, s) : launch_fold_t<U, 0, 0, GEN>(a, grid, s);
}

static int fold(const void *x, int dtype, int n, int m, const uint64_t *rows, void *u, uint64_t *basis, bool gen,
                uint64_t smask, uint64_t state, uint64_t thr, hipStream_t s)
{
    if (dtype != FWHT_I32 && dtype != FWHT_I64) return fail(FWHT_E_INVAL, "dtype must be FWHT_I32 or FWHT_I64");
    const int nmax = gen ? kFoldMaxNGen : kFoldMaxNStored;
    if (n < 0 || n > nmax) return fail(FWHT_E_RANGE, "fold needs 0 <= n <= %d", nmax);
    if (m < 0 || m > n || m > kFoldMaxM) return fail(FWHT_E_RANGE, "fold needs 0 <= m <= min(n, %d)", kFoldMaxM);
    if (!u || (!gen && !x)) return fail(FWHT_E_INVAL, "signal or output is NULL");
    if (m > 0 && (!rows || !basis)) return fail(FWHT_E_INVAL, "rows or basis is NULL");
    if ((((uintptr_t)u) & 15) || (!gen && (((uintptr_t)x) & 15)))
        return fail(FWHT_E_INVAL, "signal and output must be 16-byte aligned");
    const uint64_t nmask = n == 64 ? ~0ull : ((1ull << n) - 1);
    for (int t = 0; t < m; ++t)
        if (rows[t] & ~nmask) return fail(FWHT_E_INVAL, "row %d has bits at or above n = %d", t, n);
    if (gen && (smask & ~nmask)) return fail(FWHT_E_INVAL, "planted mask has bits at or above n = %d", n);

    uint64_t can[kFoldMaxM] = {};
    if (m > 0 && !canonical_basis(rows, n, m, can)) return fail(FWHT_E_INVAL, "rows are linearly dependent");

    FoldArgs a{};
    a.x = x;
    a.u = u;
    a.s = smask;
    a.state = state;
    a.thr32 = thr > 0xFFFFFFFFull ? 0u : (uint32_t)thr;  // thr >= 2^32: every noise bit is 1
    a.flip = thr > 0xFFFFFFFFull ? 1u : 0u;
    const int esz = dtype == FWHT_I32 ? 4 : 8;
    const int vbmax = (gen || esz == 4) ? 2 : 1;
    int vb = 0;
    while (vb < vbmax && vb < m && (can[vb] & (~can[vb] + 1)) == (1ull << vb)) ++vb;  // pivot p_vb = vb
    // Only whole vectors: VB is either the full vector width or 0.
    if (vb != vbmax) vb = 0;
    // pivots and the non-pivot positions
    uint64_t pivmask = 0;
    for (int t = 0; t < m; ++t) pivmask |= can[t] & (~can[t] + 1);
    int nq = 0;
    for (int q = 0; q < n; ++q) {
        if ((pivmask >> q) & 1u) continue;
        uint64_t gm = 1ull << q;
        for (int t = 0; t < m; ++t)
            if ((can[t] >> q) & 1u) gm |= can[t] & (~can[t] + 1);
        a.gamma[nq++] = gm;
    }
    for (int t = vb; t < m; ++t) a.dep[t - vb] = can[t] & (~can[t] + 1);
    const int nm = n - m;
    const int jb = m - vb;
    // Split each run's preimage over 2^cbits threads so that about 2^21
    // threads run, each walking at least 16 steps of h (8 for the generated
    // source) where there are that many; a generated chunk counts its -1
    // entries in 32 bits.
    int cb = std::max(0, 21 - jb);
    cb = std::min(cb, std::max(0, nm - (gen ? 3 : 4)));
    if (gen) cb = std::max(cb, nm - 31);
    cb = std::min(cb, nm);
    if (jb + cb > 38) return fail(FWHT_E_RANGE, "fold too large for one launch");
    a.jbits = (uint32_t)jb;
    a.nvec = 1ull << jb;
    a.cbits = (uint32_t)cb;
    a.lbits = (uint32_t)(nm - cb);
    a.atomic = cb > 0 ? 1u : 0u;
    // stored vectors: sixteen loads in flight per thread where h has the bits
    const int ub = (!gen && vb > 0 && a.lbits >= 4) ? 4 : (a.lbits >= 3 ? 3 : 0);
    const uint64_t threads = 1ull << (jb + cb);
    const uint32_t grid = (uint32_t)((threads + 255) / 256);

    hipError_t e = hipSuccess;
    if (a.atomic) {
        const uint64_t bytes = (uint64_t)esz << m;
        if (bytes >= 16) {
            const uint64_t nv = bytes / 16;
            const uint64_t zg = std::min<uint64_t>((nv + 255) / 256, 1u << 20);
            hipLaunchKernelGGL(fold_zero_kernel, dim3((uint32_t)zg), dim3(256), 0, s, (uint4 *)u, nv);
        } else {
            hipLaunchKernelGGL(fold_zero_small_kernel, dim3(1), dim3(256), 0, s, (unsigned char *)u, bytes);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "fold zero");
    }
    if (esz == 4)
        e = gen ? launch_fold_u<uint32_t, true>(a, vb, ub, grid, s) : launch_fold_u<uint32_t, false>(a, vb, ub, grid, s);
    else
        e = gen ? launch_fold_u<uint64_t, true>(a, vb, ub, grid, s) : launch_fold_u<uint64_t, false>(a, vb, ub, grid, s);
    if (e != hipSuccess) return hip_fail(e, "fold launch");
    for (int t = 0; t < m; ++t) basis[t] = can[t];
    return FWHT_OK;
}

}  // namespace fwht

extern "C" {

int fwht_fold(const void *x, int dtype, int n, int m, const uint64_t *rows, void *u, uint64_t *basis, void *stream)
{
    return fwht::fold(x, dtype, n, m, rows, u, basis, false, 0, 0, 0, (hipStream_t)stream);
}

int fwht_fold_planted(int dtype, int n, int m, const uint64_t *rows, uint64_t mask, uint64_t state, uint64_t thr,
                      void *u, uint64_t *basis, void *stream)
{
    return fwht::fold(nullptr, dtype, n, m, rows, u, basis, true, mask, state, thr, (hipStream_t)stream);
}

int fwht_subspace_hits(uint64_t *idx, uint64_t cap, const uint64_t *count, int m, const uint64_t *basis, void *stream)
{
    if (!count) return fwht::fail(FWHT_E_INVAL, "count is NULL");
    if (cap > 0 && !idx) return fwht::fail(FWHT_E_INVAL, "idx is NULL with cap > 0");
    if (m < 0 || m > fwht::kFoldMaxM) return fwht::fail(FWHT_E_RANGE, "m out of range");
    if (m > 0 && !basis) return fwht::fail(FWHT_E_INVAL, "basis is NULL");
    if (cap == 0) return FWHT_OK;
    fwht::RemapArgs a{};
    a.idx = idx;
    a.count = count;
    a.cap = cap;
    a.m = (uint32_t)m;
    for (int t = 0; t < m; ++t) a.basis[t] = basis[t];
    const uint64_t grid = std::min<uint64_t>((cap + 255) / 256, 1024);
    hipLaunchKernelGGL(fwht::remap_hits_kernel, dim3((uint32_t)grid), dim3(256), 0, (hipStream_t)stream, a);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FWHT_OK : fwht::hip_fail(e, "subspace hits");
}

}  // extern "C"
