// fwht_omega.hip -- the prime-factor-count signal x_i = Omega(i) (the number
// of prime factors of i counted with multiplicity; Omega(0) = Omega(1) = 0),
// the practical distribution whose transform section 4.3 announces.
//
// Segmented sieve in LDS.  A workgroup owns a segment of S = 2^15 consecutive
// integers [L, L + S) with one 32-bit word each.  Every odd prime power
// q = p^k <= N (p <= sqrt(N), N = 2^n - 1) adds (1 << 26) + round(log2(p) 2^16)
// to the words of its multiples: the top six bits count prime factors, the
// low 26 bits sum their base-2 logarithms in fixed point.  The factor 2 comes
// from the trailing zeros of i.  What is left of i after the sieved factors is
// 1 or a single prime above sqrt(N) (two such primes would exceed N); it is
// at least 3, so it shows as a logarithm gap of more than 1 between log2(i)
// and the sum, far above the rounding of either (below 2^-10).
//
// Load balance: the multiples of q in a segment are cut into chunks of at most
// 32, and each (q, chunk) pair is an item; items are dealt round-robin to the
// 1024 threads (at most 16 each).  Workgroups are persistent (one per CU, the
// segment taking 128 KiB of LDS) and walk the segments with a fixed stride D,
// so each item's residue r = L mod q is carried in a register from one segment
// to the next as r <- (r + D mod q) mod q.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "fwht_internal.hpp"

namespace fwht {

constexpr int kOmegaSegBits = 15;
constexpr uint32_t kOmegaSeg = 1u << kOmegaSegBits;
constexpr int kOmegaThreads = 1024;
constexpr int kOmegaMaxItemsPerThread = 16;
constexpr uint32_t kOmegaChunk = 32;  // multiples per item and segment
constexpr int kOmegaMaxN = 32;

struct OmegaItem {
    uint32_t q;   // prime power
    uint32_t d;   // (grid stride in integers) mod q
    uint32_t w;   // (1 << 26) + round(log2(p) * 2^16)
    uint32_t c0;  // first multiple of this chunk, counted from the segment's first
};

template <class T>
__global__ void __launch_bounds__(kOmegaThreads, 1)
    omega_kernel(T *__restrict__ out, const OmegaItem *__restrict__ items, uint32_t nitems, uint32_t nseg,
                 uint32_t len)
{
    __shared__ uint32_t seg[kOmegaSeg];
    const uint32_t t = threadIdx.x;
    uint32_t r[kOmegaMaxItemsPerThread];
#pragma unroll
    for (int k = 0; k < kOmegaMaxItemsPerThread; ++k) {
        const uint32_t it = t + (uint32_t)k * kOmegaThreads;
        r[k] = it < nitems ? (uint32_t)(((uint64_t)blockIdx.x * kOmegaSeg) % items[it].q) : 0u;
    }
    for (uint32_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
        for (uint32_t j = t; j < len; j += kOmegaThreads) seg[j] = 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kOmegaMaxItemsPerThread; ++k) {
            const uint32_t it = t + (uint32_t)k * kOmegaThreads;
            if (it < nitems) {
                const OmegaItem m = items[it];
                const uint64_t f = r[k] ? (uint64_t)(m.q - r[k]) : 0ull;  // first multiple of q at or after L
                const uint64_t j0 = f + (uint64_t)m.c0 * m.q;
                const uint64_t j1 = std::min<uint64_t>(len, j0 + (uint64_t)kOmegaChunk * m.q);
                for (uint64_t j = j0; j < j1; j += m.q) atomicAdd(&seg[(uint32_t)j], m.w);
                r[k] = r[k] >= m.q - m.d ? r[k] - (m.q - m.d) : r[k] + m.d;
            }
        }
        __syncthreads();
        const uint32_t L = sg * kOmegaSeg;  // n <= 32: every index fits in 32 bits
        T *o = out + L;
        for (uint32_t j = t; j < len; j += kOmegaThreads) {
            const uint32_t i = L + j;
            const uint32_t wd = seg[j];
            int32_t om = 0;
            if (i > 1) {
                const uint32_t tz = (uint32_t)__builtin_ctz(i);
                const float logsum = (float)((wd & 0x3FFFFFFu) + (tz << 16)) * (1.0f / 65536.0f);
                // native log2 (relative error ~2^-22): the gap is ~0 or >= log2(3)
                const float gap = __log2f((float)i) - logsum;
                om = (int32_t)((wd >> 26) + tz) + (gap > 1.0f ? 1 : 0);
            }
            o[j] = (T)om;
        }
        __syncthreads();  // the next segment clears the words read above
    }
}

static int omega(void *data, int dtype, int n, hipStream_t s)
{
    if (!data) return fail(FWHT_E_INVAL, "data is NULL");
    if (((uintptr_t)data) & 15) return fail(FWHT_E_INVAL, "data must be 16-byte aligned");
    if (dtype != FWHT_I32 && dtype != FWHT_I64) return fail(FWHT_E_INVAL, "dtype must be FWHT_I32 or FWHT_I64");
    if (n < 0 || n > kOmegaMaxN) return fail(FWHT_E_RANGE, "prime-factor counts need 0 <= n <= %d", kOmegaMaxN);
    const uint64_t total = 1ull << n;
    const uint64_t N = total - 1;
    const uint32_t len = (uint32_t)std::min<uint64_t>(total, kOmegaSeg);
    const uint32_t nseg = (uint32_t)(total / len);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    const uint32_t grid = std::min<uint32_t>(nseg, (uint32_t)std::max(cus, 1));
    const uint64_t D = (uint64_t)grid * kOmegaSeg;  // integers between a workgroup's segments

    // odd primes p <= sqrt(N) by a sieve of Eratosthenes
    uint64_t root = (uint64_t)std::sqrt((double)N);
    while (root * root > N) --root;
    while ((root + 1) * (root + 1) <= N) ++root;
    std::vector<uint8_t> comp(root + 1, 0);
    std::vector<OmegaItem> items;
    for (uint64_t p = 3; p <= root; p += 2) {
        if (comp[p]) continue;
        for (uint64_t j = p * p; j <= root; j += 2 * p) comp[j] = 1;
        const uint32_t w = (1u << 26) + (uint32_t)std::lround(std::log2((double)p) * 65536.0);
        for (uint64_t q = p; q <= N; q *= p) {
            const uint64_t per_seg = (len + q - 1) / q;  // most multiples of q in one segment
            const uint64_t chunks = (per_seg + kOmegaChunk - 1) / kOmegaChunk;
            for (uint64_t c = 0; c < chunks; ++c)
                items.push_back(OmegaItem{(uint32_t)q, (uint32_t)(D % q), w, (uint32_t)(c * kOmegaChunk)});
            if (q > N / p) break;
        }
    }
    // Items with equal work side by side: thread t takes items t, t + 1024, ...,
    // so the lanes of a wave walk loops of the same length.
    auto work = [len](const OmegaItem &m) {
        const uint64_t per_seg = ((uint64_t)len + m.q - 1) / m.q;
        return std::min<uint64_t>(kOmegaChunk, per_seg - m.c0);
    };
    std::stable_sort(items.begin(), items.end(),
                     [&](const OmegaItem &a, const OmegaItem &b) { return work(a) > work(b); });
    if (items.size() > (size_t)kOmegaThreads * kOmegaMaxItemsPerThread)
        return fail(FWHT_E_RANGE, "too many sieve items (%zu)", items.size());

    // Items in stream-ordered memory: allocated, filled, read and released in
    // the order of `s`, so concurrent calls never share them.
    void *d_items = nullptr;
    const size_t bytes = std::max<size_t>(items.size(), 1) * sizeof(OmegaItem);
    e = hipMallocAsync(&d_items, bytes, s);
    if (e != hipSuccess) return fail(FWHT_E_NOMEM, "prime-factor counts: %s", hipGetErrorString(e));
    if (!items.empty()) {
        e = hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(OmegaItem), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);  // `items` is pageable and local
    }
    if (e != hipSuccess) {
        (void)hipFreeAsync(d_items, s);
        return hip_fail(e, "prime-factor counts upload");
    }
    if (dtype == FWHT_I32)
        hipLaunchKernelGGL(omega_kernel<int32_t>, dim3(grid), dim3(kOmegaThreads), 0, s, (int32_t *)data,
                           (const OmegaItem *)d_items, (uint32_t)items.size(), nseg, len);
    else
        hipLaunchKernelGGL(omega_kernel<int64_t>, dim3(grid), dim3(kOmegaThreads), 0, s, (int64_t *)data,
                           (const OmegaItem *)d_items, (uint32_t)items.size(), nseg, len);
    e = hipGetLastError();
    (void)hipFreeAsync(d_items, s);
    return e == hipSuccess ? FWHT_OK : hip_fail(e, "prime-factor counts launch");
}

}  // namespace fwht

extern "C" int fwht_prime_omega(void *data, int dtype, int n, void *stream)
{
    return fwht::omega(data, dtype, n, (hipStream_t)stream);
}
