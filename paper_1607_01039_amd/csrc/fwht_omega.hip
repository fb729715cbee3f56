// fwht_omega.hip -- the prime-factor-count signal x_i = Omega(i) (the number
// of prime factors of i counted with multiplicity; Omega(0) = Omega(1) = 0),
// the practical distribution whose transform section 4.3 announces.
//
// Segmented sieve in LDS.  A workgroup owns a segment of S = 2^15 consecutive
// integers [L, L + S), 16 bits each (two to a 32-bit word, 64 KiB).  Every odd
// prime power q = p^k <= N (p <= sqrt(N), N = 2^n - 1) adds
// (1 << 11) + round(32 log2(p)) to the entries of its multiples: bits 11..15
// count prime factors (at most 20 odd ones below 2^32), bits 0..10 sum their
// base-2 logarithms in units of 1/32 (below 2048 because i < 2^32), so an
// entry never carries into its neighbour.  The factor 2 comes from the
// trailing zeros of i.  What is left of i after the sieved factors is 1 or a
// single prime: one above sqrt(N) (two would exceed N), or one above the cube
// root of N whose square is not sieved (see the table); it is at least 3, so
// it shows as a logarithm gap of at least log2(3) = 1.58 between log2(i) and
// the sum, while the rounding of the sum stays below 20 / 64 = 0.31: a gap
// above 0.8 adds the last factor.
//
// Load balance: the multiples of q in a segment are dealt to C = ceil(count / 32)
// chunks (chunk c takes every C-th multiple from the c-th, so that adjacent
// lanes hit adjacent multiples and distinct LDS banks), and each (q, chunk)
// pair is an item; items sorted by work are dealt
// round-robin to the 1024 threads.  Workgroups are persistent (two per CU, so
// that the atomics of one overlap the stores of the other).  Each item finds
// its first multiple from L mod q, with the quotient taken from L times the
// FP64 reciprocal of q (exact or one off, then corrected).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "fwht_internal.hpp"

namespace fwht {

constexpr int kOmegaSegBits = 15;
constexpr uint32_t kOmegaSeg = 1u << kOmegaSegBits;
constexpr int kOmegaThreads = 1024;
constexpr int kOmegaBlocksPerCU = 2;
constexpr int kOmegaMaxItems = 1 << 16;
constexpr uint32_t kOmegaChunk = 32;  // multiples per item and segment
constexpr int kOmegaMaxN = 32;

struct OmegaItem {
    uint32_t q;   // prime power
    uint32_t w;   // (1 << 11) + round(32 log2(p))
    uint32_t c0;  // this chunk takes multiples c0, c0 + cs, c0 + 2 cs, ... (counted from the
    uint32_t cs;  // segment's first): adjacent lanes hit adjacent multiples, i.e. distinct banks
    double inv;   // 1 / q
};

template <class T>
// two workgroups of 16 waves per CU: 8 waves per SIMD
__global__ void __launch_bounds__(kOmegaThreads, kOmegaBlocksPerCU * kOmegaThreads / 256)
    omega_kernel(T *__restrict__ out, const OmegaItem *__restrict__ items, uint32_t nitems, uint32_t nseg,
                 uint32_t len)
{
    __shared__ uint32_t seg[kOmegaSeg / 2];
    const uint32_t t = threadIdx.x;
    const uint32_t words = (len + 1) / 2;
    for (uint32_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
        const uint32_t L = sg * kOmegaSeg;  // n <= 32: every index fits in 32 bits
        for (uint32_t j = t; j < words; j += kOmegaThreads) seg[j] = 0;
        __syncthreads();
        // four items per round, their loads issued together
        for (uint32_t it0 = t; it0 < nitems; it0 += 4 * kOmegaThreads) {
            OmegaItem mm[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t it = it0 + (uint32_t)u * kOmegaThreads;
                mm[u] = items[it < nitems ? it : it0];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (it0 + (uint32_t)u * kOmegaThreads >= nitems) break;
                const OmegaItem &m = mm[u];
                // L mod q: the FP64 quotient estimate is exact or one off
                const uint32_t qe = (uint32_t)((double)L * m.inv);
                int64_t rr = (int64_t)L - (int64_t)qe * m.q;
                rr = rr < 0 ? rr + m.q : (rr >= (int64_t)m.q ? rr - m.q : rr);
                const uint64_t f = rr ? (uint64_t)(m.q - rr) : 0ull;  // first multiple of q at or after L
                const uint64_t j0 = f + (uint64_t)m.c0 * m.q;
                if (j0 < len) {
                    // Entry j is the low (j even) or high half of word j / 2.
                    // Along an even step the half never changes, so each walk
                    // adds one pre-shifted value over word indices; an odd
                    // step is walked as two interleaved walks of twice the
                    // step, one per half.  Steps of len or more leave the
                    // segment after one add (32-bit walk: j < 2^15).
                    const uint64_t step64 = (uint64_t)m.cs * m.q;
                    const bool odd = step64 & 1u;
                    const uint64_t st = odd ? 2 * step64 : step64;
                    const uint32_t wstep = st < len ? (uint32_t)(st >> 1) : words;
                    const uint64_t j1 = j0 + step64;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const uint64_t js = h ? j1 : j0;
                        if (h && (!odd || js >= len)) break;
                        const uint32_t add = m.w << (((uint32_t)js & 1u) * 16u);
                        for (uint32_t wi = (uint32_t)js >> 1; wi < words; wi += wstep) atomicAdd(&seg[wi], add);
                    }
                }
            }
        }
        __syncthreads();
        T *o = out + L;
        for (uint32_t w = t; w < words; w += kOmegaThreads) {
            const uint32_t two = seg[w];
            int32_t om[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t i = L + 2 * w + h;
                const uint32_t e = (two >> (16 * h)) & 0xFFFFu;
                om[h] = 0;
                if (i > 1) {
                    const uint32_t tz = (uint32_t)__builtin_ctz(i);
                    const float logsum = (float)((e & 2047u) + (tz << 5)) * (1.0f / 32.0f);
                    // native log2 (relative error ~2^-22): the gap is below 0.31 or above 1.27
                    const float gap = __log2f((float)i) - logsum;
                    om[h] = (int32_t)((e >> 11) + tz) + (gap > 0.8f ? 1 : 0);
                }
            }
            if (2 * w + 1 < len) {  // both entries: one 8- or 16-byte store
                if constexpr (sizeof(T) == 8)
                    *reinterpret_cast<longlong2 *>(o + 2 * w) = make_longlong2(om[0], om[1]);
                else
                    *reinterpret_cast<int2 *>(o + 2 * w) = make_int2(om[0], om[1]);
            } else {
                o[2 * w] = (T)om[0];
            }
        }
        __syncthreads();  // the next segment clears the words read above
    }
}

// The item table of one (device, n): built on the host at the first call and
// kept in device memory until the process ends (read-only afterwards, so
// concurrent calls share it); at most 15,387 items of 24 bytes.
struct OmegaTable {
    OmegaItem *items = nullptr;
    uint32_t count = 0;
};
static std::mutex g_omega_mu;
static std::map<std::pair<int, int>, OmegaTable> g_omega_tables;

static int omega_table(int dev, int n, uint32_t len, OmegaTable &out)
{
    std::lock_guard<std::mutex> lock(g_omega_mu);
    auto it = g_omega_tables.find({dev, n});
    if (it != g_omega_tables.end()) {
        out = it->second;
        return FWHT_OK;
    }
    const uint64_t N = (1ull << n) - 1;
    // odd primes p <= sqrt(N) by a sieve of Eratosthenes
    uint64_t root = (uint64_t)std::sqrt((double)N);
    while (root * root > N) --root;
    while ((root + 1) * (root + 1) <= N) ++root;
    std::vector<uint8_t> comp(root + 1, 0);
    std::vector<OmegaItem> items;
    for (uint64_t p = 3; p <= root; p += 2) {
        if (comp[p]) continue;
        for (uint64_t j = p * p; j <= root; j += 2 * p) comp[j] = 1;
        const uint32_t w = (1u << 11) + (uint32_t)std::lround(std::log2((double)p) * 32.0);
        // The square of a prime above the cube root of N is left out: such a p
        // divides i at most twice (p^3 > N), and where it does, nothing above
        // sqrt(N) divides i too (p^2 P > N), so the one factor p left over is
        // counted by the logarithm gap like a prime above sqrt(N).
        const bool skip_square = p > N / p / p;
        for (uint64_t q = p, k = 1; q <= N; q *= p, ++k) {
            if (!(k == 2 && skip_square)) {
                const uint64_t per_seg = (len + q - 1) / q;  // most multiples of q in one segment
                const uint64_t chunks = (per_seg + kOmegaChunk - 1) / kOmegaChunk;
                for (uint64_t c = 0; c < chunks; ++c)
                    items.push_back(OmegaItem{(uint32_t)q, w, (uint32_t)c, (uint32_t)chunks, 1.0 / (double)q});
            }
            if (q > N / p) break;
        }
    }
    // Items with equal work side by side: thread t takes items t, t + 1024, ...,
    // so the lanes of a wave walk loops of the same length.
    auto work = [len](const OmegaItem &m) {
        const uint64_t per_seg = ((uint64_t)len + m.q - 1) / m.q;
        return (per_seg - m.c0 + m.cs - 1) / m.cs;
    };
    std::stable_sort(items.begin(), items.end(),
                     [&](const OmegaItem &a, const OmegaItem &b) { return work(a) > work(b); });
    if (items.size() > (size_t)kOmegaMaxItems) return fail(FWHT_E_RANGE, "too many sieve items (%zu)", items.size());
    OmegaTable t;
    t.count = (uint32_t)items.size();
    hipError_t e = hipMalloc((void **)&t.items, std::max<size_t>(items.size(), 1) * sizeof(OmegaItem));
    if (e != hipSuccess) return fail(FWHT_E_NOMEM, "prime-factor counts: %s", hipGetErrorString(e));
    if (!items.empty()) {
        e = hipMemcpy(t.items, items.data(), items.size() * sizeof(OmegaItem), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(t.items);
            return hip_fail(e, "prime-factor counts upload");
        }
    }
    g_omega_tables[{dev, n}] = t;
    out = t;
    return FWHT_OK;
}

static int omega(void *data, int dtype, int n, hipStream_t s)
{
    if (!data) return fail(FWHT_E_INVAL, "data is NULL");
    if (((uintptr_t)data) & 15) return fail(FWHT_E_INVAL, "data must be 16-byte aligned");
    if (dtype != FWHT_I32 && dtype != FWHT_I64) return fail(FWHT_E_INVAL, "dtype must be FWHT_I32 or FWHT_I64");
    if (n < 0 || n > kOmegaMaxN) return fail(FWHT_E_RANGE, "prime-factor counts need 0 <= n <= %d", kOmegaMaxN);
    const uint64_t total = 1ull << n;
    const uint32_t len = (uint32_t)std::min<uint64_t>(total, kOmegaSeg);
    const uint32_t nseg = (uint32_t)(total / len);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    const uint32_t grid = std::min<uint32_t>(nseg, (uint32_t)std::max(cus, 1) * kOmegaBlocksPerCU);
    OmegaTable tab;
    const int rc = omega_table(dev, n, len, tab);
    if (rc != FWHT_OK) return rc;
    if (dtype == FWHT_I32)
        hipLaunchKernelGGL(omega_kernel<int32_t>, dim3(grid), dim3(kOmegaThreads), 0, s, (int32_t *)data, tab.items,
                           tab.count, nseg, len);
    else
        hipLaunchKernelGGL(omega_kernel<int64_t>, dim3(grid), dim3(kOmegaThreads), 0, s, (int64_t *)data, tab.items,
                           tab.count, nseg, len);
    e = hipGetLastError();
    return e == hipSuccess ? FWHT_OK : hip_fail(e, "prime-factor counts launch");
}

}  // namespace fwht

extern "C" int fwht_prime_omega(void *data, int dtype, int n, void *stream)
{
    return fwht::omega(data, dtype, n, (hipStream_t)stream);
}
