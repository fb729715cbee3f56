// fwht_batched.hip -- host side of the batched persistent transform: work-list
// planning, device buffers, and a cached HIP graph per request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <list>
#include <mutex>
#include <vector>

#include "fwht_internal.hpp"
#include "wht_batched.hpp"

namespace fwht {

__global__ void __launch_bounds__(BATCH_NT, 1) batched_kernel(BArgs a)
{
    BatchedKernel<BATCH_TB, BATCH_NT>::run(a);
}

namespace {

constexpr int BTB = BATCH_TB;  // tile bits of the batched kernel
constexpr int BNT = BATCH_NT;  // threads per block

struct Plan {
    // key
    float *data = nullptr;
    int32_t count = 0;
    int normalize = 0, prec = 0;
    uint64_t hash = 0;
    std::vector<int64_t> off;  // the request itself, compared on a hash match
    std::vector<int32_t> lg;
    // device state
    BItem *items = nullptr;
    int64_t *segs = nullptr;
    int32_t nitems = 0;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

std::mutex g_mu;
std::list<Plan> g_plans;  // most recent first
constexpr size_t kMaxPlans = 8;
hipStream_t g_capture = nullptr;

// Cache key of the host arrays: a multiply-xorshift hash over 8-byte words
// (a byte-wise hash of 4096 offsets and sizes took tens of microseconds,
// spent on the host before every replay).  A plan matches only when the
// hash and then the stored arrays themselves are equal, so a collision can
// never replay another request's graph.
uint64_t hash_words(const void *p, size_t n, uint64_t h)
{
    const unsigned char *c = (const unsigned char *)p;
    size_t i = 0;
    for (; i + 8 <= n; i += 8) {
        uint64_t w;
        memcpy(&w, c + i, 8);
        h = (h ^ w) * 0x9E3779B97F4A7C15ull;
        h ^= h >> 29;
    }
    uint64_t w = 0;
    memcpy(&w, c + i, n - i);
    h = (h ^ w ^ (uint64_t)n) * 0x9E3779B97F4A7C15ull;
    return h ^ (h >> 31);
}

void release(Plan &p)
{
    if (p.exec) (void)hipGraphExecDestroy(p.exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    if (p.items) (void)hipFree(p.items);
    if (p.segs) (void)hipFree(p.segs);
    p = Plan{};
}

int grid_size(int prec, int *out)
{
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    if (prec == FWHT_PREC_FP32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_kernel, BNT, 0);
    else
        e = batched_mfma_occupancy(prec, &per);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    *out = cus * std::max(per, 1);
    return FWHT_OK;
}

// Tiles in hand-out order: transforms sorted by decreasing size; each tile
// gathers 2^(16-m) transforms of one size 2^m (the last of a size may hold
// fewer).
void build_items(const int64_t *off, const int32_t *lg, int32_t count, std::vector<BItem> &items,
                 std::vector<int64_t> &segs)
{
    std::vector<int32_t> order((size_t)count);
    for (int32_t i = 0; i < count; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return lg[a] > lg[b]; });
    size_t k = 0;
    while (k < order.size()) {
        const int32_t m = lg[order[k]];
        const int32_t per = 1 << (BTB - m);
        BItem it{m, (int32_t)segs.size(), 0, 0};
        while (k < order.size() && lg[order[k]] == m && it.nseg < per) {
            segs.push_back(off[order[k]]);
            ++it.nseg;
            ++k;
        }
        items.push_back(it);
    }
}

int make_plan(Plan &p, float *data, const int64_t *off, const int32_t *lg, int32_t count, int normalize, int prec)
{
    std::vector<BItem> items;
    std::vector<int64_t> segs;
    build_items(off, lg, count, items, segs);
    p.nitems = (int32_t)items.size();
    hipError_t e = hipMalloc(&p.items, sizeof(BItem) * items.size());
    if (e == hipSuccess) e = hipMalloc(&p.segs, sizeof(int64_t) * segs.size());
    if (e != hipSuccess) return fail(FWHT_E_NOMEM, "batched plan: %s", hipGetErrorString(e));
    e = hipMemcpy(p.items, items.data(), sizeof(BItem) * items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p.segs, segs.data(), sizeof(int64_t) * segs.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batched plan upload");

    int grid = 0;
    int rc = grid_size(prec, &grid);
    if (rc) return rc;
    if (grid > p.nitems) grid = p.nitems;
    if (!g_capture) {
        e = hipStreamCreateWithFlags(&g_capture, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "capture stream");
    }
    BArgs a{};
    a.data = data;
    a.items = p.items;
    a.segs = p.segs;
    a.nitems = p.nitems;
    a.normalize = normalize;
    // The graph: the persistent kernel alone (work is assigned statically,
    // so there is no counter to reset between replays).
    e = hipStreamBeginCapture(g_capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    const hipError_t le = launch_batched(prec, a, grid, g_capture);
    e = hipStreamEndCapture(g_capture, &p.graph);
    if (le != hipSuccess) return hip_fail(le, "batched launch (capture)");
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiate(&p.exec, p.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    return FWHT_OK;
}

}  // namespace

hipError_t launch_batched(int prec, const BArgs &a, int grid, hipStream_t s)
{
    if (prec == FWHT_PREC_FP32)
        hipLaunchKernelGGL(batched_kernel, dim3(grid), dim3(BNT), 0, s, a);
    else
        return launch_batched_mfma(prec, a, grid, s);
    return hipGetLastError();
}

int batched(float *data, const int64_t *off, const int32_t *lg, int32_t count, int normalize, int prec,
            hipStream_t s)
{
    uint64_t h = hash_words(off, sizeof(int64_t) * (size_t)count, 0xcbf29ce484222325ull);
    h = hash_words(lg, sizeof(int32_t) * (size_t)count, h);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_plans.begin();
    for (; it != g_plans.end(); ++it)
        if (it->data == data && it->count == count && it->normalize == normalize && it->prec == prec &&
            it->hash == h && !memcmp(it->off.data(), off, sizeof(int64_t) * (size_t)count) &&
            !memcmp(it->lg.data(), lg, sizeof(int32_t) * (size_t)count))
            break;
    if (it == g_plans.end()) {
        if (g_plans.size() >= kMaxPlans) {
            // An evicted plan's graph may still be in flight on some stream.
            (void)hipDeviceSynchronize();
            release(g_plans.back());
            g_plans.pop_back();
        }
        g_plans.push_front(Plan{});
        Plan &p = g_plans.front();
        p.data = data;
        p.count = count;
        p.normalize = normalize;
        p.prec = prec;
        p.hash = h;
        p.off.assign(off, off + count);
        p.lg.assign(lg, lg + count);
        int rc = make_plan(p, data, off, lg, count, normalize, prec);
        if (rc) {
            release(p);
            g_plans.pop_front();
            return rc;
        }
        it = g_plans.begin();
    } else if (it != g_plans.begin()) {
        g_plans.splice(g_plans.begin(), g_plans, it);
        it = g_plans.begin();
    }
    hipError_t e = hipGraphLaunch(it->exec, s);
    return e == hipSuccess ? FWHT_OK : hip_fail(e, "graph launch");
}

}  // namespace fwht

// ---------------------------------------------------------------- no-alloc
// The allocation-free variant: the work list goes to a fixed device array
// (tiles first, the segment table after them) instead of a cached plan.
namespace fwht {
namespace {

constexpr size_t kNaItemBytes = sizeof(BItem) * FWHT_NOALLOC_MAX_TRANSFORMS;
constexpr size_t kNaScratchBytes = kNaItemBytes + sizeof(int64_t) * FWHT_NOALLOC_MAX_TRANSFORMS;
static_assert(sizeof(BItem) == 16, "work-list layout");

// One copy per GPU, for the life of the process.  In host code `scratch`
// names a host-side stand-in: kernels get the device address found by
// hipGetSymbolAddress, never the name.
static __device__ __align__(256) unsigned char scratch[kNaScratchBytes];

constexpr int kNaMaxDevices = 64;
struct NoAllocDevice {
    unsigned char *ptr = nullptr;  // device address of this GPU's scratch
    int grid[3] = {0, 0, 0};       // persistent grid per precision
};
std::mutex g_na_mu;
NoAllocDevice g_na_dev[kNaMaxDevices];
// host side of the work list (one call at a time, under g_na_mu)
BItem g_na_items[FWHT_NOALLOC_MAX_TRANSFORMS];
int64_t g_na_segs[FWHT_NOALLOC_MAX_TRANSFORMS];

// The tiles of build_items (largest transforms first, a size's transforms
// in the caller's order, 2^(16-m) of them per tile) by a counting sort into
// the fixed host arrays.
int32_t build_items_fixed(const int64_t *off, const int32_t *lg, int32_t count)
{
    int32_t start[BTB + 2] = {0};
    for (int32_t t = 0; t < count; ++t) ++start[lg[t]];
    int32_t pos = 0;
    for (int m = BTB; m >= 0; --m) {
        const int32_t c = start[m];
        start[m] = pos;
        pos += c;
    }
    int32_t next[BTB + 1];
    for (int m = 0; m <= BTB; ++m) next[m] = start[m];
    for (int32_t t = 0; t < count; ++t) g_na_segs[next[lg[t]]++] = off[t];
    int32_t nitems = 0;
    for (int m = BTB; m >= 0; --m) {
        const int32_t per = 1 << (BTB - m);
        for (int32_t k = start[m]; k < next[m]; k += per)
            g_na_items[nitems++] = BItem{m, k, std::min(per, next[m] - k), 0};
    }
    return nitems;
}

}  // namespace

int batched_noalloc(float *data, const int64_t *off, const int32_t *lg, int32_t count, int normalize, int prec,
                    hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_na_mu);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    if (dev < 0 || dev >= kNaMaxDevices) return fail(FWHT_E_UNSUPPORTED, "device %d beyond %d", dev, kNaMaxDevices);
    NoAllocDevice &D = g_na_dev[dev];
    if (!D.ptr) {  // first call on this device, with it current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "scratch address");
        D.ptr = static_cast<unsigned char *>(p);
    }
    if (!D.grid[prec]) {
        int rc = grid_size(prec, &D.grid[prec]);
        if (rc) return rc;
    }
    const int32_t nitems = build_items_fixed(off, lg, count);
    BItem *d_items = reinterpret_cast<BItem *>(D.ptr);
    int64_t *d_segs = reinterpret_cast<int64_t *>(D.ptr + kNaItemBytes);
    e = hipMemcpyAsync(d_items, g_na_items, sizeof(BItem) * (size_t)nitems, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_segs, g_na_segs, sizeof(int64_t) * (size_t)count, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "work-list copy");
    BArgs a{};
    a.data = data;
    a.items = d_items;
    a.segs = d_segs;
    a.nitems = nitems;
    a.normalize = normalize;
    e = launch_batched(prec, a, std::min(D.grid[prec], nitems), s);
    return e == hipSuccess ? FWHT_OK : hip_fail(e, "batched launch");
}

}  // namespace fwht

namespace {

int check_batched_args(const float *data, const int64_t *offsets, const int32_t *log2n, int32_t count, int prec)
{
    using namespace fwht;
    if (!data || !offsets || !log2n) return fail(FWHT_E_INVAL, "NULL argument");
    if (((uintptr_t)data) & 15) return fail(FWHT_E_INVAL, "data must be 16-byte aligned");
    if (count < 1) return fail(FWHT_E_INVAL, "count must be >= 1");
    if (prec != FWHT_PREC_FP32 && prec != FWHT_PREC_FP16_MFMA && prec != FWHT_PREC_BF16_MFMA)
        return fail(FWHT_E_INVAL, "unknown precision %d", prec);
    for (int32_t t = 0; t < count; ++t) {
        if (log2n[t] < 2 || log2n[t] > 16) return fail(FWHT_E_RANGE, "log2n[%d] = %d outside [2, 16]", t, log2n[t]);
        if (offsets[t] < 0 || (offsets[t] & 3)) return fail(FWHT_E_INVAL, "offsets[%d] must be >= 0 and a multiple of 4", t);
    }
    return FWHT_OK;
}

}  // namespace

extern "C" int fwht_batched(float *data, const int64_t *offsets, const int32_t *log2n, int32_t count,
                            int normalize, int prec, void *stream)
{
    const int rc = check_batched_args(data, offsets, log2n, count, prec);
    if (rc) return rc;
    return fwht::batched(data, offsets, log2n, count, normalize, prec, (hipStream_t)stream);
}

extern "C" int fwht_batched_noalloc(float *data, const int64_t *offsets, const int32_t *log2n, int32_t count,
                                    int normalize, int prec, void *stream)
{
    if (count > FWHT_NOALLOC_MAX_TRANSFORMS)
        return fwht::fail(FWHT_E_RANGE, "count = %d above the limit of %d", count, FWHT_NOALLOC_MAX_TRANSFORMS);
    const int rc = check_batched_args(data, offsets, log2n, count, prec);
    if (rc) return rc;
    return fwht::batched_noalloc(data, offsets, log2n, count, normalize, prec, (hipStream_t)stream);
}
