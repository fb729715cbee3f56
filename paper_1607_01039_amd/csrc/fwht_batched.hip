// fwht_batched.hip -- host side of the batched persistent transform: tile
// groups, work-list planning, device buffers, a cached HIP graph per
// request, and the allocation-free variant.
//
// Transforms are routed by size to tile groups: a group "tb:lo-hi" gathers
// the transforms of 2^lo .. 2^hi entries into tiles of 2^tb entries (2^16
// tiles in 1024 threads, one workgroup per CU; 2^15 tiles in 512 threads and
// 2^14 tiles in 256 threads, two and four workgroups per CU, so that one
// workgroup's loads and stores overlap another's LDS phases).  Each group is
// one persistent launch.  A request's work list is built and uploaded once
// and cached; later calls with the same request launch its kernels straight
// from the cached list, or (fwht_set_batched_graphs) replay a HIP graph
// captured from those launches.  Direct launches are the default: measured
// on this stack, replaying a one-kernel graph costs 15 us of host time and
// 12 us more latency than launching the kernel itself (2.5 us and 6.8 us).
// The FP32 grouping comes from the tuned table ("batched fp32 <groups>") or
// fwht_set_batched_tiles; the matrix-core kernels use 2^16 tiles only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <list>
#include <mutex>
#include <string>
#include <vector>

#include "fwht_internal.hpp"
#include "wht_batched.hpp"

namespace fwht {

template <int TB, int NT>
__global__ void __launch_bounds__(NT, 1024 / NT) batched_kernel(BArgs a)
{
    BatchedKernel<TB, NT>::run(a);
}

namespace {

constexpr int BTB = BATCH_TB;  // largest tile: 2^16 entries

// ------------------------------------------------------------- tile groups
std::mutex g_tiles_mu;
bool g_tiles_set[3] = {false, false, false};
TilePlan g_tiles_override[3];

TilePlan default_tiles(int prec)
{
    TilePlan p;
    if (prec == FWHT_PREC_FP32) {
        const std::string *tuned = tuned_batched_tiles(prec);
        std::string why;
        if (tuned && parse_tiles(prec, *tuned, p, why)) return p;
    }
    p.n = 1;
    p.g[0] = TileGroup{BTB, 2, BTB};
    return p;
}

TilePlan tiles_for(int prec)
{
    std::lock_guard<std::mutex> lk(g_tiles_mu);
    return g_tiles_set[prec] ? g_tiles_override[prec] : default_tiles(prec);
}

bool same_tiles(const TilePlan &a, const TilePlan &b)
{
    if (a.n != b.n) return false;
    for (int i = 0; i < a.n; ++i)
        if (a.g[i].tb != b.g[i].tb || a.g[i].lo != b.g[i].lo || a.g[i].hi != b.g[i].hi) return false;
    return true;
}

hipError_t group_occupancy(int prec, int tb, int *per)
{
    if (prec != FWHT_PREC_FP32) return batched_mfma_occupancy(prec, per);
    if (tb == 16) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, batched_kernel<16, 1024>, 1024, 0);
    if (tb == 15) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, batched_kernel<15, 512>, 512, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, batched_kernel<14, 256>, 256, 0);
}

// Persistent grid of a group: the resident workgroups of its kernel.
int grid_size(int prec, int tb, int *out)
{
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    e = group_occupancy(prec, tb, &per);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    *out = cus * std::max(per, 1);
    return FWHT_OK;
}

hipError_t launch_group(int prec, int tb, const BArgs &a, int grid, hipStream_t s)
{
    if (prec != FWHT_PREC_FP32) return tb == 16 ? launch_batched_mfma(prec, a, grid, s) : hipErrorInvalidValue;
    if (tb == 16)
        hipLaunchKernelGGL((batched_kernel<16, 1024>), dim3(grid), dim3(1024), 0, s, a);
    else if (tb == 15)
        hipLaunchKernelGGL((batched_kernel<15, 512>), dim3(grid), dim3(512), 0, s, a);
    else if (tb == 14)
        hipLaunchKernelGGL((batched_kernel<14, 256>), dim3(grid), dim3(256), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Work list of one request: for each group, its tiles in hand-out order
// (transforms sorted by decreasing size, a size's transforms in the caller's
// order, 2^(tb - m) transforms of size 2^m per tile; the last tile of a size
// may hold fewer), written to items[] and the segment table (entry offsets,
// indexed by BItem::seg0) to segs[].  A counting sort over the sizes; a work
// list never has more tiles than transforms.
struct GroupRange {
    int32_t item0 = 0, nitems = 0;
};

void build_work_list(const TilePlan &tp, const int64_t *off, const int32_t *lg, int32_t count, BItem *items,
                     int64_t *segs, GroupRange *gr)
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
    for (int32_t t = 0; t < count; ++t) segs[next[lg[t]]++] = off[t];
    int32_t nitems = 0;
    for (int gi = 0; gi < tp.n; ++gi) {
        const TileGroup &G = tp.g[gi];
        gr[gi].item0 = nitems;
        for (int m = G.hi; m >= G.lo; --m) {
            const int32_t per = 1 << (G.tb - m);
            for (int32_t k = start[m]; k < next[m]; k += per)
                items[nitems++] = BItem{m, k, std::min(per, next[m] - k), 0};
        }
        gr[gi].nitems = nitems - gr[gi].item0;
    }
}

// Launch every non-empty group of a work list already in device memory.
hipError_t launch_work_list(int prec, const TilePlan &tp, const GroupRange *gr, const int *grid, float *data,
                            const BItem *items, const int64_t *segs, int normalize, hipStream_t s)
{
    for (int gi = 0; gi < tp.n; ++gi) {
        if (!gr[gi].nitems) continue;
        BArgs a{};
        a.data = data;
        a.items = items + gr[gi].item0;
        a.segs = segs;
        a.nitems = gr[gi].nitems;
        a.normalize = normalize;
        const hipError_t e = launch_group(prec, tp.g[gi].tb, a, std::min(grid[gi], gr[gi].nitems), s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------- cached graph path
struct Plan {
    // key
    float *data = nullptr;
    int32_t count = 0;
    int normalize = 0, prec = 0;
    TilePlan tiles;
    std::vector<int64_t> off;  // the request itself
    std::vector<int32_t> lg;
    // device state
    BItem *items = nullptr;
    int64_t *segs = nullptr;
    GroupRange gr[3];
    int grid[3] = {0, 0, 0};
    hipGraphExec_t exec = nullptr;  // captured on the first replay in graph mode
    hipGraph_t graph = nullptr;
};

std::mutex g_mu;
std::list<Plan> g_plans;  // most recent first
constexpr size_t kMaxPlans = 8;
hipStream_t g_capture = nullptr;
std::atomic<int> g_use_graphs{0};

void release(Plan &p)
{
    if (p.exec) (void)hipGraphExecDestroy(p.exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    if (p.items) (void)hipFree(p.items);
    if (p.segs) (void)hipFree(p.segs);
    p = Plan{};
}

int make_plan(Plan &p, const int64_t *off, const int32_t *lg, int32_t count, int prec)
{
    std::vector<BItem> items((size_t)count);
    std::vector<int64_t> segs((size_t)count);
    build_work_list(p.tiles, off, lg, count, items.data(), segs.data(), p.gr);
    const size_t nitems = (size_t)(p.gr[p.tiles.n - 1].item0 + p.gr[p.tiles.n - 1].nitems);
    hipError_t e = hipMalloc(&p.items, sizeof(BItem) * nitems);
    if (e == hipSuccess) e = hipMalloc(&p.segs, sizeof(int64_t) * segs.size());
    if (e != hipSuccess) return fail(FWHT_E_NOMEM, "batched plan: %s", hipGetErrorString(e));
    e = hipMemcpy(p.items, items.data(), sizeof(BItem) * nitems, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p.segs, segs.data(), sizeof(int64_t) * segs.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batched plan upload");

    for (int gi = 0; gi < p.tiles.n; ++gi) {
        const int rc = grid_size(prec, p.tiles.g[gi].tb, &p.grid[gi]);
        if (rc) return rc;
    }
    return FWHT_OK;
}

// The graph of a plan: the persistent launch of each group, one after another
// (work is assigned statically, so there is no counter to reset between
// replays).
int capture_graph(Plan &p)
{
    hipError_t e = hipSuccess;
    if (p.graph) {  // left by an earlier capture that failed to instantiate
        (void)hipGraphDestroy(p.graph);
        p.graph = nullptr;
    }
    if (!g_capture) {
        e = hipStreamCreateWithFlags(&g_capture, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "capture stream");
    }
    e = hipStreamBeginCapture(g_capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    const hipError_t le =
        launch_work_list(p.prec, p.tiles, p.gr, p.grid, p.data, p.items, p.segs, p.normalize, g_capture);
    e = hipStreamEndCapture(g_capture, &p.graph);
    if (le != hipSuccess) return hip_fail(le, "batched launch (capture)");
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiate(&p.exec, p.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    return FWHT_OK;
}

}  // namespace

// "tb:lo-hi" (or "tb:m") groups separated by commas; every size 2^2 .. 2^16
// in exactly one group, lo <= hi <= tb; tb in {14, 15, 16}, and only 16 for
// the matrix-core precisions.
bool parse_tiles(int prec, const std::string &spec, TilePlan &out, std::string &why)
{
    TilePlan p;
    int covered[BTB + 1] = {0};
    size_t pos = 0;
    while (pos <= spec.size()) {
        size_t e = spec.find(',', pos);
        const std::string tok = spec.substr(pos, e == std::string::npos ? std::string::npos : e - pos);
        pos = e == std::string::npos ? spec.size() + 1 : e + 1;
        if (tok.empty()) continue;
        int tb = 0, lo = 0, hi = 0, used = 0;
        if (sscanf(tok.c_str(), "%d:%d-%d%n", &tb, &lo, &hi, &used) == 3 && used == (int)tok.size()) {
        } else if (sscanf(tok.c_str(), "%d:%d%n", &tb, &lo, &used) == 2 && used == (int)tok.size()) {
            hi = lo;
        } else {
            why = "bad group '" + tok + "'";
            return false;
        }
        if (tb < 14 || tb > BTB || (prec != FWHT_PREC_FP32 && tb != BTB)) {
            why = "unsupported tile size in '" + tok + "'";
            return false;
        }
        if (lo < 2 || lo > hi || hi > tb) {
            why = "size range outside [2, tile] in '" + tok + "'";
            return false;
        }
        if (p.n == 3) {
            why = "at most three groups";
            return false;
        }
        for (int m = lo; m <= hi; ++m) ++covered[m];
        p.g[p.n++] = TileGroup{tb, lo, hi};
    }
    for (int m = 2; m <= BTB; ++m)
        if (covered[m] != 1) {
            why = "every size 2^2 .. 2^16 must be in exactly one group";
            return false;
        }
    out = p;
    return true;
}

std::string tiles_to_string(const TilePlan &p)
{
    std::string s;
    for (int i = 0; i < p.n; ++i) {
        if (i) s += ",";
        s += std::to_string(p.g[i].tb) + ":" + std::to_string(p.g[i].lo);
        if (p.g[i].hi != p.g[i].lo) s += "-" + std::to_string(p.g[i].hi);
    }
    return s;
}

int batched(float *data, const int64_t *off, const int32_t *lg, int32_t count, int normalize, int prec,
            hipStream_t s)
{
    const TilePlan tiles = tiles_for(prec);
    std::lock_guard<std::mutex> lk(g_mu);
    // A plan matches only when its request is the same, arrays included: a
    // straight comparison (1 us for 4096 transforms) costs less than any
    // hash of them, whose dependency chain took 13 us.
    auto it = g_plans.begin();
    for (; it != g_plans.end(); ++it)
        if (it->data == data && it->count == count && it->normalize == normalize && it->prec == prec &&
            same_tiles(it->tiles, tiles) && !memcmp(it->lg.data(), lg, sizeof(int32_t) * (size_t)count) &&
            !memcmp(it->off.data(), off, sizeof(int64_t) * (size_t)count))
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
        p.tiles = tiles;
        p.off.assign(off, off + count);
        p.lg.assign(lg, lg + count);
        int rc = make_plan(p, off, lg, count, prec);
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
    if (g_use_graphs.load(std::memory_order_relaxed)) {
        if (!it->exec) {
            const int rc = capture_graph(*it);
            if (rc) return rc;
        }
        const hipError_t e = hipGraphLaunch(it->exec, s);
        return e == hipSuccess ? FWHT_OK : hip_fail(e, "graph launch");
    }
    const hipError_t e =
        launch_work_list(prec, it->tiles, it->gr, it->grid, data, it->items, it->segs, normalize, s);
    return e == hipSuccess ? FWHT_OK : hip_fail(e, "batched launch");
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
    int grid[3][BTB + 1] = {};     // persistent grid per precision and tile size
};
std::mutex g_na_mu;
NoAllocDevice g_na_dev[kNaMaxDevices];
// host side of the work list (one call at a time, under g_na_mu)
BItem g_na_items[FWHT_NOALLOC_MAX_TRANSFORMS];
int64_t g_na_segs[FWHT_NOALLOC_MAX_TRANSFORMS];

}  // namespace

int batched_noalloc(float *data, const int64_t *off, const int32_t *lg, int32_t count, int normalize, int prec,
                    hipStream_t s)
{
    const TilePlan tiles = tiles_for(prec);
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
    int grid[3] = {0, 0, 0};
    for (int gi = 0; gi < tiles.n; ++gi) {
        int &g = D.grid[prec][tiles.g[gi].tb];
        if (!g) {
            const int rc = grid_size(prec, tiles.g[gi].tb, &g);
            if (rc) return rc;
        }
        grid[gi] = g;
    }
    GroupRange gr[3];
    build_work_list(tiles, off, lg, count, g_na_items, g_na_segs, gr);
    const int32_t nitems = gr[tiles.n - 1].item0 + gr[tiles.n - 1].nitems;
    BItem *d_items = reinterpret_cast<BItem *>(D.ptr);
    int64_t *d_segs = reinterpret_cast<int64_t *>(D.ptr + kNaItemBytes);
    e = hipMemcpyAsync(d_items, g_na_items, sizeof(BItem) * (size_t)nitems, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_segs, g_na_segs, sizeof(int64_t) * (size_t)count, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "work-list copy");
    e = launch_work_list(prec, tiles, gr, grid, data, d_items, d_segs, normalize, s);
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

extern "C" int fwht_set_batched_tiles(int prec, const char *spec)
{
    using namespace fwht;
    if (prec != FWHT_PREC_FP32 && prec != FWHT_PREC_FP16_MFMA && prec != FWHT_PREC_BF16_MFMA)
        return fail(FWHT_E_INVAL, "unknown precision %d", prec);
    TilePlan p;
    std::string why;
    if (spec && !parse_tiles(prec, spec, p, why)) return fail(FWHT_E_INVAL, "bad tile groups '%s': %s", spec, why.c_str());
    std::lock_guard<std::mutex> lk(g_tiles_mu);
    g_tiles_set[prec] = spec != nullptr;
    g_tiles_override[prec] = p;
    return FWHT_OK;
}

extern "C" int fwht_get_batched_tiles(int prec, char *buf, int len)
{
    using namespace fwht;
    if (prec != FWHT_PREC_FP32 && prec != FWHT_PREC_FP16_MFMA && prec != FWHT_PREC_BF16_MFMA)
        return fail(FWHT_E_INVAL, "unknown precision %d", prec);
    if (!buf || len < 1) return fail(FWHT_E_INVAL, "NULL or empty buffer");
    const std::string s = tiles_to_string(tiles_for(prec));
    if ((int)s.size() + 1 > len) return fail(FWHT_E_CAPACITY, "buffer of %d bytes too small", len);
    memcpy(buf, s.c_str(), s.size() + 1);
    return FWHT_OK;
}

extern "C" int fwht_set_batched_graphs(int on)
{
    fwht::g_use_graphs.store(on != 0, std::memory_order_relaxed);
    return FWHT_OK;
}

extern "C" int fwht_get_batched_graphs(void) { return fwht::g_use_graphs.load(std::memory_order_relaxed); }
