// fwht_internal.hpp -- declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "fwht.h"

namespace fwht {

struct PassArgs;
struct BArgs;

// One compiled tile-kernel variant (see wht_tile.hpp): tiles of 2^TB entries,
// 2^CB contiguous columns, NT threads; COLS = contiguous pass.
struct Variant {
    const char *name;
    int TB, CB, NT;
    bool cols;
    hipError_t (*launch)(void *buf, const PassArgs &a, hipStream_t s);
    // register-resident tiles (wht_contig16.hpp) transform every bit they
    // own: a contiguous one only as a first pass followed by strided passes
    // (it carries no epilogue), a strided one only at its full height
    bool whole = false;
};

// One pass of a schedule: variant `v` transforms global bits [lo, lo + r).
struct Pass {
    const Variant *v;
    int lo, r;
};

// What the last pass applies before storing.
struct Epilogue {
    int do_scale = 0;
    float scale = 1.f;
    int thresh = 0;
    int64_t T = 0;
    float Tf = 0.f;
    uint64_t *idx = nullptr;
    void *val = nullptr;
    uint64_t cap = 0;
    uint64_t *count = nullptr;
    uint32_t kshift = 0, kL = 0;  // hit-index remap (see PassArgs)
    uint64_t kbase = 0;
    int clear_count = 0;  // run_passes clears *count before the first append
};

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

const std::vector<Variant> &registry(int dtype);
std::vector<Variant> variants_u32();
std::vector<Variant> variants_u64();
std::vector<Variant> variants_f32();
bool parse_schedule(int dtype, int n, const std::string &spec, std::vector<Pass> &out, std::string &why);
std::string schedule_for(int dtype, int n);
const std::string *tuned_schedule(int dtype, int n);
// src != nullptr: the first pass reads src and writes buf (out of place; the
// two must not overlap), the others work in place on buf
int run_passes(void *buf, int dtype, int n, uint64_t batch, const Epilogue &epi, hipStream_t s,
               const void *src = nullptr);
int run_strided_range(void *buf, int dtype, uint64_t total, int lo, int nbits, const Epilogue &epi, hipStream_t s);
int zero_count(uint64_t *count, hipStream_t s);
float float_threshold(double T);

// batched persistent path (fwht_batched.hip, fwht_mfma.hip): transforms of
// 2^lo .. 2^hi entries go to tiles of 2^tb entries
struct TileGroup {
    int tb = 16, lo = 2, hi = 16;
};
struct TilePlan {
    int n = 0;
    TileGroup g[3];
};
bool parse_tiles(int prec, const std::string &spec, TilePlan &out, std::string &why);
const std::string *tuned_batched_tiles(int prec);
hipError_t launch_batched_mfma(int prec, const BArgs &a, int grid, hipStream_t s);
hipError_t batched_mfma_occupancy(int prec, int *blocks_per_cu);
int batched(float *data, const int64_t *off, const int32_t *lg, int32_t count, int normalize, int prec,
            hipStream_t s);

// streamed Kronecker path (pinned host data), fwht_stream.hip
int streamed_int(void *host, int dtype, int n, const fwht_thresh_t *th, hipStream_t s);
// MFMA uniform-size float path, fwht_batched.hip
int mfma_uniform(float *data, int n, uint64_t batch, int normalize, int prec, hipStream_t s);

}  // namespace fwht
