// fwht_tune.hip -- the autotuned schedule table.
//
// Text file, one entry per line: "<dtype> <n> <schedule> [ms]" with dtype in
// {int32, int64, float32}, or "batched <fp32|fp16|bf16> <tile groups> [ms]"
// for the batched transform; '#' starts a comment.  Looked up at
// $FWHT_TUNE_TABLE if set, else tune/gfx950.txt in the library's directory.
// Entries that do not parse against the compiled variants are ignored.
#include <dlfcn.h>

#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "fwht_internal.hpp"

namespace fwht {

static std::once_flag g_tune_once;
static std::map<std::pair<int, int>, std::string> g_tuned;
static std::string g_tuned_tiles[3];  // "batched <precision> <tile groups>"
static std::string g_tune_path;

static void load_table()
{
    const char *env = getenv("FWHT_TUNE_TABLE");
    std::string path;
    if (env && *env) {
        path = env;
    } else {
        Dl_info info;
        if (dladdr((void *)&load_table, &info) && info.dli_fname) {
            std::string lib = info.dli_fname;
            size_t sl = lib.rfind('/');
            path = (sl == std::string::npos ? std::string(".") : lib.substr(0, sl)) + "/tune/gfx950.txt";
        }
    }
    g_tune_path = path;
    std::ifstream in(path);
    if (!in) return;
    std::string line;
    while (std::getline(in, line)) {
        size_t h = line.find('#');
        if (h != std::string::npos) line = line.substr(0, h);
        std::istringstream ls(line);
        std::string dt, spec;
        int n = -1;
        if (line.compare(0, 8, "batched ") == 0) {
            std::string prec;
            ls >> dt >> prec >> spec;
            const int p = prec == "fp32" ? FWHT_PREC_FP32 : prec == "fp16" ? FWHT_PREC_FP16_MFMA
                          : prec == "bf16" ? FWHT_PREC_BF16_MFMA : -1;
            TilePlan tp;
            std::string why;
            if (p >= 0 && parse_tiles(p, spec, tp, why)) g_tuned_tiles[p] = spec;
            continue;
        }
        if (!(ls >> dt >> n >> spec)) continue;
        int d = dt == "int32" ? FWHT_I32 : dt == "int64" ? FWHT_I64 : dt == "float32" ? FWHT_F32 : -1;
        if (d < 0 || n < 1 || n > 40) continue;
        std::vector<Pass> p;
        std::string why;
        if (!parse_schedule(d, n, spec, p, why)) continue;
        g_tuned[{d, n}] = spec;
    }
}

const std::string *tuned_batched_tiles(int prec)
{
    std::call_once(g_tune_once, load_table);
    return prec >= 0 && prec < 3 && !g_tuned_tiles[prec].empty() ? &g_tuned_tiles[prec] : nullptr;
}

const std::string *tuned_schedule(int dtype, int n)
{
    std::call_once(g_tune_once, load_table);
    auto it = g_tuned.find({dtype, n});
    return it == g_tuned.end() ? nullptr : &it->second;
}

}  // namespace fwht
