// Tuning table of the re-arrangement kernels.
//
// The table is a text file written by the autotuner
// (paper_2003_09133_amd/autotune.py): one entry per line,
//   <batched 0|1> <esize> <row class> <variant> <threads> <rows_in_flight>
//   <tile_bytes> <vec_per_thread> <nontemporal> <persistent> <grid>
//   <waves_per_eu> <schedule>
// '#' starts a comment.  The row class of a shape is floor(log2(ny*nz*esize)),
// the size class of an x-row in bytes: the kernels' work decomposition, and so
// their best configuration, follows the row size.  A shape takes the entry of
// its own class, else the entry of the nearest class (same batched flag; a
// class step counts twice as much as a different element size), else the
// built-in defaults below.  The table is read once, from $LFBP_TUNE_TABLE if
// set, else from lfbp_tune.txt next to liblfbp.so.
#include "lfbp_tune.h"

#include <dlfcn.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lfbp_validate.h"

namespace lfbp {

namespace {

struct Entry {
    int batched, esize, cls;
    lfbp_gather_config cfg;
};

std::once_flag g_once;
std::vector<Entry> g_table;

std::string table_path()
{
    const char* env = std::getenv("LFBP_TUNE_TABLE");
    if (env && *env) return env;
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&tuned_config), &info) && info.dli_fname) {
        std::string p(info.dli_fname);
        const size_t slash = p.find_last_of('/');
        return (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) + "/lfbp_tune.txt";
    }
    return "lfbp_tune.txt";
}

void load_table()
{
    FILE* fh = std::fopen(table_path().c_str(), "r");
    if (!fh) return;
    char line[512];
    while (std::fgets(line, sizeof(line), fh)) {
        char* hash = std::strchr(line, '#');
        if (hash) *hash = 0;
        Entry e;
        std::memset(&e, 0, sizeof(e));
        lfbp_gather_config& c = e.cfg;
        int extra = 0;
        const int n = std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d %d %d %d %d", &e.batched, &e.esize, &e.cls,
                                  &c.variant, &c.block_threads, &c.rows_in_flight, &c.tile_bytes,
                                  &c.vec_per_thread, &c.nontemporal, &c.persistent, &c.grid, &c.waves_per_eu,
                                  &c.schedule, &extra);
        if (n != 13) continue;
        const bool ok = (e.batched == 0 || e.batched == 1) && (e.esize == 2 || e.esize == 4) && e.cls >= 0 &&
                        e.cls < 64 && c.variant >= LFBP_GATHER_DIRECT && c.variant <= LFBP_GATHER_WIDE &&
                        c.block_threads > 0 && c.rows_in_flight > 0 && c.vec_per_thread > 0 && c.nontemporal > 0 &&
                        c.persistent > 0 && c.waves_per_eu > 0 && c.schedule > 0 && check_config(&c) == LFBP_OK;
        if (ok) g_table.push_back(e);
    }
    std::fclose(fh);
}

}  // namespace

int row_class(const lfbp_shape& s, int esize)
{
    uint64_t b = uint64_t(s.ny) * uint64_t(s.nz) * uint64_t(esize);
    int c = 0;
    while (b > 1) {
        b >>= 1;
        ++c;
    }
    return c;
}

lfbp_gather_config tuned_config(const lfbp_shape& s, int esize, bool batched)
{
    std::call_once(g_once, load_table);
    const int cls = row_class(s, esize);
    const Entry* best = nullptr;
    int best_score = 0;
    for (const Entry& e : g_table) {
        if (e.batched != int(batched)) continue;
        const int score = 2 * (e.cls > cls ? e.cls - cls : cls - e.cls) + (e.esize != esize ? 1 : 0);
        if (!best || score < best_score) {
            best = &e;
            best_score = score;
        }
    }
    if (best) return best->cfg;
    lfbp_gather_config c;
    c.variant = LFBP_GATHER_WIDE;
    c.block_threads = batched ? 128 : 256;
    c.rows_in_flight = 2;
    c.tile_bytes = 16384;
    c.vec_per_thread = 4;
    c.nontemporal = batched ? 2 : 1;
    c.persistent = 2;
    c.grid = 0;
    c.waves_per_eu = 8;
    c.schedule = 1;
    return c;
}

}  // namespace lfbp
