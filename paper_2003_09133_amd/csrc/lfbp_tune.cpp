// Tuning table of the re-arrangement kernels.
//
// The table is a text file written by the autotuner
// (paper_2003_09133_amd/autotune.py): one entry per line,
//   <batched 0|1> <esize> <W> <nx> <variant> <threads> <rows_in_flight> <tile_bytes>
//   <vec_per_thread> <nontemporal> <persistent> <grid>
// '#' starts a comment.  It is read once, from $LFBP_TUNE_TABLE if set, else
// from lfbp_tune.txt next to liblfbp.so.  Shapes without an entry use the
// built-in defaults below.
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
    int batched, esize, W, nx;
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
        const int n = std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d %d %d", &e.batched, &e.esize, &e.W, &e.nx,
                                  &c.variant, &c.block_threads, &c.rows_in_flight, &c.tile_bytes,
                                  &c.vec_per_thread, &c.nontemporal, &c.persistent, &c.grid);
        if (n != 12) continue;
        const bool ok = c.variant >= LFBP_GATHER_DIRECT && c.variant <= LFBP_GATHER_WIDE && c.block_threads > 0 &&
                        c.rows_in_flight > 0 && c.vec_per_thread > 0 && c.nontemporal > 0 && c.persistent > 0 &&
                        check_config(&c) == LFBP_OK;
        if (ok) g_table.push_back(e);
    }
    std::fclose(fh);
}

}  // namespace

lfbp_gather_config tuned_config(const lfbp_shape& s, int esize, bool batched)
{
    std::call_once(g_once, load_table);
    const int W = int(s.ny * s.nz), nx = int(s.nx);
    for (const Entry& e : g_table)
        if (e.batched == int(batched) && e.esize == esize && e.W == W && e.nx == nx) return e.cfg;
    lfbp_gather_config c;
    c.variant = LFBP_GATHER_WIDE;
    c.block_threads = 256;
    c.rows_in_flight = 2;
    c.tile_bytes = 16384;
    c.vec_per_thread = 4;
    c.nontemporal = 1;
    c.persistent = batched ? 1 : 2;
    c.grid = 0;
    return c;
}

}  // namespace lfbp
