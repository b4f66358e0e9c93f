// Tuning table of the re-arrangement kernels.
//
// The table is a text file written by the autotuner
// (paper_2003_09133_amd/autotune.py), one entry per line, of two kinds:
//   shape <batched 0|1> <esize> <ns> <nt> <nx> <ny> <nz> <config>
//   class <batched 0|1> <esize> <row class> <config>
// where <config> is <variant> <threads> <rows_in_flight> <tile_bytes>
// <vec_per_thread> <nontemporal> <persistent> <grid> <waves_per_eu>
// <schedule>.  '#' starts a comment.  A shape entry serves that exact shape
// (for a batch: the shape of its largest problem).  The row class of a shape
// is floor(log2(ny*nz*esize)), the size class of an x-row in bytes: the
// kernels' work decomposition follows the row size.  A shape with no entry of
// its own takes the entry of its row class, else the entry of the nearest
// class (same batched flag; a class step counts twice as much as a different
// element size), else the built-in defaults below.  The table is read once,
// from $LFBP_TUNE_TABLE if set, else from lfbp_tune.txt next to liblfbp.so.
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
    int batched, esize, cls;  // cls < 0: a shape entry
    int64_t dims[5];
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

// Parse the ten configuration fields at p; true if all are present, valid
// and nothing follows them.
bool parse_config(const char* p, lfbp_gather_config& c)
{
    int extra = 0;
    const int n = std::sscanf(p, "%d %d %d %d %d %d %d %d %d %d %d", &c.variant, &c.block_threads,
                              &c.rows_in_flight, &c.tile_bytes, &c.vec_per_thread, &c.nontemporal, &c.persistent,
                              &c.grid, &c.waves_per_eu, &c.schedule, &extra);
    return n == 10 && c.variant >= LFBP_GATHER_DIRECT && c.variant <= LFBP_GATHER_WIDE && c.block_threads > 0 &&
           c.rows_in_flight > 0 && c.vec_per_thread > 0 && c.nontemporal > 0 && c.persistent > 0 &&
           c.waves_per_eu > 0 && c.schedule > 0 && check_config(&c) == LFBP_OK;
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
        char kind[16] = {0};
        int used = 0;
        if (std::sscanf(line, "%15s %d %d%n", kind, &e.batched, &e.esize, &used) != 3) continue;
        if ((e.batched != 0 && e.batched != 1) || (e.esize != 2 && e.esize != 4)) continue;
        const char* rest = line + used;
        int more = 0;
        if (std::strcmp(kind, "class") == 0) {
            if (std::sscanf(rest, "%d%n", &e.cls, &more) != 1 || e.cls < 0 || e.cls >= 64) continue;
        } else if (std::strcmp(kind, "shape") == 0) {
            long long d[5];
            if (std::sscanf(rest, "%lld %lld %lld %lld %lld%n", &d[0], &d[1], &d[2], &d[3], &d[4], &more) != 5)
                continue;
            for (int i = 0; i < 5; ++i) e.dims[i] = d[i];
            e.cls = -1;
        } else {
            continue;
        }
        if (parse_config(rest + more, e.cfg)) g_table.push_back(e);
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
    const int64_t dims[5] = {s.ns, s.nt, s.nx, s.ny, s.nz};
    for (const Entry& e : g_table)
        if (e.cls < 0 && e.batched == int(batched) && e.esize == esize && std::memcmp(e.dims, dims, sizeof(dims)) == 0)
            return e.cfg;
    const int cls = row_class(s, esize);
    const Entry* best = nullptr;
    int best_score = 0;
    for (const Entry& e : g_table) {
        if (e.cls < 0 || e.batched != int(batched)) continue;
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
