// Host runtime and C ABI of the H -> H' calls of liblfbp.so: argument checks,
// kernel choice and work decomposition, batched plans (device descriptor
// tables + captured hipGraphs), device set-up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "lfbp.h"
#include "lfbp_internal.h"
#include "lfbp_tune.h"
#include "lfbp_validate.h"

namespace lfbp {

hipError_t launch_gather(const GatherDesc& d, int esize, const LaunchPlan& p, hipStream_t stream);
hipError_t launch_gather_batched(const BatchArgs& a, uint32_t maxW, int esize, const LaunchPlan& p,
                                 hipStream_t stream);
hipError_t set_gather_smem_limits(int max_bytes);
hipError_t set_inplace_smem_limits(int max_bytes);
hipError_t launch_inplace(void* H, const lfbp_shape& s, int esize, int max_lds, hipStream_t stream);
hipError_t set_colmajor_smem_limits(int max_bytes);
hipError_t launch_colmajor(const void* H, void* Ht, const lfbp_shape& s, int esize, int max_lds, hipStream_t stream);
int gather_occupancy(const LaunchPlan& p, uint32_t W, int esize, bool batched);
namespace {

// ---------------------------------------------------------------- device setup

std::once_flag g_init_once;
hipError_t g_init_err = hipSuccess;
int g_max_lds = 65536;  // dynamic LDS a workgroup may use (device limit, read at init)
int g_cus = 256;

}  // namespace

namespace {

// Dynamic LDS limits of every kernel that may use more than the default 64 KB.
hipError_t set_smem_limits(int max_bytes)
{
    hipError_t e = set_gather_smem_limits(max_bytes);
    if (e == hipSuccess) e = set_inplace_smem_limits(max_bytes);
    if (e == hipSuccess) e = set_colmajor_smem_limits(max_bytes);
    return e;
}

}  // namespace

// Once per process: device limits, kernels' LDS limits.
hipError_t ensure_init()
{
    std::call_once(g_init_once, [] {
        int dev = 0, lds = 0, cus = 0;
        g_init_err = hipGetDevice(&dev);
        if (g_init_err != hipSuccess) return;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
            g_max_lds = lds;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            g_cus = cus;
        g_init_err = set_smem_limits(g_max_lds);
        if (g_init_err != hipSuccess && g_max_lds > 65536) {
            (void)hipGetLastError();
            g_max_lds = 65536;
            g_init_err = set_smem_limits(g_max_lds);
        }
    });
    return g_init_err;
}

namespace {

int round16(int64_t b) { return int((b + 15) / 16 * 16); }

// ---------------------------------------------------------------- work decomposition

// Complete a (possibly partial) user configuration with the tuned values.
lfbp_gather_config resolve_config(const lfbp_shape& s, int esize, const lfbp_gather_config* user, bool batched)
{
    lfbp_gather_config c = tuned_config(s, esize, batched);  // every field set
    if (user) {
        if (user->variant) c.variant = user->variant;
        if (user->block_threads) c.block_threads = user->block_threads;
        if (user->rows_in_flight) c.rows_in_flight = user->rows_in_flight;
        if (user->tile_bytes) c.tile_bytes = user->tile_bytes;
        if (user->vec_per_thread) c.vec_per_thread = user->vec_per_thread;
        if (user->nontemporal) c.nontemporal = user->nontemporal;
        if (user->persistent) c.persistent = user->persistent;
        if (user->grid) c.grid = user->grid;
    }
    return c;
}

// Rows per work unit and dynamic LDS of config c for rows of W elements.
// Falls back WIDE -> STAGED -> DIRECT when a row does not fit.  ntab = row
// tables the WIDE kernel keeps (2 when pipelined).
void decompose(uint32_t W, int es, lfbp_gather_config& c, uint32_t& rows, int& lds)
{
    const int64_t ve = 16 / es;
    if (c.variant == LFBP_GATHER_WIDE) {
        const int64_t vpr = (int64_t(W) + 2 * ve - 2) / ve;
        const int ntab = c.persistent == 1 ? 2 : 1;
        int64_t r = int64_t(c.vec_per_thread) * c.block_threads / vpr;
        auto need = [&](int64_t rr) { return int64_t(ntab) * rr * 16 + round16((rr * W + 2 * ve) * es); };
        while (r > 0 && need(r) > g_max_lds) --r;
        if (r > 0) {
            rows = uint32_t(r);
            lds = int(need(r));
            return;
        }
        c.variant = LFBP_GATHER_STAGED;
    }
    if (c.variant == LFBP_GATHER_STAGED) {
        int tile = std::min(c.tile_bytes, g_max_lds);
        int64_t r = (int64_t(tile) - 2 * 16) / (int64_t(W) * es);
        if (r < 1 && int64_t(W) * es + 32 <= g_max_lds) {
            tile = round16(int64_t(W) * es + 32);
            r = 1;
        }
        if (r >= 1) {
            rows = uint32_t(r);
            lds = tile;
            return;
        }
        c.variant = LFBP_GATHER_DIRECT;
    }
    rows = uint32_t(c.block_threads / 64 * c.rows_in_flight);
    lds = 0;
}

GatherDesc make_desc(const void* H, void* Ht, const lfbp_shape& s, int es, uint32_t rows)
{
    GatherDesc d;
    std::memset(&d, 0, sizeof(d));
    d.H = H;
    d.Ht = Ht;
    d.E = shape_elems(s);
    d.ns = uint32_t(s.ns);
    d.nt = uint32_t(s.nt);
    d.nx = uint32_t(s.nx);
    d.ny = uint32_t(s.ny);
    d.nz = uint32_t(s.nz);
    d.W = d.ny * d.nz;
    d.NB = d.ns * d.nt;
    d.nrows = d.NB * d.nx;
    const uint32_t hs = (d.ns - 1) / 2, ht = (d.nt - 1) / 2;
    d.a_off = (d.nx - hs % d.nx) % d.nx;  // s' - hs == s' + a_off (mod nx)
    d.b_off = (d.ny - ht % d.ny) % d.ny;
    d.fnx = make_fastdiv(d.nx);
    d.fny = make_fastdiv(d.ny);
    d.fnt = make_fastdiv(d.nt);
    d.rows_per_unit = std::max<uint32_t>(1, std::min(rows, d.nrows));
    d.nunits = (d.nrows + d.rows_per_unit - 1) / d.rows_per_unit;
    const uint32_t ve = 16 / uint32_t(es);
    d.phase_in = uint32_t((reinterpret_cast<uintptr_t>(H) / uintptr_t(es)) % ve);
    d.phase_out = uint32_t((reinterpret_cast<uintptr_t>(Ht) / uintptr_t(es)) % ve);
    d.vpr = (d.W + 2 * ve - 2) / ve;
    d.fvpr = make_fastdiv(d.vpr);
    d.xcd_remap = 1;
    return d;
}

LaunchPlan make_plan(const lfbp_gather_config& c, int lds)
{
    LaunchPlan p;
    p.variant = c.variant;
    p.threads = c.block_threads;
    p.rows_in_flight = c.rows_in_flight;
    p.vec_per_thread = c.vec_per_thread;
    p.lds_bytes = lds;
    p.nontemporal = c.nontemporal;
    p.persistent = c.persistent;
    p.grid = 0;
    return p;
}

// Largest grid whose work-items (grid x threads) fit the 32-bit dispatch size,
// a multiple of 8 (one share per XCD).  The kernels stride over their units,
// so a grid this size still covers every unit.
uint64_t max_grid(int threads)
{
    return ((uint64_t(1) << 32) - 1) / uint64_t(std::max(threads, 64)) / 8 * 8;
}

// Grid of a launch over `units` work units.
int grid_for(const lfbp_gather_config& c, LaunchPlan& p, uint32_t units, uint32_t W, int es, bool batched)
{
    if (c.persistent != 1) return int(std::min<uint64_t>(units, max_grid(p.threads)));
    int g = c.grid;
    if (g <= 0) g = g_cus * gather_occupancy(p, W, es, batched);  // a multiple of 8: one share per XCD
    return int(std::min<uint64_t>(uint64_t(g), units));
}

// ---------------------------------------------------------------- batched plans

struct BatchPlan {
    int device = -1;
    std::vector<lfbp_problem> probs;
    lfbp_dtype dtype = LFBP_F32;
    lfbp_gather_config key{};
    int use_graph = 1;
    GatherDesc* descs_dev = nullptr;      // only for batches beyond kInlineProblems
    uint32_t* unit_start_dev = nullptr;
    uint32_t maxW = 0;
    BatchArgs args{};
    LaunchPlan plan{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~BatchPlan()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (descs_dev) (void)hipFree(descs_dev);
        if (unit_start_dev) (void)hipFree(unit_start_dev);
    }
};

std::mutex g_plan_mu;
std::vector<std::unique_ptr<BatchPlan>> g_plans;

bool same_table(const BatchPlan& p, int dev, const lfbp_problem* probs, int32_t count, lfbp_dtype dt,
                const lfbp_gather_config& key, int use_graph)
{
    if (p.device != dev || p.dtype != dt || p.probs.size() != size_t(count) || p.use_graph != use_graph) return false;
    if (std::memcmp(&p.key, &key, sizeof(key)) != 0) return false;
    return std::memcmp(p.probs.data(), probs, sizeof(lfbp_problem) * size_t(count)) == 0;
}

lfbp_status build_plan(BatchPlan& bp, const lfbp_problem* probs, int32_t count, lfbp_dtype dt,
                       const lfbp_gather_config* user, int use_graph)
{
    const int es = dtype_size(dt);
    // One kernel configuration for the whole batch: the tuned choice of the
    // largest problem; each problem's work unit is then sized for it.
    int big = 0;
    for (int32_t i = 1; i < count; ++i)
        if (shape_elems(probs[i].shape) > shape_elems(probs[big].shape)) big = i;
    lfbp_gather_config c = resolve_config(probs[big].shape, es, user, true);
    // Every problem must fit the chosen variant; the first one that does not
    // moves the whole batch down (WIDE -> STAGED -> DIRECT).
    uint32_t maxW = 0;
    for (int32_t i = 0; i < count; ++i) {
        const uint32_t W = uint32_t(probs[i].shape.ny * probs[i].shape.nz);
        maxW = std::max(maxW, W);
        uint32_t r;
        int l;
        decompose(W, es, c, r, l);
    }
    std::vector<uint32_t> rows(static_cast<size_t>(count));
    int lds = 0;
    uint32_t max_rows = 0;
    for (int32_t i = 0; i < count; ++i) {
        const uint32_t W = uint32_t(probs[i].shape.ny * probs[i].shape.nz);
        lfbp_gather_config ci = c;
        int l = 0;
        decompose(W, es, ci, rows[size_t(i)], l);
        max_rows = std::max(max_rows, rows[size_t(i)]);
        if (c.variant == LFBP_GATHER_WIDE) {
            const int64_t ve = 16 / es;
            l = round16((int64_t(rows[size_t(i)]) * W + 2 * ve) * es);  // tile only; tables added below
        }
        lds = std::max(lds, l);
    }
    if (c.variant == LFBP_GATHER_WIDE) lds += (c.persistent == 1 ? 2 : 1) * int(max_rows) * 16;
    if (lds > g_max_lds) return LFBP_ESHAPE;
    std::vector<GatherDesc> descs(static_cast<size_t>(count));
    std::vector<uint32_t> start(static_cast<size_t>(count) + 1, 0);
    for (int32_t i = 0; i < count; ++i) {
        descs[size_t(i)] = make_desc(probs[i].H, probs[i].Ht, probs[i].shape, es, rows[size_t(i)]);
        const uint64_t next = uint64_t(start[size_t(i)]) + descs[size_t(i)].nunits;
        if (next >= (uint64_t(1) << 31)) return LFBP_ESHAPE;
        start[size_t(i) + 1] = uint32_t(next);
    }
    const uint32_t total = start[size_t(count)];
    LaunchPlan lp = make_plan(c, lds);
    lp.grid = grid_for(c, lp, total, maxW, es, true);
    BatchArgs& a = bp.args;
    std::memset(&a, 0, sizeof(a));
    a.count = uint32_t(count);
    a.total = total;
    a.max_rows = max_rows;
    a.nt = c.nontemporal == 1 ? 1 : 0;
    if (uint32_t(count) <= kInlineProblems) {
        for (int32_t i = 0; i < count; ++i) a.d[i] = descs[size_t(i)];
        for (int32_t i = 0; i <= count; ++i) a.start[i] = start[size_t(i)];
    } else {
        if (hipMalloc(reinterpret_cast<void**>(&bp.descs_dev), sizeof(GatherDesc) * size_t(count)) != hipSuccess)
            return LFBP_ENOMEM;
        if (hipMalloc(reinterpret_cast<void**>(&bp.unit_start_dev), sizeof(uint32_t) * (size_t(count) + 1)) !=
            hipSuccess)
            return LFBP_ENOMEM;
        if (hipMemcpy(bp.descs_dev, descs.data(), sizeof(GatherDesc) * size_t(count), hipMemcpyHostToDevice) !=
            hipSuccess)
            return LFBP_EDEVICE;
        if (hipMemcpy(bp.unit_start_dev, start.data(), sizeof(uint32_t) * (size_t(count) + 1),
                      hipMemcpyHostToDevice) != hipSuccess)
            return LFBP_EDEVICE;
        a.table = bp.descs_dev;
        a.table_start = bp.unit_start_dev;
    }
    bp.maxW = maxW;
    bp.plan = lp;
    bp.dtype = dt;
    bp.use_graph = use_graph;
    bp.probs.assign(probs, probs + count);
    if (use_graph) {
        hipStream_t cs = nullptr;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return LFBP_EDEVICE;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t le = launch_gather_batched(bp.args, bp.maxW, es, lp, cs);
            e = hipStreamEndCapture(cs, &bp.graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&bp.exec, bp.graph, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) return LFBP_EDEVICE;
    }
    return LFBP_OK;
}

lfbp_status validate_batch(const lfbp_problem* probs, int32_t count, lfbp_dtype dt)
{
    if (!probs || count <= 0) return LFBP_EINVAL;
    const int es = dtype_size(dt);
    if (es == 0) return LFBP_EDTYPE;
    for (int32_t i = 0; i < count; ++i) {
        const lfbp_status st = check_gather(probs[i].H, probs[i].Ht, probs[i].shape, dt);
        if (st != LFBP_OK) return st;
    }
    // No output may overlap any input or any other output (inputs may overlap
    // each other).  Sweep the byte ranges in address order: a range that starts
    // before the furthest end seen so far of a conflicting kind overlaps it.
    struct Range {
        uint64_t begin, end;
        bool out;
    };
    std::vector<Range> r;
    r.reserve(2 * static_cast<size_t>(count));
    for (int32_t i = 0; i < count; ++i) {
        const uint64_t b = shape_elems(probs[i].shape) * uint64_t(es);
        const uint64_t h = reinterpret_cast<uint64_t>(probs[i].H), o = reinterpret_cast<uint64_t>(probs[i].Ht);
        r.push_back({h, h + b, false});
        r.push_back({o, o + b, true});
    }
    std::sort(r.begin(), r.end(), [](const Range& a, const Range& b) { return a.begin < b.begin; });
    uint64_t end_in = 0, end_out = 0;
    for (const Range& x : r) {
        if (x.begin < end_out || (x.out && x.begin < end_in)) return LFBP_EALIAS;
        if (x.out)
            end_out = std::max(end_out, x.end);
        else
            end_in = std::max(end_in, x.end);
    }
    return LFBP_OK;
}

}  // namespace
}  // namespace lfbp

using namespace lfbp;

extern "C" {

const char* lfbp_status_string(lfbp_status s)
{
    switch (s) {
        case LFBP_OK: return "ok";
        case LFBP_EINVAL: return "invalid argument (null pointer, count, image size or config field)";
        case LFBP_ESHAPE: return "invalid shape (dimension < 1, even ns/nt/nx/ny, or size limit exceeded)";
        case LFBP_EDTYPE: return "unsupported element type";
        case LFBP_EALIAS: return "input and output memory overlap";
        case LFBP_EDEVICE: return "HIP device error";
        case LFBP_ENOMEM: return "out of memory";
        case LFBP_EALIGN: return "pointer not aligned to its element size";
        default: return "unknown status";
    }
}

const char* lfbp_version(void) { return "lfbp 0.2 gfx950"; }

lfbp_status lfbp_default_config(lfbp_shape shape, lfbp_dtype dtype, lfbp_gather_config* cfg)
{
    if (!cfg) return LFBP_EINVAL;
    const int es = dtype_size(dtype);
    if (es == 0) return LFBP_EDTYPE;
    const lfbp_status st = check_shape(shape, es);
    if (st != LFBP_OK) return st;
    lfbp_gather_config c = resolve_config(shape, es, nullptr, false);
    uint32_t rows = 0;
    int lds = 0;
    decompose(uint32_t(shape.ny * shape.nz), es, c, rows, lds);
    if (c.grid == 0) {
        const GatherDesc d = make_desc(nullptr, nullptr, shape, es, rows);
        c.grid = c.persistent == 1 ? g_cus : int(std::min<uint64_t>(d.nunits, max_grid(c.block_threads)));
    }
    *cfg = c;
    return LFBP_OK;
}

lfbp_status lfbp_compute_Ht_config(const void* H, void* Ht, lfbp_shape shape, lfbp_dtype dtype,
                                   const lfbp_gather_config* cfg, void* stream)
{
    lfbp_status st = check_gather(H, Ht, shape, dtype);
    if (st != LFBP_OK) return st;
    st = check_config(cfg);
    if (st != LFBP_OK) return st;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    const int es = dtype_size(dtype);
    lfbp_gather_config c = resolve_config(shape, es, cfg, false);
    uint32_t rows = 0;
    int lds = 0;
    const uint32_t W = uint32_t(shape.ny * shape.nz);
    decompose(W, es, c, rows, lds);
    const GatherDesc d = make_desc(H, Ht, shape, es, rows);
    LaunchPlan p = make_plan(c, lds);
    p.grid = grid_for(c, p, d.nunits, W, es, false);
    return launch_gather(d, es, p, static_cast<hipStream_t>(stream)) == hipSuccess ? LFBP_OK : LFBP_EDEVICE;
}

lfbp_status lfbp_compute_Ht(const void* H, void* Ht, lfbp_shape shape, lfbp_dtype dtype, void* stream)
{
    return lfbp_compute_Ht_config(H, Ht, shape, dtype, nullptr, stream);
}

lfbp_status lfbp_compute_Ht_batched_config(const lfbp_problem* problems, int32_t count, lfbp_dtype dtype,
                                           const lfbp_gather_config* cfg, int32_t use_graph, void* stream)
{
    lfbp_status st = validate_batch(problems, count, dtype);
    if (st != LFBP_OK) return st;
    st = check_config(cfg);
    if (st != LFBP_OK) return st;
    if (use_graph != 0 && use_graph != 1) return LFBP_EINVAL;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LFBP_EDEVICE;
    lfbp_gather_config key{};
    if (cfg) key = *cfg;
    std::lock_guard<std::mutex> lock(g_plan_mu);
    BatchPlan* plan = nullptr;
    for (auto& p : g_plans)
        if (same_table(*p, dev, problems, count, dtype, key, use_graph)) {
            plan = p.get();
            break;
        }
    if (!plan) {
        auto bp = std::make_unique<BatchPlan>();
        bp->device = dev;
        bp->key = key;
        st = build_plan(*bp, problems, count, dtype, cfg, use_graph);
        if (st != LFBP_OK) return st;
        g_plans.push_back(std::move(bp));
        plan = g_plans.back().get();
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (plan->use_graph)
        e = hipGraphLaunch(plan->exec, s);
    else
        e = launch_gather_batched(plan->args, plan->maxW, dtype_size(dtype), plan->plan, s);
    return e == hipSuccess ? LFBP_OK : LFBP_EDEVICE;
}

lfbp_status lfbp_compute_Ht_batched(const lfbp_problem* problems, int32_t count, lfbp_dtype dtype, void* stream)
{
    // a direct launch: replaying the plan's one-kernel graph costs more host
    // time per call than launching the kernel (measured on small tables)
    return lfbp_compute_Ht_batched_config(problems, count, dtype, nullptr, 0, stream);
}

lfbp_status lfbp_compute_Ht_inplace(void* H, lfbp_shape shape, lfbp_dtype dtype, void* stream)
{
    if (!H) return LFBP_EINVAL;
    const int es = dtype_size(dtype);
    if (es == 0) return LFBP_EDTYPE;
    const lfbp_status st = check_shape(shape, es);
    if (st != LFBP_OK) return st;
    if (reinterpret_cast<uintptr_t>(H) % uintptr_t(es)) return LFBP_EALIGN;
    // one x-row of block O and its partner row must fit the LDS together
    if (uint64_t(shape.ny) * uint64_t(shape.nz) * uint64_t(es) * 2 > uint64_t(kInplaceMinLds)) return LFBP_ESHAPE;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return launch_inplace(H, shape, es, g_max_lds, static_cast<hipStream_t>(stream)) == hipSuccess ? LFBP_OK
                                                                                               : LFBP_EDEVICE;
}

lfbp_status lfbp_compute_Ht_colmajor(const void* H, void* Ht, lfbp_shape shape, lfbp_dtype dtype, void* stream)
{
    const lfbp_status st = check_gather(H, Ht, shape, dtype);
    if (st != LFBP_OK) return st;
    const int es = dtype_size(dtype);
    // nx <= 2048: a 16-byte vector of each of the nx rows of an input plane
    // and the kernel's row table fit in the 64 KB of LDS every device
    // provides; the grid (at most one workgroup per s-position of every
    // plane) must fit the 32-bit grid size
    if (shape.nx > 2048) return LFBP_ESHAPE;
    const uint64_t planes = uint64_t(shape.nt) * uint64_t(shape.ny) * uint64_t(shape.nz);
    if (planes * uint64_t(shape.ns) >= (uint64_t(1) << 31)) return LFBP_ESHAPE;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return launch_colmajor(H, Ht, shape, es, g_max_lds, static_cast<hipStream_t>(stream)) == hipSuccess
               ? LFBP_OK
               : LFBP_EDEVICE;
}

void lfbp_release_plans(void)
{
    std::lock_guard<std::mutex> lock(g_plan_mu);
    g_plans.clear();
}

}  // extern "C"
