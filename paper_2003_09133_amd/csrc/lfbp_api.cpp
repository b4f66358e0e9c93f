// Host runtime and C ABI of liblfbp.so: argument checks, kernel choice,
// batched plans (device descriptor tables + captured hipGraphs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "lfbp.h"
#include "lfbp_internal.h"
#include "lfbp_tune.h"
#include "lfbp_validate.h"

namespace lfbp {

hipError_t launch_gather(const GatherDesc& d, int esize, const LaunchPlan& p, hipStream_t stream);
hipError_t launch_gather_batched(const GatherDesc* descs_dev, const uint32_t* unit_start_dev, uint32_t count,
                                 uint32_t maxW, int esize, const LaunchPlan& p, hipStream_t stream);
hipError_t set_gather_smem_limits(int max_bytes);
int batched_occupancy(int variant, uint32_t maxW, int esize, int U, int threads, int smem);
hipError_t launch_forward(const float* H, const lfbp_shape& s, const float* g, int64_t R, int64_t C, float* f,
                          hipStream_t stream);
hipError_t launch_backward(const float* Ht, const lfbp_shape& s, const float* f, int64_t R, int64_t C, float* g,
                           hipStream_t stream);
hipError_t project_init();

namespace {

constexpr int kMaxTile = 65536;

// One-time per-process setup of kernel attributes (dynamic LDS limits).
std::once_flag g_init_once;
hipError_t g_init_err = hipSuccess;

hipError_t ensure_init()
{
    std::call_once(g_init_once, [] {
        g_init_err = set_gather_smem_limits(kMaxTile);
        if (g_init_err == hipSuccess) g_init_err = project_init();
    });
    return g_init_err;
}

// Rows of W elements that fit a tile of tile_bytes with the two alignment
// vectors of slack.
uint32_t rows_for_tile(uint32_t W, int esize, int tile_bytes)
{
    const int64_t usable = int64_t(tile_bytes) - 2 * 16;
    const int64_t rows = usable / (int64_t(W) * esize);
    return rows < 1 ? 0 : uint32_t(rows);
}

// Complete a (possibly partial) configuration for one problem.
lfbp_gather_config resolve_config(const lfbp_shape& s, int esize, const lfbp_gather_config* user)
{
    lfbp_gather_config c = tuned_config(s, esize);  // never has zero fields
    if (user) {
        if (user->variant) c.variant = user->variant;
        if (user->block_threads) c.block_threads = user->block_threads;
        if (user->rows_in_flight) c.rows_in_flight = user->rows_in_flight;
        if (user->tile_bytes) c.tile_bytes = user->tile_bytes;
        if (user->nontemporal) c.nontemporal = user->nontemporal;
        if (user->grid) c.grid = user->grid;
        else if (user->variant || user->block_threads || user->rows_in_flight || user->tile_bytes)
            c.grid = 0;  // a different work split: let the unit count decide
    }
    const uint32_t W = uint32_t(s.ny * s.nz);
    // A staged tile must hold at least one row; otherwise copy rows directly.
    if (c.variant == LFBP_GATHER_STAGED && rows_for_tile(W, esize, c.tile_bytes) == 0) {
        if (int64_t(W) * esize + 32 <= kMaxTile)
            c.tile_bytes = int(((int64_t(W) * esize + 32 + 15) / 16) * 16);
        else
            c.variant = LFBP_GATHER_DIRECT;
    }
    return c;
}

GatherDesc make_desc(const void* H, void* Ht, const lfbp_shape& s, int esize, const lfbp_gather_config& c)
{
    GatherDesc d;
    std::memset(&d, 0, sizeof(d));
    d.H = H;
    d.Ht = Ht;
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
    if (c.variant == LFBP_GATHER_STAGED)
        d.rows_per_unit = rows_for_tile(d.W, esize, c.tile_bytes);
    else
        d.rows_per_unit = uint32_t(c.block_threads / 64) * uint32_t(c.rows_in_flight);
    d.rows_per_unit = std::max<uint32_t>(1, std::min(d.rows_per_unit, d.nrows));
    d.nunits = (d.nrows + d.rows_per_unit - 1) / d.rows_per_unit;
    const uint32_t ve = 16 / uint32_t(esize);
    d.phase_out = uint32_t((reinterpret_cast<uintptr_t>(Ht) / uintptr_t(esize)) % ve);
    return d;
}

LaunchPlan make_plan(const lfbp_gather_config& c, uint32_t units)
{
    LaunchPlan p;
    p.variant = c.variant;
    p.threads = c.block_threads;
    p.rows_in_flight = c.rows_in_flight;
    p.tile_bytes = c.variant == LFBP_GATHER_STAGED ? c.tile_bytes : 0;
    p.nontemporal = c.nontemporal;
    p.grid = c.grid > 0 ? int(std::min<uint32_t>(uint32_t(c.grid), units)) : int(units);
    return p;
}

// ---------------------------------------------------------------- batched plans

struct BatchPlan {
    int device = -1;
    std::vector<lfbp_problem> probs;
    lfbp_dtype dtype = LFBP_F32;
    lfbp_gather_config cfg{};
    int use_graph = 1;
    GatherDesc* descs_dev = nullptr;
    uint32_t* unit_start_dev = nullptr;
    uint32_t count = 0, maxW = 0;
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
                const lfbp_gather_config& cfg, int use_graph)
{
    if (p.device != dev || p.dtype != dt || p.probs.size() != size_t(count) || p.use_graph != use_graph) return false;
    if (std::memcmp(&p.cfg, &cfg, sizeof(cfg)) != 0) return false;
    return std::memcmp(p.probs.data(), probs, sizeof(lfbp_problem) * size_t(count)) == 0;
}

lfbp_status build_plan(BatchPlan& bp, const lfbp_problem* probs, int32_t count, lfbp_dtype dt,
                       const lfbp_gather_config* user, int use_graph)
{
    const int es = dtype_size(dt);
    // One variant, workgroup size and rows-in-flight for the whole batch: take
    // the tuned choice of the largest problem, then size each problem's work
    // unit for that choice.
    int big = 0;
    for (int32_t i = 1; i < count; ++i)
        if (shape_elems(probs[i].shape) > shape_elems(probs[big].shape)) big = i;
    lfbp_gather_config c = resolve_config(probs[big].shape, es, user);
    std::vector<GatherDesc> descs(static_cast<size_t>(count));
    std::vector<uint32_t> start(static_cast<size_t>(count) + 1, 0);
    uint32_t maxW = 0;
    int tile = 0;
    for (int32_t i = 0; i < count; ++i) {
        const uint32_t W = uint32_t(probs[i].shape.ny * probs[i].shape.nz);
        maxW = std::max(maxW, W);
        if (c.variant == LFBP_GATHER_STAGED && rows_for_tile(W, es, c.tile_bytes) == 0) {
            if (int64_t(W) * es + 32 <= kMaxTile)
                c.tile_bytes = int(((int64_t(W) * es + 32 + 15) / 16) * 16);
            else
                c.variant = LFBP_GATHER_DIRECT;
        }
    }
    for (int32_t i = 0; i < count; ++i) {
        descs[size_t(i)] = make_desc(probs[i].H, probs[i].Ht, probs[i].shape, es, c);
        const uint64_t next = uint64_t(start[size_t(i)]) + descs[size_t(i)].nunits;
        if (next >= (uint64_t(1) << 31)) return LFBP_ESHAPE;
        start[size_t(i) + 1] = uint32_t(next);
    }
    tile = c.variant == LFBP_GATHER_STAGED ? c.tile_bytes : 0;
    const uint32_t total = start[size_t(count)];
    LaunchPlan lp = make_plan(c, total);
    lp.tile_bytes = tile;
    if (c.grid <= 0) {
        // persistent grid: every workgroup slot of the device, once
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess) return LFBP_EDEVICE;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return LFBP_EDEVICE;
        const int per_cu = std::max(1, batched_occupancy(c.variant, maxW, es, c.rows_in_flight, c.block_threads, tile));
        lp.grid = int(std::min<uint64_t>(uint64_t(cus) * uint64_t(per_cu), total));
    }
    if (hipMalloc(reinterpret_cast<void**>(&bp.descs_dev), sizeof(GatherDesc) * size_t(count)) != hipSuccess)
        return LFBP_ENOMEM;
    if (hipMalloc(reinterpret_cast<void**>(&bp.unit_start_dev), sizeof(uint32_t) * (size_t(count) + 1)) != hipSuccess)
        return LFBP_ENOMEM;
    if (hipMemcpy(bp.descs_dev, descs.data(), sizeof(GatherDesc) * size_t(count), hipMemcpyHostToDevice) != hipSuccess)
        return LFBP_EDEVICE;
    if (hipMemcpy(bp.unit_start_dev, start.data(), sizeof(uint32_t) * (size_t(count) + 1), hipMemcpyHostToDevice) !=
        hipSuccess)
        return LFBP_EDEVICE;
    bp.count = uint32_t(count);
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
            const hipError_t le = launch_gather_batched(bp.descs_dev, bp.unit_start_dev, bp.count, bp.maxW, es, lp, cs);
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
    // no output may overlap any input or any other output
    for (int32_t i = 0; i < count; ++i) {
        const uint64_t bi = shape_elems(probs[i].shape) * uint64_t(es);
        for (int32_t j = 0; j < count; ++j) {
            if (i == j) continue;
            const uint64_t bj = shape_elems(probs[j].shape) * uint64_t(es);
            if (ranges_overlap(probs[i].Ht, bi, probs[j].H, bj)) return LFBP_EALIAS;
            if (j > i && ranges_overlap(probs[i].Ht, bi, probs[j].Ht, bj)) return LFBP_EALIAS;
        }
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

const char* lfbp_version(void) { return "lfbp 0.1 gfx950"; }

lfbp_status lfbp_default_config(lfbp_shape shape, lfbp_dtype dtype, lfbp_gather_config* cfg)
{
    if (!cfg) return LFBP_EINVAL;
    const int es = dtype_size(dtype);
    if (es == 0) return LFBP_EDTYPE;
    const lfbp_status st = check_shape(shape, es);
    if (st != LFBP_OK) return st;
    *cfg = resolve_config(shape, es, nullptr);
    if (cfg->grid == 0) {
        const GatherDesc d = make_desc(nullptr, nullptr, shape, es, *cfg);
        cfg->grid = int(d.nunits);
    }
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
    const lfbp_gather_config c = resolve_config(shape, es, cfg);
    const GatherDesc d = make_desc(H, Ht, shape, es, c);
    const LaunchPlan p = make_plan(c, d.nunits);
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
        bp->cfg = key;
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
        e = launch_gather_batched(plan->descs_dev, plan->unit_start_dev, plan->count, plan->maxW,
                                  dtype_size(dtype), plan->plan, s);
    return e == hipSuccess ? LFBP_OK : LFBP_EDEVICE;
}

lfbp_status lfbp_compute_Ht_batched(const lfbp_problem* problems, int32_t count, lfbp_dtype dtype, void* stream)
{
    return lfbp_compute_Ht_batched_config(problems, count, dtype, nullptr, 1, stream);
}

void lfbp_release_plans(void)
{
    std::lock_guard<std::mutex> lock(g_plan_mu);
    g_plans.clear();
}

lfbp_status lfbp_forward(const float* H, lfbp_shape shape, const float* g, int64_t R, int64_t C, float* f,
                         void* stream)
{
    const lfbp_status st = check_project(H, shape, g, shape.nz * R * C, R, C, f, R * C);
    if (st != LFBP_OK) return st;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return launch_forward(H, shape, g, R, C, f, static_cast<hipStream_t>(stream)) == hipSuccess ? LFBP_OK
                                                                                             : LFBP_EDEVICE;
}

lfbp_status lfbp_backward(const float* Ht, lfbp_shape shape, const float* f, int64_t R, int64_t C, float* g,
                          void* stream)
{
    const lfbp_status st = check_project(Ht, shape, f, R * C, R, C, g, shape.nz * R * C);
    if (st != LFBP_OK) return st;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    return launch_backward(Ht, shape, f, R, C, g, static_cast<hipStream_t>(stream)) == hipSuccess ? LFBP_OK
                                                                                              : LFBP_EDEVICE;
}

}  // extern "C"
