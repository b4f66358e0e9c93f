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
hipError_t put_words(uint32_t* dst, const uint32_t* src, size_t n, hipStream_t stream);
hipError_t noalloc_scratch(void** ptr, size_t* bytes);
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
int g_cu_lds = 65536;   // LDS of one compute unit (read at init)
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
        int cu_lds = 0;
        if (hipDeviceGetAttribute(&cu_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess &&
            cu_lds > 0)
            g_cu_lds = cu_lds;
        g_cu_lds = std::max(g_cu_lds, g_max_lds);
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
        if (user->waves_per_eu) c.waves_per_eu = user->waves_per_eu;
        if (user->schedule) c.schedule = user->schedule;
    }
    return c;
}

// LDS a workgroup of config c reserves so that at most c.waves_per_eu
// wavefronts run per SIMD: k = 4*waves_per_eu*64/threads workgroups per CU
// (4 SIMDs), enforced by reserving just over 1/(k+1) of the CU's LDS each.
int occupancy_lds(int lds, const lfbp_gather_config& c)
{
    if (c.waves_per_eu >= 8) return lds;
    const int k = std::max(1, 4 * c.waves_per_eu * 64 / c.block_threads);
    const int pad = round16(int64_t(g_cu_lds) / (k + 1) + 1);
    return std::max(lds, std::min(pad, g_max_lds));
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

// Rows per unit of a WIDE unit of about `vecs` 16-byte loads over rows of W
// elements, within the LDS (ntab row tables); 0 if not even one row fits.
uint32_t wide_rows(uint32_t W, int es, int64_t vecs, int ntab)
{
    const int64_t ve = 16 / es;
    const int64_t vpr = (int64_t(W) + 2 * ve - 2) / ve;
    int64_t r = std::max<int64_t>(1, vecs / vpr);
    auto need = [&](int64_t rr) { return int64_t(ntab) * rr * 16 + round16((rr * W + 2 * ve) * es); };
    while (r > 0 && need(r) > g_max_lds) --r;
    return uint32_t(r);
}

// Everything a batched launch needs, computed on the host from the problem
// table (no HIP call): descriptors sorted largest first, each with its own
// work-unit size; the per-XCD walks; the kernel choice and grid.
struct BatchLayout {
    std::vector<GatherDesc> descs;
    std::vector<uint32_t> xstart;  // [kXcds][count+1]
    BatchArgs args{};              // everything but the table pointers
    LaunchPlan plan{};
    uint32_t maxW = 0;
};

lfbp_status layout_batch(const lfbp_problem* probs, int32_t count, int es, const lfbp_gather_config* user,
                         BatchLayout& L)
{
    std::vector<int32_t> order(static_cast<size_t>(count));
    for (int32_t i = 0; i < count; ++i) order[size_t(i)] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t i, int32_t j) {
        return shape_elems(probs[i].shape) > shape_elems(probs[j].shape);
    });
    // One kernel for the whole batch: the tuned batched choice for the largest
    // problem.  Every problem must fit the chosen variant; the first one that
    // does not moves the whole batch down (WIDE -> STAGED -> DIRECT).
    lfbp_gather_config c = resolve_config(probs[order[0]].shape, es, user, true);
    uint32_t maxW = 0;
    for (int32_t i = 0; i < count; ++i) {
        const uint32_t W = uint32_t(probs[i].shape.ny * probs[i].shape.nz);
        maxW = std::max(maxW, W);
        uint32_t r;
        int l;
        decompose(W, es, c, r, l);
    }
    // Work-unit size per problem.  WIDE: a unit holds as many 16-byte loads as
    // the tuned plain kernel for that problem's shape class uses per unit (at
    // most the batched kernel's vec_per_thread per thread), unless the caller
    // fixed the vector count; others: as the common configuration gives.
    const int ntab = c.persistent == 1 ? 2 : 1;
    const int64_t cap = int64_t(c.block_threads) * c.vec_per_thread;
    const bool own_units = c.variant == LFBP_GATHER_WIDE && !(user && user->vec_per_thread);
    std::vector<uint32_t> rows(static_cast<size_t>(count));
    int lds = 0;
    uint32_t max_rows = 0;
    for (int32_t k = 0; k < count; ++k) {
        const lfbp_shape& sh = probs[order[size_t(k)]].shape;
        const uint32_t W = uint32_t(sh.ny * sh.nz);
        uint32_t r = 0;
        int l = 0;
        if (c.variant == LFBP_GATHER_WIDE) {
            int64_t vecs = cap;
            if (own_units) {
                const lfbp_gather_config pc = tuned_config(sh, es, false);
                if (pc.variant == LFBP_GATHER_WIDE)
                    vecs = std::min<int64_t>(cap, int64_t(pc.block_threads) * pc.vec_per_thread);
            }
            r = wide_rows(W, es, vecs, ntab);
            if (r == 0) return LFBP_ESHAPE;
            const int64_t ve = 16 / es;
            l = round16((int64_t(r) * W + 2 * ve) * es);  // tile only; tables added below
        } else {
            lfbp_gather_config ci = c;
            decompose(W, es, ci, r, l);
        }
        rows[size_t(k)] = r;
        max_rows = std::max(max_rows, r);
        lds = std::max(lds, l);
    }
    if (c.variant == LFBP_GATHER_WIDE) lds += ntab * int(max_rows) * 16;
    if (lds > g_max_lds) return LFBP_ESHAPE;
    lds = occupancy_lds(lds, c);
    L.descs.resize(static_cast<size_t>(count));
    for (int32_t k = 0; k < count; ++k) {
        const lfbp_problem& pb = probs[order[size_t(k)]];
        L.descs[size_t(k)] = make_desc(pb.H, pb.Ht, pb.shape, es, rows[size_t(k)]);
    }
    BatchArgs& a = L.args;
    std::memset(&a, 0, sizeof(a));
    L.xstart.assign(size_t(kXcds) * (size_t(count) + 1), 0);
    a.linear = c.schedule == 2 ? 1 : 0;
    uint64_t nslots = 0;
    if (a.linear) {
        // one walk over every unit in launch order (row 0 of the prefix table)
        uint64_t cum = 0;
        for (int32_t k = 0; k < count; ++k) {
            L.xstart[size_t(k)] = uint32_t(cum);
            cum += L.descs[size_t(k)].nunits;
            if (cum >= (uint64_t(1) << 31)) return LFBP_ESHAPE;
        }
        L.xstart[size_t(count)] = uint32_t(cum);
        a.xtotal[0] = uint32_t(cum);
        nslots = cum;
    } else {
        uint64_t slots = 0;
        for (uint32_t x = 0; x < kXcds; ++x) {
            uint64_t cum = 0;
            for (int32_t k = 0; k < count; ++k) {
                L.xstart[x * (size_t(count) + 1) + size_t(k)] = uint32_t(cum);
                cum += xcd_share(L.descs[size_t(k)].nunits, x);
                if (cum >= (uint64_t(1) << 28)) return LFBP_ESHAPE;  // kXcds * slots < 2^31
            }
            L.xstart[x * (size_t(count) + 1) + size_t(count)] = uint32_t(cum);
            a.xtotal[x] = uint32_t(cum);
            slots = std::max(slots, cum);
        }
        nslots = uint64_t(kXcds) * slots;
    }
    a.count = uint32_t(count);
    a.nslots = uint32_t(nslots);
    a.max_rows = max_rows;
    a.nt = c.nontemporal == 1 ? 1 : 0;
    if (uint32_t(count) <= kInlineProblems) {
        for (int32_t k = 0; k < count; ++k) a.d[k] = L.descs[size_t(k)];
        for (uint32_t x = 0; x < kXcds; ++x)
            for (int32_t k = 0; k <= count; ++k) a.xstart[x][k] = L.xstart[x * (size_t(count) + 1) + size_t(k)];
    }
    LaunchPlan lp = make_plan(c, lds);
    if (c.persistent != 1) {
        lp.grid = int(std::min<uint64_t>(nslots, max_grid(lp.threads)));
    } else {
        // a multiple of kXcds, so that every workgroup stays on one XCD's walk
        uint64_t g = c.grid > 0 ? uint64_t(c.grid) : uint64_t(g_cus) * gather_occupancy(lp, maxW, es, true);
        g = std::max<uint64_t>(kXcds, g / kXcds * kXcds);
        lp.grid = int(std::min<uint64_t>(g, nslots));
    }
    L.plan = lp;
    L.maxW = maxW;
    return LFBP_OK;
}

// Upload a layout's descriptor table and per-XCD walks into `table` (device
// memory of table_bytes(count) bytes) on `stream`, and point the launch
// arguments at it.
size_t table_bytes(int32_t count) { return batch_table_bytes(size_t(count)); }

hipError_t upload_table(BatchLayout& L, void* table, hipStream_t stream)
{
    const size_t dbytes = sizeof(GatherDesc) * L.descs.size();
    static_assert(sizeof(GatherDesc) % sizeof(uint32_t) == 0, "descriptor is whole words");
    uint32_t* words = static_cast<uint32_t*>(table);
    hipError_t e = put_words(words, reinterpret_cast<const uint32_t*>(L.descs.data()), dbytes / 4, stream);
    if (e == hipSuccess) e = put_words(words + dbytes / 4, L.xstart.data(), L.xstart.size(), stream);
    L.args.table = static_cast<const GatherDesc*>(table);
    L.args.table_xstart = words + dbytes / 4;
    return e;
}

// hipEventQuery without leaving "not ready" behind as the thread's last error
// (the launch checks read hipGetLastError).
bool event_done(hipEvent_t e)
{
    const hipError_t r = hipEventQuery(e);
    if (r == hipErrorNotReady) {
        (void)hipGetLastError();
        return false;
    }
    return true;
}

bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// A cached batched plan.  Plans are keyed on the exact problem table (pointers
// and shapes), the configuration and graph use, and are immutable once made,
// so one plan may be launched from several streams and threads at once.
struct BatchPlan {
    int device = -1;
    std::vector<lfbp_problem> probs;
    lfbp_dtype dtype = LFBP_F32;
    lfbp_gather_config key{};
    int use_graph = 0;
    BatchLayout layout;
    void* table = nullptr;             // device table, batches beyond kInlineProblems
    hipStream_t upload_stream = nullptr;
    hipEvent_t ready = nullptr;        // table written (recorded on upload_stream)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<std::pair<hipStream_t, hipEvent_t>> uses;  // last launch on each stream
    bool pinned = false;               // used by a captured call: kept until lfbp_release_plans
    uint64_t tick = 0;

    bool holds_device() const { return table != nullptr || exec != nullptr; }

    // Every launch (and the upload) of this plan has finished.
    bool idle() const
    {
        if (ready && !event_done(ready)) return false;
        for (const auto& u : uses)
            if (!event_done(u.second)) return false;
        return true;
    }

    void wait_idle() const
    {
        if (ready) (void)hipEventSynchronize(ready);
        for (const auto& u : uses) (void)hipEventSynchronize(u.second);
    }

    ~BatchPlan()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto& u : uses) (void)hipEventDestroy(u.second);
        if (ready) (void)hipEventDestroy(ready);
        if (table) (void)hipFree(table);
    }
};

// At most kMaxPlans plans are kept; the least recently used one is dropped
// first.  A dropped plan that holds device memory or a graph is retired and
// freed once every launch of it has finished (checked without blocking on
// later calls).  Plans used by a captured call are never dropped.
constexpr size_t kMaxPlans = 32;
std::mutex g_plan_mu;
std::vector<std::unique_ptr<BatchPlan>> g_plans;
std::vector<std::unique_ptr<BatchPlan>> g_retired;
uint64_t g_tick = 0;

bool same_table(const BatchPlan& p, int dev, const lfbp_problem* probs, int32_t count, lfbp_dtype dt,
                const lfbp_gather_config& key, int use_graph)
{
    if (p.device != dev || p.dtype != dt || p.probs.size() != size_t(count) || p.use_graph != use_graph) return false;
    if (std::memcmp(&p.key, &key, sizeof(key)) != 0) return false;
    return std::memcmp(p.probs.data(), probs, sizeof(lfbp_problem) * size_t(count)) == 0;
}

void reap_retired()
{
    for (size_t i = 0; i < g_retired.size();) {
        if (g_retired[i]->idle()) {
            g_retired[i] = std::move(g_retired.back());
            g_retired.pop_back();
        } else {
            ++i;
        }
    }
}

void evict_plans()
{
    while (g_plans.size() > kMaxPlans) {
        size_t victim = g_plans.size();
        for (size_t i = 0; i < g_plans.size(); ++i)
            if (!g_plans[i]->pinned && (victim == g_plans.size() || g_plans[i]->tick < g_plans[victim]->tick))
                victim = i;
        if (victim == g_plans.size()) return;  // every plan pinned
        std::unique_ptr<BatchPlan> p = std::move(g_plans[victim]);
        g_plans.erase(g_plans.begin() + std::ptrdiff_t(victim));
        if (p->holds_device() && !p->idle()) g_retired.push_back(std::move(p));
    }
}

lfbp_status build_plan(BatchPlan& bp, const lfbp_problem* probs, int32_t count, lfbp_dtype dt,
                       const lfbp_gather_config* user, int use_graph, hipStream_t stream)
{
    const int es = dtype_size(dt);
    const lfbp_status st = layout_batch(probs, count, es, user, bp.layout);
    if (st != LFBP_OK) return st;
    bp.dtype = dt;
    bp.use_graph = use_graph;
    bp.probs.assign(probs, probs + count);
    if (uint32_t(count) > kInlineProblems) {
        if (hipMalloc(&bp.table, table_bytes(count)) != hipSuccess) {
            (void)hipGetLastError();
            bp.table = nullptr;
            return LFBP_ENOMEM;
        }
        if (upload_table(bp.layout, bp.table, stream) != hipSuccess) return LFBP_EDEVICE;
        if (hipEventCreateWithFlags(&bp.ready, hipEventDisableTiming) != hipSuccess) return LFBP_EDEVICE;
        if (hipEventRecord(bp.ready, stream) != hipSuccess) return LFBP_EDEVICE;
        bp.upload_stream = stream;
    }
    if (use_graph) {
        hipStream_t cs = nullptr;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return LFBP_EDEVICE;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t le = launch_gather_batched(bp.layout.args, bp.layout.maxW, es, bp.layout.plan, cs);
            e = hipStreamEndCapture(cs, &bp.graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&bp.exec, bp.graph, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) return LFBP_EDEVICE;
    }
    return LFBP_OK;
}

// Record that `plan` was launched on stream s (not under capture).
lfbp_status note_use(BatchPlan& plan, hipStream_t s)
{
    if (!plan.holds_device()) return LFBP_OK;
    hipEvent_t ev = nullptr;
    for (auto& u : plan.uses)
        if (u.first == s) ev = u.second;
    if (!ev) {
        // forget finished launches on other streams before adding one
        for (size_t i = 0; i < plan.uses.size();) {
            if (event_done(plan.uses[i].second)) {
                (void)hipEventDestroy(plan.uses[i].second);
                plan.uses[i] = plan.uses.back();
                plan.uses.pop_back();
            } else {
                ++i;
            }
        }
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return LFBP_EDEVICE;
        plan.uses.emplace_back(s, ev);
    }
    return hipEventRecord(ev, s) == hipSuccess ? LFBP_OK : LFBP_EDEVICE;
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
        case LFBP_ECAPTURE: return "the call would allocate while its stream is being captured";
        case LFBP_ESCRATCH: return "the call needs more than the library's fixed device scratch holds";
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
    // the device's LDS size decides the work decomposition, as in a launch
    // (with no device, the 64 KB every device provides)
    (void)ensure_init();
    lfbp_gather_config c = resolve_config(shape, es, nullptr, false);
    uint32_t rows = 0;
    int lds = 0;
    const uint32_t W = uint32_t(shape.ny * shape.nz);
    decompose(W, es, c, rows, lds);
    const GatherDesc d = make_desc(nullptr, nullptr, shape, es, rows);
    LaunchPlan p = make_plan(c, occupancy_lds(lds, c));
    c.grid = grid_for(c, p, d.nunits, W, es, false);
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
    GatherDesc d = make_desc(H, Ht, shape, es, rows);
    d.xcd_remap = c.schedule == 2 ? 0 : 1;
    LaunchPlan p = make_plan(c, occupancy_lds(lds, c));
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
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool in_capture = capturing(s);
    lfbp_gather_config key{};
    if (cfg) key = *cfg;
    std::lock_guard<std::mutex> lock(g_plan_mu);
    reap_retired();
    BatchPlan* plan = nullptr;
    for (auto& p : g_plans)
        if (same_table(*p, dev, problems, count, dtype, key, use_graph)) {
            plan = p.get();
            break;
        }
    if (!plan) {
        // a plan with device memory cannot be made inside a capture (the
        // allocation would end the caller's capture)
        if (in_capture && (uint32_t(count) > kInlineProblems || use_graph)) return LFBP_ECAPTURE;
        auto bp = std::make_unique<BatchPlan>();
        bp->device = dev;
        bp->key = key;
        st = build_plan(*bp, problems, count, dtype, cfg, use_graph, s);
        if (st != LFBP_OK) return st;
        g_plans.push_back(std::move(bp));
        plan = g_plans.back().get();
    } else if (plan->ready && plan->upload_stream != s && !event_done(plan->ready)) {
        // the table is still being written on the stream of the plan's first
        // call: order this launch after it
        const hipError_t e = in_capture ? hipEventSynchronize(plan->ready) : hipStreamWaitEvent(s, plan->ready, 0);
        if (e != hipSuccess) return LFBP_EDEVICE;
    }
    plan->tick = ++g_tick;
    hipError_t e;
    if (plan->use_graph)
        e = hipGraphLaunch(plan->exec, s);
    else
        e = launch_gather_batched(plan->layout.args, plan->layout.maxW, dtype_size(dtype), plan->layout.plan, s);
    if (e != hipSuccess) return LFBP_EDEVICE;
    if (in_capture)
        plan->pinned = true;
    else if (note_use(*plan, s) != LFBP_OK)
        return LFBP_EDEVICE;
    evict_plans();
    return LFBP_OK;
}

lfbp_status lfbp_compute_Ht_batched(const lfbp_problem* problems, int32_t count, lfbp_dtype dtype, void* stream)
{
    // a direct launch: replaying the plan's one-kernel graph costs more host
    // time per call than launching the kernel (measured on small tables)
    return lfbp_compute_Ht_batched_config(problems, count, dtype, nullptr, 0, stream);
}

lfbp_status lfbp_compute_Ht_batched_noalloc(const lfbp_problem* problems, int32_t count, lfbp_dtype dtype,
                                             void* stream)
{
    lfbp_status st = validate_batch(problems, count, dtype);
    if (st != LFBP_OK) return st;
    if (count > LFBP_NOALLOC_MAX_PROBLEMS) return LFBP_ESCRATCH;
    if (ensure_init() != hipSuccess) return LFBP_EDEVICE;
    const int es = dtype_size(dtype);
    BatchLayout L;
    st = layout_batch(problems, count, es, nullptr, L);
    if (st != LFBP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (uint32_t(count) > kInlineProblems) {
        // the descriptor table goes to the library's fixed device scratch
        void* table = nullptr;
        size_t bytes = 0;
        if (noalloc_scratch(&table, &bytes) != hipSuccess) return LFBP_EDEVICE;
        if (table_bytes(count) > bytes) return LFBP_ESCRATCH;
        if (upload_table(L, table, s) != hipSuccess) return LFBP_EDEVICE;
    }
    return launch_gather_batched(L.args, L.maxW, es, L.plan, s) == hipSuccess ? LFBP_OK : LFBP_EDEVICE;
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
    for (auto& p : g_plans) p->wait_idle();
    for (auto& p : g_retired) p->wait_idle();
    g_plans.clear();
    g_retired.clear();
}

int32_t lfbp_plan_count(void)
{
    std::lock_guard<std::mutex> lock(g_plan_mu);
    reap_retired();
    return int32_t(g_plans.size() + g_retired.size());
}

}  // extern "C"
