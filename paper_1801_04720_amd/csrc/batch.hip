// Batched plain SGM over many stereo pairs of uneven size and disparity range
// (paper Sec. 3.1, applied pair by pair; the batching is this library's, the
// paper processes one pair at a time).
//
// A batch plan sorts the pairs by size class, packs them into waves whose
// workspace fits a memory budget, and writes one aggregation task table per
// (wave, size class) into a plan-owned device buffer.  A run enqueues, wave by
// wave: census of all images, both cost volumes of every pair, one aggregation
// launch per size class (both views of all its pairs; the class's tuning picks
// chains per block, prefetch depth, task order and persistence), WTA of the
// right views, WTA + sub-pixel + LR check of the left views.  The run only
// launches kernels on one stream, so it is captured once into a HIP graph
// (sf_batch_capture) and replayed with one sf_batch_launch.
//
// The autotuner times candidate tunings of the aggregation on one pair of a
// size class (synthetic costs) and returns the fastest.
#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <tuple>

#include "plan.hpp"
#include "sf_internal.hpp"
#include "sgm_tasks.hpp"
#include "stages.hpp"

namespace sf {

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

struct BatchGroup {
    int cls = 0;
    std::vector<int> pairs;
    size_t views_off = 0, tasks_off = 0, counter_off = 0;  // byte offsets into d_tables
    int ntasks = 0;
};

struct BatchData {
    std::vector<sf_pair> pairs;
    std::vector<size_t> pair_off;  // offset of each pair's region in the workspace
    std::vector<std::vector<BatchGroup>> waves;
    std::vector<sf_agg_tuning> tuning;  // per class
    std::vector<std::tuple<int, int, int>> classes;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int ncu = 0;  // compute units, queried at plan creation (not during capture)
};

struct PairLayout {
    size_t cen[2], cost[2], slab[2], wtar, total;
};

static PairLayout pair_layout(int H, int W, int D)
{
    PairLayout L{};
    const size_t npx = (size_t)H * W, ncell = npx * D;
    size_t o = 0;
    for (int v = 0; v < 2; ++v) { L.cen[v] = o; o += al256(npx * 8); }
    for (int v = 0; v < 2; ++v) { L.cost[v] = o; o += al256(ncell); }
    for (int v = 0; v < 2; ++v) { L.slab[v] = o; o += al256(8 * ncell); }
    L.wtar = o; o += al256(npx * 2);
    L.total = o;
    return L;
}

__global__ void fill_random_cost_kernel(uint8_t *p, size_t n, uint32_t seed)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t st = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) {
        uint32_t h = (uint32_t)i * 2654435761u ^ seed;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        p[i] = (uint8_t)(h % 63u);
    }
}

static void order_tasks(std::vector<AggTask> &tasks, const std::vector<int> &lens, int order)
{
    if (order == 0) sort_tasks_longest_first(tasks, lens);
    // order 1: view-major, directions in table order (as generated).
}

static int check_tuning(const sf_agg_tuning &t)
{
    if (t.chains_per_block != 4 && t.chains_per_block != 8 && t.chains_per_block != 16)
        return fail(SF_EINVAL, "tuning: chains_per_block must be 4, 8 or 16");
    if (t.prefetch != 4 && t.prefetch != 8) return fail(SF_EINVAL, "tuning: prefetch must be 4 or 8");
    if (t.order != 0 && t.order != 1) return fail(SF_EINVAL, "tuning: order must be 0 or 1");
    if (t.persistent_per_cu < 0 || t.persistent_per_cu > 32)
        return fail(SF_EINVAL, "tuning: persistent_per_cu must be in [0, 32]");
    if (t.packed != 0 && t.packed != 1) return fail(SF_EINVAL, "tuning: packed must be 0 or 1");
    return SF_OK;
}

static int cu_count()
{
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return ncu;
}

// As in the frame: 6-bit packed costs when the class's tuning asks for them,
// D = 128 or 256, and the workspace keeps the cost volumes (256-byte offsets)
// 4-byte aligned.
static bool batch_packed(int packed, int D, const void *ws)
{
    return packed && cost_packable(D) && (reinterpret_cast<uintptr_t>(ws) & 3) == 0;
}

static int batch_enqueue(Plan *p, uint8_t *ws, hipStream_t st)
{
    BatchData &B = *p->batch;
    uint8_t *tab = static_cast<uint8_t *>(p->d_tables);
    const int ncu = B.ncu;
    int rc;
    for (const auto &wave : B.waves) {
        // Census and costs, per size class in chunks of 4 pairs (8 images / views).
        for (const BatchGroup &g : wave) {
            const auto [H, W, D] = B.classes[g.cls];
            const PairLayout L = pair_layout(H, W, D);
            for (size_t c0 = 0; c0 < g.pairs.size(); c0 += 4) {
                CensusArgs ca{};
                CostArgs co{};
                int n = 0;
                for (size_t c = c0; c < g.pairs.size() && c < c0 + 4; ++c, ++n) {
                    const sf_pair &pr = B.pairs[g.pairs[c]];
                    uint8_t *base = ws + B.pair_off[g.pairs[c]];
                    uint64_t *cl = reinterpret_cast<uint64_t *>(base + L.cen[0]);
                    uint64_t *cr = reinterpret_cast<uint64_t *>(base + L.cen[1]);
                    ca.img[2 * n] = pr.left;
                    ca.img[2 * n + 1] = pr.right;
                    ca.out[2 * n] = cl;
                    ca.out[2 * n + 1] = cr;
                    ca.pitch[2 * n] = ca.pitch[2 * n + 1] = pr.pitch;
                    co.base[2 * n] = cl; co.match[2 * n] = cr; co.right[2 * n] = 0;
                    co.base[2 * n + 1] = cr; co.match[2 * n + 1] = cl; co.right[2 * n + 1] = 1;
                    co.cost[2 * n] = base + L.cost[0];
                    co.cost[2 * n + 1] = base + L.cost[1];
                }
                ca.n = co.n = 2 * n;
                ca.H = co.H = H;
                ca.W = co.W = W;
                co.D = D;
                co.packed = batch_packed(B.tuning[g.cls].packed, D, ws);
                if ((rc = launch_census(ca, st))) return rc;
                if ((rc = launch_cost(co, st))) return rc;
            }
        }
        // Aggregation: one launch per size class.
        for (const BatchGroup &g : wave) {
            const auto [H, W, D] = B.classes[g.cls];
            const sf_agg_tuning &t = B.tuning[g.cls];
            (void)H; (void)W;
            if ((rc = launch_agg_tasks(reinterpret_cast<AggView *>(tab + g.views_off),
                                       reinterpret_cast<AggTask *>(tab + g.tasks_off), g.ntasks,
                                       D / 16, ws, reinterpret_cast<int *>(tab + g.counter_off),
                                       t.persistent_per_cu * ncu, st, t.chains_per_block, t.prefetch,
                                       nullptr, batch_packed(t.packed, D, ws))))
                return rc;
        }
        // WTA of the right views, then WTA + LR check of the left views.
        for (int side = 1; side >= 0; --side) {
            for (const BatchGroup &g : wave) {
                const auto [H, W, D] = B.classes[g.cls];
                const PairLayout L = pair_layout(H, W, D);
                for (size_t c0 = 0; c0 < g.pairs.size(); c0 += STAGE_MAXV) {
                    WtaArgs wa{};
                    int n = 0;
                    for (size_t c = c0; c < g.pairs.size() && c < c0 + STAGE_MAXV; ++c, ++n) {
                        const sf_pair &pr = B.pairs[g.pairs[c]];
                        uint8_t *base = ws + B.pair_off[g.pairs[c]];
                        WtaView &v = wa.v[n];
                        v.nslab = 8; v.H = H; v.W = W; v.D = D; v.P2 = p->P2; v.tol = p->tol;
                        if (side == 1) {
                            v.slab = base + L.slab[1];
                            v.wta = reinterpret_cast<int16_t *>(base + L.wtar);
                            v.right_only = 1;
                        } else {
                            v.slab = base + L.slab[0];
                            v.wta_r = reinterpret_cast<const int16_t *>(base + L.wtar);
                            v.wta = pr.wta;
                            v.disp = pr.disp;
                            v.valid = pr.valid;
                            v.right_only = 0;
                        }
                    }
                    wa.n = n;
                    if ((rc = launch_wta_slabs(wa, st))) return rc;
                }
            }
        }
    }
    return SF_OK;
}

}  // namespace sf

using namespace sf;

extern "C" int sf_batch_plan_create(const sf_pair *pairs, int n, int P1, int P2, int lr_tol,
                                    const sf_agg_tuning *tunings, int ntunings, size_t mem_budget,
                                    sf_plan *out)
{
    clear_error();
    SF_REQUIRE(out, SF_EINVAL, "sf_batch_plan_create: NULL out");
    *out = nullptr;
    SF_REQUIRE(pairs && n > 0, SF_EINVAL, "sf_batch_plan_create: no pairs");
    SF_REQUIRE(P1 >= 0 && P2 >= P1, SF_EINVAL, "sf_batch_plan_create: need 0 <= P1 <= P2");
    SF_REQUIRE(SF_CMAX + P2 <= 255, SF_EUNSUPPORTED,
               "sf_batch_plan_create: batches need 62 + P2 <= 255 (u8 path costs)");
    SF_REQUIRE(lr_tol >= 0, SF_EINVAL, "sf_batch_plan_create: lr_tol < 0");
    SF_REQUIRE(!tunings || ntunings >= 0, SF_EINVAL, "sf_batch_plan_create: ntunings < 0");
    for (int i = 0; i < n; ++i) {
        const sf_pair &q = pairs[i];
        SF_REQUIRE(q.left && q.right && q.disp && q.valid, SF_EINVAL, "sf_batch_plan_create: NULL pointer in a pair");
        SF_REQUIRE(q.H > 0 && q.W > 0 && q.H <= 65535 && (long long)q.H * q.W <= (1LL << 28), SF_EINVAL,
                   "sf_batch_plan_create: pair size out of range");
        SF_REQUIRE((long long)q.H * q.W * q.D <= 0x7FFFFFFFLL, SF_EINVAL,
                   "sf_batch_plan_create: H * W * D of a pair must stay below 2^31");
        SF_REQUIRE(q.pitch >= q.W, SF_EINVAL, "sf_batch_plan_create: pitch < W");
        SF_REQUIRE(q.D >= 32 && q.D <= SF_DMAX && q.D % 32 == 0, SF_EUNSUPPORTED,
                   "sf_batch_plan_create: D must be a multiple of 32 in [32, 256]");
    }
    Plan *p = new (std::nothrow) Plan();
    BatchData *B = new (std::nothrow) BatchData();
    if (!p || !B) {
        delete p;
        delete B;
        return fail(SF_ENOMEM, "sf_batch_plan_create: out of host memory");
    }
    p->kind = Plan::BATCH;
    p->P1 = P1;
    p->P2 = P2;
    p->tol = lr_tol;
    p->batch = B;
    B->pairs.assign(pairs, pairs + n);
    B->ncu = cu_count();
    // Size classes in order of first appearance; pairs grouped by class.
    std::map<std::tuple<int, int, int>, int> cls_of;
    std::vector<int> pair_cls(n);
    for (int i = 0; i < n; ++i) {
        auto key = std::make_tuple(pairs[i].H, pairs[i].W, pairs[i].D);
        auto it = cls_of.find(key);
        if (it == cls_of.end()) {
            it = cls_of.emplace(key, (int)B->classes.size()).first;
            B->classes.push_back(key);
        }
        pair_cls[i] = it->second;
    }
    const int ncls = (int)B->classes.size();
    B->tuning.assign(ncls, sf_agg_tuning{16, 8, 0, 0, 0});
    for (int c = 0; c < ncls && tunings && c < ntunings; ++c) {
        int rc = check_tuning(tunings[c]);
        if (rc) {
            sf_plan_destroy(reinterpret_cast<sf_plan>(p));
            return rc;
        }
        B->tuning[c] = tunings[c];
    }
    // Waves: pairs in class order, a new wave when the budget would overflow.
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pair_cls[a] < pair_cls[b]; });
    B->pair_off.assign(n, 0);
    size_t wave_bytes = 0, max_wave = 0;
    B->waves.emplace_back();
    for (int i : order) {
        const size_t need = pair_layout(pairs[i].H, pairs[i].W, pairs[i].D).total;
        if (wave_bytes > 0 && mem_budget > 0 && wave_bytes + need > mem_budget) {
            B->waves.emplace_back();
            wave_bytes = 0;
        }
        auto &wave = B->waves.back();
        if (wave.empty() || wave.back().cls != pair_cls[i]) {
            wave.emplace_back();
            wave.back().cls = pair_cls[i];
        }
        wave.back().pairs.push_back(i);
        B->pair_off[i] = wave_bytes;
        wave_bytes += need;
        max_wave = std::max(max_wave, wave_bytes);
    }
    p->ws_bytes = max_wave;
    // Task tables of every (wave, class) group in one device buffer.
    std::vector<uint8_t> host;
    auto put = [&](const void *src, size_t bytes) {
        const size_t off = al256(host.size());
        host.resize(off + bytes);
        std::memcpy(host.data() + off, src, bytes);
        return off;
    };
    for (auto &wave : B->waves) {
        for (BatchGroup &g : wave) {
            const auto [H, W, D] = B->classes[g.cls];
            const PairLayout L = pair_layout(H, W, D);
            const sf_agg_tuning &t = B->tuning[g.cls];
            std::vector<AggView> views;
            std::vector<AggTask> tasks;
            std::vector<int> lens;
            for (int pi : g.pairs) {
                for (int side = 0; side < 2; ++side) {
                    AggView v{};
                    v.cost_off = B->pair_off[pi] + L.cost[side];
                    v.slab_off = B->pair_off[pi] + L.slab[side];
                    v.H = H; v.W = W; v.K = D / 16; v.P1 = P1; v.P2 = P2; v.ndir = 8;
                    for (int r = 0; r < 8; ++r) v.dir[r] = r;
                    append_agg_tasks(tasks, lens, (int)views.size(), v, t.chains_per_block);
                    views.push_back(v);
                }
            }
            order_tasks(tasks, lens, t.order);
            g.views_off = put(views.data(), views.size() * sizeof(AggView));
            g.tasks_off = put(tasks.data(), tasks.size() * sizeof(AggTask));
            int zero = 0;
            g.counter_off = put(&zero, sizeof(int));
            g.ntasks = (int)tasks.size();
        }
    }
    if (hipMalloc(&p->d_tables, host.size() + 256) != hipSuccess ||
        hipMemcpy(p->d_tables, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
        sf_plan_destroy(reinterpret_cast<sf_plan>(p));
        return fail(SF_EHIP, "sf_batch_plan_create: task table upload failed");
    }
    *out = reinterpret_cast<sf_plan>(p);
    return SF_OK;
}

extern "C" int sf_batch_plan_info(sf_plan plan, int *nwaves, int *nclasses)
{
    clear_error();
    SF_REQUIRE(plan, SF_EINVAL, "sf_batch_plan_info: NULL plan");
    Plan *p = reinterpret_cast<Plan *>(plan);
    SF_REQUIRE(p->kind == Plan::BATCH, SF_EINVAL, "sf_batch_plan_info: not a batch plan");
    if (nwaves) *nwaves = (int)p->batch->waves.size();
    if (nclasses) *nclasses = (int)p->batch->classes.size();
    return SF_OK;
}

extern "C" int sf_batch_run(sf_plan plan, void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    SF_REQUIRE(plan, SF_EINVAL, "sf_batch_run: NULL plan");
    Plan *p = reinterpret_cast<Plan *>(plan);
    SF_REQUIRE(p->kind == Plan::BATCH, SF_EINVAL, "sf_batch_run: not a batch plan");
    SF_REQUIRE(workspace, SF_EINVAL, "sf_batch_run: NULL workspace");
    SF_REQUIRE(ws_bytes >= p->ws_bytes, SF_ENOMEM, "sf_batch_run: workspace too small");
    return batch_enqueue(p, static_cast<uint8_t *>(workspace), as_stream(stream));
}

extern "C" int sf_batch_capture(sf_plan plan, void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    SF_REQUIRE(plan, SF_EINVAL, "sf_batch_capture: NULL plan");
    Plan *p = reinterpret_cast<Plan *>(plan);
    SF_REQUIRE(p->kind == Plan::BATCH, SF_EINVAL, "sf_batch_capture: not a batch plan");
    SF_REQUIRE(workspace, SF_EINVAL, "sf_batch_capture: NULL workspace");
    SF_REQUIRE(ws_bytes >= p->ws_bytes, SF_ENOMEM, "sf_batch_capture: workspace too small");
    SF_REQUIRE(stream, SF_EINVAL, "sf_batch_capture: capture needs a non-default stream");
    BatchData &B = *p->batch;
    if (B.exec) { (void)hipGraphExecDestroy(B.exec); B.exec = nullptr; }
    if (B.graph) { (void)hipGraphDestroy(B.graph); B.graph = nullptr; }
    hipStream_t st = as_stream(stream);
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(SF_EHIP, "sf_batch_capture: hipStreamBeginCapture failed");
    const int rc = batch_enqueue(p, static_cast<uint8_t *>(workspace), st);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) return fail(SF_EHIP, "sf_batch_capture: hipStreamEndCapture failed");
    if (hipGraphInstantiate(&B.exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(SF_EHIP, "sf_batch_capture: hipGraphInstantiate failed");
    }
    B.graph = g;
    return SF_OK;
}

extern "C" int sf_batch_launch(sf_plan plan, void *stream)
{
    clear_error();
    SF_REQUIRE(plan, SF_EINVAL, "sf_batch_launch: NULL plan");
    Plan *p = reinterpret_cast<Plan *>(plan);
    SF_REQUIRE(p->kind == Plan::BATCH && p->batch->exec, SF_EINVAL,
               "sf_batch_launch: no captured graph (call sf_batch_capture first)");
    ProfScope prof("batch_graph", as_stream(stream));
    if (hipGraphLaunch(p->batch->exec, as_stream(stream)) != hipSuccess)
        return fail(SF_EHIP, "sf_batch_launch: hipGraphLaunch failed");
    return SF_OK;
}

namespace sf {
void destroy_batch(BatchData *b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
}
}  // namespace sf

extern "C" int sf_agg_autotune(int H, int W, int D, int P1, int P2, int nviews, void *stream,
                               sf_agg_tuning *best, float *best_ms)
{
    clear_error();
    SF_REQUIRE(best, SF_EINVAL, "sf_agg_autotune: NULL best");
    SF_REQUIRE(H > 0 && W > 0 && (long long)H * W <= (1LL << 28), SF_EINVAL, "sf_agg_autotune: bad size");
    SF_REQUIRE((long long)H * W * D <= 0x7FFFFFFFLL, SF_EINVAL,
               "sf_agg_autotune: H * W * D must stay below 2^31");
    SF_REQUIRE(D >= 32 && D <= SF_DMAX && D % 32 == 0, SF_EUNSUPPORTED, "sf_agg_autotune: bad D");
    SF_REQUIRE(P1 >= 0 && P2 >= P1 && SF_CMAX + P2 <= 255, SF_EINVAL, "sf_agg_autotune: bad P1/P2");
    SF_REQUIRE(nviews >= 1 && nviews <= 8, SF_EINVAL, "sf_agg_autotune: nviews must be in [1, 8]");
    hipStream_t st = as_stream(stream);
    // nviews views of synthetic costs, each with its cost volume and 8 slabs.
    const size_t ncell = (size_t)H * W * D;
    const size_t vbytes = al256(ncell) + al256(8 * ncell);
    uint8_t *ws = nullptr;
    if (hipMalloc(&ws, vbytes * nviews) != hipSuccess) return fail(SF_EHIP, "sf_agg_autotune: hipMalloc");
    for (int v = 0; v < nviews; ++v)
        hipLaunchKernelGGL(fill_random_cost_kernel, dim3(4096), dim3(256), 0, st, ws + v * vbytes, ncell,
                           1234u + v);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipFree(ws);
        return fail(SF_EHIP, "sf_agg_autotune: hipEventCreate");
    }
    const int ncu = cu_count();
    float best_t = 1e30f;
    int rc = SF_OK;
    const int cpbs[3] = {4, 8, 16}, prefs[2] = {4, 8}, pers[3] = {0, 4, 8};
    for (int cpb : cpbs)
        for (int order = 0; order < 2 && rc == SF_OK; ++order) {
            std::vector<AggView> views;
            std::vector<AggTask> tasks;
            std::vector<int> lens;
            for (int side = 0; side < nviews; ++side) {
                AggView v{};
                v.cost_off = side * vbytes;
                v.slab_off = side * vbytes + al256(ncell);
                v.H = H; v.W = W; v.K = D / 16; v.P1 = P1; v.P2 = P2; v.ndir = 8;
                for (int r = 0; r < 8; ++r) v.dir[r] = r;
                append_agg_tasks(tasks, lens, side, v, cpb);
                views.push_back(v);
            }
            order_tasks(tasks, lens, order);
            uint8_t *tab = nullptr;
            const size_t bv = al256(views.size() * sizeof(AggView)), bt = al256(tasks.size() * sizeof(AggTask));
            if (hipMalloc(&tab, bv + bt + 256) != hipSuccess) { rc = fail(SF_EHIP, "sf_agg_autotune: hipMalloc"); break; }
            // The tables and the persistent counter (which starts at 0) must be in
            // place before any launch reads them.
            if (hipMemcpy(tab, views.data(), views.size() * sizeof(AggView), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(tab + bv, tasks.data(), tasks.size() * sizeof(AggTask), hipMemcpyHostToDevice) !=
                    hipSuccess ||
                hipMemset(tab + bv + bt, 0, sizeof(int)) != hipSuccess) {
                rc = fail(SF_EHIP, "sf_agg_autotune: task table upload");
                (void)hipFree(tab);
                break;
            }
            for (int pf : prefs)
                for (int pp : pers)
                    for (int pk = 0; pk <= (cost_packable(D) ? 1 : 0) && rc == SF_OK; ++pk) {
                    auto go = [&]() {
                        return launch_agg_tasks(reinterpret_cast<AggView *>(tab),
                                                reinterpret_cast<AggTask *>(tab + bv), (int)tasks.size(),
                                                D / 16, ws, reinterpret_cast<int *>(tab + bv + bt), pp * ncu,
                                                st, cpb, pf, nullptr, batch_packed(pk, D, ws));
                    };
                    if ((rc = go())) break;
                    float tms[5];
                    for (int rep = 0; rep < 5 && rc == SF_OK; ++rep) {
                        // As in a frame, the cost volumes have just been written
                        // when the aggregation starts (they may sit in the last-level cache).
                        for (int v = 0; v < nviews; ++v)
                            hipLaunchKernelGGL(fill_random_cost_kernel, dim3(4096), dim3(256), 0, st,
                                               ws + v * vbytes, ncell, 1234u + v);
                        if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(SF_EHIP, "sf_agg_autotune: event"); break; }
                        if ((rc = go())) break;
                        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&tms[rep], e0, e1) != hipSuccess)
                            rc = fail(SF_EHIP, "sf_agg_autotune: event timing");
                    }
                    if (rc) break;
                    std::sort(tms, tms + 5);
                    if (tms[2] < best_t) {
                        best_t = tms[2];
                        *best = sf_agg_tuning{cpb, pf, order, pp, pk};
                    }
                }
            (void)hipFree(tab);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(ws);
    if (rc) return rc;
    if (best_ms) *best_ms = best_t;
    return SF_OK;
}
