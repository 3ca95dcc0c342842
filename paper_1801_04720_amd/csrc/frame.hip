// Fused plain scene-flow frame (paper Sec. 3: SGM on the stereo pairs at t0
// and t1 with the left-right check, Sec. 3.3: combination with the flow).
//
// A frame plan fixes the size and parameters, lays out the caller's workspace
// and holds the aggregation task table of the four views (L0, R0, L1, R1 as
// bases) in a small device buffer written once at plan creation.  A run
// enqueues six launches: census of the 4 images, 4 cost volumes, one
// aggregation over all 4 views (u8 slabs), WTA of both right views, WTA +
// sub-pixel + LR check of both left views (slabs summed on the fly, S never
// written), and the combination.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "sf_internal.hpp"
#include "sgm_tasks.hpp"
#include "stages.hpp"
#include "plan.hpp"

namespace sf {

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Whether a run aggregates from 6-bit packed costs: the tuning asks for them,
// D = 128 or 256, and the workspace keeps the cost volumes (at 256-byte
// offsets) 4-byte aligned.  The cost and aggregation launches of a run take
// the same answer.
static bool frame_packed(const sf_agg_tuning &t, int D, const void *ws)
{
    return t.packed && cost_packable(D) && (reinterpret_cast<uintptr_t>(ws) & 3) == 0;
}

int plan_upload_tables(Plan &p, const std::vector<AggView> &views, const std::vector<AggTask> &tasks)
{
    p.ntasks = (int)tasks.size();
    p.nviews = (int)views.size();
    const size_t bv = views.size() * sizeof(AggView), bt = tasks.size() * sizeof(AggTask);
    if (hipMalloc(&p.d_tables, align256(bv) + bt + 256) != hipSuccess)
        return fail(SF_EHIP, "plan: hipMalloc of the task table failed");
    p.d_views = reinterpret_cast<AggView *>(p.d_tables);
    p.d_tasks = reinterpret_cast<AggTask *>(static_cast<uint8_t *>(p.d_tables) + align256(bv));
    p.d_counter = reinterpret_cast<int *>(static_cast<uint8_t *>(p.d_tables) + align256(bv) + bt);
    if (hipMemcpy(p.d_views, views.data(), bv, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p.d_tasks, tasks.data(), bt, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(p.d_counter, 0, sizeof(int)) != hipSuccess)  // the persistent launches keep it at 0
        return fail(SF_EHIP, "plan: upload of the task table failed");
    return SF_OK;
}

int cu_count_dev()
{
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return ncu;
}

}  // namespace sf

using namespace sf;

extern "C" int sf_frame_plan_create(int H, int W, int D, int P1, int P2, int lr_tol, int flags,
                                    const sf_agg_tuning *tuning, sf_plan *out)
{
    clear_error();
    SF_REQUIRE(out, SF_EINVAL, "sf_frame_plan_create: NULL out");
    *out = nullptr;
    SF_REQUIRE(H > 0 && W > 0, SF_EINVAL, "sf_frame_plan_create: H and W must be positive");
    SF_REQUIRE(H <= 65535 && (long long)H * W <= (1LL << 28), SF_EINVAL,
               "sf_frame_plan_create: image too large");
    SF_REQUIRE(P1 >= 0 && P2 >= P1, SF_EINVAL, "sf_frame_plan_create: need 0 <= P1 <= P2");
    SF_REQUIRE(SF_CMAX + P2 <= 255, SF_EUNSUPPORTED,
               "sf_frame_plan_create: the fused frame needs 62 + P2 <= 255 (u8 path costs)");
    SF_REQUIRE(lr_tol >= 0, SF_EINVAL, "sf_frame_plan_create: lr_tol < 0");
    SF_REQUIRE(D >= 32 && D <= SF_DMAX && D % 32 == 0, SF_EUNSUPPORTED,
               "sf_frame_plan_create: D must be a multiple of 32 in [32, 256]");
    SF_REQUIRE((long long)H * W * D <= 0x7FFFFFFFLL, SF_EINVAL,
               "sf_frame_plan_create: H * W * D must stay below 2^31 (32-bit volume offsets)");
    SF_REQUIRE((flags & ~(SF_FRAME_PERSISTENT | SF_FRAME_LEARNED | SF_FRAME_DIAG | SF_FRAME_MEDIAN |
                          SF_FRAME_ADAPTIVE_P2)) == 0,
               SF_EINVAL, "sf_frame_plan_create: unknown flags");
    SF_REQUIRE(!((flags & SF_FRAME_DIAG) && (flags & SF_FRAME_LEARNED)), SF_EINVAL,
               "sf_frame_plan_create: SF_FRAME_DIAG and SF_FRAME_LEARNED exclude each other");
    SF_REQUIRE(!(flags & SF_FRAME_DIAG) || W <= 4096, SF_EUNSUPPORTED,
               "sf_frame_plan_create: SF_FRAME_DIAG needs W <= 4096");
    sf_agg_tuning tun{16, 8, 0, (flags & SF_FRAME_PERSISTENT) ? 8 : 0, 0};
    if (tuning) {
        tun = *tuning;
        SF_REQUIRE(tun.chains_per_block == 4 || tun.chains_per_block == 8 || tun.chains_per_block == 16,
                   SF_EINVAL, "sf_frame_plan_create: chains_per_block must be 4, 8 or 16");
        SF_REQUIRE(tun.prefetch == 4 || tun.prefetch == 8, SF_EINVAL,
                   "sf_frame_plan_create: prefetch must be 4 or 8");
        SF_REQUIRE(tun.order == 0 || tun.order == 1, SF_EINVAL, "sf_frame_plan_create: order must be 0 or 1");
        SF_REQUIRE(tun.persistent_per_cu >= 0 && tun.persistent_per_cu <= 32, SF_EINVAL,
                   "sf_frame_plan_create: persistent_per_cu must be in [0, 32]");
        SF_REQUIRE(tun.packed == 0 || tun.packed == 1, SF_EINVAL, "sf_frame_plan_create: packed must be 0 or 1");
    }
    Plan *p = new (std::nothrow) Plan();
    if (!p) return fail(SF_ENOMEM, "sf_frame_plan_create: out of host memory");
    p->kind = Plan::FRAME;
    p->learned = (flags & SF_FRAME_LEARNED) != 0;
    p->diag = (flags & SF_FRAME_DIAG) != 0;
    p->median = (flags & SF_FRAME_MEDIAN) != 0;
    p->adaptive = (flags & SF_FRAME_ADAPTIVE_P2) != 0;
    p->H = H;
    p->W = W;
    p->D = D;
    p->P1 = P1;
    p->P2 = P2;
    p->tol = lr_tol;
    // Views aggregated: plain = L0, R0, L1, R1 bases; learned and diag = L0, L1 bases only.
    const int nv = (p->learned || p->diag) ? 2 : 4;
    const size_t npx = (size_t)H * W, ncell = npx * D;
    size_t off = 0;
    for (int i = 0; i < 4; ++i) { p->off_cen[i] = off; off += align256(npx * 8); }
    for (int i = 0; i < nv; ++i) { p->off_cost[i] = off; off += align256(ncell); }
    for (int i = 0; i < nv; ++i) { p->off_slab[i] = off; off += align256(8 * ncell); }
    for (int i = 0; i < 2; ++i) { p->off_wtar[i] = off; off += align256(npx * 2); }
    for (int i = 0; i < 2; ++i) { p->off_wtal[i] = off; off += align256(npx * 2); }
    if (p->learned || p->median)
        for (int i = 0; i < 2; ++i) { p->off_dsub[i] = off; off += align256(npx * 4); }
    if (p->learned) {
        p->off_feat = off; off += align256(2 * npx * 16);
        for (int i = 0; i < 2; ++i) { p->off_vtmp[i] = off; off += align256(npx); }
        p->off_logit = off; off += align256(2 * npx * 4);
        p->off_lrws = off; off += align256(lrnet_forward_ws_bytes(2, H, W));
    }
    p->ws_bytes = off;
    std::vector<AggView> views(nv);
    std::vector<AggTask> tasks;
    std::vector<int> lens;
    for (int i = 0; i < nv; ++i) {
        AggView &v = views[i];
        v.cost_off = p->off_cost[i];
        v.slab_off = p->off_slab[i];
        v.H = H;
        v.W = W;
        v.K = D / 16;
        v.P1 = P1;
        v.P2 = P2;
        v.ndir = 8;
        for (int r = 0; r < 8; ++r) v.dir[r] = r;
        append_agg_tasks(tasks, lens, i, v, tun.chains_per_block);
    }
    if (tun.order == 0) sort_tasks_longest_first(tasks, lens);
    int rc = plan_upload_tables(*p, views, tasks);
    if (rc) {
        sf_plan_destroy(reinterpret_cast<sf_plan>(p));
        return rc;
    }
    p->tuning = tun;
    p->persistent_blocks = tun.persistent_per_cu > 0 ? tun.persistent_per_cu * cu_count_dev() : 0;
    *out = reinterpret_cast<sf_plan>(p);
    return SF_OK;
}

extern "C" size_t sf_plan_workspace_bytes(sf_plan plan)
{
    return plan ? reinterpret_cast<Plan *>(plan)->ws_bytes : 0;
}

extern "C" int sf_plan_destroy(sf_plan plan)
{
    if (!plan) return SF_OK;
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (p->d_tables) (void)hipFree(p->d_tables);
    if (p->batch) destroy_batch(p->batch);
    delete p;
    return SF_OK;
}

extern "C" int sf_frame_run(sf_plan plan, const uint8_t *L0, const uint8_t *R0, const uint8_t *L1,
                            const uint8_t *R1, int pitch, const float *flow, const sf_camera *cam,
                            float *disp0, uint8_t *valid0, float *disp1, uint8_t *valid1,
                            float *sf4, uint8_t *valid, float *xyz0, float *motion,
                            void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    SF_REQUIRE(plan, SF_EINVAL, "sf_frame_run: NULL plan");
    Plan *p = reinterpret_cast<Plan *>(plan);
    SF_REQUIRE(p->kind == Plan::FRAME && !p->learned, SF_EINVAL,
               "sf_frame_run: not a plain frame plan");
    SF_REQUIRE(L0 && R0 && L1 && R1 && flow && disp0 && valid0 && disp1 && valid1 && sf4 && valid,
               SF_EINVAL, "sf_frame_run: NULL pointer");
    SF_REQUIRE(pitch >= p->W, SF_EINVAL, "sf_frame_run: pitch < W");
    SF_REQUIRE((long long)p->H * pitch <= 0x7FFFFFFFLL, SF_EINVAL, "sf_frame_run: H * pitch too large");
    SF_REQUIRE(!cam || (xyz0 && motion), SF_EINVAL, "sf_frame_run: camera given without xyz0/motion");
    if (cam) SF_REQUIRE(cam->f != 0.0f, SF_EINVAL, "sf_frame_run: focal length is zero");
    SF_REQUIRE(workspace, SF_EINVAL, "sf_frame_run: NULL workspace");
    SF_REQUIRE(ws_bytes >= p->ws_bytes, SF_ENOMEM, "sf_frame_run: workspace too small");
    hipStream_t st = as_stream(stream);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    const int H = p->H, W = p->W, D = p->D;
    auto at = [&](size_t off) { return ws + off; };
    const bool packed = frame_packed(p->tuning, D, ws);
    const uint8_t *img[4] = {L0, R0, L1, R1};
    uint64_t *cen[4];
    for (int i = 0; i < 4; ++i) cen[i] = reinterpret_cast<uint64_t *>(at(p->off_cen[i]));

    CensusArgs ca{};
    for (int i = 0; i < 4; ++i) { ca.img[i] = img[i]; ca.out[i] = cen[i]; ca.pitch[i] = pitch; }
    ca.n = 4; ca.H = H; ca.W = W;
    int rc = launch_census(ca, st);
    if (rc) return rc;

    float *dsp[2] = {disp0, disp1};
    uint8_t *vld[2] = {valid0, valid1};
    int16_t *wtar[2], *wtal[2];
    for (int t = 0; t < 2; ++t) {
        wtar[t] = reinterpret_cast<int16_t *>(at(p->off_wtar[t]));
        wtal[t] = reinterpret_cast<int16_t *>(at(p->off_wtal[t]));
    }
    // With the median, the WTA writes the dense sub-pixel map to scratch and the
    // median kernel writes the masked result.
    float *wdsp[2];
    for (int t = 0; t < 2; ++t)
        wdsp[t] = p->median ? reinterpret_cast<float *>(at(p->off_dsub[t])) : dsp[t];

    if (p->diag) {
        // Views: 0 = L0 base, 1 = L1 base; right maps by the diagonal search.
        CostArgs co{};
        for (int t = 0; t < 2; ++t) {
            co.base[t] = cen[2 * t];
            co.match[t] = cen[2 * t + 1];
            co.right[t] = 0;
            co.cost[t] = at(p->off_cost[t]);
        }
        co.n = 2; co.H = H; co.W = W; co.D = D;
        co.packed = packed;
        if ((rc = launch_cost(co, st))) return rc;
        AggImages ims{};
        if (p->adaptive) {
            ims.n = 2;
            for (int t = 0; t < 2; ++t) { ims.img[t] = img[2 * t]; ims.pitch[t] = pitch; }
        }
        if ((rc = launch_agg_tasks(p->d_views, p->d_tasks, p->ntasks, D / 16, ws, p->d_counter,
                                   p->persistent_blocks, st, p->tuning.chains_per_block,
                                   p->tuning.prefetch, &ims, packed)))
            return rc;
        WtaArgs wd{};
        for (int t = 0; t < 2; ++t) {
            WtaView &v = wd.v[t];
            v.slab = at(p->off_slab[t]);
            v.wta = wtal[t];
            v.wta_r_out = wtar[t];
            v.disp = wdsp[t];
            v.valid = vld[t];
            v.dense = p->median ? 1 : 0;
            v.nslab = 8; v.H = H; v.W = W; v.D = D; v.P2 = p->P2; v.tol = p->tol;
        }
        wd.n = 2;
        if ((rc = launch_wta_diag_slabs(wd, st))) return rc;
    } else {
        // Views: 0 = L0 base, 1 = R0 base, 2 = L1 base, 3 = R1 base.
        CostArgs co{};
        for (int t = 0; t < 2; ++t) {
            co.base[2 * t] = cen[2 * t];      co.match[2 * t] = cen[2 * t + 1];  co.right[2 * t] = 0;
            co.base[2 * t + 1] = cen[2 * t + 1]; co.match[2 * t + 1] = cen[2 * t]; co.right[2 * t + 1] = 1;
        }
        for (int i = 0; i < 4; ++i) co.cost[i] = at(p->off_cost[i]);
        co.n = 4; co.H = H; co.W = W; co.D = D;
        co.packed = packed;
        if ((rc = launch_cost(co, st))) return rc;

        // Each view's base image: L0, R0, L1, R1.
        AggImages ims{};
        if (p->adaptive) {
            ims.n = 4;
            for (int i = 0; i < 4; ++i) { ims.img[i] = img[i]; ims.pitch[i] = pitch; }
        }
        if ((rc = launch_agg_tasks(p->d_views, p->d_tasks, p->ntasks, D / 16, ws, p->d_counter,
                                   p->persistent_blocks, st, p->tuning.chains_per_block,
                                   p->tuning.prefetch, &ims, packed)))
            return rc;

        WtaArgs wr{};
        for (int t = 0; t < 2; ++t) {
            WtaView &v = wr.v[t];
            v.slab = at(p->off_slab[2 * t + 1]);
            v.wta = wtar[t];
            v.nslab = 8; v.H = H; v.W = W; v.D = D; v.P2 = p->P2; v.tol = p->tol; v.right_only = 1;
        }
        wr.n = 2;
        if ((rc = launch_wta_slabs(wr, st))) return rc;

        WtaArgs wl{};
        for (int t = 0; t < 2; ++t) {
            WtaView &v = wl.v[t];
            v.slab = at(p->off_slab[2 * t]);
            v.wta_r = wtar[t];
            v.wta = wtal[t];
            v.disp = wdsp[t];
            v.valid = vld[t];
            v.dense = p->median ? 1 : 0;
            v.nslab = 8; v.H = H; v.W = W; v.D = D; v.P2 = p->P2; v.tol = p->tol; v.right_only = 0;
        }
        wl.n = 2;
        if ((rc = launch_wta_slabs(wl, st))) return rc;
    }
    if (p->median)
        for (int t = 0; t < 2; ++t)
            if ((rc = launch_median_mask(wdsp[t], vld[t], H, W, dsp[t], st))) return rc;

    return launch_combine(disp0, valid0, disp1, valid1, flow, H, W, cam, sf4, valid, xyz0, motion, st);
}

extern "C" int sf_frame_run_learned(sf_plan plan, const uint8_t *L0, const uint8_t *R0,
                                    const uint8_t *L1, const uint8_t *R1, int pitch,
                                    const float *flow, const sf_camera *cam, const float *lr_params,
                                    float *disp0, uint8_t *valid0, float *disp1, uint8_t *valid1,
                                    float *sf4, uint8_t *valid, float *xyz0, float *motion,
                                    void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    SF_REQUIRE(plan, SF_EINVAL, "sf_frame_run_learned: NULL plan");
    Plan *p = reinterpret_cast<Plan *>(plan);
    SF_REQUIRE(p->kind == Plan::FRAME && p->learned, SF_EINVAL,
               "sf_frame_run_learned: not a learned frame plan");
    SF_REQUIRE(L0 && R0 && L1 && R1 && flow && lr_params && disp0 && valid0 && disp1 && valid1 &&
                   sf4 && valid,
               SF_EINVAL, "sf_frame_run_learned: NULL pointer");
    SF_REQUIRE(pitch >= p->W, SF_EINVAL, "sf_frame_run_learned: pitch < W");
    SF_REQUIRE((long long)p->H * pitch <= 0x7FFFFFFFLL, SF_EINVAL,
               "sf_frame_run_learned: H * pitch too large");
    SF_REQUIRE(!cam || (xyz0 && motion), SF_EINVAL,
               "sf_frame_run_learned: camera given without xyz0/motion");
    if (cam) SF_REQUIRE(cam->f != 0.0f, SF_EINVAL, "sf_frame_run_learned: focal length is zero");
    SF_REQUIRE(workspace, SF_EINVAL, "sf_frame_run_learned: NULL workspace");
    SF_REQUIRE(ws_bytes >= p->ws_bytes, SF_ENOMEM, "sf_frame_run_learned: workspace too small");
    hipStream_t st = as_stream(stream);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    const int H = p->H, W = p->W, D = p->D;
    auto at = [&](size_t off) { return ws + off; };
    const bool packed = frame_packed(p->tuning, D, ws);
    const uint8_t *img[4] = {L0, R0, L1, R1};
    uint64_t *cen[4];
    for (int i = 0; i < 4; ++i) cen[i] = reinterpret_cast<uint64_t *>(at(p->off_cen[i]));
    CensusArgs ca{};
    for (int i = 0; i < 4; ++i) { ca.img[i] = img[i]; ca.out[i] = cen[i]; ca.pitch[i] = pitch; }
    ca.n = 4; ca.H = H; ca.W = W;
    // The census launch also packs the network's weight fragments (one launch fewer).
    ca.pack_prm = lr_params;
    lrnet_pack_targets(at(p->off_lrws), &ca.pack_frag, &ca.pack_fl);
    int rc = launch_census(ca, st);
    if (rc) return rc;
    // Left-base cost volumes only: views 0 = L0 base, 1 = L1 base.
    CostArgs co{};
    for (int t = 0; t < 2; ++t) {
        co.base[t] = cen[2 * t];
        co.match[t] = cen[2 * t + 1];
        co.right[t] = 0;
        co.cost[t] = at(p->off_cost[t]);
    }
    co.n = 2; co.H = H; co.W = W; co.D = D;
    co.packed = packed;
    if ((rc = launch_cost(co, st))) return rc;
    AggImages ims{};
    if (p->adaptive) {
        ims.n = 2;
        for (int t = 0; t < 2; ++t) { ims.img[t] = img[2 * t]; ims.pitch[t] = pitch; }
    }
    if ((rc = launch_agg_tasks(p->d_views, p->d_tasks, p->ntasks, D / 16, ws, p->d_counter,
                               p->persistent_blocks, st, p->tuning.chains_per_block,
                               p->tuning.prefetch, &ims, packed)))
        return rc;
    // WTA + sub-pixel + features of both left maps (no right view).
    float *feat = reinterpret_cast<float *>(at(p->off_feat));
    WtaArgs wl{};
    for (int t = 0; t < 2; ++t) {
        WtaView &v = wl.v[t];
        v.slab = at(p->off_slab[t]);
        v.wta_r = nullptr;
        v.img = img[2 * t];
        v.pitch = pitch;
        v.wta = reinterpret_cast<int16_t *>(at(p->off_wtal[t]));
        v.disp = reinterpret_cast<float *>(at(p->off_dsub[t]));
        v.valid = at(p->off_vtmp[t]);
        v.feat = feat + (size_t)t * H * W * 4;
        v.nslab = 8; v.H = H; v.W = W; v.D = D; v.P2 = p->P2; v.tol = p->tol; v.right_only = 0;
    }
    wl.n = 2;
    if ((rc = launch_wta_slabs(wl, st))) return rc;
    // The network writes each map's learned mask and masked disparities itself.
    float *logits = reinterpret_cast<float *>(at(p->off_logit));
    float *dsp[2] = {disp0, disp1};
    uint8_t *vld[2] = {valid0, valid1};
    LrMaskOut mo{};
    for (int t = 0; t < 2; ++t) {
        mo.wta[t] = reinterpret_cast<const int16_t *>(at(p->off_wtal[t]));
        mo.dsub[t] = reinterpret_cast<const float *>(at(p->off_dsub[t]));
        mo.valid[t] = vld[t];
        mo.disp[t] = dsp[t];
    }
    if ((rc = lrnet_forward(lr_params, feat, 2, H, W, logits, at(p->off_lrws), st, &mo, true))) return rc;
    if (p->median)
        for (int t = 0; t < 2; ++t)
            if ((rc = launch_median_mask(mo.dsub[t], vld[t], H, W, dsp[t], st))) return rc;
    return launch_combine(disp0, valid0, disp1, valid1, flow, H, W, cam, sf4, valid, xyz0, motion, st);
}

// --- frame autotuner ----------------------------------------------------------
namespace {
// Seeded bytes (hash of the word index) or zeros, for the autotuner's inputs.
__global__ void tune_fill_kernel(uint32_t *p, size_t nwords, uint32_t seed, int random)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords;
         i += (size_t)gridDim.x * blockDim.x) {
        uint32_t h = 0;
        if (random) {
            h = (uint32_t)i * 0x9E3779B1u ^ seed;
            h ^= h >> 15;
            h *= 0x2C1B3C6Du;
            h ^= h >> 12;
        }
        p[i] = h;
    }
}

size_t al256f(size_t v) { return (v + 255) & ~(size_t)255; }
}  // namespace

extern "C" int sf_frame_autotune(int H, int W, int D, int P1, int P2, int lr_tol, int flags,
                                 void *stream, sf_agg_tuning *best, float *best_ms)
{
    clear_error();
    SF_REQUIRE(best, SF_EINVAL, "sf_frame_autotune: NULL best");
    sf_plan probe = nullptr;
    int rc = sf_frame_plan_create(H, W, D, P1, P2, lr_tol, flags, nullptr, &probe);
    if (rc) return rc;
    const size_t ws_bytes = sf_plan_workspace_bytes(probe);
    sf_plan_destroy(probe);
    const bool learned = (flags & SF_FRAME_LEARNED) != 0;
    hipStream_t st = as_stream(stream);
    // One allocation: 4 images, flow, network parameters, the outputs, the workspace.
    const size_t npx = (size_t)H * W;
    size_t off = 0;
    const size_t o_img = off; off += al256f(4 * npx);
    const size_t o_flow = off; off += al256f(npx * 8);
    const size_t o_prm = off; off += al256f((size_t)sf_lrnet_nparams() * 4);
    const size_t o_d0 = off; off += al256f(npx * 4);
    const size_t o_v0 = off; off += al256f(npx);
    const size_t o_d1 = off; off += al256f(npx * 4);
    const size_t o_v1 = off; off += al256f(npx);
    const size_t o_sf = off; off += al256f(npx * 16);
    const size_t o_v = off; off += al256f(npx);
    const size_t o_xyz = off; off += al256f(npx * 12);
    const size_t o_mot = off; off += al256f(npx * 12);
    const size_t o_ws = off; off += al256f(ws_bytes);
    uint8_t *buf = nullptr;
    if (hipMalloc(&buf, off) != hipSuccess) return fail(SF_EHIP, "sf_frame_autotune: hipMalloc");
    hipLaunchKernelGGL(tune_fill_kernel, dim3(2048), dim3(256), 0, st, reinterpret_cast<uint32_t *>(buf),
                       o_ws / 4, 0x5EEDu, 0);
    hipLaunchKernelGGL(tune_fill_kernel, dim3(2048), dim3(256), 0, st,
                       reinterpret_cast<uint32_t *>(buf + o_img), (4 * npx) / 4, 0x5EEDu, 1);
    const uint8_t *img[4];
    for (int i = 0; i < 4; ++i) img[i] = buf + o_img + i * npx;
    const sf_camera cam{721.5f, 0.54f, 0.5f * (float)(W - 1), 0.5f * (float)(H - 1)};
    auto run = [&](sf_plan pl) {
        float *d0 = reinterpret_cast<float *>(buf + o_d0), *d1 = reinterpret_cast<float *>(buf + o_d1);
        float *sf = reinterpret_cast<float *>(buf + o_sf), *xyz = reinterpret_cast<float *>(buf + o_xyz);
        float *mot = reinterpret_cast<float *>(buf + o_mot);
        const float *flow = reinterpret_cast<const float *>(buf + o_flow);
        if (learned)
            return sf_frame_run_learned(pl, img[0], img[1], img[2], img[3], W, flow, &cam,
                                        reinterpret_cast<const float *>(buf + o_prm), d0, buf + o_v0, d1,
                                        buf + o_v1, sf, buf + o_v, xyz, mot, buf + o_ws, ws_bytes, stream);
        return sf_frame_run(pl, img[0], img[1], img[2], img[3], W, flow, &cam, d0, buf + o_v0, d1,
                            buf + o_v1, sf, buf + o_v, xyz, mot, buf + o_ws, ws_bytes, stream);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipFree(buf);
        return fail(SF_EHIP, "sf_frame_autotune: hipEventCreate");
    }
    float best_t = 1e30f;
    // Candidates: packed costs (where D allows) x chains per block x order x prefetch x
    // persistent blocks per CU.
    std::vector<sf_agg_tuning> cand;
    for (int pk = 0; pk <= (cost_packable(D) ? 1 : 0); ++pk)
        for (int cpb : {4, 8, 16})
            for (int order : {0, 1})
                for (int pf : {4, 8})
                    for (int pp : {0, 4, 8}) cand.push_back(sf_agg_tuning{cpb, pf, order, pp, pk});
    constexpr int REPS = 5, FRAMES = 3;
    for (size_t c = 0; c < cand.size() && rc == SF_OK; ++c) {
        sf_plan pl = nullptr;
        if ((rc = sf_frame_plan_create(H, W, D, P1, P2, lr_tol, flags, &cand[c], &pl))) break;
        for (int w = 0; w < 2 && rc == SF_OK; ++w) rc = run(pl);
        float tms[REPS];
        for (int r = 0; r < REPS && rc == SF_OK; ++r) {
            if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(SF_EHIP, "sf_frame_autotune: event"); break; }
            for (int f = 0; f < FRAMES && rc == SF_OK; ++f) rc = run(pl);
            if (rc) break;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&tms[r], e0, e1) != hipSuccess)
                rc = fail(SF_EHIP, "sf_frame_autotune: event timing");
            tms[r] /= FRAMES;
        }
        sf_plan_destroy(pl);
        if (rc) break;
        std::sort(tms, tms + REPS);
        if (tms[REPS / 2] < best_t) {
            best_t = tms[REPS / 2];
            *best = cand[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    if (rc) return rc;
    if (best_ms) *best_ms = best_t;
    return SF_OK;
}
