// Host-side plan objects behind the opaque sf_plan handle.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "sf.h"
#include "sgm_tasks.hpp"

namespace sf {

struct BatchData;
void destroy_batch(BatchData *b);

struct Plan {
    enum Kind { FRAME, BATCH, LRNET } kind = FRAME;
    int H = 0, W = 0, D = 0, P1 = 0, P2 = 0, tol = 0;
    size_t ws_bytes = 0;
    // Frame workspace layout (byte offsets).
    size_t off_cen[4] = {}, off_cost[4] = {}, off_slab[4] = {}, off_wtar[2] = {}, off_wtal[2] = {};
    // Learned frame: features [2][H][W][4], sub-pixel maps, logits, scratch masks, net workspace.
    bool learned = false, diag = false, median = false, adaptive = false;
    size_t off_feat = 0, off_dsub[2] = {}, off_logit = 0, off_vtmp[2] = {}, off_lrws = 0;
    // Aggregation task table (plan-owned device memory).
    void *d_tables = nullptr;
    AggView *d_views = nullptr;
    AggTask *d_tasks = nullptr;
    int *d_counter = nullptr;
    int ntasks = 0, nviews = 0;
    int persistent_blocks = 0;
    sf_agg_tuning tuning{16, 8, 0, 0};
    // Batch plans: pairs, waves, per-class tunings, captured graph.
    BatchData *batch = nullptr;
};

int plan_upload_tables(Plan &p, const std::vector<AggView> &views, const std::vector<AggTask> &tasks);
int cu_count_dev();

}  // namespace sf
