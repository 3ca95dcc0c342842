// Multi-view aggregation task tables (shared by the frame and batch paths).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

namespace sf {

// One view to aggregate.  Pointers are base + offset, where base is a kernel
// argument (the caller's workspace) so a table stays valid for any workspace
// address when the offsets are relative, or base = 0 and offsets absolute.
struct AggView {
    uint64_t cost_off;  // cost volume [H][W][16 K] u8
    uint64_t slab_off;  // ndir slabs [ndir][H][W][16 K] u8
    int H, W, K;        // D = 16 K
    int P1, P2;
    int ndir;
    int dir[8];         // direction of slab slot s
};

// Up to 16 consecutive chains (lines line0 ..) of one direction slot of a view.
struct AggTask {
    int view, slot, line0, nlines;
};

// Base images of the views of a launch, for the intensity-adaptive large-jump
// penalty (n = 0: constant P2).  img[v] is view v's base image [H][pitch[v]].
constexpr int AGG_MAX_IMG = 8;
struct AggImages {
    const uint8_t *img[AGG_MAX_IMG];
    int pitch[AGG_MAX_IMG];
    int n;
};

int chains_of(int r, int H, int W);
void append_agg_tasks(std::vector<AggTask> &tasks, std::vector<int> &task_len, int view,
                      const AggView &v, int chains_per_task = 16);
void sort_tasks_longest_first(std::vector<AggTask> &tasks, const std::vector<int> &task_len);
// persistent_blocks > 0: persistent launch with that many blocks pulling from
// *d_counter, which must be 0 before the first launch (the kernel leaves it at
// 0 again); 0: one block per task.  Launches sharing a counter must not overlap.
// chains_per_block in {4, 8, 16} must match the table's chains per task;
// prefetch (cost steps in flight per chain) in {4, 8}.
// images: NULL or n = 0 for the constant P2; otherwise every view index of the
// table must be < n.
// packed: the cost volumes hold 6-bit costs (CostArgs::packed; K = 8 or 16).
int launch_agg_tasks(const AggView *d_views, const AggTask *d_tasks, int ntasks, int K,
                     uint8_t *base, int *d_counter, int persistent_blocks, hipStream_t st,
                     int chains_per_block = 16, int prefetch = 8, const AggImages *images = nullptr,
                     bool packed = false);

}  // namespace sf
