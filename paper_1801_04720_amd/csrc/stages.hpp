// Launch helpers of the per-pixel stages, each covering several images or
// views of one size in one launch (the views travel in the kernel arguments).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sf.h"

namespace sf {

constexpr int STAGE_MAXV = 8;  // views per launch

struct CensusArgs {
    const uint8_t *img[STAGE_MAXV];
    uint64_t *out[STAGE_MAXV];
    int pitch[STAGE_MAXV];
    int n, H, W;
    // Optional extra job (pack_prm != NULL, n < STAGE_MAXV): pack the network's
    // weight fragments from pack_prm into the targets of lrnet_pack_targets.
    const float *pack_prm;
    uint4 *pack_frag;
    float *pack_fl;
};

// packed = 1 (D = 128 or 256, cost volumes 4-byte aligned): the volume holds
// 6-bit costs, 0.75 D bytes per pixel, each run of 16 disparities d = 16c ..
// 16c + 15 as 16 consecutive 6-bit fields (LSB first) in the 12 bytes at byte
// 12c of its pixel (cost_packed_bytes gives the volume size).  The fused frame
// and batch paths aggregate from it; the C ABI keeps one byte per cost.
struct CostArgs {
    const uint64_t *base[STAGE_MAXV];
    const uint64_t *match[STAGE_MAXV];
    uint8_t *cost[STAGE_MAXV];
    int right[STAGE_MAXV];
    int n, H, W, D;
    int vec;  // store width in bytes (16, 4 or 1), set by launch_cost from D and the pointers' alignment
    int packed;
};

inline bool cost_packable(int D) { return D == 128 || D == 256; }
inline size_t cost_packed_bytes(int H, int W, int D) { return (size_t)H * W * (size_t)(3 * D / 4); }

// WTA over the sum of nslab u8 slabs [nslab][H][W][D] (D a multiple of 8;
// launch_wta_slabs needs nslab = 8, the diagonal-search launch takes 1..8).
// right_only: write d* to wta only.  Otherwise d*, sub-pixel disparity, the LR
// check against wta_r (NULL: no check, valid := 1) and optional features.
// dense: disp holds the sub-pixel disparity everywhere (valid still written).
// The diagonal-search launch ignores wta_r and may write the right map to
// wta_r_out.
struct WtaView {
    const uint8_t *slab;
    const int16_t *wta_r;
    const uint8_t *img;
    int16_t *wta;
    float *disp;
    uint8_t *valid;
    float *feat;
    int16_t *wta_r_out;
    int nslab, H, W, D, P2, tol, pitch, right_only, dense;
};

struct WtaArgs {
    WtaView v[STAGE_MAXV];
    int blk0[STAGE_MAXV + 1];  // first block of each view; blk0[n] = grid size (set by the launchers)
    int n;
};

int launch_census(const CensusArgs &a, hipStream_t st);
int launch_cost(const CostArgs &a, hipStream_t st);
int launch_wta_slabs(const WtaArgs &a, hipStream_t st);  // computes the block offsets itself
int launch_wta_diag_slabs(WtaArgs &a, hipStream_t st);  // fills blk0; W <= 4096
// out = 3x3 median of dense (clamp-to-edge), or -1 where mask is 0 (mask may be NULL).
int launch_median_mask(const float *dense, const uint8_t *mask, int H, int W, float *out,
                       hipStream_t st);
size_t lrnet_forward_ws_bytes(int B, int H, int W);
// Learned mask written by the network's own last step (maps b < 2): valid =
// logit > 0 and x - wta >= 0, disp = valid ? dsub : -1 (as launch_lr_mask).
struct LrMaskOut {
    const int16_t *wta[2];
    const float *dsub[2];
    uint8_t *valid[2];
    float *disp[2];
};
// Where the inference workspace holds the packed weight fragments.
void lrnet_pack_targets(uint8_t *ws, uint4 **frag, float **fl);
// prepacked: the fragments in ws already hold params (packed by an earlier
// launch on the stream), so no packing launch precedes the network's.
int lrnet_forward(const float *params, const float *feat, int B, int H, int W, float *logits,
                  uint8_t *ws, hipStream_t st, const LrMaskOut *mask = nullptr,
                  bool prepacked = false);
int launch_lr_mask(const float *logits, const int16_t *wta, const float *dsub, int H, int W,
                   uint8_t *valid, float *disp, hipStream_t st);
int launch_combine(const float *disp0, const uint8_t *valid0, const float *disp1,
                   const uint8_t *valid1, const float *flow, int H, int W, const sf_camera *cam,
                   float *sf4, uint8_t *valid, float *xyz0, float *motion, hipStream_t st);

}  // namespace sf
