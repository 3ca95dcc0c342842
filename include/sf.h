/*
 * sf.h - C ABI of the MI355X (gfx950) stereo / scene-flow hot path.
 *
 * The method: two rectified, temporally adjacent stereo pairs on one image
 * domain Omega (paper, Sec. 3); a disparity map D: Omega -> R+ per time step by
 * semi-global matching over eight paths with a left-right consistency check
 * that leaves it non-dense (Sec. 3.1, Eq. 1); a flow field F: Omega -> R^2
 * (Sec. 3.2, supplied by the caller); and the combination into the scene-flow
 * map S: Omega -> R^4, S(x) = (u, v, d0, d1) with d1 read bilinearly at
 * x + F(x), undefined where x + F(x) leaves Omega or a disparity is invalid
 * (Sec. 3.3, case definition and bilinear equation).
 *
 * Conventions shared by every entry point:
 *   - All array arguments are DEVICE pointers to caller-owned memory unless a
 *     comment says "host".  The library never allocates or frees them; where
 *     scratch memory is needed the caller passes a workspace and its size.
 *   - Images and maps are row-major [H][W]; cost and aggregated-cost volumes
 *     are [H][W][D] with the disparity index fastest.
 *   - Calls enqueue work on `stream` (a hipStream_t; NULL = default stream)
 *     and return without synchronising.
 *   - Arguments are validated on the host before anything is launched.  On
 *     failure nothing is enqueued and the status is returned; sf_last_error()
 *     then holds a message for the calling thread.
 *   - Direction numbering for path masks, r = (rx, ry), predecessor p - r:
 *       0:(+1,0) 1:(-1,0) 2:(0,+1) 3:(0,-1) 4:(+1,+1) 5:(-1,+1) 6:(+1,-1) 7:(-1,-1)
 */
#ifndef SF_H
#define SF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SF_OK 0
#define SF_EINVAL 1        /* bad argument: NULL pointer, size <= 0, pitch < W, P2 < P1 ... */
#define SF_EUNSUPPORTED 2  /* valid for the method, not supported by these kernels (e.g. D) */
#define SF_EHIP 3          /* HIP runtime / launch error */
#define SF_ENOMEM 4        /* workspace smaller than the required size */

#define SF_ABI_VERSION 1
#define SF_DMAX 256        /* largest disparity range the kernels accept */
#define SF_CMAX 62         /* largest Hamming cost of the 9x7 census (62 bits) */

int sf_abi_version(void);
/* Message describing the last failure of an sf_* call on this thread ("" if none). */
const char *sf_last_error(void);

/* ---------------------------------------------------------------------------
 * Census transform (the matching cost of SGM, Sec. 3.1; the paper names none).
 * 9 wide x 7 tall window; neighbours in row-major order with the centre
 * skipped; bit = 1 iff neighbour < centre; the first neighbour lands in bit 61
 * and the last in bit 0 (bits 63..62 are zero); pixels outside the image take
 * the nearest edge pixel.
 *   img    [H][pitch] uint8, pitch >= W
 *   census [H][W] uint64 (output)
 * Errors: SF_EINVAL for NULL pointers, H or W <= 0, pitch < W. */
int sf_census(const uint8_t *img, int H, int W, int pitch, uint64_t *census, void *stream);

/* ---------------------------------------------------------------------------
 * Matching-cost volume: Hamming distance between the base pixel's census and
 * the match pixel's, for every disparity d in [0, D).
 *   base_is_right = 0: base = left view, match pixel (x - d, y)
 *   base_is_right = 1: base = right view, match pixel (x + d, y)
 * A match pixel outside the image costs SF_CMAX (62).
 *   cen_base, cen_match [H][W] uint64;  cost [H][W][D] uint8 (output)
 * Errors: SF_EINVAL (NULL, H/W <= 0, D < 1 or D > SF_DMAX). */
int sf_cost(const uint64_t *cen_base, const uint64_t *cen_match, int H, int W, int D,
            int base_is_right, uint8_t *cost, void *stream);

/* ---------------------------------------------------------------------------
 * Semi-global aggregation over the selected paths (Sec. 3.1: eight paths
 * radiating from each pixel; recurrence of the cited SGM method).  For each
 * direction r in path_mask, with predecessor p - r:
 *   Lr(p, d) = C(p, d)                                   if p - r is outside
 *   Lr(p, d) = C(p, d) + min(Lr(p-r, d), Lr(p-r, d-1) + P1, Lr(p-r, d+1) + P1,
 *                            M + P2) - M,   M = min_k Lr(p-r, k)   otherwise
 * (terms with d +- 1 outside [0, D) dropped) and S(p, d) = sum_r Lr(p, d).
 * All values are exact integers: Lr <= 62 + P2 and S <= 8 (62 + P2).
 *   cost      [H][W][D] uint8 (values <= 62)
 *   S         [H][W][D] uint16 (output)
 *   workspace device scratch of at least sf_sgm_workspace_bytes(H, W, D) bytes
 * Supported: D a multiple of 32 in [32, 256]; 0 <= P1 <= P2 <= 8000;
 * path_mask in [1, 255]; H * W * D < 2^31 (the kernels use 32-bit offsets).
 * Errors: SF_EINVAL (NULL, H/W <= 0, P2 < P1, P2 > 8000, mask 0 or > 255),
 * SF_EUNSUPPORTED (D), SF_ENOMEM (ws_bytes too small). */
size_t sf_sgm_workspace_bytes(int H, int W, int D);
/* Tuning knob for the aggregation's output stage: 0 = automatic (u8 slabs + sum
 * while 62 + P2 <= 255, packed atomics otherwise), 1 = u8 slabs + sum,
 * 2 = packed 32-bit atomics into a zero-filled S.  Results are identical.
 * Process-wide; not thread-safe.  Errors: SF_EINVAL for other modes. */
int sf_sgm_set_epilogue(int mode);
int sf_sgm_aggregate(const uint8_t *cost, int H, int W, int D, int P1, int P2,
                     uint32_t path_mask, uint16_t *S, void *workspace, size_t ws_bytes,
                     void *stream);
/* The same aggregation with the matching cost computed inside the path walk
 * from the two census images (Sec. 3.1 paths; cost as sf_cost: the Hamming
 * distance of the base pixel's census to the match pixel's, x - d for a left
 * base, x + d for a right base, SF_CMAX where the match pixel is outside the
 * image), so no cost volume is read or written.  S equals
 * sf_cost(cen_base, cen_match, ...) followed by sf_sgm_aggregate.
 *   cen_base, cen_match [H][W] uint64 (as sf_census writes them)
 *   base_is_right 0 or 1; other arguments, limits and errors as sf_sgm_aggregate
 *   (SF_EINVAL also for a NULL census or base_is_right outside {0, 1}). */
int sf_sgm_aggregate_census(const uint64_t *cen_base, const uint64_t *cen_match, int H, int W, int D,
                            int base_is_right, int P1, int P2, uint32_t path_mask, uint16_t *S,
                            void *workspace, size_t ws_bytes, void *stream);
/* Intensity-adaptive variant of the cited SGM method: the large-jump penalty at
 * p is taken from the base image along the path,
 *   P2(p, r) = P2                          if g = |I(p) - I(p - r)| = 0
 *            = max(P1, floor(P2 / g))      otherwise,
 * in place of the constant P2 (path starts have no predecessor and Lr = C).
 *   img [H][pitch] uint8, the base image of the cost volume (pitch >= W,
 *   H * pitch < 2^31); other arguments, limits and errors as sf_sgm_aggregate. */
int sf_sgm_aggregate_adaptive(const uint8_t *cost, const uint8_t *img, int pitch, int H, int W,
                              int D, int P1, int P2, uint32_t path_mask, uint16_t *S,
                              void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Winner-take-all, sub-pixel refinement, left-right check (Sec. 3.1: the
 * check compares two computed disparity maps and removes inconsistent pixels,
 * leaving a non-dense map) and, optionally, the learned stand-in's features.
 *   d*      = smallest d with S(p, d) = min_k S(p, k)
 *   d_sub   = d* + (S(d*-1) - S(d*+1)) / (2 (S(d*-1) - 2 S(d*) + S(d*+1)))
 *             when 0 < d* < D-1 and the denominator is > 0, else d*
 *             (one FP32 division, one FP32 addition)
 *   valid   = q = x - d*_L >= 0 and |d*_L(x, y) - d*_R(q, y)| <= lr_tol
 *   disp    = d_sub where valid, -1.0f elsewhere; the uint8 mask is authoritative
 * Arguments:
 *   S_left    [H][W][D] uint16, left-view aggregated costs
 *   S_right   [H][W][D] uint16 right-view costs, or NULL: no check, valid := 1
 *   wta_left  [H][W] int16 (output) d*_L, unmasked
 *   wta_right [H][W] int16 (output) d*_R; required iff S_right != NULL
 *   disp      [H][W] float (output);  valid [H][W] uint8 (output)
 *   feat      [H][W][4] float (output) or NULL; needs img_left (pitch >= W):
 *             k=0 I_L/255, k=1 d* / (D-1), k=2 S(d*)/(8 (62+P2)),
 *             k=3 S2/max(S(d*),1) with S2 = min of S over |d - d*| >= 2
 *             (S(d*) when no such d); FP32 divisions
 * Supported D: any in [1, SF_DMAX].  Errors: SF_EINVAL. */
int sf_wta_lr(const uint16_t *S_left, const uint16_t *S_right, const uint8_t *img_left, int pitch,
              int H, int W, int D, int P2, int lr_tol, int16_t *wta_left, int16_t *wta_right,
              float *disp, uint8_t *valid, float *feat, void *stream);

/* ---------------------------------------------------------------------------
 * Variants of the cited SGM method (the paper's disparity step names SGM and
 * its left-right check; these are that method's own options).
 *
 * sf_wta_right_diag: the right view's disparity without a right-view
 * aggregation, found on the diagonal of the left volume:
 *   d*_R(q, y) = smallest d in [0, D) with q + d <= W-1 minimising S_L(q + d, y, d)
 *   S_left [H][W][D] uint16;  wta_right [H][W] int16 (output).
 *   Supported D: [1, SF_DMAX].  Errors: SF_EINVAL.
 *
 * sf_lr_check: the left-right check of sf_wta_lr on given maps:
 *   valid = q = x - wta_left >= 0 and |wta_left(x, y) - wta_right(q, y)| <= lr_tol;
 *   disp = dsub where valid, -1.0f elsewhere.
 *   wta_left, wta_right [H][W] int16; dsub [H][W] float; valid [H][W] uint8 and
 *   disp [H][W] float (outputs).  Errors: SF_EINVAL.
 *
 * sf_median3x3: 3x3 median post-filter of a disparity map:
 *   out(x, y) = 5th smallest of in(x+i, y+j), i, j in {-1, 0, 1}, coordinates
 *   clamped to the image (bit-exact: the result is one of the nine inputs);
 *   with mask != NULL, out = -1.0f where mask is 0.  in, out [H][W] float,
 *   distinct buffers; mask [H][W] uint8 or NULL.  Errors: SF_EINVAL. */
int sf_wta_right_diag(const uint16_t *S_left, int H, int W, int D, int16_t *wta_right, void *stream);
int sf_lr_check(const int16_t *wta_left, const int16_t *wta_right, const float *dsub, int H, int W,
                int lr_tol, uint8_t *valid, float *disp, void *stream);
int sf_median3x3(const float *in, const uint8_t *mask, int H, int W, float *out, void *stream);

/* ---------------------------------------------------------------------------
 * Combination and triangulation (Sec. 3.3).
 * For each pixel x = (x, y): (u, v) = flow, x' = x + u, y' = y + v.
 * S(x) = (u, v, d0 = disp0(x), d1) is defined iff valid0(x), 0 <= x' <= W-1 and
 * 0 <= y' <= H-1 (NaN fails), and the four taps (x0,y0) (x1,y0) (x0,y1) (x1,y1)
 * with x0 = floor(x'), y0 = floor(y'), x1 = min(x0+1, W-1), y1 = min(y0+1, H-1)
 * are valid in valid1.  d1 is the bilinear equation of Sec. 3.3 with
 * fx = x' - x0, fy = y' - y0, its four terms ((D*w1)*w2) summed in the printed
 * order, in FP32.
 * With a camera (host pointer, NULL = no 3-D output): where S is defined and
 * d0 > 0 and d1 > 0, Z = (f*B)/d, X = ((x - cx) Z)/f, Y = ((y - cy) Z)/f;
 * xyz0 = P0 from (x, y, d0); motion = P1 - P0 with P1 from (x', y', d1).
 *   disp0, disp1 [H][W] float; valid0, valid1 [H][W] uint8; flow [H][W][2] float
 *   sf4 [H][W][4] float (output; 4x NaN where undefined)
 *   valid [H][W] uint8 (output): bit 0 = S defined, bit 1 = 3-D defined
 *   xyz0, motion [H][W][3] float (outputs, NaN where undefined); ignored if cam NULL
 * Errors: SF_EINVAL. */
typedef struct {
    float f;   /* focal length, px */
    float B;   /* baseline, m */
    float cx;  /* principal point, px */
    float cy;
} sf_camera;

int sf_combine(const float *disp0, const uint8_t *valid0, const float *disp1,
               const uint8_t *valid1, const float *flow, int H, int W, const sf_camera *cam,
               float *sf4, uint8_t *valid, float *xyz0, float *motion, void *stream);

/* ---------------------------------------------------------------------------
 * Plans.  A plan is a host object fixing sizes and parameters of a fused
 * multi-stage run; it owns a small device buffer with its aggregation task
 * table (allocated and written once by the create call, freed by destroy) and
 * lays out the caller's workspace, whose size sf_plan_workspace_bytes reports.
 * Runs allocate nothing and enqueue only kernel launches, so they can be
 * captured in a HIP graph.  A plan may be run concurrently on different
 * streams only with different workspaces, and only if its aggregation tuning
 * is not persistent: persistent launches pull tasks from a counter in the
 * plan's buffer, which each launch leaves at zero for the next one, so runs of
 * such a plan must follow one another (one stream, or ordered by events). */
typedef struct sf_plan_s *sf_plan;

/* Tuning of the multi-view aggregation launch (frame and batch plans):
 *   chains_per_block  4, 8 or 16 chains (16-lane rows) per block
 *   prefetch          4 or 8 cost steps in flight per chain
 *   order             0 = tasks longest chains first, 1 = view by view
 *   persistent_per_cu 0 = one block per task; k > 0 = k blocks per CU pulling
 *                     tasks from a counter
 *   packed            0 = the run's internal cost volumes hold one byte per
 *                     cost; 1 = 6-bit costs, 0.75 D bytes per pixel, where D
 *                     is 128 or 256 (otherwise bytes): a quarter fewer bytes
 *                     written by the cost stage and re-read by each of the
 *                     eight directions, for a few more instructions per step
 * Every tuning gives identical results. */
typedef struct {
    int chains_per_block, prefetch, order, persistent_per_cu, packed;
} sf_agg_tuning;
size_t sf_plan_workspace_bytes(sf_plan plan);
int sf_plan_destroy(sf_plan plan);

/* Plain scene-flow frame (Sec. 3 and Sec. 3.3 end to end): the stereo pairs at
 * t0 and t1 go through census, left- and right-base costs, 8-path aggregation,
 * WTA + sub-pixel + LR check (as sf_wta_lr, but summing the per-direction path
 * costs on the fly instead of materialising S), then sf_combine's
 * combination and triangulation with the given flow.
 *   flags: SF_FRAME_PERSISTENT = persistent aggregation blocks pulling tasks
 *          from a counter (same results); SF_FRAME_LEARNED = the learned
 *          frame (sf_frame_run_learned): the right-view aggregations are
 *          skipped and the LR check is replaced by the network's mask;
 *          SF_FRAME_DIAG = plain frame whose right maps come from the
 *          diagonal search in the left volumes (sf_wta_right_diag), so the
 *          right-view aggregations are skipped (not with LEARNED; W <= 4096);
 *          SF_FRAME_MEDIAN = each left map's sub-pixel disparities pass the
 *          3x3 median (sf_median3x3) before the mask is applied;
 *          SF_FRAME_ADAPTIVE_P2 = intensity-adaptive large-jump penalty in
 *          every aggregation (sf_sgm_aggregate_adaptive; each view's base
 *          image: L0, R0, L1, R1).
 * Supported: D a multiple of 32 in [32, 256]; 62 + P2 <= 255; H <= 65535;
 * H * W * D < 2^31.
 * Errors: SF_EINVAL, SF_EUNSUPPORTED, SF_EHIP (device table upload). */
#define SF_FRAME_PERSISTENT 1
#define SF_FRAME_LEARNED 2
#define SF_FRAME_DIAG 4
#define SF_FRAME_MEDIAN 8
#define SF_FRAME_ADAPTIVE_P2 16
int sf_frame_plan_create(int H, int W, int D, int P1, int P2, int lr_tol, int flags,
                         const sf_agg_tuning *tuning /* host, NULL = default */, sf_plan *plan);
/* L0, R0, L1, R1 [H][pitch] uint8; flow [H][W][2]; cam host pointer or NULL.
 * Outputs: disp0/valid0 (t0 map), disp1/valid1 (t1 map), as sf_wta_lr;
 * sf4/valid/xyz0/motion as sf_combine.  Errors: SF_EINVAL, SF_ENOMEM
 * (workspace smaller than sf_plan_workspace_bytes), SF_EHIP. */
int sf_frame_run(sf_plan plan, const uint8_t *L0, const uint8_t *R0, const uint8_t *L1,
                 const uint8_t *R1, int pitch, const float *flow, const sf_camera *cam,
                 float *disp0, uint8_t *valid0, float *disp1, uint8_t *valid1, float *sf4,
                 uint8_t *valid, float *xyz0, float *motion, void *workspace, size_t ws_bytes,
                 void *stream);

/* Frame autotuner: times whole frames (sf_frame_run, or sf_frame_run_learned
 * with zero network parameters) of a plan with the given size, penalties and
 * flags for every candidate aggregation tuning (chains per block x prefetch x
 * order x persistence x packed costs where D allows), on seeded synthetic
 * images, and returns the tuning with the fastest median frame and that time
 * in ms.  In a frame the aggregation
 * shares the memory system with the cost and WTA stages, so this choice can
 * differ from sf_agg_autotune's.  Allocates and frees its own buffers;
 * synchronises the stream.  Errors: those of sf_frame_plan_create, SF_EINVAL
 * (NULL best), SF_EHIP. */
int sf_frame_autotune(int H, int W, int D, int P1, int P2, int lr_tol, int flags, void *stream,
                      sf_agg_tuning *best, float *best_ms);

/* Learned frame (plan created with SF_FRAME_LEARNED): as sf_frame_run, except
 * that only the two left-base views are aggregated, WTA also writes the
 * network's features, and each map's validity is sf_lrnet_mask of
 * sf_lrnet_forward (lr_params: device FP32 parameters, see below) instead of
 * the left-right check. */
int sf_frame_run_learned(sf_plan plan, const uint8_t *L0, const uint8_t *R0, const uint8_t *L1,
                         const uint8_t *R1, int pitch, const float *flow, const sf_camera *cam,
                         const float *lr_params, float *disp0, uint8_t *valid0, float *disp1,
                         uint8_t *valid1, float *sf4, uint8_t *valid, float *xyz0, float *motion,
                         void *workspace, size_t ws_bytes, void *stream);

/* Judge of the learned stand-in against the left-right check it imitates
 * (Sec. 3.1): *count (device u32, output) = the number of i < n where a[i] and
 * b[i] (device uint8 masks, any alignment) are both zero or both nonzero.
 * One small launch on `stream`; the count is deterministic and needs no
 * clearing.  SF_EINVAL on a NULL pointer or n <= 0. */
int sf_mask_agreement(const uint8_t *a, const uint8_t *b, int n, uint32_t *count, void *stream);

/* ---------------------------------------------------------------------------
 * Batched plain SGM: many stereo pairs of uneven size and disparity range, each
 * processed exactly as a plain pair (census, both cost volumes, 8-path
 * aggregation of both views, WTA + sub-pixel + LR check; same results as
 * sf_census .. sf_wta_lr on that pair alone).  The plan groups pairs by size
 * class and packs them into waves whose workspace fits mem_budget bytes (0 =
 * one wave); each wave runs one aggregation launch per size class from a
 * device task table.  Device pointers in the pair descriptors are fixed at plan
 * creation and must stay valid while the plan is used.
 * Tuning of the aggregation per size class (sf_agg_tuning; classes numbered in
 * order of first appearance in `pairs`; NULL / missing = {16, 8, 0, 0, 0}).
 * Supported: D a multiple of 32 in [32, 256]; 62 + P2 <= 255; H * W * D < 2^31 per pair.
 * Errors: SF_EINVAL, SF_EUNSUPPORTED, SF_EHIP (table upload). */
typedef struct {
    int H, W, D, pitch;
    const uint8_t *left, *right; /* [H][pitch] */
    int16_t *wta;                /* [H][W] d*_L or NULL */
    float *disp;                 /* [H][W] d_sub or -1 */
    uint8_t *valid;              /* [H][W] LR-check mask */
} sf_pair;

int sf_batch_plan_create(const sf_pair *pairs /* host array */, int n, int P1, int P2, int lr_tol,
                         const sf_agg_tuning *tunings /* host, per class */, int ntunings,
                         size_t mem_budget, sf_plan *plan);
int sf_batch_plan_info(sf_plan plan, int *nwaves, int *nclasses);
/* Enqueue the whole batch on stream (eager). */
int sf_batch_run(sf_plan plan, void *workspace, size_t ws_bytes, void *stream);
/* Capture the whole batch on a non-default stream into a HIP graph owned by the
 * plan (the workspace address is baked in), then replay it with one call. */
int sf_batch_capture(sf_plan plan, void *workspace, size_t ws_bytes, void *stream);
int sf_batch_launch(sf_plan plan, void *stream);
/* Autotuner: times every candidate tuning (chains per block x prefetch x order x
 * persistence x packed costs where D allows) of one aggregation launch over
 * nviews views of H x W x D (synthetic costs; 2 = a stereo pair, 4 = a
 * scene-flow frame) on `stream`, and returns the fastest and its median time over five runs, each started right
 * after the cost volumes were rewritten (as in a frame, where the cost stage
 * precedes the aggregation).  Allocates and frees its own scratch;
 * synchronises the stream. */
int sf_agg_autotune(int H, int W, int D, int P1, int P2, int nviews, void *stream,
                    sf_agg_tuning *best, float *best_ms);

/* ---------------------------------------------------------------------------
 * Learned stand-in for the left-right check (the check is the paper's, Sec.
 * 3.1; the network is not: it predicts from the left view alone which pixels
 * the check would keep, so the right-view aggregation can be skipped).
 * Network: 3x3 cross-correlations with zero padding, channels 4 -> 16 -> 16 ->
 * 16 -> 1, ReLU after the first three; layer inputs and weights rounded to
 * BF16 (nearest even), biases FP32, FP32 sums; logit output.
 * Parameters: flat FP32 vector of sf_lrnet_nparams() = 5377 values, W1[16][4][3][3]
 * b1[16] W2[16][16][3][3] b2[16] W3[16][16][3][3] b3[16] W4[1][16][3][3] b4[1].
 * Features: feat [B][H][W][4] FP32 as written by sf_wta_lr.
 * workspace: sf_lrnet_workspace_bytes(B, H, W, train) bytes of device memory.
 * Errors: SF_EINVAL (NULL, sizes), SF_ENOMEM (workspace). */
int sf_lrnet_nparams(void);
size_t sf_lrnet_workspace_bytes(int B, int H, int W, int train);
/* logits [B][H][W] FP32 (output). */
int sf_lrnet_forward(const float *params, const float *feat, int B, int H, int W, float *logits,
                     void *workspace, size_t ws_bytes, void *stream);
/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): sf_lrnet_forward without a
 * workspace argument.  Its only scratch (the packed weight fragments, 13,568
 * bytes for any B, H, W) lives in a 16 KiB array of the library in each GPU's
 * memory, held until the process ends; the call allocates nothing.  Every
 * call on one GPU shares that array and overwrites it completely before
 * reading it, so calls that overlap on one GPU (different streams, or
 * different threads) race and must be ordered by the caller.  Same results
 * and limits as sf_lrnet_forward (SF_EINVAL on NULL pointers or sizes beyond
 * B <= 65535, B*H*W <= 2^30); SF_EHIP if the array's device address cannot
 * be looked up. */
int sf_lrnet_forward_noalloc(const float *params, const float *feat, int B, int H, int W,
                             float *logits, void *stream);
/* Learned mask of one map: valid = logit > 0 and x - d* >= 0 (a match pixel
 * outside the image can never pass the check); disp = d_sub where valid, else
 * -1.0f.  wta [H][W] int16 d*, dsub [H][W] FP32. */
int sf_lrnet_mask(const float *logits, const int16_t *wta, const float *dsub, int H, int W,
                  uint8_t *valid, float *disp, void *stream);
/* Mean binary cross-entropy of sigmoid(logit) against label [B][H][W] in {0,1}
 * and its gradient: grad [5377] FP32 (output), loss [1] FP32 (output, device).
 * Backward: dL/dz4 = (sigmoid(z4) - y)/N in FP32; BF16 rounding passed straight
 * through; the gradients w.r.t. the pre-activations of layers 3..1 are rounded
 * to BF16; weight and bias gradients are FP32 sums reduced in a fixed order
 * (bit-reproducible run to run). */
int sf_lrnet_grad(const float *params, const float *feat, const uint8_t *label, int B, int H, int W,
                  float *grad, float *loss, void *workspace, size_t ws_bytes, void *stream);
/* The same backward from a given dL/dz4 [B][H][W] FP32 (device, caller-owned)
 * instead of the loss: the forward recomputes the activations, then the four
 * layers' gradients follow exactly as in sf_lrnet_grad.  grad [5377] FP32
 * (output).  Workspace: sf_lrnet_workspace_bytes(B, H, W, 1).  SF_EINVAL on a
 * NULL pointer or a bad size, SF_ENOMEM on a short workspace. */
int sf_lrnet_backward(const float *params, const float *feat, const float *dz4, int B, int H, int W,
                      float *grad, void *workspace, size_t ws_bytes, void *stream);
/* Adam in FP32, in place, in this order: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g g;
 * w -= (lr m/(1-b1t)) / (sqrt(v/(1-b2t)) + eps); b1t, b2t = b1, b2 to the step count. */
int sf_lrnet_adam(float *params, float *m, float *v, const float *grad, int n, float lr, float b1,
                  float b2, float eps, float b1t, float b2t, void *stream);

/* ---------------------------------------------------------------------------
 * Kernel timer for benchmarking.  While enabled, each timed launch (census,
 * cost, sgm_paths, slab_sum, wta_right, wta_left, combine, ...) records a pair
 * of HIP events on its own stream; sf_prof_query waits for and sums those of one
 * kernel name.  At most max_launches launches are recorded per enable.  The
 * events are created by sf_prof_enable (call it outside any timed region).
 * sf_prof_only(name) restricts the recording to launches of that name (NULL:
 * all), so that a timed region carries the events of one kernel only.
 * Process-wide, single-threaded use.  Errors: SF_EINVAL, SF_EHIP. */
int sf_prof_enable(int max_launches);
int sf_prof_only(const char *kernel);
int sf_prof_disable(void);
int sf_prof_query(const char *kernel, double *total_ms, int *launches);

/* ---------------------------------------------------------------------------
 * Checked builds (libsf_checked.so: the same library built with index checks).
 * At the accesses whose indices come from data (bilinear taps at x + F(x), the
 * LR check's d*_R(x - d*), flow candidates, densification sources, the
 * temporal check's chained pixel, each chain step's cost and slab bytes) a
 * failed check sets one bit per site in device memory; the access proceeds as
 * in the normal build and nothing traps.
 *   sf_debug_checked: 1 for a checked build, 0 otherwise.
 *   sf_debug_check: waits for the device, then *bits = the sites whose checks
 *     failed since the last clear on the current device (bit 0 taps, 1
 *     temporal, 2 LR check, 3 flow samples, 4 densification, 5 chain costs,
 *     6 chain slabs, 31 self-test); clear != 0 resets them.  0 in a normal
 *     build.  Errors: SF_EINVAL (NULL), SF_EHIP.
 *   sf_debug_selftest: enqueues a kernel that checks i < n for i = 0 .. n and
 *     reads no memory, so a checked build records bit 31.  Errors: SF_EINVAL
 *     (n outside [0, 2^24)), SF_EHIP. */
int sf_debug_checked(void);
int sf_debug_check(uint32_t *bits, int clear);
int sf_debug_selftest(int n, void *stream);

/* ---------------------------------------------------------------------------
 * Densification of the sparse scene-flow map (the paper reports a dense
 * version interpolated by the benchmark and names a better interpolation as
 * future work, Sec. 4; the fill rule is this library's own):
 *   - an undefined pixel takes all four values (u, v, d0, d1) of the nearest
 *     defined pixel to its left or right in the same row; when both exist, the
 *     one with the smaller d0 (the farther surface), ties to the left;
 *   - a row with no defined pixel copies the nearest row that has one, pixel by
 *     pixel (ties to the row above).
 *   sf4 [H][W][4] float, valid [H][W] uint8 (bit 0 = defined), as sf_combine
 *   writes them; out [H][W][4] float (output, distinct from sf4; both 16-byte
 *   aligned); fill [H][W] uint8 (output): 1 defined, 2 filled from the row,
 *   3 copied from another row, 0 (with NaNs) only when nothing is defined.
 *   workspace: at least sf_densify_workspace_bytes(H) bytes of device scratch.
 * Supported: W <= 8192.  Errors: SF_EINVAL, SF_EUNSUPPORTED, SF_ENOMEM. */
size_t sf_densify_workspace_bytes(int H);
int sf_densify(const float *sf4, const uint8_t *valid, int H, int W, float *out, uint8_t *fill,
               void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Temporal validation over more than two frame pairs (the paper's future work:
 * more frame pairs with an intermediate validation of the correspondences; the
 * rule is this library's).  sf4_a / valid_a is the scene flow between t_k and
 * t_k+1 (as sf_combine writes it), sf4_b / valid_b the one between t_k+1 and
 * t_k+2.  out(x) = 1 iff S_a(x) = (u, v, d0, d1) is defined, the chained pixel
 * q = (floor(x + u + 0.5), floor(y + v + 0.5)) lies in the image, S_b(q) =
 * (u', v', d0', d1') is defined, |u - u'| <= tau_f, |v - v'| <= tau_f and
 * |(d1 - d0) - (d1' - d0')| <= tau_d (FP32, in this order); else 0.
 *   sf4_a, sf4_b [H][W][4] float (16-byte aligned); valid_a, valid_b, out
 *   [H][W] uint8.  Errors: SF_EINVAL. */
int sf_temporal_check(const float *sf4_a, const uint8_t *valid_a, const float *sf4_b,
                      const uint8_t *valid_b, int H, int W, float tau_f, float tau_d, uint8_t *out,
                      void *stream);

/* ---------------------------------------------------------------------------
 * Optical-flow stand-in for the flow input of the combination.  The paper
 * takes its flow from Flow Fields+ (Sec. 3.2: coarse-level matches propagated
 * to neighbours and refined by random search under a patch data term, lifted
 * level by level, filtered by consistency with the inverse flow); this is a
 * method of the same outline with choices of its own, all integer:
 *   - pyramid of `levels` levels, each the 2x2 box mean (a+b+c+d+2)/4 of the
 *     finer one (odd borders clamped);
 *   - data term at each level: the 9x7 census of sf_census; the cost of
 *     integer flow f at x is sum over o in {-2,0,2}^2 of the Hamming distance
 *     of census0(x + o) and census1(x + f + o), coordinates clamped; targets
 *     outside the image are no candidates;
 *   - `iters` iterations per level, each updating all pixels from the previous
 *     field: own f, the f of the neighbours at distance 1 then 4 (left, right,
 *     up, down), then random search around the best so far with radii
 *     R_l >> k (R_l = max(1, R >> l), capped at fine_radius on every level
 *     but the coarsest when fine_radius > 0), offsets from SplitMix64 output
 *     (seed, counter (((l*64 + iter)*64 + k)*65536 + y/8)*65536 + x/8, one
 *     offset per 8x8 tile) as
 *     ((h & 0xFFFF) mod (2r+1)) - r and (((h >> 16) & 0xFFFF) mod (2r+1)) - r;
 *     the first candidate with the lowest cost wins;
 *   - f = 0 on the coarsest level; f(x, y) = 2 f_coarser(x/2, y/2), target
 *     clamped into the image, when moving one level finer;
 *   - forward flow F (L0 -> L1, seed) and backward flow B (L1 -> L0, seed ^
 *     0x5bd1e995); flow(x) = F(x) if |F(x) + B(x + F(x))| <= tol in both
 *     components, else NaN (the combination then leaves S undefined there).
 *   L0, L1 [H][pitch] uint8; F, B [H][W][2] int16 (outputs, 4-byte aligned);
 *   flow [H][W][2] float (output, 8-byte aligned); workspace of at least
 *   sf_flow_workspace_bytes(H, W, levels) bytes.
 * Supported: H, W <= 16383; levels in [1, 16]; iters in [1, 63]; R in
 * [1, 16383]; fine_radius >= 0.  Errors: SF_EINVAL, SF_ENOMEM, SF_EHIP. */
size_t sf_flow_workspace_bytes(int H, int W, int levels);
int sf_flow(const uint8_t *L0, const uint8_t *L1, int pitch, int H, int W, int levels, int iters,
            int R, int fine_radius, uint64_t seed, int tol, int16_t *F, int16_t *B, float *flow,
            void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Machine-balance probes (not part of the method): the measured ceilings the
 * kernels' roofline fractions are also quoted against.
 *
 * sf_probe_stream: mode 0 copies `bytes` from src to dst, mode 1 only reads
 * src, mode 2 only writes dst (16-byte non-temporal accesses).  bytes a
 * multiple of 16, pointers 16-byte aligned device memory (dst unused in mode 1,
 * src unused in mode 2).  Errors: SF_EINVAL, SF_EHIP.
 *
 * sf_probe_pk_u16: `blocks` blocks of 256 threads; each thread runs `iters`
 * iterations of 8 packed 16-bit adds and 8 packed 16-bit mins (the
 * instruction mix of the path-cost recurrence), i.e. blocks*256*iters*32
 * 16-bit element operations, and writes a checksum to out[blocks*256]
 * (uint32, device).  Errors: SF_EINVAL, SF_EHIP. */
int sf_probe_stream(const void *src, void *dst, size_t bytes, int mode, void *stream);
int sf_probe_pk_u16(uint32_t *out, int blocks, int iters, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SF_H */
