/*
 * bm.h -- C ABI of the MI355X block-matching library (libbm.so).
 *
 * Block matching (BM), Sec. III-A Eq. (equ:bm): for every reference patch X_i of an image,
 * return the K candidate patches X_j of its search window with the smallest squared
 * Euclidean distance ||X_j - X_i||_F^2.  The library evaluates each distance through
 * Lemma 2 (Sec. III-B): d = ||X_j||^2 + ||X_i||^2 - 2 <X_i, X_j>, where the squared patch
 * norms come from a box filter (the entries of h_X (.) h_X) and the inner products are the
 * window-restricted Self-Convolution cross term C_i of Eq. (eq:selfConv), footnote to
 * Eq. (eq:unifySelfConv).  Selection is Theorem 1 with the Euclidean H: the support of the
 * K largest b_i = vec(C_i) - h_X(.)h_X / 2, i.e. the K smallest distances.
 *
 * Conventions shared by every call
 * --------------------------------
 * Image       planar C x H x W float32 (channel-major, then rows, then columns), device
 *             memory, owned by the caller.  Multi-channel patches are joint P x P x C
 *             blocks and distances sum over channels (Sec. IV, channel sum S(.)).
 * References  top-left corners on the grid {0, s, 2s, ...} in each axis; n_ref =
 *             (floor((H-P)/s)+1) * (floor((W-P)/s)+1), numbered row-major.
 * Candidates  every valid patch position (stride 1) whose offset from the reference lies in
 *             [-a, b]^2 with a = floor(window/2), b = window - 1 - a (odd windows: [-r, r],
 *             r = (window-1)/2; even windows one more offset before the reference than
 *             after), intersected with the image (never shifted).
 *             The reference is its own candidate (distance 0).
 * Output      idx[i*K + k] = qy*W + qx (int32) and dist[i*K + k] (float32, clamped at 0),
 *             sorted ascending by the key (dist, idx); rows with fewer than K candidates
 *             are padded with idx = -1, dist = +inf.  Device memory, owned by the caller.
 * Streams     `stream` is a hipStream_t passed as void* (NULL = the null stream).  Device
 *             calls are asynchronous on that stream, like kernel launches.
 * Errors      every call returns bm_status; BM_OK is 0.  Argument checks happen on the host
 *             before anything is enqueued.  bm_last_error() returns a thread-local message
 *             for the last failing call on the calling thread.
 */
#ifndef BM_H_
#define BM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bm_status;
#define BM_OK 0
#define BM_EINVAL (-1)      /* invalid argument (the message names it)               */
#define BM_ENOMEM (-2)      /* device or host allocation failed                       */
#define BM_EDEVICE (-3)     /* HIP runtime error (launch, copy, no device)            */
#define BM_EAGAIN (-4)      /* bm_poll: result not ready yet                          */
#define BM_EBUSY (-5)       /* bm_submit: admission refused (budget or slots)         */
#define BM_ENOTFOUND (-6)   /* unknown ticket                                          */
#define BM_ECANCELED (-7)   /* ticket was cancelled                                    */
#define BM_ENOTSUP (-8)     /* valid request outside what the library supports         */

/* Arithmetic of the cross term <X_i, X_j>.  Norms and the distance assembly are float32
 * in every form.  The split forms write x = hi + lo (hi = round(x), lo = round(x - hi)) and
 * accumulate the products of the parts in float32 on the matrix cores. */
#define BM_PREC_FP32 0      /* float32 products, float32 accumulation                 */
#define BM_PREC_BF16X4 1    /* bfloat16 hi/lo split, all four products hi*hi + hi*lo +
                               lo*hi + lo*lo, i.e. the exact cross term of the image
                               rounded to hi + lo (16 significant bits); the norm map of
                               such a plan (bm_norms) holds the norms of the same rounded
                               values, so Lemma 2's cancellation is exact for the rounded
                               patches and the result differs from the float32 one only
                               by the distance between rounded and original patches     */
#define BM_PREC_FP16X3 2    /* float16 hi/lo split after a power-of-two pre-scale,
                               chosen per 4 x 4 block of references from the largest
                               |x| around it (a property of the image, not of the call);
                               three products hi*hi + hi*lo + lo*hi (22 significant bits) */

/* bm_desc.flags */
#define BM_FLAG_CENTER 1u   /* subtract a per-channel mean before the cross term (the
                               distance is translation invariant; reduces cancellation) */
#define BM_FLAG_NCC 2u      /* rank by normalized cross-correlation (Sec. III-A,
                               Eq. (equ:cor); Lemma 1, Theorem 1 item 3): keep the K
                               candidates with the largest <X_i, X_j> / (||X_i|| ||X_j||);
                               dist reports 2 - 2 NCC in [0, 4] (the squared distance of the
                               unit-normalised patches), ascending; NCC is 0 when either
                               patch has zero norm.  Needs the specialised kernel (C <= 4,
                               patch 3..8, K <= 32, 17 <= 3*stride + window <= 48; BM_ENOTSUP
                               otherwise); not combinable with BM_FLAG_CENTER (BM_EINVAL). */

/* One BM problem, following the paper's statement of BM: image, patch size sqrt(n),
 * stride, search window, K (Sec. III-A; Sec. V-A fixes 6x6 patches, stride 1, 30x30).
 *
 * 3D search (Sec. IV, 3D Self-Convolution; the multi-channel setups of Sec. V-A): with
 * window_depth = c >= 1 the image is a volume of q = channels planes (frames, modalities),
 * a patch is a d x P x P block of d = patch_depth consecutive planes, and the search window
 * is Wn x Wn x c.  References: every depth z = 0..q-d times the 2D reference grid, numbered
 * z * (2D reference count) + grid index (n_ref = (q-d+1) * 2D count).  Candidates of depth
 * z: depths z - (c-1)/2 .. z - (c-1)/2 + c - 1 (integer division; c = 9: z-4..z+4, c = 2:
 * z..z+1) intersected with 0..q-d, never shifted, times the clipped 2D window.  Returned
 * indices are volume positions (z' * H + y) * W + x; order and padding as in 2D.  Needs the
 * specialised kernel's envelope for a d-channel image (d <= 4, patch 3..8 (5..8 split),
 * K <= 32, 17 <= 3*stride + window <= 48), no flags (BM_ENOTSUP otherwise); q * H * W < 2^31.
 * Both fields 0: the plain 2D problem. */
typedef struct {
  int32_t height, width, channels; /* image H, W, C; 1 <= C <= 8 (3D: q <= 65536)       */
  int32_t patch;                   /* patch side P, 1 <= P <= 16, P <= min(H, W)        */
  int32_t stride;                  /* reference-grid stride s >= 1                      */
  int32_t window;                  /* window side Wn >= 1: candidate offsets -floor(Wn/2)
                                      .. Wn - 1 - floor(Wn/2) per axis (odd Wn: -r..r;
                                      even Wn, e.g. the paper's 30: -Wn/2 .. Wn/2 - 1)   */
  int32_t k;                       /* neighbours kept, 1 <= K <= 64                     */
  int32_t precision;               /* BM_PREC_*                                         */
  uint32_t flags;                  /* BM_FLAG_*                                         */
  int32_t patch_depth;             /* 3D: planes per patch d, 1 <= d <= min(4, q); 2D: 0 */
  int32_t window_depth;            /* 3D: depth window c >= 1; 2D: 0                    */
} bm_desc;

typedef struct bm_plan_s* bm_plan_t;

/* Validate `desc`, pick the kernel configuration for its shape (the autotuner's choice
 * when a tuned entry exists, else the built-in rule), and allocate the plan-owned
 * workspace on the current device.  Errors: BM_EINVAL (bad field), BM_ENOTSUP,
 * BM_ENOMEM, BM_EDEVICE.  The plan is immutable afterwards. */
bm_status bm_plan(const bm_desc* desc, bm_plan_t* out);

/* Number of references, and the workspace bytes a caller must pass to bm_match to avoid
 * the plan-owned one.  Either output pointer may be NULL. */
bm_status bm_plan_info(bm_plan_t plan, int64_t* n_ref, int64_t* workspace_bytes);

/* Run BM on one image: patch norms (box filter), then the fused cross-term / distance /
 * top-K kernel.  d_img: C*H*W floats (3D: the q*H*W volume); d_idx, d_dist: n_ref*K each.  d_workspace: NULL to
 * use the plan's own (then calls on one plan must not overlap in time), or
 * workspace_bytes of device memory owned by the caller.  Asynchronous on `stream`. */
bm_status bm_match(bm_plan_t plan, const float* d_img, int32_t* d_idx, float* d_dist,
                   void* d_workspace, void* stream);

/* bm_match for callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same kernels and results as
 * bm_match, with the workspace in a fixed device array of BM_NOALLOC_MAX_WORKSPACE bytes
 * that the library holds on each device it runs on until the process ends.  The call
 * allocates nothing (no hipMalloc, no host allocation on the call path after the first
 * call on a device, which looks up the array's address).  The plan must have been made on
 * the current device.  BM_EINVAL if the plan's workspace_bytes exceed the maximum (the
 * message names both sizes) or on NULL pointers.  Every call on a device shares that
 * device's array, so calls that overlap in time on one device (other streams, other
 * threads) race; the caller serialises them.  Asynchronous on `stream`. */
#define BM_NOALLOC_MAX_WORKSPACE (32ll << 20)
bm_status bm_match_noalloc(bm_plan_t plan, const float* d_img, int32_t* d_idx, float* d_dist,
                           void* stream);

/* Patch-norm map alone (the box filter, h_X (.) h_X of Sec. III-B): d_norm receives
 * (H-P+1)*(W-P+1) floats, row-major (3D plans: one such map per slab z = 0..q-d, stacked by
 * z, each the norms of the d-plane blocks at that depth).  BM_PREC_BF16X4 plans: the norms
 * of the image rounded to the bfloat16 hi + lo split (each value x becomes hi + lo).  It
 * also writes the plan's own workspace (centring
 * constants, and the per-tile maxima of |x| that BM_PREC_FP16X3 reads), which the next
 * bm_cross_topk on the same plan consumes: such pairs on one plan must not overlap in
 * time.  Asynchronous on `stream`. */
bm_status bm_norms(bm_plan_t plan, const float* d_img, float* d_norm, void* stream);

/* Second step of bm_match on its own: the fused cross-term / distance / top-K kernel,
 * given the norm map that bm_norms wrote for the same image (d_norm, (H-P+1)*(W-P+1)
 * floats).  Together the two calls compute exactly what bm_match computes.
 * Asynchronous on `stream`. */
bm_status bm_cross_topk(bm_plan_t plan, const float* d_img, const float* d_norm,
                        int32_t* d_idx, float* d_dist, void* stream);

/* Many images of uneven shapes: one norm launch over all images, then one persistent
 * launch per kernel tier present (a device counter hands out 4 x 4 reference blocks,
 * costliest images first).  Tiers group block shapes that share registers and workgroup
 * size: float32 images with 1..3 channels form one tier, 4 channels another; the split
 * forms put 1 channel in one tier and 2..4 channels in another.  Images whose shape only
 * the generic float32 kernel covers get a launch of their own.  Every image's results are
 * bitwise those of bm_match with the same plan.  Entry b uses plans[b], d_imgs[b],
 * d_idx[b], d_dist[b] (plans may repeat).  d_workspace must hold bm_batch_workspace()
 * bytes or be NULL (then the library allocates and frees it inside the call, which
 * synchronises `stream`); a workspace must not be reused before the call's work has
 * finished on `stream`.  n = 0 is a no-op.  Errors: BM_EINVAL (NULL plan or pointer, plan
 * from another device), BM_ENOTSUP, BM_ENOMEM, BM_EDEVICE. */
/* 3D plans: BM_ENOTSUP. */
bm_status bm_match_batch(int32_t n, const bm_plan_t* plans, const float* const* d_imgs,
                         int32_t* const* d_idx, float* const* d_dist, void* d_workspace,
                         void* stream);
bm_status bm_batch_workspace(int32_t n, const bm_plan_t* plans, int64_t* bytes);

bm_status bm_plan_destroy(bm_plan_t plan);

/* ---- patch groups -------------------------------------------------------------------- */
/* Group gather (Sec. IV: Y_i = [X_{S_i(1)}, ..., X_{S_i(K)}]): for every reference i and
 * k < K, d_groups[((i*K + k)*C + c)*P*P + l*P + m] = X_c[qy + l][qx + m] where
 * d_idx[i*K + k] = qy*W + qx (the output layout of bm_match).  An index of -1, or one that
 * names no valid patch position, gives a zero patch.  d_idx: n_ref*K int32; d_groups:
 * n_ref*K*C*P*P floats.  Asynchronous on `stream`. */
/* 3D plans: BM_ENOTSUP. */
bm_status bm_gather(bm_plan_t plan, const float* d_img, const int32_t* d_idx, float* d_groups,
                    void* stream);

/* Aggregation (Sec. IV, image reconstruction): deposit every group patch d_groups[i][k]
 * (layout as bm_gather) at the location d_idx[i*K + k] (skipped when it names no valid
 * position), summing overlaps, and divide each pixel by the number of deposited patches
 * covering it; pixels no patch covers are 0.  d_out: C*H*W floats.  Sums are formed in
 * 64-bit fixed point with an exponent taken from the largest |value| (exact to one rounding
 * per deposit, independent of ordering: bitwise deterministic); values must be finite.
 * d_workspace: bm_aggregate_workspace bytes, or NULL (the library allocates and frees it,
 * which synchronises `stream`).  Asynchronous on `stream`. */
/* 3D plans: BM_ENOTSUP. */
bm_status bm_aggregate_workspace(bm_plan_t plan, int64_t* bytes);
bm_status bm_aggregate(bm_plan_t plan, const float* d_groups, const int32_t* d_idx, float* d_out,
                       void* d_workspace, void* stream);

/* ---- non-local means ---------------------------------------------------------------- */
/* Non-local means over each reference's search window (Sec. III-A, Eq. (equ:nlm);
 * Prop. 1): w_ij = exp(-||X_j - X_i||^2 / b^2) for every in-window candidate X_j, Theta_i =
 * sum_j w_ij, and the recovered patch Y_i = sum_j w_ij X_j / Theta_i.  The distances come
 * from Lemma 2 as in bm_match; the weighted sum is a second matrix-core contraction.
 * d_patch receives n_ref * C * P * P floats (reference-major in grid order, then channel,
 * row, column); d_theta (may be NULL) n_ref floats.  The plan must be float32 without
 * flags and inside the specialised kernel's envelope (C <= 4, patch 3..8,
 * 3*stride + window in 17..48; BM_ENOTSUP otherwise); its K is not used.  b: finite,
 * > 0 (BM_EINVAL otherwise).  d_workspace as in bm_match.  3D plans: BM_ENOTSUP.
 * Asynchronous on `stream`. */
bm_status bm_nlm(bm_plan_t plan, const float* d_img, float b, float* d_patch, float* d_theta,
                 void* d_workspace, void* stream);

/* ---- autotuning ------------------------------------------------------------------- */
/* Time every kernel configuration that can run desc's shape class (waves per reference
 * block or wave grid, bounding-sweep row step, candidate-buffer capacity) on the current
 * device, `reps` launches each, on d_img (C*H*W device floats) or, if d_img is NULL, on a
 * built-in structured test image.  The fastest is remembered for the shape class (channels,
 * patch, stride, window, K/16, precision, coarse grid size) and used by later bm_plan calls
 * in this process; with the environment variable BM_TUNE_CACHE naming a file it is also
 * appended there and read back by later processes.  out_cfg (may be NULL) receives the
 * configuration string.  A 3D descriptor is tuned as the 2D problem of one d-plane slab
 * (the first d planes of d_img), which is the configuration 3D plans look up.
 * Synchronous.  Errors: BM_EINVAL, BM_ENOMEM, BM_EDEVICE. */
bm_status bm_autotune(const bm_desc* desc, const float* d_img, int32_t reps, char* out_cfg,
                      int32_t out_len);

/* Configuration string of a plan and where it came from (0 built-in rule, 1 autotuner
 * table, 2 the BM_CFG environment override used for tuning experiments). */
bm_status bm_plan_config(bm_plan_t plan, char* out_cfg, int32_t out_len, int32_t* source);

/* ---- serving ---------------------------------------------------------------------- */
typedef struct bm_server_s* bm_server_t;

typedef struct {
  int64_t hbm_budget_bytes;  /* device bytes the server may hold for admitted requests */
  int32_t max_inflight;      /* admitted (device-resident) requests at most            */
  int32_t max_queue;         /* queued, not yet admitted requests at most               */
  int32_t max_step;          /* requests launched together as one step at most (the
                                work of one batch launch); 0 = 8.  A step also takes at
                                most half of max_inflight (at least 1), so that a next step
                                can be admitted while one runs                             */
} bm_server_cfg;

typedef struct {
  double queue_s;   /* submit -> admitted                                             */
  double device_s;  /* admitted -> result on the host                                  */
  double total_s;   /* submit -> result ready                                          */
  int64_t n_ref;
} bm_request_stats;

/* Start a server on the current device: one device arena of hbm_budget_bytes (>= 1 MiB)
 * sub-allocated per request (image, norm map, outputs) so that admission never calls the
 * device allocator, a pinned host arena for queued images and returned results (the
 * budget, clamped to [256 MiB, 8 GiB]), and a scheduler thread.  The scheduler admits
 * queued requests in arrival order while their footprint fits the arena and fewer than
 * max_inflight are admitted, launches newly admitted requests together as one step (at
 * most 8, and at most max_inflight / 2), copies in on an input stream, runs the
 * uneven-batch launch on one of two compute streams and copies results out on an output
 * stream; steps overlap.  Requests are computed exactly as bm_match computes them.
 * Errors: BM_EINVAL (cfg out of range), BM_ENOMEM, BM_EDEVICE. */
bm_status bm_server_create(const bm_server_cfg* cfg, bm_server_t* out);

/* Queue one request; the host image (C*H*W floats) is copied before the call returns.
 * Thread-safe.  BM_EBUSY when max_queue requests wait, the host arena is full, or the
 * request alone exceeds the device budget; BM_EINVAL / BM_ENOTSUP as bm_plan (3D
 * descriptors: BM_ENOTSUP). */
bm_status bm_submit(bm_server_t srv, const bm_desc* desc, const float* host_img,
                    uint64_t* ticket);

/* Non-blocking, thread-safe.  BM_EAGAIN while pending; BM_OK once done: copies n_ref*K
 * results into the caller's host buffers (either may be NULL), fills stats (may be NULL)
 * and retires the ticket.  BM_ENOTFOUND for unknown or retired tickets, BM_ECANCELED if
 * cancelled; a request that failed returns its error (e.g. BM_ENOTSUP, BM_EDEVICE) and is
 * retired. */
bm_status bm_poll(bm_server_t srv, uint64_t ticket, int32_t* host_idx, float* host_dist,
                  bm_request_stats* stats);

/* Cancel a ticket: a queued request is dropped at once; an admitted one finishes on the
 * device and its results are discarded.  Either way bm_poll then returns BM_ECANCELED. */
bm_status bm_cancel(bm_server_t srv, uint64_t ticket);

/* Stop accepting, wait for admitted work to finish, drop queued requests, stop the
 * scheduler and free both arenas; every ticket of the server becomes invalid. */
bm_status bm_server_destroy(bm_server_t srv);

const char* bm_status_str(bm_status s);
const char* bm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BM_H_ */
