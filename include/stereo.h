/*
 * stereo.h - C interface of the MI355X stereo-matching library.
 *
 * The library computes the disparity map of a rectified stereo pair by the
 * method of Chang & Maruyama, "Real-Time High-Quality Stereo Matching System
 * on a GPU" (arXiv 2212.00488): gray-scale and 2x mean-pool downscale
 * (Sec. III-A, Eq. 2), absolute-difference plus mini-census matching cost
 * (Sec. III-B, Eq. 3-6), cross-based aggregation along x then y (Sec. III-C,
 * Eq. 7-8), winner-take-all for the left- and right-based maps (Eq. 9),
 * left/right cross-check into ground control points (Sec. III-D, Eq. 10),
 * median filter and bilateral filling of the other pixels (Sec. III-E,
 * Eq. 11) and bilateral upscale back to full resolution (Sec. IV, Step8).
 *
 * Conventions shared by every entry point
 *   - All image and map pointers are DEVICE pointers (HIP global memory) on
 *     the context's device, row-major, tightly packed (pitch = width).
 *   - Input images are uint8 RGB, interleaved, [H][W][3].  The output is an
 *     int16 full-resolution disparity map [H][W] for the left image, values
 *     in [0, Dmax-1] (even numbers and midpoints of the half-res map).
 *   - Dmax is the full-resolution disparity range: d in [0, Dmax-1] (Sec. II).
 *     The half-resolution search range is D = ceil(Dmax / 2).
 *   - Work is enqueued asynchronously on `stream` (0 = the null stream).  The
 *     caller keeps inputs and outputs alive and unmodified until the stream
 *     has passed the work.  Results are bit-exact and deterministic.
 *   - Every function returns 0 on success or a negative STEREO_E* code.  On
 *     error nothing is enqueued, the context stays usable and
 *     stereo_last_error() describes the failure.
 *   - A context may be used by one host thread at a time.
 */
#ifndef STEREO_H
#define STEREO_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STEREO_OK 0
#define STEREO_EINVAL (-1)  /* bad pointer, size, range or params              */
#define STEREO_ENOMEM (-2)  /* device allocation failed or mem_cap exceeded     */
#define STEREO_EHIP (-3)    /* a HIP runtime call failed                        */
#define STEREO_EUNIMPL (-4) /* not implemented                                  */

/* Largest supported full-resolution image side and disparity range. */
#define STEREO_MAX_SIDE 8192
#define STEREO_MAX_DMAX 512

/* params.flags */
#define STEREO_F_KEEP_INTERMEDIATES 1u /* keep per-call planes for stereo_get_intermediate */
#define STEREO_F_STAGE_TIMING 2u       /* time each stage with HIP events on the stream     */
#define STEREO_F_FULL_RES 4u           /* no 2x downscale / upscale: the method on the
                                          original images over d in [0, Dmax-1] (Sec. V);
                                          W <= STEREO_MAX_SIDE / 2                            */

/* Parameters of the method.  Defaults (stereo_default_params) are the paper's:
 * lambda_AD = 0.3, lambda_MC = 2.3 and T = 3 (Sec. V); arm caps 21 (x) and
 * 31 (y) and colour threshold 13 (Table II footnote, Sec. V); the bilateral
 * fill; one horizontal cap for both images.  The paper's variants: a
 * separate horizontal cap for the right image (arm_x_r, Sec. V), the two
 * simpler non-GCP fills (fill_mode, Sec. III-E) and the full-resolution
 * mode with caps 41 and 61 (STEREO_F_FULL_RES, Sec. V; it needs a smaller
 * cost_scale, e.g. 512, to meet the aggregate bound below). */
typedef struct stereo_params {
  uint32_t size;       /* must equal sizeof(stereo_params)                          */
  float lambda_ad;     /* Eq. 4, on brightness normalised to [0,1]; > 0              */
  float lambda_mc;     /* Eq. 5, on census Hamming distance; > 0                     */
  int32_t cost_scale;  /* fixed-point scale S of the cost tables, 1..1024            */
  int32_t color_delta; /* delta of Sec. III-C: arms take |I(t) - I(centre)| < delta  */
  int32_t arm_x;       /* per-side cap of the horizontal arms m, n; 0..127           */
  int32_t arm_y;       /* per-side cap of the vertical arms M, N; 0..127             */
  int32_t fill_T;      /* T of Sec. III-E (bilateral filling and upscale); >= 0      */
  uint32_t flags;      /* STEREO_F_*                                                 */
  int32_t arm_x_r;     /* horizontal cap of the right image; -1 = arm_x; 0..127      */
  int32_t fill_mode;   /* non-GCPs: 0 bilateral (Eq. 11), 1 the GCP closer in
                          distance (right on equal distance), 2 the smaller disparity */
} stereo_params;

typedef struct stereo_ctx stereo_ctx; /* opaque, owned by the library */

/* Fills *p with the paper's parameters. */
void stereo_default_params(stereo_params* p);

/* Creates a context on HIP device `device`.  mem_cap bounds the library's
 * device scratch in bytes (0 = no bound).  *out receives the context. */
int stereo_create(stereo_ctx** out, int device, size_t mem_cap);

/* Frees the context and everything it allocated.  NULL is a no-op.  The
 * caller must have synchronised every stream it used with the context. */
void stereo_destroy(stereo_ctx* ctx);

/* Text of the last error on this context ("" if none).  Valid until the next
 * call on the context. */
const char* stereo_last_error(const stereo_ctx* ctx);

/* Disparity map of one pair (the whole path of Sec. III / Sec. IV Step1-8).
 *   left, right : device, uint8 [H][W][3] RGB, rectified so that a left pixel
 *                 (x,y) matches right pixel (x-d, y) (Sec. II).
 *   W, H        : 2..STEREO_MAX_SIDE.
 *   Dmax        : 1..min(W, STEREO_MAX_DMAX).
 *   params      : NULL for the defaults; else size must match and values be
 *                 in range, including (2 max(arm_x, arm_x_r) + 1)(2 arm_y + 1)
 *                 * C_max < 2^(32 - b), where C_max is the largest table cost
 *                 and b the bits of D - 1 (D the searched range, at least 1
 *                 bit): the winner-take-all keys pack the aggregate and d.
 *   out_disp    : device, int16 [H][W].
 * Scratch for each (W, H, Dmax, params) is allocated on first use and cached. */
int stereo_disparity(stereo_ctx* ctx, const uint8_t* left, const uint8_t* right, int W, int H,
                     int Dmax, const stereo_params* params, int16_t* out_disp,
                     hipStream_t stream);

/* n independent pairs of the same shape in one launch sequence: pair i reads
 * left[i], right[i] and writes out_disp[i] (all device pointers; the pointer
 * arrays themselves are host memory read during the call).  n >= 1. */
int stereo_disparity_batch(stereo_ctx* ctx, const uint8_t* const* left,
                           const uint8_t* const* right, int n, int W, int H, int Dmax,
                           const stereo_params* params, int16_t* const* out_disp,
                           hipStream_t stream);

/* Tunes the launch geometry of the fused cost / aggregation / WTA kernel for
 * one shape: times candidate sizes of its disparity chunks (the default the
 * library's scheduling model picks, then ceil(D / k) for k = 1 .. min(D, 32))
 * on the caller's min(n, 8) pairs (device images as for
 * stereo_disparity_batch), five runs each, and keeps the fastest for later
 * calls on this context with the same W, H, Dmax, pair count and params;
 * results do not depend on it.  *chosen (may be NULL) receives the size in
 * disparities; sizes and times_ms (each may be NULL, max_times entries, host
 * memory) the candidates in trial order and their average milliseconds per
 * run, followed by 0 / -1 when room is left.  Synchronises the device; frees
 * and re-makes the shape's scratch. */
int stereo_autotune(stereo_ctx* ctx, const uint8_t* const* left, const uint8_t* const* right,
                    int n, int W, int H, int Dmax, const stereo_params* params, int* chosen,
                    int* sizes, float* times_ms, int max_times, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid allocation, harnesses that ban
 * hipMalloc): stereo_disparity for one pair, with every scratch plane carved
 * from one fixed array of STEREO_NOALLOC_MAX_BYTES per device instead of the
 * context's cached plans.  The array is allocated when the library's code is
 * loaded on the device (looked up once per device by stereo_create) and held
 * until the process ends; this call makes no device allocation, free or
 * memset (its set-up is a kernel, so it may be captured in a graph).
 *   Arguments, layouts and ownership as for stereo_disparity.  params->flags
 *   must not hold STEREO_F_KEEP_INTERMEDIATES or STEREO_F_STAGE_TIMING.
 *   Returns STEREO_EINVAL when the shape's scratch exceeds the array (the
 *   message gives both sizes; 1436x992 Dmax 145 needs about 46 MB,
 *   1920x1080 Dmax 256 about 37 MB), STEREO_EHIP when the array's address
 *   could not be found on this device.
 * Every call on one device uses the same array and each call re-initialises
 * it: calls whose work overlaps on a device (two streams, two contexts or
 * two threads) race and give wrong maps; order them on one stream. */
#define STEREO_NOALLOC_MAX_BYTES (64u << 20)
int stereo_disparity_noalloc(stereo_ctx* ctx, const uint8_t* left, const uint8_t* right, int W,
                             int H, int Dmax, const stereo_params* params, int16_t* out_disp,
                             hipStream_t stream);

/* Debug export of one plane of the last stereo_disparity call made with
 * STEREO_F_KEEP_INTERMEDIATES (pair 0 of a batch).  Copies into HOST memory
 * `dst`, which must hold at least `bytes` = the plane size; synchronises
 * `stream`.  Half-resolution planes are [Y][X] with X = ceil(W/2),
 * Y = ceil(H/2).  `d` (half-res disparity, 0..D-1) selects the plane of the
 * *_D items and is ignored otherwise. */
enum stereo_intermediate {
  STEREO_I_HALF_L = 1,    /* uint8  [Y][X] gray, downscaled (Eq. 2)                 */
  STEREO_I_HALF_R = 2,
  STEREO_I_CENSUS_L = 3,  /* uint8  [Y][X] 6-bit mini-census string                 */
  STEREO_I_CENSUS_R = 4,
  STEREO_I_ARMS_L = 5,    /* uint8  [Y][X][4] m, n, M, N                            */
  STEREO_I_ARMS_R = 6,
  STEREO_I_COST_L_D = 7,  /* uint16 [Y][X] C^L(x,y,d) (Eq. 3)                       */
  STEREO_I_COST_R_D = 8,  /* uint16 [Y][X] C^R(x,y,d) (Eq. 6)                       */
  STEREO_I_CAX_L_D = 9,   /* uint32 [Y][X] CA^L_x(x,y,d) (Eq. 7)                    */
  STEREO_I_CAX_R_D = 10,
  STEREO_I_CA_L_D = 11,   /* uint32 [Y][X] CA^L(x,y,d) (Eq. 8)                      */
  STEREO_I_CA_R_D = 12,
  STEREO_I_MINCOST_L = 13,/* uint32 [Y][X] min over d of CA^L                       */
  STEREO_I_MINCOST_R = 14,
  STEREO_I_DISP_L = 15,   /* int16  [Y][X] D^L (Eq. 9)                              */
  STEREO_I_DISP_R = 16,
  STEREO_I_GCP = 17,      /* uint8  [Y][X] 1 for ground control points (Eq. 10)     */
  STEREO_I_MEDIAN = 18,   /* int16  [Y][X] 3x3 median of D^L                        */
  STEREO_I_FILLED = 19,   /* int16  [Y][X] D+ after bilateral filling (Eq. 11)      */
  STEREO_I_LUT = 20       /* uint16 [263]: AD table [256] then census table [7]     */
};
int stereo_get_intermediate(stereo_ctx* ctx, int which, int d, void* dst, size_t bytes,
                            hipStream_t stream);

/* Device time of each stage, in the order of Sec. IV: 0 downscale (Step1),
 * 1 census + arms (Step2, Step4), 2 cost + x/y aggregation + WTA per
 * d-chunk (Step3, Step5), 3 minimum over the d-chunks (Step5), 4 cross-check
 * + median + filling (Step6, Step7), 5 upscale (Step8).  Sums, in milliseconds, over the calls made with
 * STEREO_F_STAGE_TIMING since the last reset, measured by HIP events
 * recorded on each call's stream around each stage's launch.  ms receives
 * STEREO_NUM_STAGES values; *calls (may be NULL) the number of calls.
 * Synchronises with the timed work.  reset != 0 clears the sums after
 * reading them. */
#define STEREO_NUM_STAGES 6
int stereo_stage_times(stereo_ctx* ctx, double* ms, int* calls, int reset);


/* ------------------------------------------------------------------------
 * Differentiable soft-argmin head.
 *
 * A float version of the left-based path that is smooth in the image
 * intensities and in the two cost weights, for training them by gradient
 * descent.  Per pair: gray (77 R + 150 G + 29 B) / 256 and the 3x3 mean at
 * (2x, 2y) in float (Eq. 2, unrounded); cost (Eq. 3-5 in robust form on the
 * 0..255 brightness scale)
 *   C(x,y,d) = (1 - exp(-255 |L(x,y) - R(x-d,y)| / lambda_AD))
 *            + (1 - exp(-H(x,y,d) / lambda_census)),   C = 2 for x - d < 0,
 * with H the census Hamming distance; the sum of C over the cross region of
 * (x,y) (Eq. 7-8) divided by its pixel count |S(x,y)|; and
 *   d_hat(x,y) = sum_d d p_d,  p = softmax over d in [0, D-1] of -mean / tau.
 * The census strings and the arms are those of the integer path on the
 * images quantised to floor(255 v + 1/2) (float32 arithmetic, clamped), and
 * are not differentiated.  Aggregation sums fixed-point costs (C scaled by
 * 2^k, rounded; k is the largest that keeps every cross-region sum below
 * 2^31, k = 18 for the default arms): |error of the mean| <= 2^-(k+1).
 *
 * Shared conventions: left/right are device float [n][H][W][3] RGB in [0,1],
 * contiguous per batch; half-resolution maps are device float [n][Y][X],
 * X = ceil(W/2), Y = ceil(H/2), D = ceil(Dmax/2); `lambdas` is a device
 * float[2] {lambda_AD, lambda_census}, both > 0.  Inputs must be finite.
 * Results are deterministic for fixed inputs.
 * ---------------------------------------------------------------------- */
typedef struct stereo_soft_params {
  uint32_t size;        /* must equal sizeof(stereo_soft_params)                     */
  float tau;            /* softmax temperature on the mean cost; >= 0.025            */
  int32_t color_delta;  /* delta of the frozen arms (Sec. III-C), 0..256             */
  int32_t arm_x;        /* per-side cap of m, n; 0..31                               */
  int32_t arm_y;        /* per-side cap of M, N; 0..63                               */
  int32_t slab;         /* disparities recomputed per backward slab; 0 = automatic   */
  uint32_t flags;       /* STEREO_SOFT_F_*                                           */
} stereo_soft_params;

/* stereo_soft_params.flags.  REUSE_FEATURES, for stereo_soft_backward: left
 * and right hold the same data as in the last stereo_soft_forward made on
 * this context and stream with these parameters (as in an autograd
 * backward, which keeps the forward's inputs unchanged); the backward then
 * reuses that forward's half images, census strings, arms and support sizes
 * instead of recomputing them.  The library checks that the last feature
 * pass on the plan was for the same two pointers and recomputes otherwise;
 * that the data behind them is unchanged is the caller's promise.  If that
 * forward also saved its weights (SAVE_WEIGHTS) for the same left, right and
 * lambdas pointers, the backward forms dL/dCA from them instead of
 * recomputing the aggregate; lambdas must then hold the forward's values too.
 * SAVE_WEIGHTS, for stereo_soft_forward: keep the softmax weight of every
 * pixel and disparity (n * X * Y * D floats of the context's scratch, in the
 * planes the backward's slabs use; ignored when one slab cannot hold all D)
 * for a following backward with REUSE_FEATURES.  Any later forward or
 * backward with other inputs on the same context, stream and parameters
 * replaces or drops them. */
#define STEREO_SOFT_F_REUSE_FEATURES 1u
#define STEREO_SOFT_F_SAVE_WEIGHTS 2u

/* tau = 0.1, delta = 13, arm caps 21 and 31, automatic slab, no flags. */
void stereo_soft_default_params(stereo_soft_params* p);

/* Forward of n pairs (1..64): d_hat [n][Y][X] (half-resolution disparity) and
 * lse2 [n][Y][X] = log2 of the softmax normaliser in the kernel's scaling,
 * which stereo_soft_backward needs; both device float, caller-owned. */
int stereo_soft_forward(stereo_ctx* ctx, const float* left, const float* right, int n, int W,
                        int H, int Dmax, const float* lambdas, const stereo_soft_params* params,
                        float* d_hat, float* lse2, hipStream_t stream);

/* Gradient of a scalar loss L given g_dhat = dL/dd_hat [n][Y][X] (device):
 * writes g_left, g_right (device float [n][H][W][3]) and g_lambdas (device
 * float[2]: dL/dlambda_AD, dL/dlambda_census), all overwritten, not
 * accumulated.  d_hat and lse2 are the forward's outputs for the same
 * inputs.  The adjoint recomputes the aggregate for slabs of disparities
 * and runs the window sums backward (difference arrays and prefix sums over
 * the frozen arms); no cost volume is stored.  Scratch grows with the slab:
 * 2 * n * X * Y * 4 bytes per disparity of a slab. */
int stereo_soft_backward(stereo_ctx* ctx, const float* left, const float* right, int n, int W,
                         int H, int Dmax, const float* lambdas, const stereo_soft_params* params,
                         const float* d_hat, const float* lse2, const float* g_dhat,
                         float* g_left, float* g_right, float* g_lambdas, hipStream_t stream);

/* L1 training loss of the head: the mean over the batch of, per pair, the
 * mean of |2 d_hat(x,y) - GT(2x,2y)| over pixels with nonocc(2x,2y) != 0
 * (0 for a pair without such pixels).  gt: device int16 [n][H][W]
 * full-resolution disparity; nonocc: device uint8 [n][H][W].  loss: device
 * float[1]. */
int stereo_soft_l1_loss(stereo_ctx* ctx, const float* d_hat, const int16_t* gt,
                        const uint8_t* nonocc, int n, int W, int H, float* loss,
                        hipStream_t stream);

/* Its gradient: g_dhat [n][Y][X] = gscale * dL/dd_hat, sign(0) taken as 0;
 * gscale is a device float[1] (the upstream gradient) or NULL for 1. */
int stereo_soft_l1_grad(stereo_ctx* ctx, const float* d_hat, const int16_t* gt,
                        const uint8_t* nonocc, int n, int W, int H, const float* gscale,
                        float* g_dhat, hipStream_t stream);


/* ------------------------------------------------------------------------
 * Serving runtime.
 *
 * A persistent worker thread serves frames of mixed shapes as they arrive
 * (the real-time use of the method, Sec. I and Sec. V).  It keeps, per shape,
 * batch size and slot, device buffers, a plan and a HIP graph of the whole
 * path resident.  Whenever a slot (a stream of its own) is free and the
 * frames in flight, counted by their cost-volume size X*Y*D*4 bytes, stay
 * within mem_budget (a frame alone in flight is always admitted), it admits
 * the oldest pending frame together with the next pending frames of the same
 * shape that the budget also admits, up to max_batch, rounded down to 1, 2,
 * 4 or 8 frames, as one batched launch of the path.  Launches in different
 * slots overlap on the device and never share scratch, and the pairs of a
 * batch are computed independently, so each result is bit-identical to
 * stereo_disparity's for the same frame.  Times are host steady-clock
 * milliseconds since the server was created.
 * ---------------------------------------------------------------------- */
typedef struct stereo_server stereo_server; /* opaque */

typedef struct stereo_server_config {
  uint32_t size;       /* must equal sizeof(stereo_server_config)               */
  int32_t device;      /* HIP device                                            */
  int32_t slots;       /* launches in flight at most, 1..16, one stream each    */
  uint64_t mem_budget; /* admission budget in bytes of X*Y*D*4; 0 = none        */
  stereo_params params;/* method parameters for every frame (flags ignored)     */
  int32_t max_batch;   /* frames of one shape merged into one launch, 1..8      */
} stereo_server_config;

typedef struct stereo_server_result {
  uint64_t tag;        /* the submit call's tag                                 */
  int32_t status;      /* 0 or a STEREO_E* code (the frame was not computed)    */
  int32_t slot;        /* slot that served it (-1 on error)                      */
  double t_submit_ms;  /* stereo_server_submit called                           */
  double t_admit_ms;   /* work enqueued on the slot's stream                    */
  double t_done_ms;    /* output copied to the caller's buffer                  */
  int32_t batch;       /* frames in the launch that computed it                 */
  int32_t reserved;    /* 0                                                      */
} stereo_server_result;

/* 4 slots, no budget, batches of up to 8 frames, the paper's parameters. */
void stereo_server_default_config(stereo_server_config* cfg);

int stereo_server_create(stereo_server** out, const stereo_server_config* cfg);

/* Queues one frame.  left, right: HOST uint8 [H][W][3] (page-locked memory
 * makes the upload asynchronous); out: HOST int16 [H][W] (page-locked memory
 * receives the map by DMA; pageable memory through pinned staging and a host
 * copy).  All three must stay valid until the frame's result has been
 * returned by stereo_server_poll.  Returns STEREO_EINVAL for bad arguments or after
 * destroy began. */
int stereo_server_submit(stereo_server* srv, const uint8_t* left, const uint8_t* right, int W,
                         int H, int Dmax, int16_t* out, uint64_t tag);

/* Moves up to max finished results into res, waiting up to timeout_ms for
 * the first one; returns how many (0 if none finished in time). */
int stereo_server_poll(stereo_server* srv, stereo_server_result* res, int max, int timeout_ms);

/* Text of the last error the worker met ("" if none). */
const char* stereo_server_last_error(stereo_server* srv);

/* Serves every queued frame, then frees everything.  NULL is a no-op.
 * Results not yet polled are dropped. */
void stereo_server_destroy(stereo_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* STEREO_H */
